"""GPU parity of the per-entry hopping gradients (every stored H_ij an independent complex
number), their Hermitian tie, and the class-scale gradients dL/ds_c at scales other than 1
(0 included), against the oracle's reverse recurrence with every vector stored.
Bar: normwise 1e-10; the tie (one addition per element) bit for bit."""
import numpy as np
import pytest

import oracle as O
import paper_1705_01387_amd as P
from oracle.adjoint import class_parts, velocity_class_parts
from paper_1705_01387_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print(*a, flush=True)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def err(got, ref):
    return float(np.max(np.abs(np.asarray(got) - np.asarray(ref))) / max(np.max(np.abs(ref)), 1e-300))


def oracle_dE(Hs):
    return 1.01 * O.gershgorin_bound(Hs)


# (model, no_dictionary, expected storage mode: 0 uniform, 1 real, 2 complex, 3 table)
CASES = {
    "cubic_uniform": (lambda: I.cubic(7, W=2.0, seed=61), False, 0),
    "square_open_padded": (lambda: I.square(15, 11, W=1.5, seed=62, periodic_x=False), False, 0),
    "square_bond_real": (lambda: I.bond_disorder(I.square(13, 11, W=1.0, seed=63), 0.3, 64), True, 1),
    "square_nnn_bond_table": (lambda: I.bond_disorder(I.square(12, 10, t1=-1.0, t2=-0.2, W=1.0, seed=65), 0.3, 66),
                              False, 3),
    "honeycomb_flux_complex": (lambda: I.bond_disorder(I.honeycomb(10, 8, flux=1.0 / 80.0, W=1.0, seed=67), 0.2, 68,
                                                       0.3), True, 2),
    "honeycomb_flux_table": (lambda: I.honeycomb(10, 8, flux=1.0 / 80.0, W=1.0, seed=69), False, 3),
    # 3072 rows: 48 slices, several workgroups
    "square64x48_bond_table": (lambda: I.bond_disorder(I.square(64, 48, W=1.0, seed=82), 0.3, 83), False, 3),
}


def setup(name, scales=None):
    """Handle, oracle operators at the given class scales, and the build-time class parts."""
    mk, nodict, mode = CASES[name]
    m = mk()
    H0 = I.dense_hop(m)
    hop = H0 if scales is None else H0 * np.asarray(scales)[m.hop_class if m.hop_class is not None else 0]
    Hs, V, _ = O.operators(m.nn, m.nbr, hop, m.onsite, m.x, m.length_x)
    H1, _, _ = O.operators(m.nn, m.nbr, H0, m.onsite, m.x, m.length_x)
    dE = oracle_dE(H1)                       # DeltaE fixed at the build-time spectrum
    H = P.gpuqt_build_h_from_model(m, energy_max=dE, no_dictionary=nodict)
    assert int(H.info.hop_mode) == mode, (name, int(H.info.hop_mode))
    if scales is not None:
        import torch
        P.gpuqt_update_h_values(H, None, np.asarray(scales, dtype=np.float64))
    return m, H, Hs, V, dE


def zeros_entries(H):
    import torch
    return torch.zeros((H.n, int(H.info.max_nn), 2), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("B,M,stride", [(1, 40, 0), (2, 33, 5), (1, 2, 1), (2, 41, 1), (1, 3, 0)])
@pytest.mark.parametrize("same", [False, True])
def test_moments_entry_gradient(gpu, name, B, M, stride, same):
    """Untied per-entry gradients (and the on-site and class gradients of the same call) at
    every checkpoint stride, phiL != phiR and phiL = phiR (the same tensor); padding slots
    stay zero; the tied values match the oracle's tie of its own untied values."""
    import torch
    say(f"case: entry gradient {name} B={B} M={M} stride={stride} same={same}")
    m, H, Hs, _, dE = setup(name)
    n_class = m.n_class
    parts = class_parts(m.nn, m.nbr, m.hop, m.hop_class, n_class)
    phiL = I.random_phase(m.n, B, 70)
    phiR = phiL if same else I.random_phase(m.n, B, 71)
    w = np.random.default_rng(72).normal(size=(1, B, M))
    dL = dev(phiL)
    dR = dL if same else dev(phiR)
    gH = zeros_entries(H)
    gU, gC, _ = P.gpuqt_moments_backward(H, dL, dR, dev(w), ckpt_stride=stride, grad_hop=gH,
                                         grad_class=torch.zeros(n_class, dtype=torch.float64, device="cuda"))
    ent = O.entry_list(m.nn, m.nbr)
    rH = np.zeros((m.n * m.max_nn, 2))
    rU, rC = O.moments_gradient(Hs, phiL, phiR, dE, w[0].T, parts, ent, rH)
    rH = rH.reshape(m.n, m.max_nn, 2)
    got = host(gH)
    assert err(got, rH) < TOL
    assert err(host(gU), rU) < TOL and err(host(gC), rC) < TOL
    pad = np.arange(m.max_nn)[None, :] >= m.nn[:, None]
    assert np.all(got[pad] == 0.0)
    tied = host(P.gpuqt_tie_entry_gradient(H, gH))
    assert err(tied, O.tie_hermitian(m.nn, m.nbr, rH)) < TOL


@pytest.mark.parametrize("name", list(CASES))
def test_tie_matches_oracle(gpu, name):
    """The tie of seeded values (padding slots included) equals the oracle's, bit for bit; the
    entry point refuses an in-place tie."""
    say(f"case: tie {name}")
    m, H, _, _, _ = setup(name)
    g = np.random.default_rng(73).normal(size=(m.n, m.max_nn, 2))
    out = host(P.gpuqt_tie_entry_gradient(H, dev(g)))
    ref = O.tie_hermitian(m.nn, m.nbr, g)
    assert np.array_equal(out, ref)
    with pytest.raises(P.GpuqtError):
        d = dev(g)
        P.gpuqt_tie_entry_gradient(H, d, out=d)


VAC_NAMES = ["square_nnn_bond_table", "honeycomb_flux_complex", "square_open_padded", "cubic_uniform"]


@pytest.mark.parametrize("name", VAC_NAMES)
@pytest.mark.parametrize("B,ckpt,time_stride", [(1, 0, 1), (2, 1, 1), (2, 0, 2), (1, 1, 3)])
def test_vac_entry_gradient(gpu, name, B, ckpt, time_stride):
    """VAC rows: per-entry gradients including the velocity's share (V_ij = i dx_ij H_ij), with
    every state kept or time checkpoints, against the oracle."""
    import torch
    say(f"case: VAC entry gradient {name} B={B} ckpt={ckpt} time_stride={time_stride}")
    m, H, Hs, V, dE = setup(name)
    n_class = m.n_class
    Hc = class_parts(m.nn, m.nbr, m.hop, m.hop_class, n_class)
    Vc = velocity_class_parts(m.nn, m.nbr, m.hop, m.hop_class, n_class, m.x, m.length_x)
    phi = I.random_phase(m.n, B, 74)
    dts = [0.4, 1.1, 0.0, 0.6, 0.9]
    M = 28
    w = np.random.default_rng(75).normal(size=(len(dts), 1, B, M))
    gH = zeros_entries(H)
    gU, gC = P.gpuqt_vac_backward(H, dev(phi), dts, dev(w), ckpt_stride=ckpt, time_stride=time_stride,
                                  grad_class=torch.zeros(n_class, dtype=torch.float64, device="cuda"), grad_hop=gH)
    ent = O.entry_list(m.nn, m.nbr, m.x, m.length_x)
    rH = np.zeros((m.n * m.max_nn, 2))
    rU, rC = O.vac_gradient(Hs, V, phi, dts, dE, M, np.transpose(w[:, 0], (0, 2, 1)), 0, Hc, Vc, ent, rH)
    assert err(host(gH), rH.reshape(m.n, m.max_nn, 2)) < TOL
    assert err(host(gU), rU) < TOL and err(host(gC), rC) < TOL


SCALES = {
    "square_nnn_bond_table": [[0.6, 1.3], [1.0, 0.0], [0.0, 0.0]],
    "square_bond_real": [[0.7], [0.0]],
    "cubic_uniform": [[0.5], [0.0]],
    "honeycomb_flux_complex": [[0.8], [0.0]],
}


@pytest.mark.parametrize("name,scales", [(k, s) for k, v in SCALES.items() for s in v])
@pytest.mark.parametrize("stride", [0, 1])
def test_class_gradient_is_d_scale(gpu, name, scales, stride):
    """After gpuqt_update_h_values(scales), grad_class is dL/ds_c: the oracle's gradient for
    H(s) = sum_c s_c H_c(build time), with the build-time class parts; finite at s_c = 0."""
    import torch
    say(f"case: class scales {name} {scales} stride={stride}")
    m, H, Hs, _, dE = setup(name, scales)
    parts = class_parts(m.nn, m.nbr, I.dense_hop(m), m.hop_class, m.n_class)
    B, M = 2, 36
    phi = I.random_phase(m.n, B, 76)
    d = dev(phi)
    w = np.random.default_rng(77).normal(size=(1, B, M))
    gU, gC, _ = P.gpuqt_moments_backward(H, d, d, dev(w), ckpt_stride=stride,
                                         grad_class=torch.zeros(m.n_class, dtype=torch.float64, device="cuda"))
    rU, rC = O.moments_gradient(Hs, phi, phi, dE, w[0].T, parts)
    assert np.all(np.isfinite(host(gC)))
    assert err(host(gU), rU) < TOL and err(host(gC), rC) < TOL


@pytest.mark.parametrize("scales", [[0.8, 1.1], [0.0, 1.0]])
def test_vac_class_gradient_is_d_scale(gpu, scales):
    """The VAC class gradient (moments, evolutions and the velocity V = i dx H, whose class-c
    part scales with s_c) at scales other than 1."""
    import torch
    name = "square_nnn_bond_table"
    say(f"case: VAC class scales {scales}")
    m, H, Hs, V, dE = setup(name, scales)
    H0 = I.dense_hop(m)
    Hc = class_parts(m.nn, m.nbr, H0, m.hop_class, m.n_class)
    Vc = velocity_class_parts(m.nn, m.nbr, H0, m.hop_class, m.n_class, m.x, m.length_x)
    B, M = 1, 24
    phi = I.random_phase(m.n, B, 78)
    dts = [0.5, 0.8, 0.3]
    w = np.random.default_rng(79).normal(size=(len(dts), 1, B, M))
    gU, gC = P.gpuqt_vac_backward(H, dev(phi), dts, dev(w), ckpt_stride=0, time_stride=1,
                                  grad_class=torch.zeros(m.n_class, dtype=torch.float64, device="cuda"))
    rU, rC = O.vac_gradient(Hs, V, phi, dts, dE, M, np.transpose(w[:, 0], (0, 2, 1)), 0, Hc, Vc)
    assert err(host(gU), rU) < TOL and err(host(gC), rC) < TOL


def test_autograd_at_zero_scale(gpu):
    """torch.autograd through the moments at a class scale of 0: finite, and equal to the
    oracle's dL/ds_c there."""
    import torch
    from paper_1705_01387_amd import autograd as AG
    say("case: autograd at scale 0")
    name = "square_nnn_bond_table"
    m, H, _, _, dE = setup(name)
    scales = np.array([1.0, 0.0])
    H0 = I.dense_hop(m)
    Hs, _, _ = O.operators(m.nn, m.nbr, H0 * scales[m.hop_class], m.onsite, m.x, m.length_x)
    parts = class_parts(m.nn, m.nbr, H0, m.hop_class, m.n_class)
    phi = I.random_phase(m.n, 1, 80)
    M = 30
    wv = np.random.default_rng(81).normal(size=(1, 1, M))
    U = torch.tensor(m.onsite, dtype=torch.float64, device="cuda", requires_grad=True)
    s = torch.tensor(scales, dtype=torch.float64, requires_grad=True)
    mu = AG.Moments.apply(U, s, H, dev(phi), M)
    (mu * dev(wv)).sum().backward()
    rU, rC = O.moments_gradient(Hs, phi, phi, dE, wv[0].T, parts)
    assert np.all(np.isfinite(s.grad.numpy()))
    assert err(s.grad.numpy(), rC) < TOL and err(host(U.grad), rU) < TOL


@pytest.mark.parametrize("kind", ["moments", "vac"])
def test_entry_gradient_segments(gpu, kind):
    """Two realisations of different lattices (4 and 3 neighbour slots, real and complex
    hoppings, their own DeltaE) in one handle: each segment's per-entry gradients equal the
    oracle's for that segment alone, placed at its rows; the other segment's slots and the
    padding stay zero."""
    import torch
    say(f"case: entry gradients on two segments ({kind})")
    mods = [I.bond_disorder(I.square(9, 8, W=1.0, seed=84), 0.3, 85),
            I.bond_disorder(I.honeycomb(6, 4, flux=1.0 / 24.0, W=1.0, seed=86), 0.2, 87, 0.3)]
    cat = I.concat_segments(mods)
    offs = np.cumsum([0] + [mm.n for mm in mods])
    ops = [O.operators(mm.nn, mm.nbr, mm.hop, mm.onsite, mm.x, mm.length_x) for mm in mods]
    dEs = np.array([oracle_dE(o[0]) for o in ops])
    H = P.gpuqt_build_h(cat.nn, cat.nbr, cat.hop, cat.onsite, cat.x, 0.0, cat.volume, 0.0,
                        seg_offsets=offs, seg_energy_max=dEs, seg_length_x=[mm.length_x for mm in mods])
    B, M = 2, 30
    phi = np.concatenate([I.random_phase(mm.n, B, 88 + s) for s, mm in enumerate(mods)], axis=0)
    gH = zeros_entries(H)
    ref = np.zeros((cat.n, cat.max_nn, 2))
    if kind == "moments":
        w = np.random.default_rng(90).normal(size=(2, B, M))
        P.gpuqt_moments_backward(H, dev(phi), dev(phi), dev(w), ckpt_stride=0, grad_hop=gH)
    else:
        dts = [0.5, 0.9, 0.2]
        w = np.random.default_rng(91).normal(size=(len(dts), 2, B, M))
        P.gpuqt_vac_backward(H, dev(phi), dts, dev(w), ckpt_stride=0, time_stride=1, grad_hop=gH)
    for s, mm in enumerate(mods):
        Hs, V, _ = ops[s]
        ph = phi[offs[s]:offs[s + 1]]
        rs = np.zeros((mm.n * mm.max_nn, 2))
        if kind == "moments":
            O.moments_gradient(Hs, ph, ph, dEs[s], w[s].T, (), O.entry_list(mm.nn, mm.nbr), rs)
        else:
            O.vac_gradient(Hs, V, ph, dts, dEs[s], M, np.transpose(w[:, s], (0, 2, 1)), 0, (), (),
                           O.entry_list(mm.nn, mm.nbr, mm.x, mm.length_x), rs)
        ref[offs[s]:offs[s + 1], :mm.max_nn] = rs.reshape(mm.n, mm.max_nn, 2)
    got = host(gH)
    for s, mm in enumerate(mods):
        sl = slice(offs[s], offs[s + 1])
        assert err(got[sl], ref[sl]) < TOL, s
    assert np.all(got[offs[1]:, mods[1].max_nn:] == 0.0)
