"""The periodic-box stencils (kernel variant bits 26 and 27): detection of periodic simple
cubic boxes and of segments that are all periodic squares from the neighbour list, and
moments (and MSD rows) through the box and sheet stencil kernels against the oracle for every
block width they serve, shapes that do and do not fill their tiles, shuffled neighbour slots,
uneven segments and several workgroup counts.  Bar: normwise 1e-10."""
import numpy as np
import pytest

import oracle as O
import paper_1705_01387_amd as P
from paper_1705_01387_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = 1e-10
BOX = 1 << 26


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


def test_box_detection(gpu):
    say("case: periodic box detection")
    assert tuple(P.gpuqt_build_h_from_model(I.cubic(11, W=1.0, seed=1)).info.box) == (11, 11, 11)
    assert tuple(P.gpuqt_build_h_from_model(I.box(13, 9, 7, W=1.0, seed=2)).info.box) == (13, 9, 7)
    assert tuple(P.gpuqt_build_h_from_model(I.box(5, 4, 3, slot_seed=3)).info.box) == (5, 4, 3)
    # not a box: bond disorder (not one hopping), a square lattice, a box of side 2, two segments
    assert tuple(P.gpuqt_build_h_from_model(I.bond_disorder(I.cubic(5), 0.2, 4)).info.box) == (0, 0, 0)
    assert tuple(P.gpuqt_build_h_from_model(I.square(12, 10)).info.box) == (0, 0, 0)
    assert tuple(P.gpuqt_build_h_from_model(I.box(6, 5, 2)).info.box) == (0, 0, 0)
    mods = [I.cubic(4), I.cubic(4)]
    cat = I.concat_segments(mods)
    H = P.gpuqt_build_h(cat.nn, cat.nbr, cat.hop, cat.onsite, cat.x, 0.0, cat.volume, 0.0,
                        seg_offsets=[0, 64, 128], seg_length_x=[4.0, 4.0])
    assert tuple(H.info.box) == (0, 0, 0)


BOXES = {
    "cubic11": lambda: I.cubic(11, W=4.0, seed=11),
    "box19x13x10_shuffled": lambda: I.box(19, 13, 10, W=3.0, seed=12, slot_seed=13),
    "box3x5x4": lambda: I.box(3, 5, 4, W=2.0, seed=14),
    "box17x9x33": lambda: I.box(17, 9, 33, W=5.0, seed=15),
}


@pytest.mark.parametrize("name", list(BOXES))
@pytest.mark.parametrize("B", [2, 4, 8, 16])
def test_box_moments_match_oracle(gpu, name, B):
    """Hermitian moment sets (the step the box kernel runs) with the box bit on, at M = 2, 3
    and 65, and at three per-CU caps (different workgroup counts, so different work item
    rounds); the two-chain moments of phiL != phiR on the same handle stay right."""
    say(f"case: box moments {name} B={B}")
    m = BOXES[name]()
    Hs, _, _ = O.operators(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x)
    dE = oracle_dE(Hs)
    H = P.gpuqt_build_h_from_model(m, energy_max=dE)
    assert H.info.box[0] > 0
    phi = I.random_phase(m.n, B, 16)
    psi = I.random_phase(m.n, B, 17)
    d = dev(phi)
    for cap in (0, 1, 2, 5):
        P.gpuqt_set_variant(H, BOX | (cap << 2))
        assert H.info.kernel_variant == BOX | (cap << 2)
        for M in (2, 3, 65):
            ref = O.chebyshev_moments(Hs / dE, phi, phi, M).T
            assert err(host(P.gpuqt_moments(H, d, d, M))[0], ref) < TOL, (cap, M)
    ref2 = O.chebyshev_moments(Hs / dE, phi, psi, 40).T
    assert err(host(P.gpuqt_moments(H, d, dev(psi), 40))[0], ref2) < TOL


def test_box_msd_rows(gpu):
    """An MSD series on a box with the box bit: its rows' moment sets (Hermitian, chi) go
    through the box kernel."""
    say("case: box MSD rows B=4")
    m = I.box(14, 11, 9, W=3.0, seed=18)
    Hs, _, XH = O.operators(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x)
    dE = oracle_dE(Hs)
    H = P.gpuqt_build_h_from_model(m, energy_max=dE)
    P.gpuqt_set_variant(H, BOX)
    phi = I.random_phase(m.n, 4, 19)
    dts = [0.6, 1.1]
    got = host(P.gpuqt_msd(H, dev(phi), dts, 48))[:, 0]
    ref = O.msd_moments(Hs, XH, phi, dts, dE, 48)
    for k in range(len(dts)):
        assert err(got[k], ref[k].T) < TOL, k


def test_box_msd_detection(gpu):
    """box_msd needs +-dx on the x neighbours and 0 on the others: lattice positions give it,
    positions with a per-site jitter do not (the Hermitian box step still applies)."""
    say("case: box MSD detection")
    m = I.box(9, 7, 5)
    assert P.gpuqt_build_h_from_model(m).info.box_msd == 1
    m.x = m.x + 0.01 * np.random.default_rng(20).random(m.n)
    H = P.gpuqt_build_h_from_model(m)
    assert tuple(H.info.box) == (9, 7, 5) and H.info.box_msd == 0


@pytest.mark.parametrize("name", ["cubic11", "box19x13x10_shuffled", "box3x5x4", "box17x9x33"])
@pytest.mark.parametrize("B", [2, 4, 8, 16])
def test_box_msd_term_matches_oracle(gpu, name, B):
    """MSD rows with both box kernels (bits 26 and 27) at two caps: the fused evolution +
    commutator series runs as the box stencil, the rows' moment sets as the Hermitian one."""
    say(f"case: box MSD term {name} B={B}")
    m = BOXES[name]()
    Hs, _, XH = O.operators(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x)
    dE = oracle_dE(Hs)
    H = P.gpuqt_build_h_from_model(m, energy_max=dE)
    assert H.info.box_msd == 1
    phi = I.random_phase(m.n, B, 21)
    dts = [0.7, 1.3]
    ref = O.msd_moments(Hs, XH, phi, dts, dE, 24)
    for cap in (0, 1, 3):
        P.gpuqt_set_variant(H, BOX | (1 << 27) | (cap << 2))
        assert H.info.kernel_variant == BOX | (1 << 27) | (cap << 2)
        got = host(P.gpuqt_msd(H, dev(phi), dts, 24))[:, 0]
        for k in range(len(dts)):
            assert err(got[k], ref[k].T) < TOL, (cap, k)


def _segments(mods, dEs):
    cat = I.concat_segments(mods)
    offs = np.cumsum([0] + [mm.n for mm in mods])
    H = P.gpuqt_build_h(cat.nn, cat.nbr, cat.hop, cat.onsite, cat.x, 0.0, cat.volume, 0.0,
                        seg_offsets=offs, seg_energy_max=dEs, seg_length_x=[mm.length_x for mm in mods])
    return H, offs


def test_sheet_detection(gpu):
    """Every segment a periodic square in natural order with four neighbours: sheets = 1; a
    segment open in x, a cubic box, a square with next-nearest neighbours or a chain: 0."""
    say("case: periodic square (sheet) detection")
    sq = [I.square(13, 9, W=1.0, seed=40), I.square(5, 31, W=2.0, seed=41), I.square(3, 3, seed=42)]
    assert P.gpuqt_build_h_from_model(sq[0]).info.sheets == 1
    H, _ = _segments(sq, [6.0, 6.5, 4.5])
    assert H.info.sheets == 1 and tuple(H.info.box) == (0, 0, 0)
    H, _ = _segments([sq[0], I.square(13, 9, W=1.0, seed=43, periodic_x=False)], [6.0, 6.0])
    assert H.info.sheets == 0
    assert P.gpuqt_build_h_from_model(I.square(12, 10, t2=-0.3, seed=44)).info.sheets == 0
    assert P.gpuqt_build_h_from_model(I.cubic(7, W=1.0, seed=45)).info.sheets == 0
    assert P.gpuqt_build_h_from_model(I.chain(64, W=1.0, seed=46)).info.sheets == 0


SHEETS = {
    # strips narrower and wider than a tile (256 / B cells), ragged tails, a segment of
    # many rows (runs of rows meet inside it), rectangles both ways, the smallest square
    "uneven": lambda: [I.square(37, 5, W=2.0, seed=50), I.square(5, 41, W=3.0, seed=51),
                       I.square(300, 33, W=1.0, seed=52), I.square(3, 3, W=0.5, seed=53),
                       I.square(20, 200, W=2.5, seed=54)],
    "one": lambda: [I.square(70, 70, W=4.0, seed=55)],
}


@pytest.mark.parametrize("name", list(SHEETS))
@pytest.mark.parametrize("B", [2, 4, 8, 16])
def test_sheet_moments_match_oracle(gpu, name, B):
    """Hermitian moment sets through the sheet kernel (bit 26) on segments of periodic
    squares with per-segment DeltaE, at M = 2, 3 and 65 and four per-CU caps (different
    workgroups per segment, so different work item rounds and run lengths), each segment
    against the oracle."""
    say(f"case: sheet moments {name} B={B}")
    mods = SHEETS[name]()
    ops = [O.operators(mm.nn, mm.nbr, mm.hop, mm.onsite, mm.x, mm.length_x)[0] for mm in mods]
    dEs = [oracle_dE(Hs) for Hs in ops]
    H, offs = _segments(mods, dEs)
    assert H.info.sheets == 1
    phi = np.concatenate([I.random_phase(mm.n, B, 60 + s) for s, mm in enumerate(mods)], axis=0)
    d = dev(phi)
    for cap in (0, 1, 2, 5):
        P.gpuqt_set_variant(H, BOX | (cap << 2))
        assert H.info.kernel_variant == BOX | (cap << 2)
        for M in (2, 3, 65):
            mu = host(P.gpuqt_moments(H, d, d, M))                # [seg, B, M]
            for s, Hs in enumerate(ops):
                ph = phi[offs[s]:offs[s + 1]]
                ref = O.chebyshev_moments(Hs / dEs[s], ph, ph, M).T
                assert err(mu[s], ref) < TOL, (cap, M, s)


def test_sheet_autotune(gpu):
    """The autotuner on segments of periodic squares times the sheet kernel (times_us[6]) and
    whatever it keeps gives the oracle's moments; with bit 26 in the kept code the sheet
    kernel ran them."""
    say("case: autotune on sheets B=4")
    mods = SHEETS["uneven"]()
    ops = [O.operators(mm.nn, mm.nbr, mm.hop, mm.onsite, mm.x, mm.length_x)[0] for mm in mods]
    dEs = [oracle_dE(Hs) for Hs in ops]
    H, offs = _segments(mods, dEs)
    assert H.info.sheets == 1
    t = P.gpuqt_autotune(H, 4)
    assert t[6] > 0
    code = H.info.kernel_variant
    say(f"kept code {code}, sheet bit {(code >> 26) & 1}")
    phi = np.concatenate([I.random_phase(mm.n, 4, 80 + s) for s, mm in enumerate(mods)], axis=0)
    mu = host(P.gpuqt_moments(H, dev(phi), dev(phi), 40))
    for s, Hs in enumerate(ops):
        ph = phi[offs[s]:offs[s + 1]]
        assert err(mu[s], O.chebyshev_moments(Hs / dEs[s], ph, ph, 40).T) < TOL, s
