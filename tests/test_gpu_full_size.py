"""GPU parity at the benchmark sizes, in the launch configuration the benchmark times.

The oracle cannot run the full workloads (hours of CPU), so each test runs the
GPU path on the full lattice with the benchmark's block width and kernel forms
and compares a sample the oracle computes in seconds: the first moments of
every realisation, a few block columns (columns are independent), one time
row.  Bar as in the other parity tests: normwise relative error <= 1e-10.
"""
import sys

import numpy as np
import pytest

import oracle as O
import paper_1705_01387_amd as P
from paper_1705_01387_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def err(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def oracle_dE(Hs):
    """DeltaE as the oracle derives it from its own H: 1.01 x the Gershgorin bound."""
    return 1.01 * O.gershgorin_bound(Hs)


@pytest.fixture(scope="module")
def honeycomb2M(gpu):
    w = I.workload_honeycomb(n_vectors=1)
    m, dE = w["model"], w["energy_max"]
    H = P.gpuqt_build_h_from_model(m, energy_max=dE)
    P.gpuqt_autotune(H, 1)
    Hs, V, XH = O.operators(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x)
    assert O.gershgorin_bound(Hs) <= dE          # the workload's DeltaE bounds the spectrum
    return w, H, Hs, V, XH


def test_full_size_honeycomb_bench_forms(honeycomb2M):
    """Honeycomb 2,000,000 orbitals with Peierls phases, one vector: DOS moments through the
    Hermitian form (the same buffer as phiL and phiR, as the benchmark calls it) and VAC rows
    t = 0 and t = 15 fs through the two-chain form, M = 64; the library picks its own term
    count, the oracle its own."""
    say("case: full-size honeycomb, DOS sym M=64 + VAC 2 rows M=64")
    w, H, Hs, V, _ = honeycomb2M
    dE = w["energy_max"]
    phi = w["phis"][0]
    d = dev(phi)
    mu = host(P.gpuqt_moments(H, d, d, 64))[0, 0]
    assert err(mu, O.dos_moments(Hs, phi, dE, 64)[:, 0]) < TOL
    dts = [float(w["dt"][0])] * 2
    vac = host(P.gpuqt_vac(H, d, dts, 64, 0))[:, 0, 0]
    ref = O.vac_moments(Hs, V, phi, dts, dE, 64)[:, :, 0]
    for k in range(2):
        assert err(vac[k], ref[k]) < TOL, k


def test_full_size_honeycomb_msd_row(honeycomb2M):
    """The benchmark's MSD on the 2,000,000-orbital honeycomb lattice: the first row (t = 15 fs,
    fused evolution + commutator series with the automatic term count, about 275 terms) with
    M = 64, against the oracle's [X, U] recurrence and separate evolutions."""
    say("case: full-size honeycomb, MSD row 1 M=64")
    w, H, Hs, _, XH = honeycomb2M
    dE = w["energy_max"]
    phi = w["phis"][0]
    dt = float(w["dt"][0])
    assert P.gpuqt_auto_terms(dE * dt) == O.auto_terms(dE * dt)
    got = host(P.gpuqt_msd(H, dev(phi), [dt], 64, 0))[0, 0, 0]
    ref = O.msd_moments(Hs, XH, phi, [dt], dE, 64)[0, :, 0]
    assert err(got, ref) < TOL


def test_long_chain_honeycomb_M3000(gpu):
    """Long recurrences, M = 3000 as in the benchmark, on a mid-size honeycomb lattice with
    Peierls phases in the value-table layout (60 x 40 cells, flux 1/480): DOS moments (Hermitian
    form), the VAC rows at t = 0 and t = 15 fs (two-chain form, automatic term count) and the
    first MSD row, against the oracle's plain recurrences."""
    say("case: long chain honeycomb 60x40 M=3000")
    m = I.honeycomb(60, 40, t=-2.7, flux=1.0 / 480.0, W=2.0, seed=2101)
    Hs, V, XH = O.operators(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x)
    dE = oracle_dE(Hs)
    H = P.gpuqt_build_h_from_model(m, energy_max=dE)
    assert H.info.hop_mode == 3
    phi = I.random_phase(m.n, 1, 2102)
    d = dev(phi)
    M = 3000
    mu = host(P.gpuqt_moments(H, d, d, M))[0, 0]
    assert err(mu, O.dos_moments(Hs, phi, dE, M)[:, 0]) < TOL
    dt = 15.0 / I.HBAR_EV_FS
    vac = host(P.gpuqt_vac(H, d, [dt, dt], M, 0))[:, 0, 0]
    rv = O.vac_moments(Hs, V, phi, [dt, dt], dE, M)[:, :, 0]
    for k in range(2):
        assert err(vac[k], rv[k]) < TOL, k
    msd = host(P.gpuqt_msd(H, d, [dt], M, 0))[0, 0, 0]
    assert err(msd, O.msd_moments(Hs, XH, phi, [dt], dE, M)[0, :, 0]) < TOL


def test_full_size_cubic_B4_sampled(gpu):
    """Cubic 200^3 = 8,000,000 orbitals, W = 16, block of 4: DOS moments (Hermitian form) and
    the MSD row at t = dt = 2 (fused evolution + commutator, automatic term count) on the whole
    block, M = 64; the oracle checks columns 0 and 3.  Both periodic-box kernels are pinned
    (variant bits 26 and 27): at this size their work items go several rounds over the
    workgroups, in runs of planes that meet inside the box."""
    say("case: full-size cubic 200^3 W=16 B=4, box kernels, DOS M=64 + MSD 1 row M=64")
    w = I.workload_cubic(L=200, W=16.0, B=4)
    m, dE = w["model"], w["energy_max"]
    H = P.gpuqt_build_h_from_model(m, energy_max=dE)
    assert tuple(H.info.box) == (200, 200, 200) and H.info.box_msd == 1
    P.gpuqt_set_variant(H, (1 << 26) | (1 << 27))
    assert H.info.hop_mode == 0 and H.info.uniform_width == 6
    Hs, _, XH = O.operators(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x)
    assert O.gershgorin_bound(Hs) <= dE
    phi = w["phi"]
    d = dev(phi)
    mu = host(P.gpuqt_moments(H, d, d, 64))[0]                # [B, M]
    msd = host(P.gpuqt_msd(H, d, [2.0], 64, 0))[0, 0]           # [B, M]
    del d
    for b in (0, 3):
        col = phi[:, b:b + 1]
        assert err(mu[b], O.dos_moments(Hs, col, dE, 64)[:, 0]) < TOL, b
        assert err(msd[b], O.msd_moments(Hs, XH, col, [2.0], dE, 64)[0, :, 0]) < TOL, b


@pytest.mark.parametrize("W", [8.0, 24.0])
def test_full_size_cubic_other_disorder(gpu, W):
    """Cubic 200^3 at the two other disorder strengths of the workload, W = 8 and W = 24
    (DeltaE = 1.01 (6 + W / 2)), block of 4: the terms per step are max(60, automatic) (at
    W = 24, DeltaE dt = 36.4 needs 74 terms for machine precision), computed by the oracle and
    given to both sides; DOS moments and the first MSD row, M = 64, column 0 against the oracle."""
    say(f"case: full-size cubic 200^3 W={W} B=4, DOS M=64 + MSD 1 row M=64")
    w = I.workload_cubic(L=200, W=W, B=4)
    m, dE = w["model"], w["energy_max"]
    Hs, _, XH = O.operators(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x)
    assert O.gershgorin_bound(Hs) <= dE
    Np = max(60, O.auto_terms(dE * 2.0))
    assert Np == (74 if W == 24.0 else 60)
    H = P.gpuqt_build_h_from_model(m, energy_max=dE)
    P.gpuqt_autotune(H, 4)
    phi = w["phi"]
    d = dev(phi)
    mu = host(P.gpuqt_moments(H, d, d, 64))[0]
    msd = host(P.gpuqt_msd(H, d, [2.0], 64, Np))[0, 0]
    del d
    col = phi[:, :1]
    assert err(mu[0], O.dos_moments(Hs, col, dE, 64)[:, 0]) < TOL
    assert err(msd[0], O.msd_moments(Hs, XH, col, [2.0], dE, 64, Np)[0, :, 0]) < TOL


def test_full_size_batched_B16_sampled(gpu):
    """Eight square realisations 200^2 .. 2000^2 (8,255,182 orbitals) with per-realisation
    DeltaE, block of 16, one launch per step: the first 64 moments of every realisation for
    columns 0 and 15, through the sheet stencil kernel (variant bit 26; every segment is a
    periodic square)."""
    say("case: full-size batched 8 segments B=16, sheet kernel, DOS M=64")
    w = I.workload_batched(B=16, M=64)
    mods = w["models"]
    cat = I.concat_segments(mods)
    offs = np.cumsum([0] + [mm.n for mm in mods])
    H = P.gpuqt_build_h(cat.nn, cat.nbr, cat.hop, cat.onsite, cat.x, 0.0, cat.volume, 0.0,
                        seg_offsets=offs, seg_energy_max=w["seg_energy_max"],
                        seg_length_x=[mm.length_x for mm in mods])
    assert H.info.sheets == 1
    P.gpuqt_set_variant(H, 1 << 26)
    assert H.info.kernel_variant == 1 << 26
    d = dev(w["phi"])
    mu = host(P.gpuqt_moments(H, d, d, 64))                    # [seg, B, M]
    del d
    for s, mm in enumerate(mods):
        Hs, _, _ = O.operators(mm.nn, mm.nbr, mm.hop, mm.onsite, mm.x, mm.length_x)
        for b in (0, 15):
            col = w["phi"][offs[s]:offs[s + 1], b:b + 1]
            ref = O.dos_moments(Hs, col, float(w["seg_energy_max"][s]), 64)[:, 0]
            assert err(mu[s, b], ref) < TOL, (s, b)


def test_full_size_paper_examples_sampled(gpu):
    """The paper's examples at full size: 2000^2 square (DOS + the first two VAC rows) and the
    4,000,000-site chain with its two vectors as one block (DOS + the first two MSD rows of
    the non-uniform steps), M = 64, against the oracle."""
    say("case: full-size paper examples, M=64")
    for w, kind in ((I.workload_paper_diffusive(), "vac"), (I.workload_paper_localized(), "msd")):
        m, dE = w["model"], w["energy_max"]
        H = P.gpuqt_build_h_from_model(m, energy_max=dE)
        Hs, V, XH = O.operators(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x)
        phi = w["phi"]
        d = dev(phi)
        dts = list(w["dt"][:2])
        mu = host(P.gpuqt_moments(H, d, d, 64))[0]                       # [B, M]
        if kind == "vac":
            got = host(P.gpuqt_vac(H, d, dts, 64))[:, 0]                  # [2, B, M]
            ref = O.vac_moments(Hs, V, phi, dts, dE, 64)                  # [2, M, B]
        else:
            got = host(P.gpuqt_msd(H, d, dts, 64))[:, 0]
            ref = O.msd_moments(Hs, XH, phi, dts, dE, 64)
        assert err(mu, O.dos_moments(Hs, phi, dE, 64).T) < TOL
        for k in range(2):
            assert err(got[k], ref[k].T) < TOL, (w["name"], k)
