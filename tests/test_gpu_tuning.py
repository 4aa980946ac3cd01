"""Tuning entry points on the GPU: every slice height the tuner may pick gives oracle-exact
results, the measured slice-height build, the variant cache (miss, then hit with the same
code), the block-width choice, and the plain one-moment-per-step recurrence."""
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


LATTICES = {
    # open x: rows of different widths, so slices are padded (runtime width path)
    "square_open45x37": lambda: I.square(45, 37, W=1.5, seed=111, periodic_x=False),
    # value table with Peierls phases (fixed width 3)
    "honeycomb26x18_flux": lambda: I.honeycomb(26, 18, flux=1.0 / 234.0, W=1.0, seed=112),
    # fixed width 6, a row count that is no multiple of any slice height
    "cubic15": lambda: I.cubic(15, W=3.0, seed=113),
}


@pytest.mark.parametrize("name", list(LATTICES))
@pytest.mark.parametrize("S", [32, 64, 128, 256])
def test_slice_heights_match_oracle(gpu, name, S):
    """Moments (Hermitian and two-chain forms), the evolution + commutator series and the
    velocity at every slice height gpuqt_build_h_tuned may choose."""
    say(f"case: slice height {S} on {name}")
    m = LATTICES[name]()
    Hs, V, XH = O.operators(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x)
    dE = oracle_dE(Hs)
    H = P.gpuqt_build_h_from_model(m, energy_max=dE, slice_height=S)
    assert H.info.slice_height == S
    phi = I.random_phase(m.n, 2, 114)
    d = dev(phi)
    ref = O.chebyshev_moments(Hs / dE, phi, phi, 120).T
    assert err(host(P.gpuqt_moments(H, d, d, 120))[0], ref) < TOL
    assert err(host(P.gpuqt_moments(H, d, dev(phi), 120))[0], ref) < TOL
    po, co = P.gpuqt_evolve(H, d, 0.9, 0, with_commutator=True)
    assert err(host(po), O.evolve(Hs / dE, phi, 0.9, dE)) < TOL
    if np.max(np.abs(XH @ phi)) > 0:
        assert err(host(co), O.commutator_evolve(Hs / dE, XH / dE, phi, 0.9, dE)) < TOL
    assert err(host(P.gpuqt_apply_commutator(H, d, P.VELOCITY)), V @ phi) < 1e-13


def test_build_h_tuned_picks_a_height_and_keeps_results(gpu):
    say("case: slice height chosen by measurement")
    m = I.square(300, 280, W=2.0, seed=115)
    Hs, _, _ = O.operators(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x)
    dE = oracle_dE(Hs)
    H = P.gpuqt_build_h_tuned(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x, m.volume, dE, B=4)
    S = H.slice_tuning["slice_height"]
    assert S in (32, 64, 128, 256) and H.info.slice_height == S
    us = H.slice_tuning["us_per_step"]
    assert all(us[k] > 0 for k in (32, 64, 128, 256)) and us[S] == min(us.values())
    phi = I.random_phase(m.n, 4, 116)
    d = dev(phi)
    assert err(host(P.gpuqt_moments(H, d, d, 64))[0], O.chebyshev_moments(Hs / dE, phi, phi, 64).T) < TOL


def test_autotune_cache_miss_then_hit(gpu):
    """A miss measures and stores the choice under the handle's key; a second handle of the
    same configuration gets the same code from the cache without measuring; the cache file
    round-trips."""
    import os
    import tempfile
    say("case: tuning cache")
    P.gpuqt_tune_cache_clear()
    try:
        m = I.cubic(14, W=2.0, seed=117)
        H1 = P.gpuqt_build_h_from_model(m)
        t, hit = P.gpuqt_autotune_cached(H1, 2)
        assert not hit and np.all(t[:2] > 0)
        code = H1.info.kernel_variant
        H2 = P.gpuqt_build_h_from_model(m)
        key = P.gpuqt_tune_cache_key(H2, 2)
        assert key == P.gpuqt_tune_cache_key(H1, 2) and key.startswith("gfx") and key.endswith(" B2")
        t2, hit2 = P.gpuqt_autotune_cached(H2, 2)
        assert hit2 and np.all(t2 == 0) and H2.info.kernel_variant == code
        with tempfile.TemporaryDirectory() as td:
            path = os.path.join(td, "cache.tsv")
            P.gpuqt_tune_cache_save(path)
            P.gpuqt_tune_cache_clear()
            P.gpuqt_tune_cache_load(path)
        H3 = P.gpuqt_build_h_from_model(m)
        _, hit3 = P.gpuqt_autotune_cached(H3, 2)
        assert hit3 and H3.info.kernel_variant == code
        # the moments do not depend on where the variant came from
        phi = dev(I.random_phase(m.n, 2, 118))
        assert np.array_equal(host(P.gpuqt_moments(H1, phi, phi, 40)), host(P.gpuqt_moments(H3, phi, phi, 40)))
    finally:
        P.gpuqt_tune_cache_clear()
        P.gpuqt_tune_cache_load(P.TUNE_CACHE_PATH)


def test_autotune_block_width(gpu):
    """The block width for 6 vectors is one of 1, 2, 4 (the widths not above 6), each tried
    width has a positive per-vector time, the chosen one the least, and the handle is left
    with the variant cached for it."""
    say("case: block width for 6 vectors")
    P.gpuqt_tune_cache_clear()
    try:
        m = I.square(200, 180, W=1.0, seed=119)
        H = P.gpuqt_build_h_from_model(m)
        B, us = P.gpuqt_autotune_block(H, 6)
        assert B in (1, 2, 4)
        assert np.all(us[:3] > 0) and np.all(us[3:] == 0) and us[B.bit_length() - 1] == us[:3].min()
        code = H.info.kernel_variant
        H2 = P.gpuqt_build_h_from_model(m)
        _, hit = P.gpuqt_autotune_cached(H2, B)
        assert hit and H2.info.kernel_variant == code
    finally:
        P.gpuqt_tune_cache_clear()
        P.gpuqt_tune_cache_load(P.TUNE_CACHE_PATH)


@pytest.mark.parametrize("B", [1, 4])
def test_plain_recurrence_entry_point(gpu, B):
    """gpuqt_moments_plain (the one-moment-per-step recurrence) against the oracle for
    phiL = phiR and phiL != phiR, odd and even M down to 1, on a flux honeycomb lattice."""
    say(f"case: plain recurrence B={B}")
    m = I.honeycomb(22, 16, flux=1.0 / 176.0, W=1.2, seed=120)
    Hs, _, _ = O.operators(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x)
    dE = oracle_dE(Hs)
    H = P.gpuqt_build_h_from_model(m, energy_max=dE)
    a = I.random_phase(m.n, B, 121)
    b = I.random_phase(m.n, B, 122)
    for M in (1, 2, 3, 250, 301):
        for L, R in ((a, a), (a, b)):
            got = host(P.gpuqt_moments_plain(H, dev(L), dev(R), M))[0]
            assert err(got, O.chebyshev_moments(Hs / dE, L, R, M).T) < TOL, M
    d = dev(a)
    assert np.array_equal(host(P.gpuqt_moments_plain(H, d, d, 200)), host(P.gpuqt_moments_plain(H, d, d, 200)))
