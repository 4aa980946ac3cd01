"""The allocation-free moments entry point against gpuqt_moments with a caller workspace:
two calls in a row (the second on a smaller lattice, block and moment count), the size
limit, and replays of a captured HIP graph of it."""
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


def _case(m, B, M, seed, same):
    import torch
    H = P.gpuqt_build_h_from_model(m)
    a = dev(I.random_phase(m.n, B, seed))
    b = a if same else dev(I.random_phase(m.n, B, seed + 1))
    ws = torch.empty(P.gpuqt_workspace_size(H, P.OP_MOMENTS, B, M, 0), dtype=torch.uint8, device="cuda")
    ref = P.gpuqt_moments(H, a, b, M, ws=ws)
    mu = torch.full((H.n_segments, B, M), complex(7.0, -3.0), dtype=torch.complex128, device="cuda")
    P.gpuqt_moments_noalloc(H, a, b, M, mu)
    return H, a, b, host(ref), host(mu)


def test_noalloc_matches_workspace_entry_point(gpu):
    """Two calls in a row, the second smaller: each equals gpuqt_moments (same kernels and
    variant: bit for bit) and both match the oracle."""
    say("case: no-alloc moments, square 300x280 B=4 M=300 then square 41x37 B=1 M=77")
    runs = [(I.square(300, 280, W=1.5, seed=131), 4, 300, 132, True),
            (I.square(41, 37, W=2.0, seed=133), 1, 77, 134, False)]
    for m, B, M, seed, same in runs:
        H, a, b, ref, got = _case(m, B, M, seed, same)
        assert np.array_equal(got, ref), (m.name, B, M)
        assert err(got, ref) < TOL
        Hs, _, _ = O.operators(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x)
        dE = float(H.energy_max[0])
        assert abs(dE - 1.01 * O.gershgorin_bound(Hs)) <= 1e-15 * dE
        cols = (0, B - 1)
        for c in cols:
            ra = host(a)[:, c:c + 1]
            rb = host(b)[:, c:c + 1]
            assert err(got[0, c], O.chebyshev_moments(Hs / dE, ra, rb, M)[:, 0]) < TOL


def test_noalloc_rejects_sizes_beyond_its_array(gpu):
    """A lattice whose moments workspace exceeds the fixed array: a workspace error naming the
    limit, and the output left untouched."""
    import torch
    say("case: no-alloc size limit, square 1000x1000 B=4")
    m = I.square(1000, 1000, W=1.0, seed=135)
    H = P.gpuqt_build_h_from_model(m)
    need = P.gpuqt_workspace_size(H, P.OP_MOMENTS, 4, 50, 0)
    assert need > P.gpuqt_noalloc_scratch_bytes() == 64 << 20
    phi = dev(I.random_phase(m.n, 4, 136))
    mu = torch.zeros((1, 4, 50), dtype=torch.complex128, device="cuda")
    with pytest.raises(P.GpuqtError) as e:
        P.gpuqt_moments_noalloc(H, phi, phi, 50, mu)
    assert e.value.status == 4 and str(64 << 20) in str(e.value)
    torch.cuda.synchronize()
    assert float(mu.abs().max()) == 0.0


def test_noalloc_graph_replays(gpu):
    """Captured into a HIP graph (capture fails on any allocation) and replayed three times
    with eager work, including other no-alloc calls on the same array, between replays: every
    replay equals the eager result."""
    import torch
    say("case: no-alloc moments in a captured graph")
    m = I.honeycomb(30, 20, flux=1.0 / 300.0, W=1.0, seed=137)
    H = P.gpuqt_build_h_from_model(m)
    phi = dev(I.random_phase(m.n, 2, 138))
    M = 160
    eager = torch.empty((1, 2, M), dtype=torch.complex128, device="cuda")
    P.gpuqt_moments_noalloc(H, phi, phi, M, eager)
    torch.cuda.synchronize()
    ref = host(eager)
    out = torch.empty_like(eager)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        P.gpuqt_moments_noalloc(H, phi, phi, M, out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        P.gpuqt_moments_noalloc(H, phi, phi, M, out)
    other = P.gpuqt_build_h_from_model(I.square(50, 20, W=3.0, seed=139))
    ophi = dev(I.random_phase(other.n, 1, 140))
    omu = torch.empty((1, 1, 90), dtype=torch.complex128, device="cuda")
    for rep in range(3):
        out.fill_(complex(1.0, 1.0))
        P.gpuqt_moments_noalloc(other, ophi, ophi, 90, omu)     # the same array, other contents
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(out), ref), rep
