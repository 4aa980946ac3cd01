"""Row schedule of the sparse kernels (host only): every row is visited exactly once, by a
workgroup of its own segment, in the plain and in the banded order; the banded order brings
rows one period apart into the same or neighbouring iterations."""
import numpy as np
import pytest

import paper_1705_01387_amd as P


def _check_cover(offs, blk, it):
    n = int(offs[-1])
    assert blk.shape == (n,) and np.all(blk >= 0) and np.all(it >= 0)
    seg_of_row = np.repeat(np.arange(len(offs) - 1), np.diff(offs))
    owners = {}
    for s in range(len(offs) - 1):
        owners[s] = set(np.unique(blk[seg_of_row == s]).tolist())
    for s in owners:
        for t in owners:
            if s != t:
                assert not (owners[s] & owners[t]), (s, t)


CASES = [
    ([0, 1], None, 0),
    ([0, 1000], None, 0),
    ([0, 3, 70, 71, 5000, 5001, 20000], None, 0),
    ([0, 20000], [1000], 128),
    ([0, 20000], [1000], 64),
    ([0, 7, 9000, 40003], [0, 300, 811], 192),       # unaligned segments and periods
    ([0, 13, 26, 130000], [1, 13, 2900], 640),
]


@pytest.mark.parametrize("offs,period,band", CASES)
@pytest.mark.parametrize("B", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("cus", [1, 3, 256])
@pytest.mark.parametrize("pencil", [False, True])
def test_schedule_visits_every_row_once(offs, period, band, B, cus, pencil):
    blk, it = P.gpuqt_schedule_rows(offs, period, band, cus, B, pencil=pencil)
    _check_cover(np.asarray(offs), blk, it)


def test_pencil_order_puts_period_neighbours_in_one_tile():
    """Cubic 200^3 in natural site order (period D = 200^2 = 625 units of 64 rows): in the
    pencil order the four wavefronts of a workgroup take the same rows of four consecutive
    periods, so for 3 of every 4 rows r the row r + D is visited by the same workgroup in
    the same iteration (another wavefront of the same compute unit); in the plain and the
    banded orders almost never."""
    n, D = 200 ** 3, 40000
    r = np.arange(n - D)
    for B, W in [(1, 8192), (4, 2880), (16, 768)]:
        blk, it = P.gpuqt_schedule_rows([0, n], [D], W, 256, B, pencil=True)
        same = np.mean((blk[r + D] == blk[r]) & (it[r + D] == it[r]))
        assert same >= 0.74, (B, same)
        b0, i0 = P.gpuqt_schedule_rows([0, n], [D], W, 256, B)
        assert np.mean((b0[r + D] == b0[r]) & (i0[r + D] == i0[r])) < 0.05, B


def test_banded_order_brings_period_neighbours_together():
    """Cubic 200^3 in natural site order (period D = 200^2): with the band widths the
    library picks for B = 4 and 16, rows D apart fall in the same or the next iteration of
    their workgroups for 90 % of rows (the rest sit at band and XCD-group boundaries);
    in the plain order they are 2-3 (B = 4) and 10 (B = 16) iterations apart."""
    n, D = 200 ** 3, 40000
    r = np.arange(n - D)
    for B, W, plain_median in [(4, 5824, 2), (16, 1600, 10)]:
        _, it0 = P.gpuqt_schedule_rows([0, n], None, 0, 256, B)
        _, it1 = P.gpuqt_schedule_rows([0, n], [D], W, 256, B)
        gap0 = np.abs(it0[r + D] - it0[r])
        gap1 = np.abs(it1[r + D] - it1[r])
        assert np.percentile(gap1, 90) <= 1, B
        assert np.median(gap0) >= plain_median, B


def test_band_wider_than_period_keeps_plain_order():
    offs = [0, 50000]
    a = P.gpuqt_schedule_rows(offs, None, 0, 256, 4)
    b = P.gpuqt_schedule_rows(offs, [1000], 1024, 256, 4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_schedule_argument_errors():
    with pytest.raises(P.GpuqtError):
        P.gpuqt_schedule_rows([0, 100], [10], 100, 256, 1)        # not a multiple of 64
    with pytest.raises(P.GpuqtError):
        P.gpuqt_schedule_rows([0, 100, 100], None, 0, 256, 1)     # empty segment
    with pytest.raises(P.GpuqtError):
        P.gpuqt_schedule_rows([0, 100], None, 0, 256, 3)          # unsupported B
