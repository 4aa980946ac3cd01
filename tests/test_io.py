"""Input folders of the paper's program (Section 4.2), read by the library's C++ reader
(host only): round trips of written folders, the documented defaults, and errors."""
import os

import numpy as np
import pytest

import paper_1705_01387_amd as P
from paper_1705_01387_amd import inputs as I
from paper_1705_01387_amd.driver import write_input_folder


def test_round_trip_complex_honeycomb(tmp_path):
    m = I.honeycomb(6, 4, flux=1.0 / 24.0, W=1.0, seed=90)
    E = np.linspace(-2.5, 2.5, 11)
    dts = [0.1, 0.25, 1.0]
    write_input_folder(tmp_path, m, E, dts, energy_max=9.3, n_moments=123, n_random_vectors=3,
                       vac=True, msd=True)
    f = P.gpuqt_model_load(tmp_path)
    assert f.n == m.n and f.max_nn == m.nbr.shape[1]
    assert np.array_equal(f.nn, m.nn)
    for i in range(m.n):
        assert np.array_equal(f.nbr[i, :m.nn[i]], m.nbr[i, :m.nn[i]])
        assert np.array_equal(f.hop[i, :m.nn[i]], m.hop[i, :m.nn[i]])
    assert f.hop.dtype == np.complex128
    assert np.array_equal(f.onsite, m.onsite) and np.array_equal(f.x, m.x)
    assert f.length_x == m.length_x and f.volume == m.volume
    assert np.array_equal(f.energies, E) and np.array_equal(f.time_steps, dts)
    assert (f.energy_max, f.n_moments, f.n_random_vectors) == (9.3, 123, 3)
    assert f.calculate_vac and f.calculate_msd


def test_defaults_without_optional_files(tmp_path):
    """No hopping.in (every hopping -1), no potential.in (U = 0), no para.in: N_r = 1,
    N_m = 1000, DeltaE = 10, neither VAC nor MSD (Section 4.2)."""
    m = I.chain(9)
    m.hop = None
    m.onsite = None
    write_input_folder(tmp_path, m, [0.0, 0.5])
    os.remove(os.path.join(tmp_path, "para.in"))
    f = P.gpuqt_model_load(tmp_path)
    assert f.hop is None and f.onsite is None and f.time_steps is None
    assert (f.n_random_vectors, f.n_moments, f.energy_max) == (1, 1000, 10.0)
    assert not f.calculate_vac and not f.calculate_msd


def _folder(tmp_path):
    m = I.square(4, 3, W=1.0, seed=91)
    write_input_folder(tmp_path, m, [0.0], [1.0], msd=True)
    return tmp_path


def _expect(tmp_path, status, text):
    with pytest.raises(P.GpuqtError) as e:
        P.gpuqt_model_load(tmp_path)
    assert e.value.status == status and text in str(e.value), str(e.value)


def test_errors(tmp_path):
    d = _folder(tmp_path)
    nb = os.path.join(d, "neighbour.in")
    lines = open(nb).read().splitlines()
    # neighbour index out of range, reported with file and line
    bad = list(lines)
    bad[3] = "2 0 99"
    open(nb, "w").write("\n".join(bad) + "\n")
    _expect(d, 2, "neighbour.in:4")
    # more neighbours than the stated maximum
    bad[3] = "5 0 1 2 3 4"
    open(nb, "w").write("\n".join(bad) + "\n")
    _expect(d, 2, "neighbour count")
    # truncated file
    open(nb, "w").write("\n".join(lines[:5]) + "\n")
    _expect(d, 2, "site lines")
    open(nb, "w").write("\n".join(lines) + "\n")
    P.gpuqt_model_load(d)
    # unknown keyword in para.in
    open(os.path.join(d, "para.in"), "w").write("calculate_msd\nnumber_of_moment 10\n")
    _expect(d, 2, "unknown keyword")
    open(os.path.join(d, "para.in"), "w").write("calculate_msd\n")
    # MSD asked for without time_step.in
    os.remove(os.path.join(d, "time_step.in"))
    _expect(d, 1, "time_step.in")
    # missing required file
    os.remove(nb)
    _expect(d, 1, "neighbour.in")


GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _with_golden(tmp_path, para, time_step=None):
    """A small folder whose para.in (and time_step.in) are the paper's printed files."""
    m = I.chain(12, W=4.0, seed=92)
    write_input_folder(tmp_path, m, np.linspace(-4.0, 4.0, 5), [0.5])
    import shutil
    shutil.copy(os.path.join(GOLDEN, para), os.path.join(tmp_path, "para.in"))
    if time_step:
        shutil.copy(os.path.join(GOLDEN, time_step), os.path.join(tmp_path, "time_step.in"))
    return P.gpuqt_model_load(tmp_path)


def test_paper_para_in_of_the_diffusive_example(tmp_path):
    """Section 5.1: the file means N_m = 1000 (default), DeltaE = 6.1, N_r = 1 (default),
    VAC and MSD; the benchmark's replay of the example uses the same values."""
    f = _with_golden(tmp_path, "para_diffusive.in")
    assert (f.n_moments, f.energy_max, f.n_random_vectors) == (1000, 6.1, 1)
    assert f.calculate_vac and f.calculate_msd
    w = I.workload_paper_diffusive(L=20)
    assert (w["M"], w["energy_max"], w["phi"].shape[1], w["vac"], w["msd"]) == (1000, 6.1, 1, True, True)


def test_paper_para_and_time_steps_of_the_localized_example(tmp_path):
    """Section 5.2: N_r = 2, N_m = 500, DeltaE = 4.1, MSD only, and the 30 time steps
    0.1 .. 1.0, 1 .. 10, 10 .. 100 (total 610.5); the replay uses the same values."""
    f = _with_golden(tmp_path, "para_localized.in", "time_step_localized.in")
    assert (f.n_random_vectors, f.n_moments, f.energy_max) == (2, 500, 4.1)
    assert f.calculate_msd and not f.calculate_vac
    assert f.time_steps.shape == (30,) and abs(f.time_steps.sum() - 610.5) < 1e-9
    assert np.allclose(f.time_steps[:10], 0.1 * np.arange(1, 11)) and np.array_equal(f.time_steps[10:20], np.arange(1, 11))
    w = I.workload_paper_localized(L=1000)
    assert np.allclose(w["dt"], f.time_steps, rtol=0, atol=1e-15)
    assert (w["M"], w["energy_max"], w["phi"].shape[1], w["vac"], w["msd"]) == (500, 4.1, 2, False, True)
