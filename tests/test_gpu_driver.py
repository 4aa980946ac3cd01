"""The input-folder driver end to end on the GPU: dos.out, vac.out and msd.out of a small
honeycomb folder with Peierls phases (three vectors: a block of two and one more) against
the oracle's moments and KPM sums for the same random vectors; a second run appends."""
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_1705_01387_amd import inputs as I
from paper_1705_01387_amd.driver import main, write_input_folder

pytestmark = pytest.mark.gpu
TOL = 1e-10


def err(got, ref):
    return float(np.max(np.abs(np.asarray(got) - np.asarray(ref))) / max(np.max(np.abs(ref)), 1e-300))


def test_driver_matches_oracle_and_appends(gpu, tmp_path):
    print("case: driver honeycomb 6x4 flux, N_r=3, VAC+MSD", flush=True)
    sys.stdout.flush()
    m = I.honeycomb(6, 4, flux=1.0 / 24.0, W=1.0, seed=92)
    H, V, XH = O.operators(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x)
    dE = 1.01 * O.gershgorin_bound(H)
    E = np.linspace(-0.9 * dE, 0.9 * dE, 21)
    dts = [0.5, 1.0, 0.25]
    M = 64
    folder = tmp_path / "honeycomb"
    write_input_folder(folder, m, E, dts, energy_max=dE, n_moments=M, n_random_vectors=3, vac=True, msd=True)
    drv = tmp_path / "input.txt"
    drv.write_text(str(folder) + "\n")
    assert main([str(drv), "--seed", "7", "--block", "2"]) == 0
    dos = np.loadtxt(folder / "dos.out", ndmin=2)
    vac = np.loadtxt(folder / "vac.out", ndmin=2)
    msd = np.loadtxt(folder / "msd.out", ndmin=2)
    assert dos.shape == (3, len(E)) and vac.shape == (3 * len(dts), len(E)) and msd.shape == vac.shape
    for r in range(3):
        phi = I.random_phase(m.n, 1, 7 + r)
        ref = O.kpm_reconstruct(O.dos_moments(H, phi, dE, M)[:, 0], E, dE, m.volume)
        assert err(dos[r], ref) < TOL, r
        rv = O.kpm_reconstruct(O.vac_moments(H, V, phi, dts, dE, M)[:, :, 0].T, E, dE, m.volume).T
        rm = O.kpm_reconstruct(O.msd_moments(H, XH, phi, dts, dE, M)[:, :, 0].T, E, dE, m.volume).T
        assert err(vac[r * len(dts):(r + 1) * len(dts)], rv) < TOL, r
        assert err(msd[r * len(dts):(r + 1) * len(dts)], rm) < TOL, r
    assert main([str(drv), "--seed", "7", "--block", "4"]) == 0
    dos2 = np.loadtxt(folder / "dos.out", ndmin=2)
    assert dos2.shape == (6, len(E)) and err(dos2[3:], dos[:3]) < 1e-14
