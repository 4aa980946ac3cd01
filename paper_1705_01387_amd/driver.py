"""Run input folders of the paper's program on the GPU (Section 4.2, Section 4.3).

    python -m paper_1705_01387_amd.driver input.txt [--seed S] [--block B]

input.txt lists one input folder per line (paths relative to the current
directory, as the paper's driver file does).  For each folder the model and run
parameters are read by the library (gpuqt_model_load), the Hamiltonian is built
on the GPU, and for each of the N_r random-phase vectors the DOS (and, when
para.in asks for them, rho C_vv and rho DeltaX^2 at every time row) on the
energy grid of energy.in are appended to dos.out, vac.out and msd.out in the
folder: one row per vector in dos.out, N_t rows per vector in vac.out and
msd.out, one column per energy (Section 4.3; results of a new run are appended).

Random vectors: vector r has phases drawn by inputs.random_phase with seed
S + r.  Vectors run as blocks of up to B columns in one launch per step (the
paper runs them one at a time); the results per vector are the same.
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np

from . import _binding as P
from . import inputs as I


def write_input_folder(path, model, energies, time_steps=None, energy_max=None, n_moments=None,
                       n_random_vectors=None, vac=False, msd=False):
    """Write an inputs.Model and run parameters as the paper's input files (Section 4.2)."""
    os.makedirs(path, exist_ok=True)
    n, k = int(model.n), int(model.nbr.shape[1])
    with open(os.path.join(path, "neighbour.in"), "w") as f:
        f.write(f"{n} {k}\n")
        for i in range(n):
            c = int(model.nn[i])
            f.write(" ".join([str(c)] + [str(int(j)) for j in model.nbr[i, :c]]) + "\n")
    if model.hop is not None:
        hop = np.asarray(model.hop)
        cplx = np.iscomplexobj(hop)
        with open(os.path.join(path, "hopping.in"), "w") as f:
            f.write("complex\n" if cplx else "real\n")
            for i in range(n):
                c = int(model.nn[i])
                if cplx:
                    vals = [v for z in hop[i, :c] for v in (z.real, z.imag)]
                else:
                    vals = list(hop[i, :c])
                f.write(" ".join(repr(float(v)) for v in vals) + "\n")
    if model.onsite is not None:
        np.savetxt(os.path.join(path, "potential.in"), np.asarray(model.onsite), fmt="%.17g")
    with open(os.path.join(path, "position.in"), "w") as f:
        f.write(f"{float(model.length_x)!r} {float(model.volume)!r}\n")
        for v in model.x:
            f.write(repr(float(v)) + "\n")
    with open(os.path.join(path, "energy.in"), "w") as f:
        f.write(f"{len(energies)}\n")
        for e in energies:
            f.write(repr(float(e)) + "\n")
    if time_steps is not None:
        with open(os.path.join(path, "time_step.in"), "w") as f:
            f.write(f"{len(time_steps)}\n")
            for t in time_steps:
                f.write(repr(float(t)) + "\n")
    lines = []
    if energy_max is not None:
        lines.append(f"energy_max {float(energy_max)!r}")
    if n_moments is not None:
        lines.append(f"number_of_moments {int(n_moments)}")
    if n_random_vectors is not None:
        lines.append(f"number_of_random_vectors {int(n_random_vectors)}")
    if vac:
        lines.append("calculate_vac")
    if msd:
        lines.append("calculate_msd")
    with open(os.path.join(path, "para.in"), "w") as f:
        f.write("\n".join(lines) + "\n")


def _append(path, rows):
    with open(path, "a") as f:
        np.savetxt(f, np.atleast_2d(rows), fmt="%.15e")


def run_folder(path, seed=0, block=16, stream=None):
    """Run one input folder; appends to its dos.out / vac.out / msd.out and returns the rows."""
    import torch
    f = P.gpuqt_model_load(path)
    H = P.gpuqt_build_h(f.nn, f.nbr, f.hop, f.onsite, f.x, f.length_x, f.volume, f.energy_max,
                        stream=stream)
    dE, M, E = f.energy_max, f.n_moments, f.energies
    dts = f.time_steps if f.time_steps is not None else np.zeros(0)
    out = {"dos": [], "vac": [], "msd": []}
    r = 0
    while r < f.n_random_vectors:
        B = 1
        while B * 2 <= min(block, 16) and r + B * 2 <= f.n_random_vectors:
            B *= 2
        phi = np.concatenate([I.random_phase(f.n, 1, seed + r + b) for b in range(B)], axis=1)
        d = torch.from_numpy(phi).to("cuda")
        mu = P.gpuqt_moments(H, d, d, M, stream=stream)[0].real.contiguous()          # [B, M]
        out["dos"].append(P.gpuqt_kpm_reconstruct(mu, E, dE, f.volume, stream=stream).cpu().numpy())
        for kind, call in (("vac", P.gpuqt_vac), ("msd", P.gpuqt_msd)):
            if not getattr(f, "calculate_" + kind):
                continue
            c = call(H, d, dts, M, stream=stream)[:, 0]                                 # [N_t, B, M]
            rows = P.gpuqt_kpm_reconstruct(c.permute(1, 0, 2).reshape(-1, M), E, dE, f.volume,
                                           stream=stream)                               # [B * N_t, n_E]
            out[kind].append(rows.cpu().numpy())
        r += B
    res = {}
    for kind in ("dos", "vac", "msd"):
        if out[kind]:
            res[kind] = np.concatenate(out[kind], axis=0)
            _append(os.path.join(path, kind + ".out"), res[kind])
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("driver_file", help="file listing one input folder per line")
    ap.add_argument("--seed", type=int, default=0, help="seed of the first random-phase vector")
    ap.add_argument("--block", type=int, default=16, help="at most this many vectors per launch")
    args = ap.parse_args(argv)
    with open(args.driver_file) as fh:
        folders = [ln.strip() for ln in fh if ln.strip()]
    for folder in folders:
        print(f"[driver] {folder}", flush=True)
        res = run_folder(folder, seed=args.seed, block=args.block)
        print(f"[driver] {folder}: " + ", ".join(f"{k}.out +{v.shape[0]} rows" for k, v in res.items()),
              flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
