"""Benchmark: Chebyshev H*psi steps per second of the linear-scaling Kubo path.

Default workload (--workload honeycomb): honeycomb lattice, 1000 x 1000 unit
cells = 2,000,000 orbitals, 3 neighbours, hopping -2.7 eV with Peierls phases
for a flux of 1/2000 per hexagon (complex128 hoppings), Anderson disorder U
in [-1, 1] eV, DeltaE = 1.01 x Gershgorin bound.  One step = the whole
calculation for one random-phase vector (vectors seeded 2002, 2003, ...):
DOS moments (M = 3000), VAC moments and MSD moments over 20 time steps of
15 fs (M = 3000 per row, 275 Chebyshev-Bessel terms per step, chosen
automatically).

--workload cubic: simple cubic 200^3 = 8,000,000 orbitals, t = -1, Anderson
W = 16, a block of 4 random-phase vectors; one step = DOS moments (M = 1000)
and MSD moments over 40 steps of dt = 2 (M = 1000, automatic term count,
63) for the block.  Its working set is several GB, far beyond the 256 MB
last-level cache, so it shows the HBM roofline.

Every input is resident on the GPU before the timed region.  The value
counts Chebyshev recurrence steps applied to one vector: each moment step,
each evolution term and each velocity application counts 1, each term of
the fused evolution + commutator series counts 2 (its two chains); a step on
a block of B vectors counts B.

Also reported: the roofline of the dominant kernel (the moment step) from
HIP events around the DOS moment call of every timed step, and the CPU
oracle timed on a bounded sample of the same recurrence.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Chebyshev H·psi steps/s, HBM GB/s %peak; batched & adjoint vs plain @1e-10 err"
HBM_PEAK_GBS = 8000.0


def moment_step_bytes(info, B):
    """Algorithmic HBM bytes of one moment-step launch (gathers counted once).

    Per row: neighbour indices 4 B/entry, hoppings 0 (one value per segment),
    8 (real) or 16 (complex) B/entry, on-site term 8 B, and 4 vector streams of
    16*B B (gathered v_{n-1}, v_{n-2}, phi_L, written v_n); per slice the 8-byte
    slice offset.
    """
    hop_b = {0: 0, 1: 8, 2: 16}[int(info.hop_mode)]
    n = int(info.n)
    return int(info.nnz) * (4 + hop_b) + n * 8 + n * 64 * B + int(info.n_slices) * 8


def count_steps(M, dts, np_list, vac=True, msd=True):
    """Chebyshev H*psi steps of one vector's DOS (+ VAC) (+ MSD) calculation."""
    n_t = len(dts)
    total = M - 1
    if vac:
        total += 1 + n_t * (1 + (M - 1)) + sum(2 * (np_list[k] - 1) for k in range(n_t - 1))
    if msd:
        total += sum(2 * (np_list[k] - 1) for k in range(n_t)) + n_t * (M - 1)
    return total


def setup(name, n_vec):
    import numpy as np
    from paper_1705_01387_amd import inputs as I
    if name == "honeycomb":
        w = I.workload_honeycomb(n_vectors=n_vec)
        return dict(model=w["model"], dE=w["energy_max"], M=w["M"], dt=w["dt"], B=1, vac=True,
                    msd=True, phis=w["phis"],
                    desc="honeycomb 1000x1000 cells (2,000,000 orbitals), Peierls flux 1/2000, "
                         "W=2 eV; per vector: DOS M=3000 + VAC and MSD 20 x 15 fs, M=3000")
    if name == "cubic":
        w = I.workload_cubic(L=200, W=16.0, B=4)
        m = w["model"]
        phis = [I.random_phase(m.n, 4, 4100 + r) for r in range(n_vec)]
        return dict(model=m, dE=w["energy_max"], M=w["M"], dt=w["dt"], B=4, vac=False, msd=True,
                    phis=phis,
                    desc="cubic 200^3 (8,000,000 orbitals), W=16, block of 4 vectors; per block: "
                         "DOS M=1000 + MSD 40 x dt=2, M=1000")
    raise SystemExit(f"unknown workload {name}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="honeycomb", choices=["honeycomb", "cubic"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-moments", type=int, default=0,
                    help="moments in the CPU oracle sample (0: sized to about 15 s)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; the workload shards over "
                          "random vectors with no communication, but only --gpus 1 is run"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1705_01387_amd as P

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = setup(args.workload, args.warmup + args.steps)
    m, dE, M, dts, B = cfg["model"], cfg["dE"], cfg["M"], cfg["dt"], cfg["B"]
    H = P.gpuqt_build_h_from_model(m, energy_max=dE)
    np_list = [P.gpuqt_auto_terms(dE * abs(t)) for t in dts]
    phis = [torch.from_numpy(p).to(dev) for p in cfg["phis"]]
    ws = torch.empty(max(P.gpuqt_workspace_size(H, P.OP_VAC, B, M, max(np_list)),
                         P.gpuqt_workspace_size(H, P.OP_MSD, B, M, max(np_list)),
                         P.gpuqt_workspace_size(H, P.OP_MOMENTS, B, M, 0)),
                     dtype=torch.uint8, device=dev)
    tune_us = P.gpuqt_autotune(H, B, ws=ws)           # untimed: pick the kernel variant
    mu = torch.empty((1, B, M), dtype=torch.complex128, device=dev)
    vac = torch.empty((len(dts), 1, B, M), dtype=torch.float64, device=dev)
    msd = torch.empty_like(vac)
    ev = []

    def one_step(phi, record):
        if record:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
        P.gpuqt_moments(H, phi, phi, M, mu=mu, ws=ws)
        if record:
            e1.record()
            ev.append((e0, e1))
        if cfg["vac"]:
            P.gpuqt_vac(H, phi, dts, M, 0, out=vac, ws=ws)
        if cfg["msd"]:
            P.gpuqt_msd(H, phi, dts, M, 0, out=msd, ws=ws)

    for i in range(args.warmup):
        one_step(phis[i], False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        one_step(phis[args.warmup + i], True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    steps_per_vec = count_steps(M, dts, np_list, cfg["vac"], cfg["msd"]) * B
    value = steps_per_vec * args.steps / elapsed
    dos_ms = [a.elapsed_time(b) for a, b in ev]
    launch_s = np.mean(dos_ms) / 1e3 / (M - 1)          # moment steps per DOS call: M-1
    bytes_launch = moment_step_bytes(H.info, B)
    achieved = bytes_launch / launch_s / 1e9

    # attainable bandwidth: copy probe of 1 GiB (read 1 GiB + write 1 GiB)
    nb = 1 << 30
    src = torch.zeros(nb // 16, dtype=torch.complex128, device=dev)
    dst = torch.empty_like(src)
    P.gpuqt_copy_probe(src, dst)
    torch.cuda.synchronize()
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(10):
        P.gpuqt_copy_probe(src, dst)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * nb * 10 / (c0.elapsed_time(c1) / 1e3) / 1e9
    del src, dst

    cpu = None
    if not args.no_cpu:
        import oracle as O
        Hs, _, _ = O.operators(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x)
        phi0 = cfg["phis"][0]
        Mc = args.cpu_moments
        if Mc <= 0:                       # calibrate to about 15 s of CPU work
            tc = time.perf_counter()
            O.dos_moments(Hs, phi0, dE, 8)
            per = (time.perf_counter() - tc) / 7
            Mc = int(max(16, min(4000, 15.0 / max(per, 1e-6))))
        tc = time.perf_counter()
        O.dos_moments(Hs, phi0, dE, Mc)
        tcpu = time.perf_counter() - tc
        cpu = {"value": (Mc - 1) * B / tcpu, "unit": "Chebyshev H*psi steps/s", "cores": 1,
               "kind": "oracle",
               "sample": f"oracle DOS moment recurrence, M={Mc}, B={B}, on the full {m.n}-orbital "
                         f"lattice of this workload ({tcpu:.1f} s; scipy CSR products and numpy, "
                         f"one thread)"}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Chebyshev H*psi steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": cfg["desc"] + ", Np=auto (%d)" % np_list[0],
                   "orbitals": int(m.n), "block": B, "moments": M, "time_steps": len(dts),
                   "cheb_steps_per_step": steps_per_vec, "steps_timed": args.steps},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_moment_step (B=%d, hop mode %d, K=%d, variant %d)"
                               % (B, H.info.hop_mode, H.info.uniform_width, H.info.kernel_variant),
                     "autotune_us_per_step": [float(t) for t in tune_us],
                     "bytes_per_launch": bytes_launch, "avg_launch_us": launch_s * 1e6,
                     "copy_probe_GBs": copy_gbs},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
