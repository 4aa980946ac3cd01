"""Benchmark: Chebyshev H*psi steps per second of the linear-scaling Kubo path on one MI355X.

Default workload (--workload cubic): simple cubic lattice 200^3 = 8,000,000 orbitals,
6 neighbours, t = -1, Anderson disorder U in [-8, 8] (W = 16), DeltaE = 1.01 (6 + W/2),
a block of 4 random-phase vectors advanced together.  The MSD of this block over time steps
of dt = 2 with 60 Chebyshev-Bessel terms per step and M = 1000 moments per row is the
workload; one bench step is one time step of it: the fused evolution + commutator series
(psi <- U(dt) psi, chi <- [X, U(dt)] psi + U(dt) chi, Section 3.2, product rule) followed
by the M moments of the new chi (Section 3.3, C_n^MSD).  The state carries over from step
to step (warmup steps included), so K steps are K consecutive MSD rows.  The DOS moments
of the block (M = 1000) are timed once beside it, and the whole calculation of one block
(DOS + 40 rows) is reported as the sum.  Every input is resident in HBM before timing.

value = sparse H*psi applications per second actually launched, counted per vector (a step
on a block of B vectors counts B): a fused evolution + commutator term counts 2 (its two
chains), a step of a moment set 1 (the library reaches M moments in max(1, M/2) steps by the
Chebyshev product identities).  config.plain_equivalent_steps_per_s counts the same results
as the paper's one-moment-per-step recurrence would need them (M - 1 per set).

Also on the line:
  roofline      the kernel family with the most time (HIP events the library records on its
                own stream around each run of launches, gpuqt_set_timing): algorithmic bytes
                per launch / average launch time, against the 8 TB/s HBM peak, with the HBM
                bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE record
                when it was taken on the same kernel sources and configuration of that
                kernel family (family_config);
  single_vector the single-vector (B = 1) Chebyshev step on the same lattice, both the
                Hermitian product-identity step the library uses and the paper's plain
                one-moment-per-step recurrence (gpuqt_moments_plain);
  cpu_baseline  the CPU oracle's moment recurrence on the same lattice, one host thread and
                all host cores (median of 5 runs of 20 steps each);
  paper_examples the paper's two examples (Section 5) end to end, once;
  copy_probe_GBs a full-grid 16-byte copy kernel over 2 x 1 GiB.

Other workloads (--workload): honeycomb (2,000,000-orbital honeycomb with Peierls phases, one
vector, DOS + VAC + MSD at M = 3000: its working set fits the 256 MB last-level cache, so
the roofline is labelled "llc"); honeycomb-general (the same with every hopping stored per
entry, as an arbitrary hopping.in gives); batched (8 uneven square realisations x 16 vectors
in one launch per step, eager vs graph-captured, and vs one vector at a time); small (square
64 x 64: DOS + VAC + MSD, launch-bound, eager vs graph-captured); paper; train.
"""
import argparse
import json
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Chebyshev H·psi steps/s, HBM GB/s %peak; batched & adjoint vs plain @1e-10 err"
UNIT = "Chebyshev H*psi steps/s"
HBM_PEAK_GBS = 8000.0
LLC_BYTES = 256 << 20

# vector bytes per row and block column of one launch of each kernel family (16-byte complex
# elements, each stream counted once): gathered inputs, v_{n-2} reads, outputs, dot partners
# and series accumulators (read + write)
FAMILY_VECTOR_BYTES = {
    "moment": 64,        # x (gathered), v_{n-2}, v_n, phi_L
    "moment_sym": 48,    # x (gathered, also the dot partner), v_{n-2}, v_n
    "moment_pair": 96,   # two chains: 2 x (gathered), 2 v_{n-2}, 2 v_n
    "evolve": 80,        # x, v_{n-2}, v_n, accumulator read + write
    "msd": 160,          # two chains as moment_pair + two accumulators read + write
    "evolve_pair": 160,  # two chains as moment_pair + two accumulators read + write
}
FAMILY_KERNEL = {"moment": "k_moment_step", "moment_sym": "k_moment_step_sym",
                 "moment_pair": "k_moment_step_pair", "evolve": "k_evolve_term", "msd": "k_msd_term",
                 "evolve_pair": "k_evolve_pair_term"}
KERNEL_SOURCES = ("device_common.h", "internal.h", "kernels.hip")   # what the step kernels are built from


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def family_bytes(info, B, family="moment"):
    """Algorithmic HBM bytes of one launch of a sparse kernel family (gathers counted once).

    Matrix part, per stored entry: neighbour index 4 B and hopping 0 (one value per
    segment), 8 (real) or 16 (complex) B, plus the position difference 8 B for the
    commutator chain; in table mode (3) one 2-byte index into the table of distinct
    (column offset, hopping, dx) triples, which stays in cache.  Per row the on-site term
    8 B.  Vector part: FAMILY_VECTOR_BYTES per row and block column.
    """
    mode = int(info.hop_mode)
    n = int(info.n)
    if mode == 3:
        per_entry = 2
    else:
        per_entry = 4 + {0: 0, 1: 8, 2: 16}[mode] + (8 if family == "msd" else 0)
    if box_used(info, B, family):
        per_entry = 0          # the box stencil reads no neighbour indices
    return int(info.entries) * per_entry + n * 8 + n * FAMILY_VECTOR_BYTES[family] * B


def box_used(info, B, family):
    """Whether the family runs a periodic-box stencil kernel: the Hermitian moment step with
    variant bit 26 (a handle whose matrix is a periodic box, or whose segments are all
    periodic squares: the sheet form), the MSD term with bit 27 (a periodic box with uniform
    x steps); blocks of B >= 2."""
    if B < 2 or (int(info.box[0]) <= 0 and int(info.sheets) == 0):
        return False
    v = int(info.kernel_variant)
    if family == "moment_sym":
        return (v >> 26) & 1 == 1
    if int(info.box[0]) <= 0:
        return False
    if family == "msd":
        return (v >> 27) & 1 == 1 and int(info.box_msd) == 1
    return False


def kernel_name(info, B, family):
    """The kernel the family runs on this handle: the general one, or its box or sheet form."""
    if not box_used(info, B, family):
        return FAMILY_KERNEL[family]
    return FAMILY_KERNEL[family] + ("_box" if int(info.box[0]) > 0 else "_sheet")


SERIES_FAMILIES = ("evolve", "msd", "evolve_pair")


def family_config(v, family):
    """What the variant code v sets for one kernel family: (non-temporal loads, banded order,
    pencil order, cap on resident workgroups per CU).  Bit 0 non-temporal loads (bit 7 flips it
    for the evolution and MSD families), bit 1 banded order, bit 6 pencil order, bits 2-5 the
    per-CU cap (0 = none) unless the family has its own (3 bits per family from bit 8: 0 = the
    per-CU cap, 1 + c = cap c)."""
    from paper_1705_01387_amd._binding import K_FAMILIES
    nt = v & 1
    if family in SERIES_FAMILIES:
        nt ^= (v >> 7) & 1
    banded = (v >> 1) & 1
    cap = (v >> 2) & 15
    c = (v >> (8 + 3 * K_FAMILIES.index(family))) & 7
    if c:
        cap = c - 1
    box = (v >> 26) & 1 if family == "moment_sym" else ((v >> 27) & 1 if family == "msd" else 0)
    return nt, banded, banded & ((v >> 6) & 1), cap, box


def variant_text(v, family=None):
    """The kernel variant code v as it applies to one kernel family (family_config)."""
    if family is None:
        nt, banded, pencil, cap = v & 1, (v >> 1) & 1, ((v >> 1) & (v >> 6)) & 1, (v >> 2) & 15
    else:
        nt, banded, pencil, cap, box = family_config(v, family)
        if box:
            return "code %d: stencil form, %s" % (v, "%d workgroups/CU" % cap if cap else "full occupancy")
    order = "pencil" if pencil else ("banded" if banded else "plain")
    return "code %d: %s loads, %s row order, %s" % (v, "non-temporal" if nt else "plain", order,
                                                   "%d workgroups/CU" % cap if cap else "full occupancy")


def pick_variant(P, H, B, ws, args):
    """Autotune the kernel variant of H at block width B (through the tuning cache, so that
    the benchmark and its profiles run the same variant), or pin the one given by --variant.
    Returns (autotune times per load variant or zeros, whether the choice came from the cache)."""
    if args.variant >= 0:
        P.gpuqt_set_variant(H, args.variant)
        return [0.0] * 7, False
    t, cached = P.gpuqt_autotune_cached(H, B, ws=ws)
    return [float(x) for x in t], bool(cached)


def kernel_table(info, B, fam, elapsed_s):
    """Per family: launches, average launch time (event time of its runs / launches; the
    runs are back-to-back launches, so this includes the small gaps between them),
    algorithmic bytes per launch and the bandwidth they imply.  Returns (table, dominant)."""
    table = {}
    for f, (ms, nl) in fam.items():
        if nl <= 0:
            continue
        avg = ms / 1e3 / nl
        b = family_bytes(info, B, f)
        table[f] = {"kernel": kernel_name(info, B, f), "launches": nl, "total_ms": ms,
                    "share_of_elapsed": ms / 1e3 / elapsed_s, "avg_us": avg * 1e6,
                    "bytes_per_launch": b, "GBs": b / avg / 1e9}
    dominant = max(table, key=lambda f: table[f]["total_ms"])
    return table, dominant


def measured_traffic(name, family, bytes_launch, variant):
    """HBM bytes per launch of the dominant kernel from the committed counter record, if it was
    taken on that kernel family, on the kernel sources built now and with the same
    configuration of that family (family_config; else None: a record of another
    configuration does not describe this run's kernel)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, "paper_1705_01387_amd", "csrc")
    h = hashlib.sha256()
    for fn in KERNEL_SOURCES:
        with open(os.path.join(src, fn), "rb") as g:
            h.update(g.read())
    e = rec.get(name)
    if (not e or e.get("kernel_source_sha256") != h.hexdigest() or e.get("family") != family
            or family_config(int(e.get("variant")), family) != family_config(int(variant), family)):
        return None
    return {"bytes": e["bytes_per_launch"], "ratio_to_algorithmic": e["bytes_per_launch"] / bytes_launch,
            "fetch_kib": e["fetch_kib"], "write_kib": e["write_kib"], "scale": e["scale"],
            "variant": e["variant"], "profile": e.get("profile")}


def roofline_of(name, info, B, kernels, dominant, bound="hbm"):
    d = kernels[dominant]
    tr = measured_traffic(name, dominant, d["bytes_per_launch"], info.kernel_variant)
    return {"bound": bound, "achieved": d["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": d["GBs"] / HBM_PEAK_GBS, "traffic": None if tr is None else tr["bytes"] / 1e9,
            "traffic_detail": tr,
            "kernel": "%s (B=%d, hop mode %d, K=%d, %s)" % (kernel_name(info, B, dominant), B, info.hop_mode,
                                                          info.uniform_width,
                                                          variant_text(info.kernel_variant, dominant)),
            "bytes_per_launch": d["bytes_per_launch"], "avg_launch_us": d["avg_us"]}


def copy_probe_gbs(P, torch, dev):
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
    out = 2 * nb * 10 / (c0.elapsed_time(c1) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return out


# --------------------------------------------------------------------------
# CPU baseline: the oracle, in a fresh process that never touches the GPU
# --------------------------------------------------------------------------

def cpu_baseline(workload, timeout=600):
    """Run this file with --cpu-baseline in a child process (the oracle's worker processes are
    forked there, from a process with no GPU context) and return its JSON."""
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline", workload]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=timeout)
    if r.returncode != 0:
        log("cpu baseline failed: " + r.stderr[-400:])
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


_CPU = {}


def _cpu_runs(seed, reps, steps):
    """reps timed runs of the oracle's DOS recurrence (steps sparse steps each) on one random-phase
    vector; BLAS / OpenMP pools held to one thread."""
    import oracle as O
    from threadpoolctl import threadpool_limits
    from paper_1705_01387_amd import inputs as I
    Hs, dE, n = _CPU["H"], _CPU["dE"], _CPU["n"]
    phi = I.random_phase(n, 1, seed)
    out = []
    with threadpool_limits(limits=1):
        for _ in range(reps):
            t = time.perf_counter()
            O.dos_moments(Hs, phi, dE, steps + 1)
            out.append(time.perf_counter() - t)
    return out


def cpu_baseline_main(workload):
    import multiprocessing as mp

    import oracle as O
    from paper_1705_01387_amd import inputs as I
    if workload == "cubic":
        w = I.workload_cubic(L=200, W=16.0, B=4)
        m, dE = w["model"], w["energy_max"]
    else:
        w = I.workload_honeycomb(n_vectors=1)
        m, dE = w["model"], w["energy_max"]
    t = time.perf_counter()
    Hs, _, _ = O.operators(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x)
    setup = time.perf_counter() - t
    _CPU.update(H=Hs, dE=dE, n=m.n)
    reps, steps = 5, 20
    one = _cpu_runs(4200, reps, steps)
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    ctx = mp.get_context("fork")
    with ctx.Pool(procs) as pool:
        res = pool.starmap(_cpu_runs, [(4300 + i, reps, steps) for i in range(procs)])
    all_rate = sum(steps / statistics.median(r) for r in res)
    one_rate = steps / statistics.median(one)
    sample = (f"oracle DOS moment recurrence (scipy CSR products, numpy dots; Section 3.2) on the full "
              f"{m.n}-orbital lattice of this workload, one vector per process, {reps} runs of {steps} "
              f"steps each, median run")
    print(json.dumps({"value": all_rate, "unit": UNIT, "cores": procs, "kind": "oracle", "sample": sample,
                      "single_thread": {"value": one_rate, "cores": 1, "median_run_s": statistics.median(one)},
                      "all_cores": {"value": all_rate, "cores": procs,
                                    "median_run_s": statistics.median([statistics.median(r) for r in res])},
                      "operator_setup_s": setup}))


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def single_vector_steps(P, torch, H, n, dev, args, seed=4200):
    """The single-vector Chebyshev step on this lattice: 100 Hermitian product-identity steps
    (the library's DOS form) and 100 steps of the paper's plain recurrence, autotuned at B = 1."""
    from paper_1705_01387_amd import inputs as I
    ws = torch.empty(max(P.gpuqt_workspace_size(H, P.OP_MOMENTS, 1, 201, 0),
                         P.gpuqt_workspace_size(H, P.OP_AUTOTUNE, 1, 0, 0)), dtype=torch.uint8, device=dev)
    tune, cached = pick_variant(P, H, 1, ws, args)
    phi = torch.from_numpy(I.random_phase(n, 1, seed)).to(dev)
    mu = torch.empty((H.n_segments, 1, 201), dtype=torch.complex128, device=dev)
    out = {}
    for name, call, M in (("hermitian_step", P.gpuqt_moments, 201), ("plain_recurrence", P.gpuqt_moments_plain, 101)):
        call(H, phi, phi, M, mu=mu[:, :, :M].contiguous() if M != 201 else mu, ws=ws)
        torch.cuda.synchronize()
        P.gpuqt_set_timing(H, True)
        for _ in range(3):
            call(H, phi, phi, M, mu=mu, ws=ws) if M == 201 else call(H, phi, phi, M, ws=ws)
        torch.cuda.synchronize()
        P.gpuqt_set_timing(H, False)
        fam = P.gpuqt_timing(H)
        f = "moment_sym" if name == "hermitian_step" else "moment"
        ms, nl = fam[f]
        avg = ms / 1e3 / nl
        b = family_bytes(H.info, 1, f)
        out[name] = {"kernel": FAMILY_KERNEL[f], "B": 1, "launches": nl, "avg_us": avg * 1e6,
                     "bytes_per_launch": b, "GBs": b / avg / 1e9, "frac": b / avg / 1e9 / HBM_PEAK_GBS,
                     "variant": variant_text(H.info.kernel_variant, f),
                     "traffic": measured_traffic("cubic_b1" if f == "moment_sym" else "cubic_b1_plain", f, b,
                                                 H.info.kernel_variant)}
    out["autotune_us"] = tune
    out["from_cache"] = cached
    del ws, phi, mu
    return out


def cubic_workload(args):
    import numpy as np
    import torch

    import paper_1705_01387_amd as P
    from paper_1705_01387_amd import inputs as I

    dev = torch.device("cuda:0")
    B, W, Np, M, dt = 4, 16.0, 60, 1000, 2.0
    w = I.workload_cubic(L=200, W=W, B=B)
    m, dE = w["model"], w["energy_max"]
    H = P.gpuqt_build_h_from_model(m, energy_max=dE)
    phi = torch.from_numpy(w["phi"]).to(dev)
    ws_m = torch.empty(max(P.gpuqt_workspace_size(H, P.OP_MOMENTS, B, M, 0),
                           P.gpuqt_workspace_size(H, P.OP_AUTOTUNE, B, 0, 0)), dtype=torch.uint8, device=dev)
    ws_e = torch.empty(P.gpuqt_workspace_size(H, P.OP_EVOLVE_COMMUTATOR, B, 0, Np), dtype=torch.uint8,
                       device=dev)
    tune_us, cached = pick_variant(P, H, B, ws_m, args)
    mu = torch.empty((1, B, M), dtype=torch.complex128, device=dev)
    psi = [phi.clone(), torch.empty_like(phi)]
    chi = [torch.zeros_like(phi), torch.empty_like(phi)]
    state = {"i": 0}

    def step():
        i = state["i"]
        P.gpuqt_evolve(H, psi[i], dt, Np, psi_out=psi[i ^ 1], chi=chi[i], chi_out=chi[i ^ 1], ws=ws_e)
        P.gpuqt_moments(H, chi[i ^ 1], chi[i ^ 1], M, mu=mu, ws=ws_m)
        state["i"] = i ^ 1

    log("setup done (%d orbitals, B=%d, variant %d%s)" % (m.n, B, H.info.kernel_variant,
                                                          " from the tuning cache" if cached else ""))
    # the DOS moments of the block, once (warm) and timed
    P.gpuqt_moments(H, phi, phi, M, mu=mu, ws=ws_m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.gpuqt_moments(H, phi, phi, M, mu=mu, ws=ws_m)
    torch.cuda.synchronize()
    dos_s = time.perf_counter() - t0
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")
    P.gpuqt_set_timing(H, True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    P.gpuqt_set_timing(H, False)
    log("timed steps done")
    fam = P.gpuqt_timing(H)
    K = max(1, M // 2)
    launched = (2 * (Np - 1) + K) * B               # per step: series terms (two chains) + moment steps
    plain = (2 * (Np - 1) + (M - 1)) * B
    kernels, dominant = kernel_table(H.info, B, fam, elapsed)
    per_step = elapsed / args.steps
    out = dict(value=launched * args.steps / elapsed, ms_per_step=per_step * 1e3,
               config={"workload": "cubic 200^3 (8,000,000 orbitals, 6 neighbours, t=-1), Anderson W=16, "
                                   "DeltaE=1.01*(6+W/2), block of 4 random-phase vectors; one step = one MSD "
                                   "time step dt=2 (fused evolution + commutator series, 60 terms) + the "
                                   "M=1000 moments of the new chi",
                       "orbitals": int(m.n), "block": B, "moments": M, "terms_per_step": Np, "dt": dt,
                       "launched_steps_per_step": launched, "plain_equivalent_steps_per_step": plain,
                       "plain_equivalent_steps_per_s": plain * args.steps / elapsed,
                       "dos_moments_s": dos_s, "full_block_calculation_s": dos_s + 40 * per_step,
                       "steps_timed": args.steps, "variant_from_tuning_cache": cached,
                       "autotune_us_per_step": tune_us},
               roofline=roofline_of("cubic", H.info, B, kernels, dominant),
               kernels=kernels)
    del ws_m, ws_e, psi, chi, mu, phi
    torch.cuda.empty_cache()
    log("single-vector steps")
    out["single_vector"] = single_vector_steps(P, torch, H, m.n, dev, args)
    H.close()
    out["roofline"]["copy_probe_GBs"] = copy_probe_gbs(P, torch, dev)
    if not args.no_paper:
        log("paper examples")
        out["paper_examples"] = paper_examples(args, passes=1)
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline("cubic")
    return out


def honeycomb_workload(args, general=False):
    import torch

    import paper_1705_01387_amd as P
    from paper_1705_01387_amd import inputs as I

    dev = torch.device("cuda:0")
    n_vec = args.warmup + args.steps
    w = I.workload_honeycomb(n_vectors=n_vec)
    m, dE, M, dts, B = w["model"], w["energy_max"], w["M"], w["dt"], 1
    H = P.gpuqt_build_h_from_model(m, energy_max=dE, no_dictionary=general)
    np_list = [P.gpuqt_auto_terms(dE * abs(t)) for t in dts]
    phis = [torch.from_numpy(p).to(dev) for p in w["phis"]]
    ws = torch.empty(max(P.gpuqt_workspace_size(H, P.OP_VAC, B, M, max(np_list)),
                         P.gpuqt_workspace_size(H, P.OP_MSD, B, M, max(np_list)),
                         P.gpuqt_workspace_size(H, P.OP_MOMENTS, B, M, 0),
                         P.gpuqt_workspace_size(H, P.OP_AUTOTUNE, B, 0, 0)), dtype=torch.uint8, device=dev)
    tune_us, cached = pick_variant(P, H, B, ws, args)
    mu = torch.empty((1, B, M), dtype=torch.complex128, device=dev)
    vac = torch.empty((len(dts), 1, B, M), dtype=torch.float64, device=dev)
    msd = torch.empty_like(vac)

    def one_step(phi):
        P.gpuqt_moments(H, phi, phi, M, mu=mu, ws=ws)
        P.gpuqt_vac(H, phi, dts, M, 0, out=vac, ws=ws)
        P.gpuqt_msd(H, phi, dts, M, 0, out=msd, ws=ws)

    log("setup done (%d orbitals, hop mode %d)" % (m.n, H.info.hop_mode))
    for i in range(args.warmup):
        one_step(phis[i])
    torch.cuda.synchronize()
    P.gpuqt_set_timing(H, True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        one_step(phis[args.warmup + i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    P.gpuqt_set_timing(H, False)
    fam = P.gpuqt_timing(H)
    K = max(1, M // 2)
    n_t = len(dts)
    launched = K + (1 + n_t * (1 + 2 * K) + sum(2 * (np_list[k] - 1) for k in range(n_t - 1))) \
        + (sum(2 * (np_list[k] - 1) for k in range(n_t)) + n_t * K)
    plain = (M - 1) + (1 + n_t * M + sum(2 * (np_list[k] - 1) for k in range(n_t - 1))) \
        + (sum(2 * (np_list[k] - 1) for k in range(n_t)) + n_t * (M - 1))
    kernels, dominant = kernel_table(H.info, B, fam, elapsed)
    # working set of the dominant launch: everything it streams
    ws_bytes = kernels[dominant]["bytes_per_launch"]
    bound = "llc" if ws_bytes <= LLC_BYTES else "hbm"
    name = "honeycomb_general" if general else "honeycomb"
    desc = ("honeycomb 1000x1000 cells (2,000,000 orbitals), Peierls flux 1/2000, W=2 eV, %s; per vector: "
            "DOS M=3000 + VAC and MSD 20 x 15 fs, M=3000, Np=auto (%d)"
            % ("hoppings stored per entry (complex128)" if general else "value-table layout", np_list[0]))
    out = dict(value=launched * args.steps / elapsed, ms_per_step=elapsed / args.steps * 1e3,
               config={"workload": desc, "orbitals": int(m.n), "block": B, "moments": M, "hop_mode": H.info.hop_mode,
                       "time_steps": n_t, "launched_steps_per_step": launched,
                       "plain_equivalent_steps_per_s": plain * args.steps / elapsed, "steps_timed": args.steps,
                       "dominant_working_set_MB": ws_bytes / 1e6, "variant_from_tuning_cache": cached,
                       "autotune_us_per_step": tune_us},
               roofline=roofline_of(name, H.info, B, kernels, dominant, bound),
               kernels=kernels)
    if bound == "llc":
        out["roofline"]["note"] = ("the dominant launch streams %.0f MB, within the 256 MB last-level "
                                   "cache: achieved bandwidth is not an HBM figure" % (ws_bytes / 1e6))
    del ws
    out["roofline"]["copy_probe_GBs"] = copy_probe_gbs(P, torch, dev)
    out["cpu_baseline"] = None if args.no_cpu else cpu_baseline("honeycomb")
    return out


def _graph_vs_eager(torch, fn, reps):
    """Seconds per call of fn eagerly and as one captured HIP graph replay."""
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    eager = (time.perf_counter() - t0) / reps
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    graph = (time.perf_counter() - t0) / reps
    return eager, graph


def small_workload(args):
    """Square 64 x 64 (4096 orbitals): DOS M=1000 + VAC and MSD over 10 steps of dt=1 (100 terms);
    every launch is a few microseconds, so the launch path decides the rate: eager calls vs
    the same calls captured once into a HIP graph and replayed."""
    import torch

    import paper_1705_01387_amd as P
    from paper_1705_01387_amd import inputs as I

    dev = torch.device("cuda:0")
    w = I.workload_square64()
    m, dE, M, dts, Np = w["model"], w["energy_max"], w["M"], list(w["dt"]), w["Np"]
    H = P.gpuqt_build_h_from_model(m, energy_max=dE)
    B = 1
    phi = torch.from_numpy(w["phi"]).to(dev)
    ws = torch.empty(max(P.gpuqt_workspace_size(H, P.OP_VAC, B, M, Np),
                         P.gpuqt_workspace_size(H, P.OP_MSD, B, M, Np),
                         P.gpuqt_workspace_size(H, P.OP_AUTOTUNE, B, 0, 0)), dtype=torch.uint8, device=dev)
    tune_us, cached = pick_variant(P, H, B, ws, args)
    mu = torch.empty((1, B, M), dtype=torch.complex128, device=dev)
    vac = torch.empty((len(dts), 1, B, M), dtype=torch.float64, device=dev)
    msd = torch.empty_like(vac)

    def calc():
        P.gpuqt_moments(H, phi, phi, M, mu=mu, ws=ws)
        P.gpuqt_vac(H, phi, dts, M, Np, out=vac, ws=ws)
        P.gpuqt_msd(H, phi, dts, M, Np, out=msd, ws=ws)

    eager, graph = _graph_vs_eager(torch, calc, max(1, args.steps))
    K = max(1, M // 2)
    n_t = len(dts)
    launched = K + (1 + n_t * (1 + 2 * K) + (n_t - 1) * 2 * (Np - 1)) + (n_t * 2 * (Np - 1) + n_t * K)
    return dict(value=launched / graph, ms_per_step=graph * 1e3,
                config={"workload": "square 64x64 (4096 orbitals), W=1, DeltaE=4.5, one vector: DOS M=1000 + VAC "
                                    "and MSD over 10 steps of dt=1 with 100 terms; value from the graph replay",
                        "orbitals": int(m.n), "launched_steps_per_step": launched, "steps_timed": args.steps,
                        "variant_from_tuning_cache": cached},
                graph_vs_eager={"eager_ms": eager * 1e3, "graph_ms": graph * 1e3, "speedup": eager / graph,
                                "eager_steps_per_s": launched / eager, "graph_steps_per_s": launched / graph,
                                "launches_per_step": launched + 2 * n_t + 1},
                roofline=None, cpu_baseline=None)


def batched_workload(args):
    import numpy as np
    import torch

    import paper_1705_01387_amd as P
    from paper_1705_01387_amd import inputs as I

    dev = torch.device("cuda:0")
    w = I.workload_batched(B=16, M=2000)
    mods, B, M = w["models"], w["B"], w["M"]
    cat = I.concat_segments(mods)
    offs = np.cumsum([0] + [mm.n for mm in mods])

    def build():
        return P.gpuqt_build_h(cat.nn, cat.nbr, cat.hop, cat.onsite, cat.x, 0.0, cat.volume, 0.0,
                               seg_offsets=offs, seg_energy_max=w["seg_energy_max"],
                               seg_length_x=[mm.length_x for mm in mods])
    H = build()
    phi = torch.from_numpy(w["phi"]).to(dev)
    ws = torch.empty(max(P.gpuqt_workspace_size(H, P.OP_MOMENTS, B, M, 0),
                         P.gpuqt_workspace_size(H, P.OP_AUTOTUNE, B, 0, 0)), dtype=torch.uint8, device=dev)
    tune_us, cached = pick_variant(P, H, B, ws, args)
    mu = torch.empty((H.n_segments, B, M), dtype=torch.complex128, device=dev)
    for _ in range(args.warmup):
        P.gpuqt_moments(H, phi, phi, M, mu=mu, ws=ws)
    torch.cuda.synchronize()
    P.gpuqt_set_timing(H, True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        P.gpuqt_moments(H, phi, phi, M, mu=mu, ws=ws)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    P.gpuqt_set_timing(H, False)
    kernels, dominant = kernel_table(H.info, B, P.gpuqt_timing(H), elapsed)
    eager, graph = _graph_vs_eager(torch, lambda: P.gpuqt_moments(H, phi, phi, M, mu=mu, ws=ws), 2)
    K = max(1, M // 2)
    value = B * K * args.steps / elapsed
    out = dict(value=value, ms_per_step=elapsed / args.steps * 1e3,
               config={"workload": "8 square realisations 200^2..2000^2 (8,255,182 orbitals), W_r in [0.5,3], "
                                   "per-realisation DeltaE, block of 16 vectors, M=2000, one launch per step",
                       "orbitals": int(H.n), "block": B, "moments": M, "segments": H.n_segments,
                       "plain_equivalent_steps_per_s": B * (M - 1) * args.steps / elapsed,
                       "steps_timed": args.steps, "variant_from_tuning_cache": cached,
                       "autotune_us_per_step": tune_us},
               roofline=roofline_of("batched", H.info, B, kernels, dominant), kernels=kernels,
               graph_vs_eager={"eager_ms": eager * 1e3, "graph_ms": graph * 1e3, "speedup": eager / graph})
    del ws
    # the same moments one vector at a time (B = 1): two vectors, same M
    H1 = build()
    ws1 = torch.empty(max(P.gpuqt_workspace_size(H1, P.OP_MOMENTS, 1, M, 0),
                          P.gpuqt_workspace_size(H1, P.OP_AUTOTUNE, 1, 0, 0)), dtype=torch.uint8, device=dev)
    pick_variant(P, H1, 1, ws1, args)
    v1 = [phi[:, b].contiguous() for b in range(2)]
    P.gpuqt_moments(H1, v1[0], v1[0], M, ws=ws1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for v in v1:
        P.gpuqt_moments(H1, v, v, M, ws=ws1)
    torch.cuda.synchronize()
    plain_vs = 2 * K / (time.perf_counter() - t1)
    out["batched_vs_single"] = {"single_vector_steps_per_s": plain_vs, "batched_vector_steps_per_s": value,
                                "speedup": value / plain_vs}
    out["cpu_baseline"] = None
    return out


def train_workload(args):
    import numpy as np
    import torch

    import paper_1705_01387_amd as P
    from paper_1705_01387_amd import inputs as I

    dev = torch.device("cuda:0")
    w = I.workload_train(512)
    m, dE, M, dts = w["model"], w["energy_max"], w["M"], list(w["dt"])
    H = P.gpuqt_build_h_from_model(m, energy_max=dE)
    phi = torch.from_numpy(w["phi"]).to(dev)
    P.gpuqt_autotune(H, 1)
    rng = np.random.default_rng(5010)
    wd = torch.from_numpy(rng.normal(size=(1, 1, M))).to(dev)
    wv = torch.from_numpy(rng.normal(size=(len(dts), 1, 1, M))).to(dev)
    gU = torch.zeros(m.n, dtype=torch.float64, device=dev)
    gC = torch.zeros(2, dtype=torch.float64, device=dev)
    np_list = [P.gpuqt_auto_terms(dE * abs(t)) for t in dts]
    tape = torch.empty(P.gpuqt_vac_tape_size(H, 1, dts, M), dtype=torch.uint8, device=dev)

    def fwd():
        P.gpuqt_moments(H, phi, phi, M)
        P.gpuqt_vac_record(H, phi, dts, M, tape=tape)

    def bwd():
        P.gpuqt_moments_backward(H, phi, phi, wd, gU, gC)
        P.gpuqt_vac_backward_tape(H, phi, dts, wv, tape, gU, gC)

    for f in (fwd, bwd):
        f()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fwd()
    torch.cuda.synchronize()
    tf = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bwd()
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / args.steps
    K = max(1, M // 2)
    n_t = len(dts)
    fwd_steps = K + 1 + n_t * (1 + 2 * K) + sum(2 * (np_list[k] - 1) for k in range(n_t - 1))
    return dict(value=fwd_steps / (tf + tb), ms_per_step=(tf + tb) * 1e3,
                config={"workload": "square 512^2 (262,144 orbitals), NN + NNN hopping classes, DeltaE=6, "
                                    "DOS M=512 + VAC 10 x dt=1; forward + adjoint (all on-site and class "
                                    "gradients; VAC forward recorded for the adjoint)", "orbitals": int(m.n),
                        "moments": M},
                adjoint_vs_forward={"forward_ms": tf * 1e3, "adjoint_ms": tb * 1e3, "ratio": tb / tf},
                roofline=None, cpu_baseline=None)


def paper_examples(args, passes=None):
    """The paper's two examples end to end on resident inputs: moments, KPM sums on the energy
    grid and running conductivities (the paper reports about 3 minutes for both on a Tesla
    K40, input and output included)."""
    import torch

    import paper_1705_01387_amd as P
    from paper_1705_01387_amd import inputs as I

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    runs = []
    for w in (I.workload_paper_diffusive(), I.workload_paper_localized()):
        m = w["model"]
        H = P.gpuqt_build_h_from_model(m, energy_max=w["energy_max"])
        B = w["phi"].shape[1]
        runs.append(dict(w=w, H=H, B=B, phi=torch.from_numpy(w["phi"]).to(dev), E=w["energies"]))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    for r in runs:
        P.gpuqt_autotune_cached(r["H"], r["B"])

    def example(r):
        w, H, B, phi, E = r["w"], r["H"], r["B"], r["phi"], r["E"]
        dE, M, dts, vol = w["energy_max"], w["M"], w["dt"], float(w["model"].volume)
        mu = P.gpuqt_moments(H, phi, phi, M)[0].real.contiguous()
        out = {"dos": P.gpuqt_kpm_reconstruct(mu, E, dE, vol)}
        for kind, call, mode in (("vac", P.gpuqt_vac, P.SIGMA_VAC), ("msd", P.gpuqt_msd, P.SIGMA_MSD)):
            if not w[kind]:
                continue
            c = call(H, phi, dts, M)[:, 0]
            rows = P.gpuqt_kpm_reconstruct(c.reshape(-1, M), E, dE, vol).reshape(len(dts), B, -1)
            out[kind] = rows
            out["sigma_" + kind] = [P.gpuqt_running_conductivity(mode, rows[:, b].contiguous(), dts)
                                    for b in range(B)]
        return out

    for r in runs:
        example(r)
    torch.cuda.synchronize()
    n = passes if passes is not None else args.steps
    per = [0.0, 0.0]
    for _ in range(n):
        for i, r in enumerate(runs):
            ta = time.perf_counter()
            example(r)
            torch.cuda.synchronize()
            per[i] += time.perf_counter() - ta
    per = [p / n for p in per]
    for r in runs:
        r["H"].close()
    return {"diffusive_s": per[0], "localized_s": per[1], "total_s": sum(per), "setup_s": setup_s,
            "passes": n, "paper_k40_total_s_context": 180.0,
            "workload": "2000^2 square W=4, DeltaE=6.1, M=1000, VAC+MSD 20 x 0.2, 601 energies, 1 vector; "
                        "4e6 chain W=4, DeltaE=4.1, M=500, MSD over 30 non-uniform steps 0.1..100, 401 "
                        "energies, 2 vectors as one block",
            "note": "the paper's about 3 minutes on a Tesla K40 include reading inputs and writing outputs; "
                    "here inputs are resident"}


def paper_workload(args):
    r = paper_examples(args)
    return dict(value=None, ms_per_step=r["total_s"] * 1e3,
                config={"workload": "the paper's two examples (Section 5): " + r["workload"],
                        "steps_timed": args.steps},
                paper_examples=r, roofline=None, cpu_baseline=None)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cubic",
                    choices=["cubic", "honeycomb", "honeycomb-general", "batched", "small", "train", "paper"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper examples on the default line")
    ap.add_argument("--variant", type=int, default=-1,
                    help="pin the kernel variant code of the timed handle instead of autotuning "
                         "(as gpuqt_h_info reports it: bits 0-1 load variant, 2-5 per-CU cap, 3 bits "
                         "per kernel family from bit 8)")
    ap.add_argument("--cpu-baseline", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_baseline:
        cpu_baseline_main(args.cpu_baseline)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; the workload shards over random vectors "
                                   "and realisations with no communication, but only --gpus 1 is run"}))
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    fn = {"cubic": cubic_workload, "honeycomb": honeycomb_workload,
          "honeycomb-general": lambda a: honeycomb_workload(a, general=True), "batched": batched_workload,
          "small": small_workload, "train": train_workload, "paper": paper_workload}[args.workload]
    r = fn(args)
    out = {"metric": METRIC, "value": r.pop("value"), "unit": UNIT, "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": r.pop("ms_per_step"),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128",
           "data": "synthetic"}
    out.update(r)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
