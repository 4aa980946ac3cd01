"""Measure kernel variants for the package's workloads on this GPU and write a tuning cache.

    python -m paper_1705_01387_amd.make_tune_cache OUT.tsv [--no-start-cache]

Runs gpuqt_autotune on the layouts of the benchmark and example workloads (cubic 200^3 at
B = 4 and B = 1, the 2,000,000-orbital honeycomb lattice in both storage modes, the uneven
square realisations at B = 16 and B = 1, the paper's two examples, the 64 x 64 square) and
saves every choice (gpuqt_tune_cache_save).  The library loads the package's tune_cache.tsv
when it starts, so the benchmark and its profiles then run the variant stored here instead
of re-deciding between variants that time within noise of each other.
"""
import os
import sys
import time

import numpy as np


def main(argv):
    if len(argv) < 2:
        print(__doc__)
        return 2
    out = argv[1]
    import torch

    import paper_1705_01387_amd as P
    from paper_1705_01387_amd import inputs as I

    if "--no-start-cache" in argv:
        P.gpuqt_tune_cache_clear()
    torch.cuda.set_device(0)

    def tune(H, B, what):
        t0 = time.perf_counter()
        times, hit = P.gpuqt_autotune_cached(H, B)
        print("%-40s B=%-2d variant %-9d %s (%.1f s) key: %s" % (what, B, H.info.kernel_variant,
                                                               "cached" if hit else "measured",
                                                               time.perf_counter() - t0,
                                                               P.gpuqt_tune_cache_key(H, B)), flush=True)

    w = I.workload_cubic(L=200, W=16.0, B=4)
    H = P.gpuqt_build_h_from_model(w["model"], energy_max=w["energy_max"])
    tune(H, 4, "cubic 200^3")
    tune(H, 1, "cubic 200^3")
    H.close()
    w = I.workload_honeycomb(n_vectors=1)
    for general in (False, True):
        H = P.gpuqt_build_h_from_model(w["model"], energy_max=w["energy_max"], no_dictionary=general)
        tune(H, 1, "honeycomb 2M" + (" per-entry" if general else ""))
        H.close()
    wb = I.workload_batched(B=16, M=16)
    cat = I.concat_segments(wb["models"])
    offs = np.cumsum([0] + [mm.n for mm in wb["models"]])
    H = P.gpuqt_build_h(cat.nn, cat.nbr, cat.hop, cat.onsite, cat.x, 0.0, cat.volume, 0.0,
                        seg_offsets=offs, seg_energy_max=wb["seg_energy_max"],
                        seg_length_x=[mm.length_x for mm in wb["models"]])
    tune(H, 16, "batched 8 segments")
    tune(H, 1, "batched 8 segments")
    H.close()
    for wp in (I.workload_paper_diffusive(), I.workload_paper_localized()):
        H = P.gpuqt_build_h_from_model(wp["model"], energy_max=wp["energy_max"])
        tune(H, wp["phi"].shape[1], wp["name"])
        H.close()
    ws = I.workload_square64()
    H = P.gpuqt_build_h_from_model(ws["model"], energy_max=ws["energy_max"])
    tune(H, 1, "square 64x64")
    H.close()
    P.gpuqt_tune_cache_save(out)
    print("wrote", os.path.abspath(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
