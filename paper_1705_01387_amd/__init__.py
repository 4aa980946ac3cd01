"""MI355X-native (gfx950) Chebyshev/KPM linear-scaling Kubo transport path.

The compute lives in libgpuqt.so (HIP kernels behind a C ABI, include/gpuqt.h);
this package binds its entry points under the same names (_binding) and holds
the seeded input generators (inputs).
"""
from ._binding import (  # noqa: F401
    GpuqtError, Hamiltonian, HInfo, LIB_PATH, lib,
    OP_MOMENTS, OP_EVOLVE, OP_EVOLVE_COMMUTATOR, OP_VAC, OP_MSD, OP_MOMENTS_BACKWARD, OP_AUTOTUNE,
    VELOCITY, COMMUTATOR_XH,
    gpuqt_build_h, gpuqt_build_h_from_model, gpuqt_workspace_size, gpuqt_moments, gpuqt_moments_plain, gpuqt_moments_noalloc, gpuqt_noalloc_scratch_bytes,
    gpuqt_evolve, gpuqt_apply_commutator, gpuqt_vac, gpuqt_msd, gpuqt_kpm_reconstruct,
    gpuqt_jackson, gpuqt_bessel, gpuqt_auto_terms, gpuqt_last_error, gpuqt_copy_probe,
    gpuqt_autotune, gpuqt_moments_backward, gpuqt_vac_backward, gpuqt_vac_backward_workspace_size,
    gpuqt_tie_entry_gradient,
    gpuqt_vac_tape_size, gpuqt_vac_record, gpuqt_vac_backward_tape, gpuqt_vac_backward_tape_workspace_size,
    gpuqt_update_h_values, gpuqt_kpm_reconstruct_adjoint, gpuqt_set_timing, gpuqt_timing, K_FAMILIES, gpuqt_set_variant,
    gpuqt_schedule_rows, gpuqt_running_conductivity, SIGMA_VAC, SIGMA_MSD, gpuqt_model_load, InputFolder,
    gpuqt_transport_lengths, gpuqt_tune_cache_key, gpuqt_autotune_cached, gpuqt_tune_cache_load,
    gpuqt_tune_cache_save, gpuqt_tune_cache_clear, gpuqt_autotune_block, TUNE_CACHE_PATH, gpuqt_build_h_tuned,
)
