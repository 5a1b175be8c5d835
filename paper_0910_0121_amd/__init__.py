"""MI355X short-range TreePM tree force (GreeM, arXiv:0910.0121) -- Python binding.

Thin ctypes marshalling over ``libtreepm.so``: every function here has the name of the C
entry point it calls (``include/treepm.h``) and does nothing but convert arguments.  Device
buffers are torch CUDA tensors (PyTorch provides device memory and streams only); host
buffers may be numpy arrays or CPU tensors.  If the library has not been built, importing
the functions raises immediately -- there is no fallback path.
"""
from ._native import (  # noqa: F401
    TREEPM_DEVICE,
    TREEPM_FP32,
    TREEPM_FP64,
    TREEPM_HOST,
    TREEPM_OPEN_DISTANCE,
    TREEPM_OPEN_FIXED,
    TREEPM_OK,
    TREEPM_PENDING,
    TreePMError,
    lib,
    make_params,
    treepm_autotune,
    treepm_build,
    treepm_ens_create,
    treepm_ens_destroy,
    treepm_ens_info,
    treepm_ensemble_poll,
    treepm_ensemble_submit,
    treepm_create,
    treepm_destroy,
    treepm_release_cached,
    treepm_export_groups,
    treepm_export_lists,
    treepm_export_nodes,
    treepm_export_sorted,
    treepm_eps_of_z,
    treepm_force_long,
    treepm_kick_drift,
    treepm_kick_short,
    treepm_timestep,
    treepm_timestep_noalloc,
    treepm_force_short,
    treepm_force_short_batch,
    treepm_ens_set_batching,
    treepm_get_stats,
    treepm_last_error,
    treepm_pairwise_f32,
    treepm_params,
    treepm_set_params,
    treepm_set_timing,
    treepm_stats,
    treepm_version,
    treepm_walk,
)
