"""MI355X-native Liouville-Lanczos magnon library (arXiv:2203.01120).

The compute path is the HIP library ``libtm.so`` (C ABI in include/tm.h);
``binding`` marshals arguments to it.  PyTorch supplies device memory and
streams only.
"""
from .binding import (  # noqa: F401
    DIRS, FLAVOURS, TM_EBREAKDOWN, TM_EINVAL, TM_FP32, TM_FP64, TM_OK, Point, SystemDesc, TmError, load,
    tm_chain_begin, tm_chain_begin_multi, tm_chain_begin_lanes, tm_chain_coeffs, tm_chain_coeffs_lanes, tm_chain_lanes, tm_tensor_run, tm_chain_end, tm_chain_restore, tm_chain_save, tm_chains_step, tm_chains_use_graphs, tm_chi, tm_chi_extrapolated, tm_chi_tensor, tm_lanczos_run, tm_structure_factor, tm_liouvillian_apply, tm_liouvillian_apply_multi, tm_liouvillian_apply_noalloc, tm_autotune_enable, tm_autotune_force, tm_autotune_report, tm_profile_enable, tm_profile_read, tm_profile_reset,
    tm_qset_info_get, tm_start_vectors, tm_system_create, tm_system_destroy, tm_system_footprint, tm_system_memory, tm_system_resident_bytes,
    tm_system_set_resident_limit,
    tm_system_set_chain_slots,
)
