"""Barnes-Hut regularized dipole sums on AMD Instinct MI355X (gfx950).

The compute path is libdps.so (hand-written HIP kernels, C ABI in
``include/dps.h``); this package is its Python binding plus a
``torch.autograd.Function`` wrapper.  PyTorch supplies device memory and
streams only.
"""
from .binding import (  # noqa: F401
    DpsError, Tree, dps_build, dps_get_kernel, dps_set_attributes, dps_query, dps_query_counts,
    dps_adjoint_zero, dps_adjoint_accumulate, dps_adjoint_finalize, dps_adjoint, dps_adjoint_noalloc,
    dps_export_tree, dps_tree_info, dps_set_launch, dps_get_launch, dps_set_split, dps_get_split,
    dps_query_channels,
    dps_adjoint_accumulate_channels, dps_adjoint_accumulate_grad, dps_adjoint_accumulate_ext,
    dps_adjoint_accumulate_from_forward,
    dps_adjoint_finalize_ext, dps_set_normals, dps_query_grid, dps_ray_march, dps_ray_march_harnack, dps_ray_resample, WANT_NORMALS, WANT_EPS, dps_check, dps_set_step_limit,
    dps_set_memory_limit, dps_destroy, LAUNCH_XCD_QUERY,
    LAUNCH_XCD_ADJOINT,
    LAUNCH_PERSISTENT_QUERY, LAUNCH_PERSISTENT_ADJOINT, LAUNCH_MARCH_WHOLE, dps_status_string, dps_last_error,
    load, LIB_PATH, EXPORTED, DPS_KERNEL_DIPOLE, DPS_KERNEL_MONOPOLE,
)
from .autograd import DipoleSum, dipole_sum  # noqa: F401
