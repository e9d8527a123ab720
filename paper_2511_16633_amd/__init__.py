"""MI355X-native ray-Born single-step inversion (Hessian-free, arXiv 2511.16633).

Thin Python binding over ``librayborn.so`` (C ABI in ``include/rayborn.h``).
Every computation runs in the library's HIP kernels; this module only
marshals arguments: torch tensors supply device memory and streams.  The
binding raises if the library has not been built; there is no fallback.
"""
from ._binding import (  # noqa: F401
    DTYPES,
    RayBornError,
    NumericError,
    lib,
    lib_path,
    geometry_struct,
    trace_opts_struct,
    invert_opts_struct,
    alloc_tables,
    trace_workspace_bytes,
    green_workspace_bytes,
    forward_workspace_bytes,
    adjoint_workspace_bytes,
    invert_workspace_bytes,
    invert_cg_workspace_bytes,
    invert_asymptotic_workspace_bytes,
    tof_workspace_bytes,
    trace_rays,
    build_green,
    born_forward,
    born_adjoint_weighted,
    born_adjoint_weighted_noalloc,
    born_hessian_banded,
    invert_frequency_set,
    invert_frequency_sets_grouped,
    invert_frequency_set_cg,
    invert_frequency_set_asymptotic,
    tof_invert,
    version,
)
