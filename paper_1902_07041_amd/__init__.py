"""pfeig: polynomial-filtered interior eigensolver on one MI355X (gfx950).

Thin Python binding of the C-ABI library ``libpfeig.so`` (declared in
``include/pfeig.h``).  The functions here carry the C names and only marshal
arguments: numpy arrays are passed as host pointers, torch tensors on the GPU
as device pointers (PFE_DEVICE_PTRS).  Every numerical step runs in the
library's HIP kernels; if the library is missing the import of any function
fails loudly (there is no fallback).
"""
from ._capi import (PFE_FP32, PFE_FP64, PFE_SMOOTH_JACKSON, PFE_SMOOTH_LANCZOS, PFE_SMOOTH_NONE,
                    Filter, PfeError, STATUS, lib_path, load_library, pfe_apply_filter,
                    pfe_apply_filter_adjoint, pfe_apply_filter_noalloc, pfe_create,
                    pfe_design_filter, pfe_destroy,
                    pfe_device_bytes, pfe_eigvec_block_gradient, pfe_estimate_bounds,
                    pfe_estimate_count, pfe_last_error, pfe_set_bounds, pfe_set_hessian,
                    pfe_set_springs, pfe_count_moments, pfe_solve_sliced, pfe_design_dirac,
                    pfe_solve_lanczos, DiracFilter, pfe_locality_order,
                    pfe_solve_interval, pfe_spring_gradient, pfe_version)

__all__ = [
    "PFE_FP32", "PFE_FP64", "PFE_SMOOTH_JACKSON", "PFE_SMOOTH_LANCZOS", "PFE_SMOOTH_NONE",
    "Filter", "PfeError", "STATUS", "lib_path", "load_library", "pfe_apply_filter",
    "pfe_apply_filter_adjoint", "pfe_apply_filter_noalloc", "pfe_create", "pfe_design_filter",
    "pfe_destroy",
    "pfe_device_bytes", "pfe_eigvec_block_gradient", "pfe_estimate_bounds", "pfe_estimate_count",
    "pfe_last_error", "pfe_set_bounds", "pfe_set_hessian", "pfe_set_springs", "pfe_solve_interval",
    "pfe_spring_gradient", "pfe_version", "pfe_count_moments", "pfe_solve_sliced",
    "pfe_design_dirac", "pfe_solve_lanczos", "DiracFilter", "pfe_locality_order",
]
