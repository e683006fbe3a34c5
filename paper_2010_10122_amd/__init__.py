"""wgrid for MI355X: the w-gridding radio-interferometry measurement operator of
Arras et al., "Efficient wide-field radio interferometry response"
(arXiv:2010.10122), as hand-written HIP kernels behind a C ABI.

    plan = Plan(uvw, freq, npix_x, npix_y, pixsize_x, pixsize_y, epsilon, "f32")
    vis = plan.degrid(dirty)        # forward operator R  (dirty2ms)
    img = plan.grid(vis)            # adjoint R^H, real part (ms2dirty)
"""
from ._lib import WgridError, WG_F32, WG_F64  # noqa: F401
from .plan import (Plan, Profiler, grid_size, kernel_map_error, kernel_params, kernel_poly,  # noqa: F401
                   kernel_psi, kernel_search, kernel_table, select_kernel)

__all__ = ["Plan", "Profiler", "WgridError", "WG_F32", "WG_F64", "grid_size", "kernel_params", "kernel_poly",
           "kernel_psi", "select_kernel", "kernel_search", "kernel_map_error", "kernel_table"]
