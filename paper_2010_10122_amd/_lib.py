"""ctypes binding of the wgrid C ABI (include/wgrid.h).  Marshalling only."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwgrid.so")

WG_OK, WG_EINVAL, WG_ENOMEM, WG_EHIP, WG_EUNSUPPORTED, WG_ESCRATCH = 0, -1, -2, -3, -4, -5
WG_SCRATCH_BYTES = 128 << 20
WG_F32, WG_F64 = 0, 1

_alloc_fn = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)
_free_fn = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("uvw", ctypes.c_void_p),
        ("freq", ctypes.c_void_p),
        ("mask", ctypes.c_void_p),
        ("n_rows", ctypes.c_int64),
        ("n_chan", ctypes.c_int64),
        ("npix_x", ctypes.c_int),
        ("npix_y", ctypes.c_int),
        ("pixsize_x", ctypes.c_double),
        ("pixsize_y", ctypes.c_double),
        ("epsilon", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("do_wgridding", ctypes.c_int),
        ("alpha", ctypes.c_int),
        ("sigma", ctypes.c_double),
        ("planes_per_batch", ctypes.c_int),
        ("column_transform", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("alloc", _alloc_fn),
        ("free", _free_fn),
        ("alloc_ctx", ctypes.c_void_p),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("alpha", ctypes.c_int),
        ("sigma", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("eps_kernel", ctypes.c_double),
        ("poly_degree", ctypes.c_int),
        ("nu", ctypes.c_int),
        ("nv", ctypes.c_int),
        ("nw", ctypes.c_int),
        ("dw", ctypes.c_double),
        ("w0", ctypes.c_double),
        ("wmin", ctypes.c_double),
        ("wmax", ctypes.c_double),
        ("npix_x", ctypes.c_int),
        ("npix_y", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("do_wgridding", ctypes.c_int),
        ("n_rows", ctypes.c_int64),
        ("n_chan", ctypes.c_int64),
        ("n_vis", ctypes.c_int64),
        ("planes_per_batch", ctypes.c_int),
        ("tile", ctypes.c_int),
        ("bytes_grid", ctypes.c_double),
        ("bytes_degrid", ctypes.c_double),
        ("predicted_seconds", ctypes.c_double),
        ("plan_bytes", ctypes.c_size_t),
        ("index_bytes", ctypes.c_size_t),
        ("workspace_bytes", ctypes.c_size_t),
        ("extra_items_grid", ctypes.c_int64),
        ("extra_items_degrid", ctypes.c_int64),
        ("rounding_error", ctypes.c_double),
        ("amplification", ctypes.c_double),
        ("poly_error", ctypes.c_double),
        ("column_transform", ctypes.c_int),
        ("col_n1", ctypes.c_int),
        ("col_n2", ctypes.c_int),
        ("col_k", ctypes.c_int),
    ]


EXPORTS = [
    "wg_plan_create", "wg_plan_destroy", "wg_plan_estimate", "wg_degrid", "wg_grid", "wg_apply_noalloc",
    "wg_plan_info",
    "wg_workspace_bytes", "wg_plan_bytes", "wg_plan_index", "wg_plan_grid_order", "wg_strerror", "wg_grid_size",
    "wg_kernel_params", "wg_select_kernel", "wg_kernel_poly", "wg_kernel_psi", "wg_kernel_search",
    "wg_kernel_map_error", "wg_kernel_table",
    "wg_profiler_create", "wg_profiler_destroy", "wg_profiler_attach", "wg_profiler_read",
    "wg_profiler_reset", "wg_kernel_kind_name",
]

KIND_NAMES = ["grid", "degrid", "fft_rows_grid", "fft_cols_grid", "fft_rows_degrid", "fft_cols_degrid",
              "image", "vis"]

_lib = None


class WgridError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} (code {code})")


def load():
    """Load libwgrid.so; raises ImportError if it has not been built (there is
    no fallback implementation)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, dp, ip = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    lib.wg_plan_create.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(vp)]
    lib.wg_plan_create.restype = ctypes.c_int
    lib.wg_plan_destroy.argtypes = [vp]
    lib.wg_plan_destroy.restype = ctypes.c_int
    sz = ctypes.POINTER(ctypes.c_size_t)
    lib.wg_plan_estimate.argtypes = [ctypes.POINTER(PlanDesc), sz, sz, sz]
    lib.wg_plan_estimate.restype = ctypes.c_int
    for fn in (lib.wg_degrid, lib.wg_grid):
        fn.argtypes = [vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        fn.restype = ctypes.c_int
    lib.wg_apply_noalloc.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    lib.wg_apply_noalloc.restype = ctypes.c_int
    lib.wg_plan_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.wg_plan_info.restype = ctypes.c_int
    lib.wg_workspace_bytes.argtypes = [vp]
    lib.wg_workspace_bytes.restype = ctypes.c_size_t
    lib.wg_plan_bytes.argtypes = [vp]
    lib.wg_plan_bytes.restype = ctypes.c_size_t
    lib.wg_plan_index.argtypes = [vp, vp, vp, vp]
    lib.wg_plan_index.restype = ctypes.c_int
    lib.wg_plan_grid_order.argtypes = [vp, vp, vp]
    lib.wg_plan_grid_order.restype = ctypes.c_int
    lib.wg_strerror.argtypes = [ctypes.c_int]
    lib.wg_strerror.restype = ctypes.c_char_p
    lib.wg_grid_size.argtypes = [ctypes.c_double, ctypes.c_int]
    lib.wg_grid_size.restype = ctypes.c_int
    lib.wg_kernel_params.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp]
    lib.wg_kernel_params.restype = ctypes.c_int
    lib.wg_select_kernel.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double, i64, ctypes.c_double, ctypes.c_double,
                                     ip, dp]
    lib.wg_select_kernel.restype = ctypes.c_int
    lib.wg_kernel_poly.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, ctypes.c_int, ip]
    lib.wg_kernel_poly.restype = ctypes.c_int
    lib.wg_kernel_psi.argtypes = [ctypes.c_int, ctypes.c_double, dp, ctypes.c_int, dp]
    lib.wg_kernel_psi.restype = ctypes.c_int
    lib.wg_kernel_search.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp]
    lib.wg_kernel_search.restype = ctypes.c_int
    lib.wg_kernel_map_error.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
    lib.wg_kernel_map_error.restype = ctypes.c_int
    lib.wg_kernel_table.argtypes = [ctypes.c_int, ip, dp, dp, dp, dp, ip]
    lib.wg_kernel_table.restype = ctypes.c_int
    lib.wg_profiler_create.argtypes = [ctypes.POINTER(vp)]
    lib.wg_profiler_create.restype = ctypes.c_int
    lib.wg_profiler_destroy.argtypes = [vp]
    lib.wg_profiler_destroy.restype = ctypes.c_int
    lib.wg_profiler_attach.argtypes = [vp]
    lib.wg_profiler_attach.restype = ctypes.c_int
    lib.wg_profiler_read.argtypes = [vp, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int64)]
    lib.wg_profiler_read.restype = ctypes.c_int
    lib.wg_profiler_reset.argtypes = [vp]
    lib.wg_profiler_reset.restype = ctypes.c_int
    lib.wg_kernel_kind_name.argtypes = [ctypes.c_int]
    lib.wg_kernel_kind_name.restype = ctypes.c_char_p
    _lib = lib
    return lib


def strerror(code):
    try:
        return load().wg_strerror(int(code)).decode()
    except ImportError:
        return f"error {code}"


def check(code, where):
    if code != WG_OK:
        raise WgridError(code, where)
