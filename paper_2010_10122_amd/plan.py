"""Python front-end of the wgrid C ABI.

``Plan`` wraps ``wg_plan_create``; ``Plan.degrid`` / ``Plan.grid`` wrap
``wg_degrid`` / ``wg_grid``.  PyTorch provides device memory and the stream;
every step of the operator runs in the HIP kernels of libwgrid.so.  The
calls follow the paper's interface (Appendix B: ``dirty2ms`` / ``ms2dirty``
with uvw, freq, pixel sizes, epsilon, do_wstacking, wgt and mask).
"""
import ctypes

import numpy as np
import torch

from . import _lib

_DTYPES = {
    _lib.WG_F32: (torch.float32, torch.complex64),
    _lib.WG_F64: (torch.float64, torch.complex128),
}


# column transform of the u axis: planner's choice, one pass, four-step
_COLUMN_TRANSFORMS = {None: 0, "auto": 0, "one-pass": 1, "four-step": 2}


def _precision_of(p):
    if p in (_lib.WG_F32, "f32", "float32", torch.float32, torch.complex64, np.float32, np.complex64):
        return _lib.WG_F32
    if p in (_lib.WG_F64, "f64", "float64", torch.float64, torch.complex128, np.float64, np.complex128):
        return _lib.WG_F64
    raise ValueError(f"unknown precision {p!r}")


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class _TorchAllocator:
    """Device-memory callbacks of the C ABI served by PyTorch's caching
    allocator, so that plan memory is pooled with the rest of the program's.
    Blocks are associated with the plan's construction stream; the ctypes
    callables must outlive the plan."""

    def __init__(self, device, stream):
        self.device = device
        self.stream = stream
        self.c_alloc = _lib._alloc_fn(self._alloc)
        self.c_free = _lib._free_fn(self._free)

    def _alloc(self, ctx, nbytes):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
        except Exception:          # out of memory: the library reports WG_ENOMEM
            return None

    def _free(self, ctx, ptr):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:          # interpreter shutdown
            pass


def _fill_desc(d, uvw, freq, mask, npix_x, npix_y, pixsize_x, pixsize_y, epsilon, precision, do_wgridding,
               alpha, sigma, planes_per_batch, stream, allocator, column_transform=None):
    d.uvw = uvw.data_ptr()
    d.freq = freq.data_ptr()
    d.mask = mask.data_ptr() if mask is not None else None
    d.n_rows = int(uvw.shape[0])
    d.n_chan = int(freq.shape[0])
    d.npix_x = int(npix_x)
    d.npix_y = int(npix_y)
    d.pixsize_x = float(pixsize_x)
    d.pixsize_y = float(pixsize_y)
    d.epsilon = float(epsilon)
    d.precision = precision
    d.do_wgridding = 1 if do_wgridding else 0
    d.alpha = int(alpha or 0)
    d.sigma = float(sigma or 0.0)
    d.planes_per_batch = int(planes_per_batch or 0)
    d.column_transform = _COLUMN_TRANSFORMS[column_transform]
    d.stream = _stream_handle(stream).value
    if allocator is not None:
        d.alloc = allocator.c_alloc
        d.free = allocator.c_free
    return d


class Plan:
    """A w-gridding operator for fixed coordinates and image geometry.

    uvw   [n_rows, 3] float64 (metres), freq [n_chan] float64 (Hz) and the
    optional mask [n_rows, n_chan] uint8 must be CUDA tensors; they are kept
    alive by the plan and must not be modified while it is in use.
    precision: "f32" (epsilon >= 1e-5) or "f64".
    alpha/sigma force a kernel of the planner's table (wg_kernel_table);
    planes_per_batch forces the w-plane batch size.
    column_transform: None/"auto", "one-pass" or "four-step" (u transform
    form; results agree to rounding).
    """

    def __init__(self, uvw, freq, npix_x, npix_y, pixsize_x, pixsize_y, epsilon, precision="f32",
                 do_wgridding=True, mask=None, alpha=None, sigma=None, planes_per_batch=None, stream=None,
                 torch_allocator=True, column_transform=None):
        lib = _lib.load()
        for name, t, dt in (("uvw", uvw, torch.float64), ("freq", freq, torch.float64)):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.is_contiguous()):
                raise TypeError(f"{name} must be a contiguous CUDA {dt} tensor")
        if uvw.dim() != 2 or uvw.shape[1] != 3 or freq.dim() != 1:
            raise ValueError("uvw must be [n_rows, 3] and freq [n_chan]")
        if mask is not None:
            if not (mask.is_cuda and mask.dtype == torch.uint8 and mask.is_contiguous()
                    and tuple(mask.shape) == (uvw.shape[0], freq.shape[0])):
                raise TypeError("mask must be a contiguous CUDA uint8 tensor [n_rows, n_chan]")
        self.uvw, self.freq, self.mask = uvw, freq, mask
        self.precision = _precision_of(precision)
        self.real_dtype, self.complex_dtype = _DTYPES[self.precision]
        self.n_rows, self.n_chan = int(uvw.shape[0]), int(freq.shape[0])
        self.npix_x, self.npix_y = int(npix_x), int(npix_y)
        self.device = uvw.device
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        # device memory of the plan comes from PyTorch's caching allocator
        # (torch_allocator=False: hipMalloc / hipFree inside the library)
        self._alloc = _TorchAllocator(self.device, stream) if torch_allocator else None
        d = _fill_desc(_lib.PlanDesc(), uvw, freq, mask, npix_x, npix_y, pixsize_x, pixsize_y, epsilon,
                       self.precision, do_wgridding, alpha, sigma, planes_per_batch, stream, self._alloc,
                       column_transform)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = lib.wg_plan_create(ctypes.byref(d), ctypes.byref(handle))
        _lib.check(rc, "wg_plan_create")
        self._h = handle
        self._lib = lib
        self.info = self._info()
        self.workspace_bytes = int(self.info["workspace_bytes"])

    def _info(self):
        inf = _lib.PlanInfo()
        _lib.check(self._lib.wg_plan_info(self._h, ctypes.byref(inf)), "wg_plan_info")
        return {name: getattr(inf, name) for name, _ in _lib.PlanInfo._fields_}

    @staticmethod
    def estimate(uvw, freq, npix_x, npix_y, pixsize_x, pixsize_y, epsilon, precision="f32", do_wgridding=True,
                 mask=None, alpha=None, sigma=None, planes_per_batch=None, stream=None, column_transform=None):
        """Device bytes (plan, peak during construction, workspace bound) of the
        plan these arguments would build, without building it
        (``wg_plan_estimate``)."""
        lib = _lib.load()
        dev = uvw.device
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        alloc = _TorchAllocator(dev, stream)
        d = _fill_desc(_lib.PlanDesc(), uvw, freq, mask, npix_x, npix_y, pixsize_x, pixsize_y, epsilon,
                       _precision_of(precision), do_wgridding, alpha, sigma, planes_per_batch, stream, alloc,
                       column_transform)
        pb, pk, wb = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        with torch.cuda.device(dev):
            rc = lib.wg_plan_estimate(ctypes.byref(d), ctypes.byref(pb), ctypes.byref(pk), ctypes.byref(wb))
        _lib.check(rc, "wg_plan_estimate")
        return {"plan_bytes": pb.value, "peak_bytes": pk.value, "workspace_bytes": wb.value}

    def close(self):
        """Release the plan's device memory.  No apply call on the plan may be
        running on any stream."""
        if getattr(self, "_h", None):
            self._lib.wg_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _workspace(self, workspace):
        # (called under the launch stream, so the block belongs to that stream)
        if workspace is None:
            return torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8, device=self.device)
        if workspace.numel() * workspace.element_size() < self.workspace_bytes or not workspace.is_cuda:
            raise ValueError("workspace too small")
        return workspace

    def _check_wgt(self, wgt):
        if wgt is None:
            return None
        if not (wgt.is_cuda and wgt.dtype == self.real_dtype and wgt.is_contiguous()
                and tuple(wgt.shape) == (self.n_rows, self.n_chan)):
            raise TypeError(f"wgt must be a contiguous CUDA {self.real_dtype} tensor [n_rows, n_chan]")
        return wgt

    def degrid(self, dirty, wgt=None, out=None, workspace=None, stream=None):
        """Forward operator (dirty2ms): visibilities [n_rows, n_chan] of ``dirty``."""
        if not (dirty.is_cuda and dirty.dtype == self.real_dtype and dirty.is_contiguous()
                and tuple(dirty.shape) == (self.npix_x, self.npix_y)):
            raise TypeError(f"dirty must be a contiguous CUDA {self.real_dtype} tensor "
                            f"[{self.npix_x}, {self.npix_y}]")
        wgt = self._check_wgt(wgt)
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.stream(st):
            if out is None:
                out = torch.empty((self.n_rows, self.n_chan), dtype=self.complex_dtype, device=self.device)
            ws = self._workspace(workspace)
            rc = self._lib.wg_degrid(self._h, _dev_ptr(dirty), _dev_ptr(wgt), _dev_ptr(out), _dev_ptr(ws),
                                     ws.numel(), _stream_handle(st))
        _lib.check(rc, "wg_degrid")
        return out

    def grid(self, vis, wgt=None, out=None, workspace=None, stream=None):
        """Adjoint operator (ms2dirty): real dirty image [npix_x, npix_y] of ``vis``."""
        if not (vis.is_cuda and vis.dtype == self.complex_dtype and vis.is_contiguous()
                and tuple(vis.shape) == (self.n_rows, self.n_chan)):
            raise TypeError(f"vis must be a contiguous CUDA {self.complex_dtype} tensor "
                            f"[{self.n_rows}, {self.n_chan}]")
        wgt = self._check_wgt(wgt)
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.stream(st):
            if out is None:
                out = torch.empty((self.npix_x, self.npix_y), dtype=self.real_dtype, device=self.device)
            ws = self._workspace(workspace)
            rc = self._lib.wg_grid(self._h, _dev_ptr(vis), _dev_ptr(wgt), _dev_ptr(out), _dev_ptr(ws),
                                   ws.numel(), _stream_handle(st))
        _lib.check(rc, "wg_grid")
        return out

    def index(self, stream=None):
        """(keys uint64 as int64 tensor, order int32 tensor) of the visibility index."""
        n = int(self.info["n_vis"])
        keys = torch.empty(n, dtype=torch.int64, device=self.device)
        order = torch.empty(n, dtype=torch.int32, device=self.device)
        _lib.check(self._lib.wg_plan_index(self._h, _dev_ptr(keys), _dev_ptr(order), _stream_handle(stream)),
                   "wg_plan_index")
        return keys, order


    def grid_order(self, stream=None):
        """Linear indices of the visibilities in the gridder's own order
        (by tile, edge rank and first plane; ``wg_plan_grid_order``)."""
        n = int(self.info["n_vis"])
        order2 = torch.empty(n, dtype=torch.int32, device=self.device)
        _lib.check(self._lib.wg_plan_grid_order(self._h, _dev_ptr(order2), _stream_handle(stream)),
                   "wg_plan_grid_order")
        return order2


class Profiler:
    """Per-kernel HIP-event timing of wg_grid / wg_degrid launches made by the
    calling thread while attached (``with Profiler() as prof: ...``)."""

    def __init__(self):
        self._lib = _lib.load()
        h = ctypes.c_void_p()
        _lib.check(self._lib.wg_profiler_create(ctypes.byref(h)), "wg_profiler_create")
        self._h = h

    def __enter__(self):
        self._lib.wg_profiler_attach(self._h)
        return self

    def __exit__(self, *exc):
        self._lib.wg_profiler_attach(None)
        return False

    def reset(self):
        _lib.check(self._lib.wg_profiler_reset(self._h), "wg_profiler_reset")

    def read(self):
        """{kind: (total_ms, launches)} for every kernel kind."""
        out = {}
        for k, name in enumerate(_lib.KIND_NAMES):
            ms, n = ctypes.c_double(), ctypes.c_int64()
            _lib.check(self._lib.wg_profiler_read(self._h, k, ctypes.byref(ms), ctypes.byref(n)),
                       "wg_profiler_read")
            out[name] = (ms.value, n.value)
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.wg_profiler_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- host-only helpers --------------------------------------------------------

def grid_size(sigma, npix):
    n = _lib.load().wg_grid_size(float(sigma), int(npix))
    _lib.check(min(n, 0), "wg_grid_size")
    return n


def kernel_params(alpha, sigma):
    e, b, m = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _lib.check(_lib.load().wg_kernel_params(int(alpha), float(sigma), ctypes.byref(e), ctypes.byref(b),
                                            ctypes.byref(m)), "wg_kernel_params")
    return e.value, b.value, m.value


def select_kernel(epsilon, precision, do_wgridding, npix_x, npix_y, pixsize_x, pixsize_y, n_vis, wmin, wmax):
    a, s = ctypes.c_int(), ctypes.c_double()
    _lib.check(_lib.load().wg_select_kernel(float(epsilon), _precision_of(precision), int(bool(do_wgridding)),
                                            int(npix_x), int(npix_y), float(pixsize_x), float(pixsize_y),
                                            int(n_vis), float(wmin), float(wmax), ctypes.byref(a),
                                            ctypes.byref(s)), "wg_select_kernel")
    return a.value, s.value


def kernel_poly(alpha, sigma, precision="f64"):
    """(coefficients [alpha, degree+1], degree) of the piecewise polynomial."""
    lib = _lib.load()
    deg = ctypes.c_int()
    _lib.check(lib.wg_kernel_poly(int(alpha), float(sigma), _precision_of(precision), None, 0,
                                  ctypes.byref(deg)), "wg_kernel_poly")
    buf = np.zeros(alpha * (deg.value + 1))
    _lib.check(lib.wg_kernel_poly(int(alpha), float(sigma), _precision_of(precision),
                                  buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), buf.size,
                                  ctypes.byref(deg)), "wg_kernel_poly")
    return buf.reshape(alpha, deg.value + 1), deg.value


def kernel_psi(alpha, sigma, k):
    k = np.ascontiguousarray(k, dtype=np.float64)
    out = np.zeros_like(k)
    _lib.check(_lib.load().wg_kernel_psi(int(alpha), float(sigma),
                                         k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), k.size,
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "wg_kernel_psi")
    return out


def kernel_search(alpha, sigma, start=None):
    """(beta, mu, eps): the sup-norm search of the map error function over the
    modified ES kernel's parameters (Sect. 3.2, eq. maperror); ``start`` an
    optional extra starting point (beta, mu)."""
    b = ctypes.c_double(start[0] if start else 0.0)
    m = ctypes.c_double(start[1] if start else 0.0)
    e = ctypes.c_double()
    _lib.check(_lib.load().wg_kernel_search(int(alpha), float(sigma), ctypes.byref(b), ctypes.byref(m),
                                            ctypes.byref(e)), "wg_kernel_search")
    return b.value, m.value, e.value


def kernel_map_error(alpha, sigma, beta, mu):
    """Supremum over the retained band of the map error function (eq. maperror)."""
    e = ctypes.c_double()
    _lib.check(_lib.load().wg_kernel_map_error(int(alpha), float(sigma), float(beta), float(mu), ctypes.byref(e)),
               "wg_kernel_map_error")
    return e.value


def kernel_table():
    """Rows (alpha, sigma, eps, beta, mu, printed) of the planner's kernel table."""
    lib = _lib.load()
    rows = []
    i = 0
    while True:
        a, s, e, b, m, pr = (ctypes.c_int(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double(),
                             ctypes.c_double(), ctypes.c_int())
        if lib.wg_kernel_table(i, ctypes.byref(a), ctypes.byref(s), ctypes.byref(e), ctypes.byref(b), ctypes.byref(m),
                               ctypes.byref(pr)) != _lib.WG_OK:
            return rows
        rows.append((a.value, s.value, e.value, b.value, m.value, bool(pr.value)))
        i += 1
