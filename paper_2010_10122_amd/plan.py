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


class Plan:
    """A w-gridding operator for fixed coordinates and image geometry.

    uvw   [n_rows, 3] float64 (metres), freq [n_chan] float64 (Hz) and the
    optional mask [n_rows, n_chan] uint8 must be CUDA tensors; they are kept
    alive by the plan and must not be modified while it is in use.
    precision: "f32" (epsilon >= 1e-5) or "f64".
    alpha/sigma force a printed Appendix-A kernel; planes_per_batch forces
    the w-plane batch size.
    """

    def __init__(self, uvw, freq, npix_x, npix_y, pixsize_x, pixsize_y, epsilon, precision="f32",
                 do_wgridding=True, mask=None, alpha=None, sigma=None, planes_per_batch=None, stream=None):
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
        d = _lib.PlanDesc()
        d.uvw = uvw.data_ptr()
        d.freq = freq.data_ptr()
        d.mask = mask.data_ptr() if mask is not None else None
        d.n_rows = self.n_rows
        d.n_chan = self.n_chan
        d.npix_x = self.npix_x
        d.npix_y = self.npix_y
        d.pixsize_x = float(pixsize_x)
        d.pixsize_y = float(pixsize_y)
        d.epsilon = float(epsilon)
        d.precision = self.precision
        d.do_wgridding = 1 if do_wgridding else 0
        d.alpha = int(alpha or 0)
        d.sigma = float(sigma or 0.0)
        d.planes_per_batch = int(planes_per_batch or 0)
        d.stream = _stream_handle(stream).value
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

    def close(self):
        if getattr(self, "_h", None):
            self._lib.wg_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _workspace(self, workspace):
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
        if out is None:
            out = torch.empty((self.n_rows, self.n_chan), dtype=self.complex_dtype, device=self.device)
        ws = self._workspace(workspace)
        rc = self._lib.wg_degrid(self._h, _dev_ptr(dirty), _dev_ptr(wgt), _dev_ptr(out), _dev_ptr(ws),
                                 ws.numel(), _stream_handle(stream))
        _lib.check(rc, "wg_degrid")
        return out

    def grid(self, vis, wgt=None, out=None, workspace=None, stream=None):
        """Adjoint operator (ms2dirty): real dirty image [npix_x, npix_y] of ``vis``."""
        if not (vis.is_cuda and vis.dtype == self.complex_dtype and vis.is_contiguous()
                and tuple(vis.shape) == (self.n_rows, self.n_chan)):
            raise TypeError(f"vis must be a contiguous CUDA {self.complex_dtype} tensor "
                            f"[{self.n_rows}, {self.n_chan}]")
        wgt = self._check_wgt(wgt)
        if out is None:
            out = torch.empty((self.npix_x, self.npix_y), dtype=self.real_dtype, device=self.device)
        ws = self._workspace(workspace)
        rc = self._lib.wg_grid(self._h, _dev_ptr(vis), _dev_ptr(wgt), _dev_ptr(out), _dev_ptr(ws),
                               ws.numel(), _stream_handle(stream))
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
