"""Oracle O1: direct FP64 evaluation of eq. (3) and of its adjoint.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Thin ctypes wrapper
around oracle/dft.c (built by oracle/build.py); weights and the flag mask are
applied here: weights multiply the visibilities after the forward operator and
before the adjoint one, masked visibilities are zero on output and excluded
on input (Appendix B, parameters ``wgt`` and ``mask``).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        _lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        i32 = ctypes.POINTER(ctypes.c_int32)
        u8 = ctypes.POINTER(ctypes.c_uint8)
        _lib.o1_forward.argtypes = [ctypes.c_int64, ctypes.c_int64, dp, dp, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int64, ip, ctypes.c_int64, i32, i32, dp, dp, dp]
        _lib.o1_adjoint.argtypes = [ctypes.c_int64, ctypes.c_int64, dp, dp, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                    dp, dp, u8, ctypes.c_int64, i32, i32, dp]
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def forward(uvw, freq, dirty, pixsize_x, pixsize_y, do_wgridding=True, wgt=None, mask=None,
            vis_idx=None, pixels=None):
    """Visibilities of the image ``dirty`` [npix_x, npix_y].

    vis_idx: optional linear indices r*nchan+c to evaluate (default: all);
    pixels:  optional (p, q) index arrays restricting the sum to those pixels
             (the other pixels must be zero, e.g. a point-source image).
    Returns complex128 [nrow, nchan] (all) or [len(vis_idx)].
    """
    lib = _load()
    uvw = np.ascontiguousarray(uvw, dtype=np.float64)
    freq = np.ascontiguousarray(freq, dtype=np.float64)
    dirty = np.asarray(dirty, dtype=np.float64)
    nrow, nchan = uvw.shape[0], freq.shape[0]
    nx, ny = dirty.shape
    full = vis_idx is None
    if full:
        vis_idx = np.arange(nrow * nchan, dtype=np.int64)
    vis_idx = np.ascontiguousarray(vis_idx, dtype=np.int64)
    if pixels is None:
        pp, qq = np.nonzero(dirty != 0.0)
    else:
        pp, qq = pixels
    pp = np.ascontiguousarray(pp, dtype=np.int32)
    qq = np.ascontiguousarray(qq, dtype=np.int32)
    vals = np.ascontiguousarray(dirty[pp, qq], dtype=np.float64)
    ore = np.zeros(len(vis_idx))
    oim = np.zeros(len(vis_idx))
    lib.o1_forward(nrow, nchan, _ptr(uvw, ctypes.c_double), _ptr(freq, ctypes.c_double),
                   nx, ny, float(pixsize_x), float(pixsize_y), int(bool(do_wgridding)),
                   len(vis_idx), _ptr(vis_idx, ctypes.c_int64), len(pp),
                   _ptr(pp, ctypes.c_int32), _ptr(qq, ctypes.c_int32), _ptr(vals, ctypes.c_double),
                   _ptr(ore, ctypes.c_double), _ptr(oim, ctypes.c_double))
    out = ore + 1j * oim
    if wgt is not None:
        out = out * np.asarray(wgt, dtype=np.float64).reshape(-1)[vis_idx]
    if mask is not None:
        out = np.where(np.asarray(mask).reshape(-1)[vis_idx] != 0, out, 0.0)
    if full:
        out = out.reshape(nrow, nchan)
    return out


def adjoint(uvw, freq, vis, npix_x, npix_y, pixsize_x, pixsize_y, do_wgridding=True,
            wgt=None, mask=None, pixels=None):
    """Real dirty image from visibilities ``vis`` [nrow, nchan].

    pixels: optional (p, q) index arrays; returns the values there instead of
    the full [npix_x, npix_y] image.
    """
    lib = _load()
    uvw = np.ascontiguousarray(uvw, dtype=np.float64)
    freq = np.ascontiguousarray(freq, dtype=np.float64)
    nrow, nchan = uvw.shape[0], freq.shape[0]
    d = np.asarray(vis, dtype=np.complex128).reshape(nrow, nchan)
    if wgt is not None:
        d = d * np.asarray(wgt, dtype=np.float64).reshape(nrow, nchan)
    vre = np.ascontiguousarray(d.real)
    vim = np.ascontiguousarray(d.imag)
    sel = None
    if mask is not None:
        sel = np.ascontiguousarray((np.asarray(mask).reshape(nrow, nchan) != 0).astype(np.uint8))
    full = pixels is None
    if full:
        pp, qq = np.meshgrid(np.arange(npix_x), np.arange(npix_y), indexing="ij")
        pp, qq = pp.ravel(), qq.ravel()
    else:
        pp, qq = pixels
    pp = np.ascontiguousarray(pp, dtype=np.int32)
    qq = np.ascontiguousarray(qq, dtype=np.int32)
    out = np.zeros(len(pp))
    lib.o1_adjoint(nrow, nchan, _ptr(uvw, ctypes.c_double), _ptr(freq, ctypes.c_double),
                   npix_x, npix_y, float(pixsize_x), float(pixsize_y), int(bool(do_wgridding)),
                   _ptr(vre, ctypes.c_double), _ptr(vim, ctypes.c_double),
                   None if sel is None else _ptr(sel, ctypes.c_uint8),
                   len(pp), _ptr(pp, ctypes.c_int32), _ptr(qq, ctypes.c_int32),
                   _ptr(out, ctypes.c_double))
    if full:
        out = out.reshape(npix_x, npix_y)
    return out
