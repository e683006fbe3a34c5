"""Oracle: plan geometry and visibility binning, plain FP64 numpy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Written from the paper's
definitions, independently of the product's host planner:

* grid size N = ceil(sigma * n) (Sect. 2, oversampled grid), rounded up to the
  smallest multiple of 16 whose prime factors are all in {2, 3, 5, 7} (reading:
  the FFT length must have small factors and whole 16-cell tiles);
* Delta w = 1 / (2 sigma max|n_lm - 1|) (Sect. 2, Nyquist condition);
* w_o = min w - Delta w (alpha - 1)/2 (eq. wcirc), and
  N_w = ceil((max w - min w)/Delta w) + alpha (reading of the non-integer
  plane count in Sect. 2), with w taken after the Hermitian fold
  (eq. Hermitian-symmetry) so that w >= 0;
* visibility binning into 16x16 uv tiles keyed by (t_u, t_v, t_w), sorted
  lexicographically, ties in (row, channel) order (Sect. 4.3).

Binning arithmetic follows one fixed sequence of correctly rounded FP64
operations (numpy applies no fused multiply-add), so that the key of every
visibility is reproducible bit for bit.
"""
import math
import numpy as np

C_LIGHT = 299792458.0     # m/s (SI exact value; the paper does not state it)
TILE = 16                 # uv tile edge in grid cells (Sect. 4.3)


def good_size(n_min):
    """Smallest N >= n_min, N % 16 == 0, all prime factors in {2,3,5,7}."""
    n = int(n_min)
    n += (-n) % TILE
    while True:
        m = n
        for p in (2, 3, 5, 7):
            while m % p == 0:
                m //= p
        if m == 1:
            return n
        n += TILE


def grid_size(sigma, npix):
    return good_size(math.ceil(sigma * npix))


def lm_grid(npix_x, npix_y, pixsize_x, pixsize_y):
    """Direction cosines of the pixel centres (Sect. 2, sets L and M) and
    n - 1 in the cancellation-free form -(l^2+m^2)/(1+n)."""
    l = (np.arange(npix_x, dtype=np.float64) - npix_x // 2) * pixsize_x
    m = (np.arange(npix_y, dtype=np.float64) - npix_y // 2) * pixsize_y
    rho = l[:, None] ** 2 + m[None, :] ** 2
    n = np.sqrt(1.0 - rho)
    nm1 = -rho / (1.0 + n)
    return l, m, n, nm1


def max_abs_nm1(npix_x, npix_y, pixsize_x, pixsize_y):
    """max over the pixel grid of |n - 1|: attained at the corner pixel (0, 0),
    which has the largest |l| and |m|."""
    l = (0 - npix_x // 2) * pixsize_x
    m = (0 - npix_y // 2) * pixsize_y
    rho = l * l + m * m
    n = math.sqrt(1.0 - rho)
    return rho / (1.0 + n)


def effective_w(uvw, freq, mask=None, do_wgridding=True):
    """|w| in wavelengths of every selected visibility (after the fold)."""
    s = np.asarray(freq, dtype=np.float64) / C_LIGHT
    w = np.abs(np.multiply.outer(uvw[:, 2], s))
    if mask is not None:
        w = w[np.asarray(mask) != 0]
    return w.ravel()


def make_plan(uvw, freq, npix_x, npix_y, pixsize_x, pixsize_y, alpha, sigma,
              do_wgridding=True, mask=None, table=None):
    """All plan quantities for a given kernel support alpha and oversampling
    sigma (the kernel row comes from Appendix A)."""
    from .kernel import table_row
    _, eps_k, beta, mu = table_row(alpha, sigma) if table is None else table
    nx = grid_size(sigma, npix_x)
    ny = grid_size(sigma, npix_y)
    p = dict(alpha=alpha, sigma=sigma, beta=beta, mu=mu, eps_k=eps_k,
             nu=nx, nv=ny, npix_x=npix_x, npix_y=npix_y,
             pixsize_x=pixsize_x, pixsize_y=pixsize_y,
             do_wgridding=bool(do_wgridding))
    if do_wgridding:
        w = effective_w(uvw, freq, mask, True)
        if w.size == 0:
            wmin = wmax = 0.0
        else:
            wmin, wmax = float(w.min()), float(w.max())
        dw = 1.0 / (2.0 * sigma * max_abs_nm1(npix_x, npix_y, pixsize_x, pixsize_y))
        w0 = wmin - dw * (alpha - 1) * 0.5
        nw = int(math.ceil((wmax - wmin) / dw)) + alpha
        p.update(wmin=wmin, wmax=wmax, dw=dw, w0=w0, nw=nw)
    else:
        p.update(wmin=0.0, wmax=0.0, dw=1.0, w0=0.0, nw=1)
    return p


def bin_visibilities(uvw, freq, plan, mask=None):
    """Binning spec: per selected visibility (row r, channel c) the tile key and
    the kernel anchor cells, in one fixed FP64 operation order.

    Returns dict with, per selected visibility in (row, chan) order:
      idx   linear index r*nchan + c       (int64)
      flip  Hermitian fold applied          (bool)
      gu, gv  grid coordinates in cells     (float64, in [0, N])
      xw    w coordinate in planes          (float64)
      iu, iv  first touched cell, wrapped   (int64, in [0, N))
      iw    first touched plane             (int64)
      key   ((iu>>4) * NTv + (iv>>4)) * N_w + iw   (uint64)
    and ``order`` = stable argsort of key.
    """
    nrow, nchan = uvw.shape[0], len(freq)
    alpha = plan["alpha"]
    nu, nv, nw = plan["nu"], plan["nv"], plan["nw"]
    half = 0.5 * alpha
    s = np.asarray(freq, dtype=np.float64) / C_LIGHT                 # [nchan]
    uu = uvw[:, 0:1] * s[None, :]
    vv = uvw[:, 1:2] * s[None, :]
    if plan["do_wgridding"]:
        ww = uvw[:, 2:3] * s[None, :]
    else:
        ww = np.zeros((nrow, nchan))
    flip = ww < 0.0
    uu = np.where(flip, -uu, uu)
    vv = np.where(flip, -vv, vv)
    ww = np.where(flip, -ww, ww)
    xu = uu * plan["pixsize_x"]
    xv = vv * plan["pixsize_y"]
    fu = xu - np.floor(xu)
    fv = xv - np.floor(xv)
    gu = fu * nu
    gv = fv * nv
    iu = np.ceil(gu - half).astype(np.int64)
    iv = np.ceil(gv - half).astype(np.int64)
    iu = np.where(iu < 0, iu + nu, iu)
    iv = np.where(iv < 0, iv + nv, iv)
    if plan["do_wgridding"]:
        xw = (ww - plan["w0"]) / plan["dw"]
        iw = np.ceil(xw - half).astype(np.int64)
    else:
        xw = np.zeros_like(ww)
        iw = np.zeros(ww.shape, dtype=np.int64)
    ntv = nv // TILE
    key = ((iu // TILE) * ntv + (iv // TILE)) * nw + iw
    sel = np.ones((nrow, nchan), dtype=bool) if mask is None else (np.asarray(mask) != 0)
    idx = np.arange(nrow * nchan, dtype=np.int64).reshape(nrow, nchan)
    out = dict(idx=idx[sel], flip=flip[sel], gu=gu[sel], gv=gv[sel], xw=xw[sel],
               iu=iu[sel], iv=iv[sel], iw=iw[sel], key=key[sel].astype(np.uint64))
    out["order"] = np.argsort(out["key"], kind="stable")
    return out
