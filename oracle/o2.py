"""Oracle O2: plain w-gridding (de)gridder in FP64 numpy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  A direct, unoptimised
transcription of the method of Sect. 3.1 at a given plan:

degridding, eqs. (R1)-(R3):
    I~_lm   = I_lm / (n_lm Psi_lm)                                  (R1)
    for every w-plane c_j = w_o + j dw:
        g_j = I~ * exp(+2 pi i c_j (n_lm - 1)) placed on the N_u x N_v grid
              at the wrapped indices (p - n_x/2) mod N_u, (q - n_y/2) mod N_v
        G_j = sum_lm g_j exp(-2 pi i (a p' / N_u + b q' / N_v))   (2-D FFT)
        d_k += phi(j - x_w) sum_ab phi(a - x_u) phi(b - x_v) G_j[a, b]  (R3)

gridding, eqs. (Rad1)-(Rad2), the same steps in reverse order with the
conjugate phases, and the real part of the image taken.

The w-screen sign follows eq. (3) / eq. (approxw2) (forward phase
exp(+2 pi i w (n - 1))); eqs. (nfft) and (R2) print the opposite sign.  The
kernel phi is evaluated directly (exp/pow), psi by quadrature, the FFT is
numpy's.  Visibilities with w < 0 are folded by eq. (Hermitian-symmetry):
(u, v, w, d) -> (-u, -v, -w, d*).
"""
import numpy as np

from .kernel import phi, psi
from .plan import bin_visibilities, lm_grid


def correction(plan):
    """n_lm * Psi_lm with Psi = psi(p'/N_u) psi(q'/N_v) psi((n-1) dw) (Sect. 2,
    definition of Psi, with the actual grid size in place of sigma n)."""
    a, b, m = plan["alpha"], plan["beta"], plan["mu"]
    nx, ny = plan["npix_x"], plan["npix_y"]
    _, _, n, nm1 = lm_grid(nx, ny, plan["pixsize_x"], plan["pixsize_y"])
    px = psi((np.arange(nx) - nx // 2) / plan["nu"], a, b, m)
    py = psi((np.arange(ny) - ny // 2) / plan["nv"], a, b, m)
    corr = n * px[:, None] * py[None, :]
    if plan["do_wgridding"]:
        pw = psi((nm1 * plan["dw"]).ravel(), a, b, m).reshape(nm1.shape)
        corr = corr * pw
    return corr, nm1


def _kernel_weights(binned, plan):
    """Per visibility: wrapped cell indices and kernel values on the u and v
    axes ([nvis, alpha]) and the first plane plus plane weights on the w axis."""
    a, b, m = plan["alpha"], plan["beta"], plan["mu"]
    half = 0.5 * a
    steps = np.arange(a)
    out = {}
    for ax, g, nn in (("u", binned["gu"], plan["nu"]), ("v", binned["gv"], plan["nv"])):
        i0 = np.ceil(g - half)                                  # unwrapped first cell
        cells = i0[:, None] + steps[None, :]
        out["w" + ax] = phi(cells - g[:, None], a, b, m)
        out["i" + ax] = np.mod(cells.astype(np.int64), nn)
    if plan["do_wgridding"]:
        xw = binned["xw"]
        j0 = np.ceil(xw - half)
        planes = j0[:, None] + steps[None, :]
        out["ww"] = phi(planes - xw[:, None], a, b, m)
        out["iw"] = planes.astype(np.int64)
    else:
        out["ww"] = np.ones((len(binned["xw"]), 1))
        out["iw"] = np.zeros((len(binned["xw"]), 1), dtype=np.int64)
    return out


def _place(plan):
    """Wrapped grid indices of the image pixels."""
    nx, ny = plan["npix_x"], plan["npix_y"]
    ia = np.mod(np.arange(nx) - nx // 2, plan["nu"])
    ib = np.mod(np.arange(ny) - ny // 2, plan["nv"])
    return ia, ib


def degrid(uvw, freq, dirty, plan, wgt=None, mask=None):
    """Forward operator R (image -> visibilities), FP64.  Returns [nrow, nchan]."""
    nrow, nchan = uvw.shape[0], len(freq)
    binned = bin_visibilities(uvw, freq, plan, mask)
    kw = _kernel_weights(binned, plan)
    corr, nm1 = correction(plan)
    itil = np.asarray(dirty, dtype=np.float64) / corr                       # (R1)
    ia, ib = _place(plan)
    nvis = len(binned["idx"])
    acc = np.zeros(nvis, dtype=np.complex128)
    nplanes = plan["nw"]
    for j in range(nplanes):
        act = np.nonzero(kw["iw"] == j)                                     # (vis, slot)
        if act[0].size == 0:
            continue
        vis_ids, slots = act
        if plan["do_wgridding"]:
            cj = plan["w0"] + j * plan["dw"]
            screen = np.exp(2j * np.pi * cj * nm1)                          # (R2)
        else:
            screen = 1.0
        g = np.zeros((plan["nu"], plan["nv"]), dtype=np.complex128)
        g[np.ix_(ia, ib)] = itil * screen
        G = np.fft.fft2(g)                                                  # e^{-2 pi i}
        wu = kw["wu"][vis_ids]
        wv = kw["wv"][vis_ids]
        cells = G[kw["iu"][vis_ids][:, :, None], kw["iv"][vis_ids][:, None, :]]
        val = np.einsum("ka,kb,kab->k", wu, wv, cells)
        acc_j = kw["ww"][vis_ids, slots] * val                              # (R3)
        np.add.at(acc, vis_ids, acc_j)
    acc = np.where(binned["flip"], np.conj(acc), acc)
    out = np.zeros(nrow * nchan, dtype=np.complex128)
    out[binned["idx"]] = acc
    out = out.reshape(nrow, nchan)
    if wgt is not None:
        out = out * wgt
    return out


def grid(uvw, freq, vis, plan, wgt=None, mask=None):
    """Adjoint operator R^dagger (visibilities -> real image), FP64."""
    nrow, nchan = uvw.shape[0], len(freq)
    binned = bin_visibilities(uvw, freq, plan, mask)
    kw = _kernel_weights(binned, plan)
    corr, nm1 = correction(plan)
    d = np.asarray(vis, dtype=np.complex128)
    if wgt is not None:
        d = d * wgt
    d = d.reshape(-1)[binned["idx"]]
    d = np.where(binned["flip"], np.conj(d), d)
    ia, ib = _place(plan)
    acc = np.zeros((plan["npix_x"], plan["npix_y"]))
    for j in range(plan["nw"]):
        act = np.nonzero(kw["iw"] == j)
        if act[0].size == 0:
            continue
        vis_ids, slots = act
        contrib = d[vis_ids] * kw["ww"][vis_ids, slots]
        w2 = kw["wu"][vis_ids][:, :, None] * kw["wv"][vis_ids][:, None, :]
        g = np.zeros((plan["nu"], plan["nv"]), dtype=np.complex128)
        rows = np.broadcast_to(kw["iu"][vis_ids][:, :, None], w2.shape)
        cols = np.broadcast_to(kw["iv"][vis_ids][:, None, :], w2.shape)
        np.add.at(g, (rows.ravel(), cols.ravel()), (contrib[:, None, None] * w2).ravel())
        H = np.fft.ifft2(g) * (plan["nu"] * plan["nv"])                    # e^{+2 pi i}  (Rad2)
        h = H[np.ix_(ia, ib)]
        if plan["do_wgridding"]:
            cj = plan["w0"] + j * plan["dw"]
            h = h * np.exp(-2j * np.pi * cj * nm1)                          # (Rad1)
        acc += h.real
    return acc / corr
