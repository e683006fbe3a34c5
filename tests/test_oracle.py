"""Pins for the oracle: each check ties it to something other than itself --
the paper's printed kernel tables, closed forms, symmetries of eq. (3),
special cases that reduce to a library FFT, and agreement between the two
independent oracles (O1 direct DFT, O2 plain gridder)."""
import math
import os

import numpy as np
import pytest

import synth
from oracle import kernel as K
from oracle import o1, o2
from oracle import plan as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


# --------------------------------------------------------------------------
# kernel: Appendix A, eq. (semicircle2), eq. (maperror)
# --------------------------------------------------------------------------

def _golden_rows():
    rows = []
    with open(os.path.join(GOLDEN, "appendix_a_kernels.csv")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            a, s, e, b, m = line.strip().split(",")
            rows.append((int(a), float(s), float(e), float(b), float(m)))
    return rows


def test_table_matches_printed_rows():
    rows = _golden_rows()
    assert len(rows) == sum(len(v) for v in K.TABLE.values()) == 86
    for a, s, e, b, m in rows:
        assert K.table_row(a, s)[1:] == (e, b, m)


@pytest.mark.parametrize("alpha", [4, 7, 8, 12, 16])
def test_map_error_reproduces_appendix_a(alpha):
    """sup_x l(x) over the retained band reproduces every printed accuracy:
    within 3% down to 1e-12, within 7% below (where FP64 cancellation inside
    l(x) limits the recomputation)."""
    for a, s, e, b, m in _golden_rows():
        if a != alpha:
            continue
        got = K.kernel_accuracy(a, s, b, m, nx=257)
        tol = 3e-2 if e >= 1e-12 else 7e-2
        assert abs(got - e) / e < tol, (a, s, e, got)


def test_map_error_detects_wrong_kernel():
    """A kernel with mu=1/2 (the one-parameter ES kernel, eq. semicircle) or a
    perturbed beta must not reach the printed accuracy of the tuned row."""
    _, e, b, m = K.table_row(8, 1.45)
    assert K.kernel_accuracy(8, 1.45, b, 0.5) > 1.3 * e
    assert K.kernel_accuracy(8, 1.45, 1.1 * b, m) > 1.3 * e


def test_psi_boxcar_closed_form():
    """beta = 0 makes phi = 1 on the support; psi(k) = sin(pi alpha k)/(pi k)."""
    k = np.linspace(0.013, 0.5, 23)
    for a in (4, 7, 16):
        assert np.allclose(K.psi(k, a, 0.0, 0.5), np.sin(np.pi * a * k) / (np.pi * k),
                           rtol=0, atol=1e-13)


def test_psi_quadrature_converged():
    for a in (4, 8, 12, 16):
        _, _, b, m = K.table_row(a, 2.0)
        k = np.linspace(0.0, 0.25, 9)
        lo = K.psi(k, a, b, m)
        hi = K.psi(k, a, b, m, q_inner=64, q_end=128)
        assert np.max(np.abs(lo - hi) / np.abs(hi)) < 1e-13


def test_phi_shape():
    a, b, m = 8, 1.871691821, 0.5161733611
    assert K.phi(0.0, a, b, m) == 1.0
    assert math.isclose(float(K.phi(a / 2, a, b, m)), math.exp(-a * b))
    assert K.phi(a / 2 + 1e-9, a, b, m) == 0.0
    t = np.linspace(-4, 4, 101)
    assert np.allclose(K.phi(t, a, b, m), K.phi(-t, a, b, m))


def test_feasible_selection():
    assert K.smallest_sigma(8, 1e-5, True) == 1.45       # 3 * 2.58e-6 <= 1e-5
    assert K.smallest_sigma(7, 1e-5, True) == 1.70
    assert K.smallest_sigma(16, 1e-10, True) == 1.35
    assert K.smallest_sigma(4, 1e-5, True) is None


# --------------------------------------------------------------------------
# plan geometry, Sect. 2
# --------------------------------------------------------------------------

def test_good_size():
    for n in range(1, 3000, 37):
        g = P.good_size(n)
        assert g >= n and g % 16 == 0
        m = g
        for p in (2, 3, 5, 7):
            while m % p == 0:
                m //= p
        assert m == 1
        # nothing smaller qualifies
        for c in range(((n + 15) // 16) * 16, g, 16):
            mm = c
            for p in (2, 3, 5, 7):
                while mm % p == 0:
                    mm //= p
            assert mm != 1
    assert P.grid_size(1.45, 2048) == 3024


def test_plane_geometry_invariants():
    c = synth.small_plain()
    pl = P.make_plan(c["uvw"], c["freq"], 64, 64, c["pixsize_x"], c["pixsize_y"], 16, 1.35)
    _, _, _, nm1 = P.lm_grid(64, 64, c["pixsize_x"], c["pixsize_y"])
    # Nyquist condition of Sect. 2 holds everywhere, with equality at the corner
    assert np.max(2 * pl["dw"] * pl["sigma"] * np.abs(nm1)) <= 1.0 + 1e-15
    assert abs(2 * pl["dw"] * pl["sigma"] * abs(nm1[0, 0]) - 1.0) < 1e-15
    b = P.bin_visibilities(c["uvw"], c["freq"], pl)
    # every visibility's alpha planes lie in [0, N_w)
    assert b["iw"].min() >= 0 and (b["iw"] + pl["alpha"] - 1).max() < pl["nw"]
    # the kernel footprint [i0, i0 + alpha) covers the point, offsets in [-a/2, -a/2+1)
    for g, i, n in ((b["gu"], b["iu"], pl["nu"]), (b["gv"], b["iv"], pl["nv"])):
        i_unwrapped = np.ceil(g - pl["alpha"] / 2)
        assert np.all(np.mod(i_unwrapped, n) == i)
        off = i_unwrapped - g
        assert np.all(off >= -pl["alpha"] / 2) and np.all(off < -pl["alpha"] / 2 + 1)
    assert np.all(b["iu"] >= 0) and np.all(b["iu"] < pl["nu"])


def test_binning_brute_force_tiny():
    """Scalar Python re-derivation of every key of a tiny input (math module,
    one visibility at a time) matches the vectorised spec, and the order is a
    stable sort by key."""
    rng = np.random.default_rng(7)
    uvw = rng.uniform(-3000, 3000, (40, 3))
    freq = np.array([0.9e9, 1.3e9, 1.7e9])
    pix = 2.0 * math.pi / 180 / 64
    mask = (rng.random((40, 3)) > 0.2).astype(np.uint8)
    pl = P.make_plan(uvw, freq, 64, 64, pix, pix, 8, 1.45, mask=mask)
    b = P.bin_visibilities(uvw, freq, pl, mask)
    keys = []
    for r in range(40):
        for ch in range(3):
            if not mask[r, ch]:
                continue
            s = freq[ch] / P.C_LIGHT
            u, v, w = uvw[r, 0] * s, uvw[r, 1] * s, uvw[r, 2] * s
            if w < 0:
                u, v, w = -u, -v, -w
            cells = []
            for x, d, n in ((u, pix, pl["nu"]), (v, pix, pl["nv"])):
                x = x * d
                g = (x - math.floor(x)) * n
                i0 = math.ceil(g - 4.0)
                cells.append(i0 + n if i0 < 0 else i0)
            iw = math.ceil((w - pl["w0"]) / pl["dw"] - 4.0)
            keys.append(((cells[0] // 16) * (pl["nv"] // 16) + cells[1] // 16) * pl["nw"] + iw)
    assert np.array_equal(np.array(keys, dtype=np.uint64), b["key"])
    srt = b["key"][b["order"]]
    assert np.all(np.diff(srt.astype(np.int64)) >= 0)
    for kv in np.unique(srt):
        pos = b["order"][srt == kv]
        assert np.all(np.diff(b["idx"][pos]) > 0)      # ties keep (row, chan) order


# --------------------------------------------------------------------------
# O1: eq. (3) and its adjoint
# --------------------------------------------------------------------------

def _tiny_case(seed=3, nrow=30, nchan=2, npix=32, do_w=True):
    rng = np.random.default_rng(seed)
    pix = 3.0 * math.pi / 180 / npix
    uvw = rng.uniform(-4000, 4000, (nrow, 3))
    freq = np.array([1.0e9, 1.4e9])[:nchan]
    img = rng.standard_normal((npix, npix))
    vis = rng.standard_normal((nrow, nchan)) + 1j * rng.standard_normal((nrow, nchan))
    return uvw, freq, img, vis, pix


def test_o1_centre_pixel_is_constant(oracle_lib):
    """A source at the phase centre (l = m = 0, n = 1) has visibility S on
    every baseline and channel, whatever u, v, w."""
    uvw, freq, _, _, pix = _tiny_case()
    img = np.zeros((32, 32))
    img[16, 16] = 2.5
    d = o1.forward(uvw, freq, img, pix, pix)
    assert np.allclose(d, 2.5, rtol=0, atol=1e-13)


def test_o1_hermitian_symmetry(oracle_lib):
    """eq. (Hermitian-symmetry): (u, v, w) -> -(u, v, w) conjugates R0 I."""
    uvw, freq, img, _, pix = _tiny_case()
    d1 = o1.forward(uvw, freq, img, pix, pix)
    d2 = o1.forward(-uvw, freq, img, pix, pix)
    assert rel(d2, np.conj(d1)) < 1e-13


def test_o1_uv_periodicity(oracle_lib):
    """For an even pixel count the pixel-grid DFT is periodic in u with period
    1/dl (wavelengths): shifting u by one period leaves eq. (3) unchanged."""
    uvw, freq, img, _, pix = _tiny_case(nchan=1)
    shifted = uvw.copy()
    lam = P.C_LIGHT / freq[0]
    shifted[:, 0] += 3.0 * lam / pix
    shifted[:, 1] -= 2.0 * lam / pix
    d1 = o1.forward(uvw, freq, img, pix, pix)
    d2 = o1.forward(shifted, freq, img, pix, pix)
    assert rel(d2, d1) < 1e-10


def test_o1_reduces_to_fft_on_grid_frequencies(oracle_lib):
    """Without w and with u = a/(n dl), v = b/(n dm) for integers a, b, eq. (3)
    is the 2-D DFT of I/n: d = (-1)^(a+b) fft2(I/n)[a mod n, b mod n]."""
    rng = np.random.default_rng(11)
    n = 32
    pix = 2.0 * math.pi / 180 / n
    lam = P.C_LIGHT / 1e9
    ab = rng.integers(-40, 40, (50, 2))
    uvw = np.zeros((50, 3))
    uvw[:, 0] = ab[:, 0] / (n * pix) * lam
    uvw[:, 1] = ab[:, 1] / (n * pix) * lam
    uvw[:, 2] = rng.uniform(-500, 500, 50)          # ignored without w
    img = rng.standard_normal((n, n))
    _, _, nn, _ = P.lm_grid(n, n, pix, pix)
    F = np.fft.fft2(img / nn)
    ref = ((-1.0) ** (ab[:, 0] + ab[:, 1])) * F[ab[:, 0] % n, ab[:, 1] % n]
    d = o1.forward(uvw, np.array([1e9]), img, pix, pix, do_wgridding=False)[:, 0]
    assert rel(d, ref) < 1e-11
    # the 1/n factor matters off-centre: without it the match fails
    F0 = np.fft.fft2(img)
    ref0 = ((-1.0) ** (ab[:, 0] + ab[:, 1])) * F0[ab[:, 0] % n, ab[:, 1] % n]
    assert rel(d, ref0) > 1e-5


def test_o1_w_term_convention(oracle_lib):
    """Reading of the sign conflict between eq. (3) and eqs. (nfft)/(R2): eq. (3)
    governs, the forward phase of a single pixel is -(u l + v m - w (n - 1))."""
    uvw = np.array([[120.0, -80.0, 2500.0]])
    pix = 1.0 * math.pi / 180 / 32
    img = np.zeros((32, 32))
    img[3, 27] = 1.0
    l, m = (3 - 16) * pix, (27 - 16) * pix
    n = math.sqrt(1 - l * l - m * m)
    s = 1e9 / P.C_LIGHT
    u, v, w = uvw[0] * s
    expect = np.exp(-2j * math.pi * (u * l + v * m - w * (n - 1))) / n
    d = o1.forward(uvw, np.array([1e9]), img, pix, pix)[0, 0]
    assert abs(d - expect) < 1e-10       # n - 1 above carries cancellation error
    assert abs(w * (n - 1)) > 0.05       # the w-term is not negligible here
    wrong = np.exp(-2j * math.pi * (u * l + v * m + w * (n - 1))) / n
    assert abs(d - wrong) > 0.5          # the opposite sign is distinguishable


def test_o1_adjointness(oracle_lib):
    """eq. (adjointness) holds for the direct operator pair to FP64 rounding."""
    for do_w in (True, False):
        uvw, freq, img, vis, pix = _tiny_case(do_w=do_w)
        d = o1.forward(uvw, freq, img, pix, pix, do_wgridding=do_w)
        im = o1.adjoint(uvw, freq, vis, 32, 32, pix, pix, do_wgridding=do_w)
        lhs = np.vdot(d, vis).real
        rhs = np.vdot(img, im)
        assert abs(lhs - rhs) / (np.linalg.norm(d) * np.linalg.norm(vis)) < 1e-14


def test_o1_weights_and_mask(oracle_lib):
    uvw, freq, img, vis, pix = _tiny_case()
    rng = np.random.default_rng(5)
    wgt = rng.uniform(0.5, 2.0, vis.shape)
    mask = (rng.random(vis.shape) > 0.3).astype(np.uint8)
    d = o1.forward(uvw, freq, img, pix, pix, wgt=wgt, mask=mask)
    d0 = o1.forward(uvw, freq, img, pix, pix)
    assert np.allclose(d, np.where(mask != 0, d0 * wgt, 0))
    im = o1.adjoint(uvw, freq, vis, 32, 32, pix, pix, wgt=wgt, mask=mask)
    im0 = o1.adjoint(uvw, freq, np.where(mask != 0, vis * wgt, 0), 32, 32, pix, pix)
    assert rel(im, im0) < 1e-13


def test_o1_spot_evaluation_matches_full(oracle_lib):
    uvw, freq, img, vis, pix = _tiny_case()
    full = o1.forward(uvw, freq, img, pix, pix)
    idx = np.array([0, 7, 33, 59])
    assert np.allclose(o1.forward(uvw, freq, img, pix, pix, vis_idx=idx), full.ravel()[idx],
                       rtol=0, atol=1e-12)
    imf = o1.adjoint(uvw, freq, vis, 32, 32, pix, pix)
    pp, qq = np.array([0, 5, 31]), np.array([3, 16, 30])
    assert np.allclose(o1.adjoint(uvw, freq, vis, 32, 32, pix, pix, pixels=(pp, qq)),
                       imf[pp, qq], rtol=0, atol=1e-12)


# --------------------------------------------------------------------------
# O2 against O1: the approximation error is bounded by the kernel accuracy
# --------------------------------------------------------------------------

@pytest.mark.parametrize("alpha,sigma", [(16, 1.35), (12, 1.9), (8, 1.45), (7, 1.5), (4, 2.0)])
def test_o2_matches_o1_small(oracle_lib, alpha, sigma):
    c = synth.small_plain()
    pl = P.make_plan(c["uvw"], c["freq"], 64, 64, c["pixsize_x"], c["pixsize_y"], alpha, sigma)
    eps = 3 * pl["eps_k"]
    d1 = o1.forward(c["uvw"], c["freq"], c["dirty"], c["pixsize_x"], c["pixsize_y"])
    d2 = o2.degrid(c["uvw"], c["freq"], c["dirty"], pl)
    assert rel(d2, d1) < eps
    i1 = o1.adjoint(c["uvw"], c["freq"], c["vis"], 64, 64, c["pixsize_x"], c["pixsize_y"])
    i2 = o2.grid(c["uvw"], c["freq"], c["vis"], pl)
    assert rel(i2, i1) < eps


@pytest.mark.parametrize("do_w", [True, False])
def test_o2_accuracy_setup(oracle_lib, do_w):
    """Sect. 5 set-up (scaled to 128^2 so that the direct sums take seconds):
    accuracy of R^dagger and R against the direct transform, and adjointness."""
    c = synth.accuracy_setup(npix=128, fov_deg=15.0, nvis=1000)
    for alpha, sigma in ((8, 1.45), (12, 1.35)):
        pl = P.make_plan(c["uvw"], c["freq"], 128, 128, c["pixsize_x"], c["pixsize_y"],
                         alpha, sigma, do_wgridding=do_w)
        eps = K.error_factor(do_w) * pl["eps_k"]
        i1 = o1.adjoint(c["uvw"], c["freq"], c["vis"], 128, 128, c["pixsize_x"], c["pixsize_y"],
                        do_wgridding=do_w)
        i2 = o2.grid(c["uvw"], c["freq"], c["vis"], pl)
        assert rel(i2, i1) < eps
        d1 = o1.forward(c["uvw"], c["freq"], c["dirty"], c["pixsize_x"], c["pixsize_y"],
                        do_wgridding=do_w)
        d2 = o2.degrid(c["uvw"], c["freq"], c["dirty"], pl)
        assert rel(d2, d1) < eps
        lhs = np.vdot(d2, c["vis"]).real
        rhs = np.vdot(c["dirty"], i2)
        e_adj = abs(lhs - rhs) / min(np.linalg.norm(c["vis"]) * np.linalg.norm(d2),
                                     np.linalg.norm(c["dirty"]) * np.linalg.norm(i2))
        assert e_adj < 1e-12


def test_o2_detects_wrong_screen_sign(oracle_lib, monkeypatch):
    """Planting the opposite w-screen sign (eq. R2 read literally) in O2 breaks
    its agreement with O1 on a wide field: the sign reading is observable."""
    c = synth.accuracy_setup(npix=64, fov_deg=20.0, nvis=300, seed=4)
    pl = P.make_plan(c["uvw"], c["freq"], 64, 64, c["pixsize_x"], c["pixsize_y"], 8, 1.45)
    d1 = o1.forward(c["uvw"], c["freq"], c["dirty"], c["pixsize_x"], c["pixsize_y"])
    good = o2.degrid(c["uvw"], c["freq"], c["dirty"], pl)
    assert rel(good, d1) < 1e-5
    real_exp = np.exp

    def flipped(z):
        z = np.asarray(z)
        return real_exp(np.conj(z)) if np.iscomplexobj(z) else real_exp(z)
    monkeypatch.setattr(o2.np, "exp", flipped)
    bad = o2.degrid(c["uvw"], c["freq"], c["dirty"], pl)
    assert rel(bad, d1) > 1e-3


def test_o2_masked_and_weighted(oracle_lib):
    c = synth.small_plain()
    rng = np.random.default_rng(9)
    wgt = rng.uniform(0.5, 1.5, c["vis"].shape)
    mask = (rng.random(c["vis"].shape) > 0.25).astype(np.uint8)
    pl = P.make_plan(c["uvw"], c["freq"], 64, 64, c["pixsize_x"], c["pixsize_y"], 12, 1.5,
                     mask=mask)
    eps = 3 * pl["eps_k"]
    d1 = o1.forward(c["uvw"], c["freq"], c["dirty"], c["pixsize_x"], c["pixsize_y"], wgt=wgt,
                    mask=mask)
    d2 = o2.degrid(c["uvw"], c["freq"], c["dirty"], pl, wgt=wgt, mask=mask)
    assert rel(d2, d1) < eps
    assert np.all(d2[mask == 0] == 0)
    i1 = o1.adjoint(c["uvw"], c["freq"], c["vis"], 64, 64, c["pixsize_x"], c["pixsize_y"],
                    wgt=wgt, mask=mask)
    i2 = o2.grid(c["uvw"], c["freq"], c["vis"], pl, wgt=wgt, mask=mask)
    assert rel(i2, i1) < eps
