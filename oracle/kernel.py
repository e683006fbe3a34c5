"""Oracle: gridding-kernel mathematics in plain FP64 numpy.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import this
module; only tests/, the smoke check and the CPU-baseline leg of the benchmark
use it.  It shares no code with the HIP path.

Contents
--------
* ``TABLE``      -- the kernel parameter tables of Appendix A (modified ES
                    kernel, alpha in {4, 7, 8, 12, 16}), transcribed by hand.
* ``phi``        -- the modified "exponential of semicircle" kernel,
                    eq. (semicircle2) in Sect. 3.2.
* ``psi``        -- its Fourier transform, psi(k) = int phi(t) e^{2 pi i k t} dt
                    (Sect. 2, definition after eq. rime3d; the 2*pi*k reading
                    is the one used by eq. approxw), by Gauss-Legendre
                    quadrature with an endpoint substitution.
* ``map_error``  -- the map error function l(x) of eq. (maperror), Sect. 3.2.
* ``feasible``   -- which table rows meet a requested accuracy.
"""
import numpy as np

# ---------------------------------------------------------------------------
# Appendix A ("Kernel parameters"): rows (sigma, eps, beta, mu) per support.
# Only the printed supports are available; the alpha=12 table has no
# sigma=1.85 row and the alpha=16 table starts at sigma=1.3.
# ---------------------------------------------------------------------------
TABLE = {
    4: [
        (1.15, 0.025654879, 1.3873426689, 0.5436851297),
        (1.20, 0.013809249, 1.3008419165, 0.5902137484),
        (1.25, 0.0085840685, 1.3274088935, 0.5953499486),
        (1.30, 0.0057322498, 1.3617063353, 0.5965631622),
        (1.35, 0.0042494419, 1.384549988, 0.5990241291),
        (1.40, 0.0033459552, 1.4405325088, 0.5924776015),
        (1.45, 0.0028187359, 1.4635220066, 0.5929442711),
        (1.50, 0.0023843943, 1.5539689162, 0.5772217314),
        (1.55, 0.0020343796, 1.5991008653, 0.5721765215),
        (1.60, 0.0017143851, 1.6581546365, 0.5644747137),
        (1.65, 0.0014730848, 1.7135331415, 0.5572788589),
        (1.70, 0.0012554492, 1.7464330378, 0.5548742415),
        (1.75, 0.0010610904, 1.7887326906, 0.5509877716),
        (1.80, 0.00090885567, 1.8122309426, 0.5502273972),
        (1.85, 0.0007757401, 1.8304451327, 0.550396716),
        (1.90, 0.0006740398, 1.8484487383, 0.5502376937),
        (1.95, 0.00058655391, 1.8742215688, 0.5489738941),
        (2.00, 0.00051911189, 1.90694363, 0.5468009434),
    ],
    7: [
        (1.15, 0.00078476028, 1.5248706519, 0.5288306317),
        (1.20, 0.00027127166, 1.5739348793, 0.5287992619),
        (1.25, 0.00012594628, 1.6245240723, 0.527921777),
        (1.30, 7.0214545e-05, 1.6835745981, 0.5257484101),
        (1.35, 4.1972457e-05, 1.7343424414, 0.5239793844),
        (1.40, 2.378019e-05, 1.7845017738, 0.5224266045),
        (1.45, 1.3863408e-05, 1.8180597789, 0.5221834768),
        (1.50, 9.1605353e-06, 1.868082272, 0.5206277502),
        (1.55, 6.479159e-06, 1.9188980015, 0.5183134674),
        (1.60, 4.6544571e-06, 1.9536166143, 0.5178695891),
        (1.65, 3.5489761e-06, 1.9786267068, 0.5178430252),
        (1.70, 2.7030348e-06, 2.0027666534, 0.5178577604),
        (1.75, 2.0533894e-06, 2.0289949199, 0.5176300336),
        (1.80, 1.6069122e-06, 2.0596412946, 0.5167551932),
        (1.85, 1.2936794e-06, 2.0720606842, 0.5178747891),
        (1.90, 1.0768664e-06, 2.090898174, 0.5181009847),
        (1.95, 9.0890421e-07, 2.1086185697, 0.5184537843),
        (2.00, 7.7488775e-07, 2.1278284187, 0.5186377792),
    ],
    8: [
        (1.15, 0.00026818611, 1.568124649, 0.5223052481),
        (1.20, 7.8028732e-05, 1.620926145, 0.5219287175),
        (1.25, 2.7460918e-05, 1.6851585171, 0.519925059),
        (1.30, 1.3421658e-05, 1.7442373315, 0.5182155619),
        (1.35, 7.5158217e-06, 1.7876782642, 0.5176319503),
        (1.40, 4.2472384e-06, 1.8294321912, 0.5171860211),
        (1.45, 2.5794802e-06, 1.871691821, 0.5161733611),
        (1.50, 1.6131994e-06, 1.9213040541, 0.5145350888),
        (1.55, 1.0974814e-06, 1.9637229131, 0.5134005827),
        (1.60, 7.531955e-07, 2.0002761373, 0.5128849282),
        (1.65, 5.5097346e-07, 2.0275645736, 0.5127082324),
        (1.70, 4.0136726e-07, 2.0498410409, 0.5130237662),
        (1.75, 2.906467e-07, 2.073158517, 0.5131757153),
        (1.80, 2.1834922e-07, 2.0907418726, 0.5136046561),
        (1.85, 1.6329905e-07, 2.1164552354, 0.5133333878),
        (1.90, 1.2828598e-07, 2.126157016, 0.5143004427),
        (1.95, 1.0171134e-07, 2.1363206613, 0.515235491),
        (2.00, 8.1881369e-08, 2.1397013368, 0.5166895497),
    ],
    12: [
        (1.15, 2.7535895e-06, 1.6661837519, 0.5098172147),
        (1.20, 5.2570038e-07, 1.7294557459, 0.5089239596),
        (1.25, 1.378658e-07, 1.7698182384, 0.5099240718),
        (1.30, 4.4329167e-08, 1.8092042442, 0.510607427),
        (1.35, 1.7038991e-08, 1.8619112597, 0.5093832337),
        (1.40, 6.5438748e-09, 1.9069147481, 0.5089479889),
        (1.45, 2.9874764e-09, 1.9318398074, 0.5098082325),
        (1.50, 1.4920459e-09, 1.9628483155, 0.5100985753),
        (1.55, 8.0989276e-10, 2.0129847811, 0.5085327805),
        (1.60, 4.1660575e-10, 2.0517921747, 0.5079102398),
        (1.65, 2.3539727e-10, 2.06983884, 0.5085131064),
        (1.70, 1.3497289e-10, 2.0887365361, 0.5090417146),
        (1.75, 8.3256938e-11, 2.106955733, 0.5095920671),
        (1.80, 5.8834619e-11, 2.1359415217, 0.5091887069),
        (1.90, 2.6412908e-11, 2.2006369514, 0.5075889699),
        (1.95, 1.7189689e-11, 2.2146741638, 0.5080017404),
        (2.00, 1.2174796e-11, 2.2431392199, 0.5075191177),
    ],
    16: [
        (1.30, 1.1509596e-10, 1.7892839755, 0.5122877693),
        (1.35, 3.2440049e-11, 1.8914441282, 0.5063521839),
        (1.40, 8.4329616e-12, 1.9296369098, 0.5065170208),
        (1.45, 3.1161739e-12, 1.9674735425, 0.5063244338),
        (1.50, 1.2100308e-12, 2.0130787701, 0.5055587965),
        (1.55, 4.6082202e-13, 2.0438032614, 0.5056309683),
        (1.60, 1.7883238e-13, 2.0329561822, 0.5089045671),
        (1.65, 9.2853815e-14, 2.0494514743, 0.5103582604),
        (1.70, 5.6614567e-14, 2.0925119791, 0.5083767402),
        (1.75, 2.875391e-14, 2.1461524027, 0.5062037834),
        (1.80, 1.6578982e-14, 2.1490040175, 0.508272183),
        (1.85, 1.1782751e-14, 2.1811826814, 0.5072570059),
        (1.90, 8.9196865e-15, 2.1981176583, 0.5075840871),
        (1.95, 6.6530006e-15, 2.234001135, 0.5060133105),
        (2.00, 5.0563492e-15, 2.2621631913, 0.5056924675),
    ],
}


def table_row(alpha, sigma):
    """(sigma, eps, beta, mu) for a printed Appendix-A row; KeyError if absent."""
    for row in TABLE[alpha]:
        if abs(row[0] - sigma) < 1e-9:
            return row
    raise KeyError((alpha, sigma))


def phi(t, alpha, beta, mu):
    """Modified ES kernel, eq. (semicircle2): exp(alpha*beta*((1-(2t/alpha)^2)^mu - 1))
    on the closed support |t| <= alpha/2, zero outside."""
    t = np.asarray(t, dtype=np.float64)
    s = 1.0 - (2.0 * t / alpha) ** 2
    inside = s >= 0.0
    sc = np.where(inside, s, 0.0)
    val = np.exp(alpha * beta * (sc ** mu - 1.0))
    return np.where(inside, val, 0.0)


def _panel_nodes(alpha, q_inner=24, q_end=48):
    """Quadrature nodes/weights on [0, alpha/2] for int_0^{alpha/2} f(t) dt.

    The half-support is cut into unit-half panels.  Interior panels use plain
    Gauss-Legendre.  The panel that touches t = alpha/2 carries the factor
    (alpha/2 - t)^mu of the kernel; substituting alpha/2 - t = h*v^4 turns it
    into v^(4 mu) times a smooth function, which Gauss-Legendre integrates to
    FP64 accuracy.
    """
    half = 0.5 * alpha
    npan = int(round(2 * half))           # panels of width 0.5
    h = half / npan
    xi, wi = np.polynomial.legendre.leggauss(q_inner)
    xe, we = np.polynomial.legendre.leggauss(q_end)
    ts, ws = [], []
    for j in range(npan - 1):
        a, b = j * h, (j + 1) * h
        ts.append(0.5 * (b - a) * xi + 0.5 * (a + b))
        ws.append(0.5 * (b - a) * wi)
    # end panel [half - h, half]: t = half - h*v^4, v in [0, 1], dt = 4 h v^3 dv
    v = 0.5 * xe + 0.5
    ts.append(half - h * v ** 4)
    ws.append(0.5 * we * 4.0 * h * v ** 3)
    return np.concatenate(ts), np.concatenate(ws)


def psi(k, alpha, beta, mu, q_inner=24, q_end=48):
    """psi(k) = int_{-alpha/2}^{alpha/2} phi(t) cos(2 pi k t) dt  (phi is even).

    Fourier transform of the kernel in the 2*pi*k convention of eq. (approxw);
    real and even in k.  Vectorised over k.
    """
    k = np.asarray(k, dtype=np.float64)
    t, w = _panel_nodes(alpha, q_inner, q_end)
    f = w * phi(t, alpha, beta, mu)
    out = 2.0 * np.cos(2.0 * np.pi * np.multiply.outer(k, t)) @ f
    return out


def map_error(x, alpha, sigma, beta, mu, q_nu=64):
    """Map error function l(x) of eq. (maperror), Sect. 3.2.

    l(x)^2 = int_0^1 | 1 - sum_a phi(a - nu) e^{2 pi i (a - nu) x} / psi(x) |^2 dnu

    where a runs over the alpha integers with a - nu in [-alpha/2, alpha/2)
    (the cells a kernel touches), nu is the fractional grid position and x the
    image coordinate in units of the grid frequency (|x| <= 1/(2 sigma) is the
    retained part of the image).  ``sigma`` only documents the intended range.
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    xg, wg = np.polynomial.legendre.leggauss(q_nu)
    # the set of cells changes at nu = frac(alpha/2): split the nu integral there
    brk = (0.5 * alpha) % 1.0
    segs = [(0.0, 1.0)] if brk == 0.0 else [(0.0, brk), (brk, 1.0)]
    nus, wts = [], []
    for a, b in segs:
        nus.append(0.5 * (b - a) * xg + 0.5 * (a + b))
        wts.append(0.5 * (b - a) * wg)
    nu = np.concatenate(nus)
    wnu = np.concatenate(wts)
    ps = psi(x, alpha, beta, mu)
    # cells: a = ceil(nu - alpha/2) + i, i = 0..alpha-1
    a0 = np.ceil(nu - 0.5 * alpha)
    off = (a0[:, None] + np.arange(alpha)[None, :]) - nu[:, None]   # a - nu
    ph = phi(off, alpha, beta, mu)                                   # [nnu, alpha]
    expo = np.exp(2j * np.pi * np.multiply.outer(off, x))             # [nnu, alpha, nx]
    s = np.einsum("ia,iax->ix", ph, expo)                             # [nnu, nx]
    err = np.abs(1.0 - s / ps[None, :]) ** 2
    return np.sqrt(wnu @ err)


def kernel_accuracy(alpha, sigma, beta, mu, nx=257):
    """Sup-norm of l(x) over the retained band 0 <= x <= 1/(2 sigma)."""
    xs = np.linspace(0.0, 0.5 / sigma, nx)
    return float(np.max(map_error(xs, alpha, sigma, beta, mu)))


def error_factor(do_wgridding):
    """Number of kernel dimensions whose errors add to first order (u, v, and w
    when w-gridding): the requested accuracy is met when factor*eps_k <= eps."""
    return 3.0 if do_wgridding else 2.0


def feasible(alpha, sigma, eps, do_wgridding):
    """True when the Appendix-A row (alpha, sigma) meets the requested eps."""
    _, ek, _, _ = table_row(alpha, sigma)
    return error_factor(do_wgridding) * ek <= eps


def smallest_sigma(alpha, eps, do_wgridding):
    """Smallest printed sigma for this alpha that meets eps, or None (Sect. 4.1:
    for each support the kernel with the smallest sufficient oversampling)."""
    fac = error_factor(do_wgridding)
    for sig, ek, _, _ in TABLE[alpha]:
        if fac * ek <= eps:
            return sig
    return None
