"""Seeded synthetic inputs shared by the tests, the benchmark and the examples.

This module only draws inputs: baseline coordinates of a synthetic array,
channel frequencies, images and visibilities.  It contains none of the
gridding method's arithmetic, so that the product and the oracle can both be
fed from it without sharing code.

Array model (a stand-in for a real measurement set; the paper's MeerKAT data
are not available): antennas on a plane at latitude -30 deg observing a phase
centre at declination -60 deg, hour angles symmetric about transit, textbook
east-north-up -> equatorial baseline rotation.  Rows are time-major (all
baselines of one dump, then the next dump), as in a measurement set.
"""
import math

import numpy as np

C_LIGHT = 299792458.0
ARCMIN = math.pi / (180.0 * 60.0)
DEG = math.pi / 180.0


def antennas_disk(rng, n_ant, diameter_m):
    """East/north positions uniform in a disk."""
    r = 0.5 * diameter_m * np.sqrt(rng.random(n_ant))
    th = 2.0 * np.pi * rng.random(n_ant)
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def antennas_logradial(rng, n_ant, r_min_m, ratio):
    """East/north positions with log-uniform radius r_min * ratio**U."""
    r = r_min_m * ratio ** rng.random(n_ant)
    th = 2.0 * np.pi * rng.random(n_ant)
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def earth_rotation_uvw(ant_en, hours, n_dumps, lat_deg=-30.0, dec_deg=-60.0):
    """uvw [n_dumps * n_baselines, 3] in metres for hour angles spread evenly
    over ``hours`` centred on transit."""
    n_ant = ant_en.shape[0]
    i, j = np.triu_indices(n_ant, k=1)
    de = ant_en[j, 0] - ant_en[i, 0]
    dn = ant_en[j, 1] - ant_en[i, 1]
    lat, dec = lat_deg * DEG, dec_deg * DEG
    lx = -math.sin(lat) * dn
    ly = de
    lz = math.cos(lat) * dn
    half = 0.5 * hours * 15.0 * DEG
    if n_dumps == 1:
        ha = np.zeros(1)
    else:
        ha = np.linspace(-half, half, n_dumps)
    sh, ch = np.sin(ha)[:, None], np.cos(ha)[:, None]
    u = sh * lx[None, :] + ch * ly[None, :]
    v = -math.sin(dec) * ch * lx[None, :] + math.sin(dec) * sh * ly[None, :] + math.cos(dec) * lz[None, :]
    w = math.cos(dec) * ch * lx[None, :] - math.cos(dec) * sh * ly[None, :] + math.sin(dec) * lz[None, :]
    return np.stack([u.ravel(), v.ravel(), w.ravel()], axis=1)


def channels(f_lo, f_hi, n_chan):
    if n_chan == 1:
        return np.array([0.5 * (f_lo + f_hi)])
    return np.linspace(f_lo, f_hi, n_chan)


def complex_gaussian(rng, shape, dtype=np.complex128):
    real_dt = np.float32 if dtype == np.complex64 else np.float64
    out = np.empty(shape, dtype=dtype)
    out.real = rng.standard_normal(shape, dtype=real_dt)
    out.imag = rng.standard_normal(shape, dtype=real_dt)
    return out


def point_sources(rng, npix_x, npix_y, n_src, dtype=np.float64):
    """Image with n_src sources at distinct random pixel centres, fluxes
    exp(N(0, 1)) (log-normal)."""
    img = np.zeros((npix_x, npix_y), dtype=dtype)
    flat = rng.choice(npix_x * npix_y, size=n_src, replace=False)
    img.ravel()[flat] = np.exp(rng.standard_normal(n_src))
    return img


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def small_plain(seed=1):
    """64x64 image, 0.5 arcmin pixels, one channel at 1 GHz, 2000 visibilities
    with u, v ~ U[-2, 2] km and w ~ U[-0.3, 0.3] km; complex Gaussian
    visibilities, N(0, 1) image."""
    rng = np.random.default_rng(seed)
    nrow = 2000
    uvw = np.empty((nrow, 3))
    uvw[:, 0:2] = rng.uniform(-2000.0, 2000.0, (nrow, 2))
    uvw[:, 2] = rng.uniform(-300.0, 300.0, nrow)
    freq = np.array([1e9])
    npix = 64
    pix = 0.5 * ARCMIN
    vis = complex_gaussian(rng, (nrow, 1))
    img = rng.standard_normal((npix, npix))
    return dict(uvw=uvw, freq=freq, npix_x=npix, npix_y=npix, pixsize_x=pix, pixsize_y=pix,
                vis=vis, dirty=img, name="plain-64x64-2000vis")


def accuracy_setup(seed=0, npix=512, fov_deg=15.0, nvis=1000, freq_hz=1e9):
    """Validation set-up of Sect. 5: npix^2 image over fov_deg^2, one channel,
    uvw uniform in [-a, a] with a = lambda / (2 pixsize) metres (reading of the
    garbled definition of a), data and image uniform in [-0.5, 0.5]."""
    rng = np.random.default_rng(seed)
    pix = fov_deg * DEG / npix
    lam = C_LIGHT / freq_hz
    a = lam / (2.0 * pix)
    uvw = rng.uniform(-a, a, (nvis, 3))
    vis = (rng.uniform(-0.5, 0.5, (nvis, 1)) + 1j * rng.uniform(-0.5, 0.5, (nvis, 1)))
    img = rng.uniform(-0.5, 0.5, (npix, npix))
    return dict(uvw=uvw, freq=np.array([freq_hz]), npix_x=npix, npix_y=npix, pixsize_x=pix,
                pixsize_y=pix, vis=vis, dirty=img, name=f"accuracy-{npix}-{fov_deg}deg-{nvis}vis")


def wide_field(seed=2, n_dumps=2880, n_chan=16, npix=2048, fov_deg=10.0, n_src=500,
               with_vis=True, vis_dtype=np.complex64):
    """Wide-field workload: 64 antennas uniform in a 5 km disk, 8 h at 10 s dumps
    (2880 x 2016 = 5,806,080 rows), 16 channels over 0.9-1.7 GHz
    (92,897,280 visibilities), 2048^2 image over 10 deg with 500 log-normal
    point sources."""
    rng = np.random.default_rng(seed)
    ant = antennas_disk(rng, 64, 5000.0)
    uvw = earth_rotation_uvw(ant, 8.0, n_dumps)
    freq = channels(0.9e9, 1.7e9, n_chan)
    pix = fov_deg * DEG / npix
    img = point_sources(rng, npix, npix, n_src)
    out = dict(uvw=uvw, freq=freq, npix_x=npix, npix_y=npix, pixsize_x=pix, pixsize_y=pix,
               dirty=img, name=f"wide-field-{npix}^2-{uvw.shape[0] * n_chan}vis")
    if with_vis:
        out["vis"] = complex_gaussian(rng, (uvw.shape[0], n_chan), vis_dtype)
    return out


def large(seed=3, n_dumps=1000, n_chan=8, npix=8192, fov_deg=30.0, with_data=True):
    """Large workload: 256 antennas with log-radial radii 20 m * 500^U (up to
    10 km), 4 h in 1000 dumps (32,640,000 rows), 8 channels over 0.9-1.7 GHz
    (261,120,000 visibilities), 8192^2 image over 30 deg; Gaussian image and
    complex64 Gaussian visibilities."""
    rng = np.random.default_rng(seed)
    ant = antennas_logradial(rng, 256, 20.0, 500.0)
    uvw = earth_rotation_uvw(ant, 4.0, n_dumps)
    freq = channels(0.9e9, 1.7e9, n_chan)
    pix = fov_deg * DEG / npix
    out = dict(uvw=uvw, freq=freq, npix_x=npix, npix_y=npix, pixsize_x=pix, pixsize_y=pix,
               name=f"large-{npix}^2-{uvw.shape[0] * n_chan}vis")
    if with_data:
        out["dirty"] = rng.standard_normal((npix, npix), dtype=np.float32)
        out["vis"] = complex_gaussian(rng, (uvw.shape[0], n_chan), np.complex64)
    return out


def differentiation(seed=5, n_dumps=620, n_chan=4, npix=1024, n_src=100, noise_frac=0.1):
    """Differentiation workload: 64 antennas (5 km disk), 2 h in 620 dumps x
    2016 baselines x 4 channels (4,999,680 visibilities), 1024^2 image with
    pixel size 10 deg / 2048 (5 deg field), a 100-source log-normal sky."""
    rng = np.random.default_rng(seed)
    ant = antennas_disk(rng, 64, 5000.0)
    uvw = earth_rotation_uvw(ant, 2.0, n_dumps)
    freq = channels(0.9e9, 1.7e9, n_chan)
    pix = 10.0 * DEG / 2048
    sky = point_sources(rng, npix, npix, n_src)
    return dict(uvw=uvw, freq=freq, npix_x=npix, npix_y=npix, pixsize_x=pix, pixsize_y=pix,
                sky=sky, noise_frac=noise_frac, rng=rng, name=f"diff-{npix}^2")


def serving_requests(seed=4, count=200, n_configs=12, sizes=(512, 1024, 2048, 4096), nvis_range=(1e5, 2e7),
                     epsilons=(1e-4, 1e-5, 1e-7, 1e-9), pixsize=10.0 * DEG / 2048, base=None):
    """Request mix of the serving workload.  ``n_configs`` operator
    configurations are drawn first (image size uniform over ``sizes``;
    visibility count log-uniform over ``nvis_range``, as a contiguous row
    range of the wide-field array with 16 channels, fewer for small counts;
    epsilon uniform over ``epsilons``, FP32 where eps >= 1e-5, else FP64), then
    ``count`` requests, each on a configuration drawn uniformly, direction
    degrid/grid 50/50, with its own data seed.  Returns (base workload,
    configurations, requests)."""
    rng = np.random.default_rng(seed)
    if base is None:
        base = wide_field(with_vis=False)
    nrow_all, nch_all = base["uvw"].shape[0], len(base["freq"])
    configs = []
    for cid in range(n_configs):
        npix = int(rng.choice(sizes))
        nvis = int(10 ** rng.uniform(np.log10(nvis_range[0]), np.log10(nvis_range[1])))
        nch = int(min(nch_all, max(1, nvis // 20000)))
        nrow = int(min(nrow_all, max(1, nvis // nch)))
        r0 = int(rng.integers(0, nrow_all - nrow + 1))
        eps = float(rng.choice(epsilons))
        configs.append(dict(cid=cid, npix=npix, pixsize=pixsize, rows=(r0, r0 + nrow), nchan=nch, epsilon=eps,
                            precision="f32" if eps >= 1e-5 else "f64"))
    reqs = []
    for rid in range(count):
        c = configs[int(rng.integers(0, n_configs))]
        reqs.append(dict(c, rid=rid, direction="degrid" if rng.random() < 0.5 else "grid",
                         seed=int(rng.integers(0, 2 ** 31))))
    return base, configs, reqs


def meerkat_like(seed=6, n_dumps=436, n_chan=2048, npix=4096, fov_deg=1.6, n_src=1000, target_vis=470e6,
                 with_mask=True):
    """Workload shaped like the benchmark set of Sect. 6 (a MeerKAT L-band
    observation that is not available here; every number below is a
    reading): 61 antennas, autocorrelations included, so 1891 baselines per
    dump; 436 dumps over 11 h, which gives the 824,476 rows of that set;
    2048 channels over 856-1712 MHz; a 4096^2 image over 1.6 deg.

    Antennas: 61 of them with radii 4 km * U^2 (a dense core, longest
    baselines near 8 km), uniform position angles; latitude -30.7 deg,
    phase centre at declination -30 deg.  Flags (mask = 0): all
    autocorrelations, six channel bands typical of L-band interference
    (band edges, mobile, navigation and satellite bands), and blocks of
    64 channels x 1 row with a flagging probability chosen so that about
    ``target_vis`` visibilities remain (470 million in Sect. 6).  Image:
    ``n_src`` point sources with log-normal fluxes."""
    rng = np.random.default_rng(seed)
    n_ant = 61
    r = 4000.0 * rng.random(n_ant) ** 2
    th = 2.0 * np.pi * rng.random(n_ant)
    ant = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
    i, j = np.triu_indices(n_ant, k=0)                   # with autocorrelations
    de = ant[j, 0] - ant[i, 0]
    dn = ant[j, 1] - ant[i, 1]
    lat, dec = -30.7 * DEG, -30.0 * DEG
    lx, ly, lz = -math.sin(lat) * dn, de, math.cos(lat) * dn
    half = 0.5 * 11.0 * 15.0 * DEG
    ha = np.linspace(-half, half, n_dumps)
    sh, ch = np.sin(ha)[:, None], np.cos(ha)[:, None]
    u = sh * lx[None, :] + ch * ly[None, :]
    v = -math.sin(dec) * ch * lx[None, :] + math.sin(dec) * sh * ly[None, :] + math.cos(dec) * lz[None, :]
    w = math.cos(dec) * ch * lx[None, :] - math.cos(dec) * sh * ly[None, :] + math.sin(dec) * lz[None, :]
    uvw = np.stack([u.ravel(), v.ravel(), w.ravel()], axis=1)
    auto = np.tile(i == j, n_dumps)
    freq = np.linspace(856e6, 1712e6, n_chan, endpoint=False) + 0.5 * 856e6 / n_chan
    pix = fov_deg * DEG / npix
    img = point_sources(rng, npix, npix, n_src)
    out = dict(uvw=uvw, freq=freq, npix_x=npix, npix_y=npix, pixsize_x=pix, pixsize_y=pix, dirty=img,
               name=f"meerkat-like-{npix}^2-{uvw.shape[0]}x{n_chan}")
    if with_mask:
        bad = np.zeros(n_chan, dtype=bool)
        for lo, hi in ((856e6, 880e6), (925e6, 960e6), (1164e6, 1300e6), (1525e6, 1630e6), (1690e6, 1712e6),
                       (1080e6, 1095e6)):
            bad |= (freq >= lo) & (freq < hi)
        nblk = (n_chan + 63) // 64
        rows_ok = ~auto
        n_ok = int(rows_ok.sum()) * int((~bad).sum())
        keep = min(1.0, target_vis / n_ok)
        blk = rng.random((uvw.shape[0], nblk)) < keep
        mask = np.repeat(blk, 64, axis=1)[:, :n_chan] & (~bad)[None, :] & rows_ok[:, None]
        out["mask"] = mask.view(np.uint8)
    return out


def flatten_channels(uvw, freq, mask, f0=None):
    """The 'flattened' form of multi-channel data used in Sect. 6.2: one
    row per selected visibility, its uvw scaled to a single reference
    frequency f0 (default: the first channel), so that the effective
    coordinates uvw * f / c are unchanged.  Returns (uvw_flat [n, 3],
    freq [1], linear indices r * n_chan + c of the selected visibilities)."""
    f0 = float(freq[0]) if f0 is None else float(f0)
    idx = np.flatnonzero(np.asarray(mask).reshape(-1))
    r = idx // len(freq)
    c = idx - r * len(freq)
    uvw_flat = uvw[r] * (np.asarray(freq)[c] / f0)[:, None]
    return uvw_flat, np.array([f0]), idx
