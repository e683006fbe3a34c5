"""GPU parity on the benchmark set-up of Sect. 6 (synthetic stand-in for the
paper's MeerKAT L-band set: 824,476 rows x 2048 channels flagged down to
470.1 million visibilities, 4096^2 over 1.6 deg):

* Sect. 6.1: FP32, eps = 1e-4, w-gridding, both directions;
* Sect. 6.2: FP64, eps = 1e-10, no w term, on the multi-channel set and on
  its flattened form (one channel, one row per selected visibility).

Degridding is checked against the direct sum (O1) on random selected
visibilities, and every flagged visibility must come out zero.  Gridding
takes an input that is zero except on 200,000 random selected
visibilities, so that the direct adjoint over just those is the exact
reference; it is checked on random pixels.
"""
import numpy as np
import pytest

import synth
from oracle import o1

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_10122_amd  # noqa: F401  (fails loudly without libwgrid.so)
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def meerkat(dev):
    c = synth.meerkat_like()
    uvw = torch.from_numpy(c["uvw"]).to(dev)
    freq = torch.from_numpy(c["freq"]).to(dev)
    mask = torch.from_numpy(c["mask"]).to(dev)
    return c, uvw, freq, mask


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def _check(c, plan, uvw_h, freq_h, mask_h, prec, eps, do_w, dev, seed):
    rng = np.random.default_rng(seed)
    rdt = torch.float32 if prec == "f32" else torch.float64
    cdt = torch.complex64 if prec == "f32" else torch.complex128
    n_total = uvw_h.shape[0] * len(freq_h)
    sel = np.flatnonzero(mask_h.reshape(-1)) if mask_h is not None else np.arange(n_total)
    # degridding: random selected visibilities against the direct sum over the sources
    vis = plan.degrid(torch.from_numpy(c["dirty"]).to(dev, rdt))
    idx = np.sort(rng.choice(sel, 400, replace=False))
    got = vis.reshape(-1)[torch.from_numpy(idx).to(dev)].cpu().numpy()
    ref = o1.forward(uvw_h, freq_h, c["dirty"], c["pixsize_x"], c["pixsize_y"], do_wgridding=do_w, vis_idx=idx,
                     pixels=np.nonzero(c["dirty"]))
    e_deg = _rel(got, ref)
    if mask_h is not None:
        flagged = np.flatnonzero(mask_h.reshape(-1) == 0)
        fidx = torch.from_numpy(rng.choice(flagged, 10000, replace=False)).to(dev)
        assert bool(torch.all(vis.reshape(-1)[fidx] == 0))
    del vis
    # gridding: input zero except on K random selected visibilities
    K = 200_000
    pick = np.sort(rng.choice(sel, K, replace=False))
    vals = synth.complex_gaussian(rng, (K,))
    v_dev = torch.zeros(n_total, dtype=cdt, device=dev)
    v_dev[torch.from_numpy(pick).to(dev)] = torch.from_numpy(vals).to(dev, cdt)
    img = plan.grid(v_dev.reshape(uvw_h.shape[0], len(freq_h)))
    del v_dev
    pp = rng.integers(0, c["npix_x"], 16)
    qq = rng.integers(0, c["npix_y"], 16)
    got_i = img[torch.from_numpy(pp).to(dev), torch.from_numpy(qq).to(dev)].cpu().numpy()
    # direct adjoint over the picked visibilities only: rows holding them, one
    # selected entry each in a mask over those rows
    rows = pick // len(freq_h)
    ur, inv_r = np.unique(rows, return_inverse=True)
    sub_vis = np.zeros((len(ur), len(freq_h)), dtype=np.complex128)
    sub_mask = np.zeros((len(ur), len(freq_h)), dtype=np.uint8)
    ch = pick - rows * len(freq_h)
    sub_vis[inv_r, ch] = vals
    sub_mask[inv_r, ch] = 1
    ref_i = o1.adjoint(uvw_h[ur], freq_h, sub_vis, c["npix_x"], c["npix_y"], c["pixsize_x"], c["pixsize_y"],
                       do_wgridding=do_w, mask=sub_mask, pixels=(pp, qq))
    e_grid = _rel(got_i, ref_i)
    return e_deg, e_grid


def test_sect61_f32_eps1e4(dev, meerkat):
    import paper_2010_10122_amd as wg
    c, uvw, freq, mask = meerkat
    print("[paper 6.1] FP32 eps=1e-4, w-gridding", flush=True)
    plan = wg.Plan(uvw, freq, c["npix_x"], c["npix_y"], c["pixsize_x"], c["pixsize_y"], 1e-4, "f32", mask=mask)
    info = plan.info
    print(f"   plan alpha={info['alpha']} sigma={info['sigma']} N={info['nu']} Nw={info['nw']} "
          f"n_vis={info['n_vis']}", flush=True)
    assert info["n_vis"] == int(c["mask"].sum())
    e_deg, e_grid = _check(c, plan, c["uvw"], c["freq"], c["mask"], "f32", 1e-4, True, dev, 61)
    print(f"   degrid {e_deg:.2e} grid {e_grid:.2e}", flush=True)
    assert e_deg < 1e-4 and e_grid < 1e-4
    plan.close()


def test_sect62_f64_eps1e10_no_w(dev, meerkat):
    import paper_2010_10122_amd as wg
    c, uvw, freq, mask = meerkat
    print("[paper 6.2] FP64 eps=1e-10, no w, multichannel", flush=True)
    plan = wg.Plan(uvw, freq, c["npix_x"], c["npix_y"], c["pixsize_x"], c["pixsize_y"], 1e-10, "f64", mask=mask,
                   do_wgridding=False)
    info = plan.info
    assert info["nw"] == 1
    print(f"   plan alpha={info['alpha']} sigma={info['sigma']} N={info['nu']}", flush=True)
    e_deg, e_grid = _check(c, plan, c["uvw"], c["freq"], c["mask"], "f64", 1e-10, False, dev, 62)
    print(f"   degrid {e_deg:.2e} grid {e_grid:.2e}", flush=True)
    assert e_deg < 1e-10 and e_grid < 1e-10
    plan.close()


def test_sect62_f64_eps1e10_no_w_flattened(dev, meerkat):
    import paper_2010_10122_amd as wg
    c, _, _, _ = meerkat
    print("[paper 6.2] FP64 eps=1e-10, no w, flattened", flush=True)
    uvw_f, freq_f, _ = synth.flatten_channels(c["uvw"], c["freq"], c["mask"])
    plan = wg.Plan(torch.from_numpy(uvw_f).to(dev), torch.from_numpy(freq_f).to(dev), c["npix_x"], c["npix_y"],
                   c["pixsize_x"], c["pixsize_y"], 1e-10, "f64", do_wgridding=False)
    info = plan.info
    print(f"   plan alpha={info['alpha']} sigma={info['sigma']} N={info['nu']} rows={uvw_f.shape[0]}", flush=True)
    assert info["n_vis"] == uvw_f.shape[0]
    e_deg, e_grid = _check(c, plan, uvw_f, freq_f, None, "f64", 1e-10, False, dev, 63)
    print(f"   degrid {e_deg:.2e} grid {e_grid:.2e}", flush=True)
    assert e_deg < 1e-10 and e_grid < 1e-10
    plan.close()
