"""GPU parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times, on sampled outputs the direct transform (O1)
evaluates one by one:

* wide field (2048^2 over 10 deg, 92,897,280 visibilities): FP32 at
  eps = 1e-5, FP64 at eps = 1e-5 (the plain FP64 form) and at eps = 1e-10,
  both directions;
* large (8192^2 over 30 deg, 261,120,000 visibilities, about 12,500
  w-planes): FP32 at eps = 1e-5, both directions.

Degridding is checked on random visibilities, gridding on random pixels;
the relative L2 error of the sample must stay below eps.  Binning (Sect.
4.3) is checked bit for bit against the oracle's binning spec on every
visibility of both workloads.
"""
import numpy as np
import pytest

import synth
from oracle import o1

from gpu_util import check_binning_full

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_10122_amd  # noqa: F401  (fails loudly without libwgrid.so)
    return torch.device("cuda:0")


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def wide():
    return synth.wide_field()


@pytest.mark.parametrize("prec,eps", [("f32", 1e-5), ("f64", 1e-5), ("f64", 1e-10)])
def test_wide_field_sampled(dev, wide, prec, eps):
    import paper_2010_10122_amd as wg
    c = wide
    print(f"[wide] {prec} eps={eps}", flush=True)
    rdt = torch.float32 if prec == "f32" else torch.float64
    cdt = torch.complex64 if prec == "f32" else torch.complex128
    uvw = torch.from_numpy(c["uvw"]).to(dev)
    freq = torch.from_numpy(c["freq"]).to(dev)
    plan = wg.Plan(uvw, freq, c["npix_x"], c["npix_y"], c["pixsize_x"], c["pixsize_y"], eps, prec)
    info = plan.info
    print(f"   plan alpha={info['alpha']} sigma={info['sigma']} N={info['nu']} Nw={info['nw']}", flush=True)
    vis = plan.degrid(torch.from_numpy(c["dirty"]).to(dev, rdt))
    img = plan.grid(torch.from_numpy(c["vis"]).to(dev, cdt))
    torch.cuda.synchronize()
    n_vis = c["uvw"].shape[0] * len(c["freq"])
    rng = np.random.default_rng(11)
    idx = rng.choice(n_vis, size=2000, replace=False)
    got = vis.reshape(-1)[torch.from_numpy(idx).to(dev)].cpu().numpy()
    # the image is 500 point sources: the direct sum runs over them only
    ref = o1.forward(c["uvw"], c["freq"], c["dirty"], c["pixsize_x"], c["pixsize_y"], vis_idx=idx)
    e_deg = _rel(got, ref)
    pp = rng.integers(0, c["npix_x"], 32)
    qq = rng.integers(0, c["npix_y"], 32)
    got_i = img[torch.from_numpy(pp).to(dev), torch.from_numpy(qq).to(dev)].cpu().numpy()
    ref_i = o1.adjoint(c["uvw"], c["freq"], c["vis"], c["npix_x"], c["npix_y"], c["pixsize_x"], c["pixsize_y"],
                       pixels=(pp, qq))
    e_grid = _rel(got_i, ref_i)
    print(f"   degrid {e_deg:.2e} (2000 vis)  grid {e_grid:.2e} (32 px)", flush=True)
    assert e_deg < eps and e_grid < eps
    plan.close()


@pytest.mark.parametrize("prec,eps", [("f32", 1e-5), ("f64", 1e-5), ("f64", 1e-10)])
def test_wide_field_binning_bit_exact(dev, wide, prec, eps):
    import paper_2010_10122_amd as wg
    c = wide
    print(f"[wide binning] {prec} eps={eps}", flush=True)
    uvw = torch.from_numpy(c["uvw"]).to(dev)
    freq = torch.from_numpy(c["freq"]).to(dev)
    plan = wg.Plan(uvw, freq, c["npix_x"], c["npix_y"], c["pixsize_x"], c["pixsize_y"], eps, prec)
    n = check_binning_full(c, plan, torch)
    print(f"   {n} keys bit-exact (alpha={plan.info['alpha']} sigma={plan.info['sigma']} "
          f"N={plan.info['nu']} Nw={plan.info['nw']})", flush=True)
    plan.close()


@pytest.fixture(scope="module")
def large(dev):
    c = synth.large()
    uvw = torch.from_numpy(c["uvw"]).to(dev)
    freq = torch.from_numpy(c["freq"]).to(dev)
    import paper_2010_10122_amd as wg
    plan = wg.Plan(uvw, freq, c["npix_x"], c["npix_y"], c["pixsize_x"], c["pixsize_y"], 1e-5, "f32")
    yield c, plan
    plan.close()


def test_large_degrid_sampled(dev, large):
    c, plan = large
    info = plan.info
    print(f"[large degrid] alpha={info['alpha']} sigma={info['sigma']} N={info['nu']} Nw={info['nw']}", flush=True)
    vis = plan.degrid(torch.from_numpy(c["dirty"]).to(dev))
    torch.cuda.synchronize()
    n_vis = c["uvw"].shape[0] * len(c["freq"])
    idx = np.random.default_rng(12).choice(n_vis, size=32, replace=False)
    got = vis.reshape(-1)[torch.from_numpy(idx).to(dev)].cpu().numpy()
    ref = o1.forward(c["uvw"], c["freq"], c["dirty"], c["pixsize_x"], c["pixsize_y"], vis_idx=idx)
    e = _rel(got, ref)
    print(f"   degrid {e:.2e} (32 vis)", flush=True)
    assert e < 1e-5


def test_large_grid_sampled(dev, large):
    c, plan = large
    print("[large grid]", flush=True)
    img = plan.grid(torch.from_numpy(c["vis"]).to(dev))
    torch.cuda.synchronize()
    rng = np.random.default_rng(13)
    pp = rng.integers(0, c["npix_x"], 16)
    qq = rng.integers(0, c["npix_y"], 16)
    got = img[torch.from_numpy(pp).to(dev), torch.from_numpy(qq).to(dev)].cpu().numpy()
    ref = o1.adjoint(c["uvw"], c["freq"], c["vis"], c["npix_x"], c["npix_y"], c["pixsize_x"], c["pixsize_y"],
                     pixels=(pp, qq))
    e = _rel(got, ref)
    print(f"   grid {e:.2e} (16 px)", flush=True)
    assert e < 1e-5


def test_large_binning_bit_exact(dev, large):
    c, plan = large
    print("[large binning]", flush=True)
    n = check_binning_full(c, plan, torch, chunk_rows=1 << 21)
    print(f"   {n} keys bit-exact", flush=True)
