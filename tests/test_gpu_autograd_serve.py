"""GPU tests of the differentiable operator and of the serving loop.

* autograd: the backward of degridding is the gridder; checked against
  central finite differences (the loss is exactly quadratic, so any step h is
  free of truncation error) and against the oracle's direct adjoint at spot
  pixels; gradient descent decreases the loss;
* serving: requests of mixed sizes, precisions and directions give bitwise
  the same result alone and in the concurrent mix, and each matches the
  oracle within its epsilon.
"""
import math

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
    import paper_2010_10122_amd  # noqa: F401
    return torch.device("cuda:0")


def _diff_case(seed=5, n_dumps=24, n_chan=4, npix=128):
    rng = np.random.default_rng(seed)
    ant = synth.antennas_disk(rng, 24, 5000.0)
    uvw = synth.earth_rotation_uvw(ant, 2.0, n_dumps)
    freq = synth.channels(0.9e9, 1.7e9, n_chan)
    pix = 5.0 * math.pi / 180 / npix
    sky = synth.point_sources(rng, npix, npix, 20)
    return uvw, freq, pix, sky, rng


@pytest.mark.parametrize("prec,eps", [("f64", 1e-10), ("f32", 1e-5)])
def test_degrid_backward_is_gridder(dev, prec, eps):
    import paper_2010_10122_amd as wg
    from paper_2010_10122_amd import autograd as ag
    uvw, freq, pix, sky, rng = _diff_case()
    n = sky.shape[0]
    rdt = torch.float64 if prec == "f64" else torch.float32
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    plan = wg.Plan(torch.from_numpy(uvw).to(dev), torch.from_numpy(freq).to(dev), n, n, pix, pix, eps, prec)
    d_true = o1.forward(uvw, freq, sky, pix, pix)
    data = d_true + 0.1 * np.std(d_true) * synth.complex_gaussian(rng, d_true.shape)
    data_t = torch.from_numpy(data).to(dev, cdt)
    x = torch.from_numpy(rng.standard_normal((n, n))).to(dev, rdt).requires_grad_(True)

    def loss_fn(img):
        # the loss is accumulated in FP64 so that the differences below
        # resolve the FP32 operator's own rounding, not the sum's
        r = ag.degrid(img, plan) - data_t
        return 0.5 * torch.sum(r.real.double() ** 2 + r.imag.double() ** 2)

    loss = loss_fn(x)
    (g,) = torch.autograd.grad(loss, x)
    g = g.detach()
    # central differences on 32 random pixels (exact for a quadratic loss)
    pix_idx = rng.choice(n * n, 32, replace=False)
    h = 1.0
    fd = []
    with torch.no_grad():
        for p in pix_idx:
            e = torch.zeros_like(x).view(-1)
            e[p] = h
            e = e.view(n, n)
            fd.append(float(loss_fn(x + e) - loss_fn(x - e)) / (2 * h))
    fd = np.array(fd)
    gp = g.view(-1)[torch.from_numpy(pix_idx).to(dev)].cpu().numpy()
    tol = 1e-8 if prec == "f64" else 1e-4
    e_fd = np.linalg.norm(fd - gp) / np.linalg.norm(gp)
    print(f"[autograd] {prec}: central differences vs backward {e_fd:.2e}", flush=True)
    assert e_fd < tol
    # backward against the oracle's direct adjoint of the residual
    with torch.no_grad():
        resid = (ag.degrid(x.detach(), plan) - data_t).cpu().numpy()
    pp, qq = pix_idx // n, pix_idx % n
    ref = o1.adjoint(uvw, freq, resid, n, n, pix, pix, pixels=(pp, qq))
    assert np.linalg.norm(gp - ref) / np.linalg.norm(ref) < eps
    plan.close()


def test_backward_full_shape_vs_direct_adjoint(dev):
    """Differentiation workload at its full shape (1024^2 FP32 image,
    4,999,680 visibilities, eps 1e-5): the autograd gradient of
    0.5 ||R x - d||^2 against central differences (FP64-accumulated loss) on
    32 pixels and against the oracle's direct adjoint of the residual
    (eq. 3, Sect. 5) on 32 pixels."""
    import paper_2010_10122_amd as wg
    from paper_2010_10122_amd import autograd as ag
    case = synth.differentiation()
    rng = np.random.default_rng(55)
    n = case["npix_x"]
    uvw = torch.from_numpy(case["uvw"]).to(dev)
    freq = torch.from_numpy(case["freq"]).to(dev)
    px = case["pixsize_x"]
    plan = wg.Plan(uvw, freq, n, n, px, px, 1e-5, "f32")
    sky = case["sky"]
    src = np.nonzero(sky)
    n_vis = case["uvw"].shape[0] * len(case["freq"])
    # data: the oracle's closed form of the 100-source sky plus 10 % noise
    d_true = o1.forward(case["uvw"], case["freq"], sky, px, px, pixels=src).reshape(-1, len(case["freq"]))
    data = d_true + 0.1 * np.std(np.abs(d_true)) * synth.complex_gaussian(rng, d_true.shape)
    data_t = torch.from_numpy(data).to(dev, torch.complex64)
    x = torch.from_numpy(rng.standard_normal((n, n))).to(dev, torch.float32).requires_grad_(True)

    def loss_fn(img):
        r = ag.degrid(img, plan) - data_t
        return 0.5 * torch.sum(r.real.double() ** 2 + r.imag.double() ** 2)

    (g,) = torch.autograd.grad(loss_fn(x), x)
    pix = rng.choice(n * n, 32, replace=False)
    gp = g.view(-1)[torch.from_numpy(pix).to(dev)].double().cpu().numpy()
    fd = []
    with torch.no_grad():
        for p in pix:
            e = torch.zeros(n * n, dtype=torch.float32, device=dev)
            e[int(p)] = 16.0
            e = e.view(n, n)
            fd.append(float(loss_fn(x + e) - loss_fn(x - e)) / 32.0)
    e_fd = float(np.linalg.norm(np.array(fd) - gp) / np.linalg.norm(gp))
    with torch.no_grad():
        resid = (ag.degrid(x.detach(), plan) - data_t).cpu().numpy()
    ref = o1.adjoint(case["uvw"], case["freq"], resid, n, n, px, px, pixels=(pix // n, pix % n))
    e_adj = float(np.linalg.norm(gp - ref) / np.linalg.norm(ref))
    print(f"[autograd full] {n_vis} vis: FD {e_fd:.2e}, vs direct adjoint {e_adj:.2e}", flush=True)
    assert e_fd < 1e-4
    assert e_adj < 1e-5
    plan.close()


def test_grid_backward_is_degridder(dev):
    import paper_2010_10122_amd as wg
    from paper_2010_10122_amd import autograd as ag
    uvw, freq, pix, sky, rng = _diff_case(seed=8)
    n = sky.shape[0]
    plan = wg.Plan(torch.from_numpy(uvw).to(dev), torch.from_numpy(freq).to(dev), n, n, pix, pix, 1e-10, "f64")
    v = torch.from_numpy(synth.complex_gaussian(rng, (uvw.shape[0], len(freq)))).to(dev).requires_grad_(True)
    w = torch.from_numpy(rng.standard_normal((n, n))).to(dev)
    out = torch.sum(ag.grid(v, plan) * w)
    (gv,) = torch.autograd.grad(out, v)
    # <Re R^H v, w> = Re <v, R w>: d/dv* gives R w
    ref = plan.degrid(w)
    assert torch.linalg.vector_norm(gv - ref) / torch.linalg.vector_norm(ref) < 1e-12
    plan.close()


def test_gradient_descent_reduces_loss(dev):
    import paper_2010_10122_amd as wg
    from paper_2010_10122_amd import autograd as ag
    uvw, freq, pix, sky, rng = _diff_case(seed=9)
    n = sky.shape[0]
    plan = wg.Plan(torch.from_numpy(uvw).to(dev), torch.from_numpy(freq).to(dev), n, n, pix, pix, 1e-5, "f32")
    data = torch.from_numpy(o1.forward(uvw, freq, sky, pix, pix)).to(dev, torch.complex64)
    lam = ag.lipschitz_estimate(plan, iters=10)
    assert lam > 0
    x, losses = ag.gradient_descent(plan, data, steps=20, step_size=1.0 / lam)
    assert losses[-1] < 0.5 * losses[0]
    assert all(b <= a * (1 + 1e-4) for a, b in zip(losses, losses[1:]))
    plan.close()


def _requests(dev, seed=4, count=14):
    from paper_2010_10122_amd.serve import Request
    rng = np.random.default_rng(seed)
    ant = synth.antennas_disk(rng, 16, 3000.0)
    uvw_all = synth.earth_rotation_uvw(ant, 4.0, 120)
    freq_all = synth.channels(0.9e9, 1.7e9, 8)
    coords = {}
    reqs = []
    for rid in range(count):
        npix = int(rng.choice([64, 128, 256]))
        eps = float(rng.choice([1e-4, 1e-5, 1e-7, 1e-9]))
        prec = "f32" if eps >= 1e-5 else "f64"
        nrow = int(rng.integers(50, 1500))
        r0 = int(rng.integers(0, len(uvw_all) - nrow))
        nch = int(rng.integers(1, 9))
        key = (r0, nrow, nch)
        if key not in coords:
            coords[key] = (torch.from_numpy(uvw_all[r0:r0 + nrow]).to(dev),
                           torch.from_numpy(freq_all[:nch]).to(dev))
        uvw, freq = coords[key]
        pix = 6.0 * math.pi / 180 / npix
        direction = "degrid" if rng.random() < 0.5 else "grid"
        rdt = torch.float32 if prec == "f32" else torch.float64
        cdt = torch.complex64 if prec == "f32" else torch.complex128
        if direction == "degrid":
            data = torch.from_numpy(rng.standard_normal((npix, npix))).to(dev, rdt)
        else:
            data = torch.from_numpy(synth.complex_gaussian(rng, (nrow, nch))).to(dev, cdt)
        reqs.append(Request(rid, direction, key, uvw, freq, npix, pix, eps, prec, data,
                            arrival=float(rid) * 1e-3))
    return reqs


def test_serving_alone_equals_mix(dev):
    from paper_2010_10122_amd.serve import Server, summarize
    reqs = _requests(dev)
    alone = {}
    srv = Server(dev, n_slots=1)
    for r in reqs:
        res, _ = srv.run([r], realtime=False)
        alone[r.rid] = res[0].output.cpu()
    srv.close()
    srv = Server(dev, n_slots=4)
    res, makespan = srv.run(reqs, realtime=True)
    srv.close()
    assert len(res) == len(reqs)
    for r in res:
        assert torch.equal(r.output.cpu(), alone[r.rid]), r.rid
    s = summarize(res, makespan)
    assert s["p99_ms"] >= s["p50_ms"] > 0
    # every result within its epsilon of the direct transform
    byid = {r.rid: r for r in reqs}
    for r in res[:6]:
        q = byid[r.rid]
        uvw = q.uvw.cpu().numpy()
        freq = q.freq.cpu().numpy()
        if q.direction == "degrid":
            ref = o1.forward(uvw, freq, q.data.cpu().numpy().astype(np.float64), q.pixsize, q.pixsize)
        else:
            ref = o1.adjoint(uvw, freq, q.data.cpu().numpy().astype(np.complex128), q.npix, q.npix, q.pixsize,
                             q.pixsize)
        got = r.output.cpu().numpy()
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < q.epsilon, (q.rid, q.direction, q.epsilon)


def test_serving_alone_equals_mix_large_images(dev):
    """Serving at the image sizes of the serving workload (512^2 to 2048^2,
    10 deg / 2048 pixels, FP32 and FP64, 2e5 to 1.6e6 visibilities of the
    wide-field array): each result is bitwise the same alone and in the
    concurrent mix, and within its epsilon of the direct transform on
    sampled outputs."""
    from paper_2010_10122_amd.serve import Request, Server
    base = synth.wide_field(n_dumps=200, with_vis=False)
    rng = np.random.default_rng(44)
    pix = 10.0 * math.pi / 180 / 2048
    reqs = []
    coords = {}
    for rid, (npix, eps, direction, nrow, nch) in enumerate([
            (512, 1e-5, "degrid", 25000, 8), (1024, 1e-9, "grid", 50000, 16), (2048, 1e-4, "grid", 100000, 16),
            (1024, 1e-5, "degrid", 100000, 16), (512, 1e-7, "degrid", 12500, 16), (2048, 1e-5, "degrid", 50000, 4),
            (512, 1e-4, "grid", 100000, 2), (1024, 1e-7, "grid", 25000, 8)]):
        r0 = int(rng.integers(0, base["uvw"].shape[0] - nrow))
        key = (r0, nrow, nch)
        coords[key] = (torch.from_numpy(np.ascontiguousarray(base["uvw"][r0:r0 + nrow])).to(dev),
                       torch.from_numpy(np.ascontiguousarray(base["freq"][:nch])).to(dev))
        prec = "f32" if eps >= 1e-5 else "f64"
        rdt = torch.float32 if prec == "f32" else torch.float64
        cdt = torch.complex64 if prec == "f32" else torch.complex128
        if direction == "degrid":
            data = torch.from_numpy(rng.standard_normal((npix, npix))).to(dev, rdt)
        else:
            data = torch.from_numpy(synth.complex_gaussian(rng, (nrow, nch))).to(dev, cdt)
        reqs.append(Request(rid, direction, key, coords[key][0], coords[key][1], npix, pix, eps, prec, data,
                            arrival=0.02 * rid))
    alone = {}
    srv = Server(dev, n_slots=1)
    for r in reqs:
        res, _ = srv.run([r], realtime=False)
        alone[r.rid] = res[0].output.cpu()
    srv.close()
    srv = Server(dev, n_slots=4)
    res, _ = srv.run(reqs, realtime=True)
    srv.close()
    assert len(res) == len(reqs)
    for r in res:
        assert torch.equal(r.output.cpu(), alone[r.rid]), r.rid
    byid = {r.rid: r for r in reqs}
    for r in res:
        q = byid[r.rid]
        uvw = q.uvw.cpu().numpy()
        freq = q.freq.cpu().numpy()
        got = r.output.cpu().numpy()
        if q.direction == "degrid":
            idx = rng.choice(uvw.shape[0] * len(freq), 64, replace=False)
            ref = o1.forward(uvw, freq, q.data.cpu().numpy().astype(np.float64), q.pixsize, q.pixsize, vis_idx=idx)
            got = got.reshape(-1)[idx]
        else:
            pp = rng.integers(0, q.npix, 16)
            qq = rng.integers(0, q.npix, 16)
            ref = o1.adjoint(uvw, freq, q.data.cpu().numpy().astype(np.complex128), q.npix, q.npix, q.pixsize,
                             q.pixsize, pixels=(pp, qq))
            got = got[pp, qq]
        e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"[serve large] rid {q.rid} {q.direction} {q.npix}^2 eps {q.epsilon:g}: {e:.2e}", flush=True)
        assert e < q.epsilon, (q.rid, q.direction, q.epsilon)
