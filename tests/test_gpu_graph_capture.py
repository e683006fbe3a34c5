"""HIP graph capture of the apply calls.

wg_degrid / wg_grid with a caller workspace, and the allocation-free
wg_apply_noalloc, are captured into one graph: degrid then grid on the
capturing stream. Each call forks onto the plan's second stream and joins
back inside the capture. The graph is replayed several times, with eager
work and a synchronisation between the replays. Every replay must equal
the eager outputs bit for bit (the apply kernels are deterministic).
"""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_10122_amd  # noqa: F401  (fails loudly without libwgrid.so)
    return torch.device("cuda:0")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _noalloc(plan, adjoint, inp, out, wgt):
    from paper_2010_10122_amd import _lib
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return _lib.load().wg_apply_noalloc(plan._h, int(adjoint), _ptr(inp), _ptr(wgt), _ptr(out), st)


@pytest.mark.parametrize("prec,eps,masked", [("f32", 1e-5, False), ("f64", 1e-9, True)])
def test_apply_graph_replays_equal_eager(dev, prec, eps, masked):
    import paper_2010_10122_amd as wg
    from paper_2010_10122_amd import _lib
    rng = np.random.default_rng(21)
    ant = synth.antennas_disk(rng, 16, 3000.0)
    uvw_h = synth.earth_rotation_uvw(ant, 6.0, 30)[:3000]
    freq_h = synth.channels(0.9e9, 1.7e9, 6)
    npix = 192
    pix = 6.0 * np.pi / 180 / npix
    mask = None
    if masked:
        mask = torch.from_numpy((rng.random((uvw_h.shape[0], len(freq_h))) > 0.2).astype(np.uint8)).to(dev)
    plan = wg.Plan(torch.from_numpy(uvw_h).to(dev), torch.from_numpy(freq_h).to(dev), npix, npix, pix, pix, eps,
                   prec, mask=mask)
    info = plan.info
    print(f"[graph] {prec} N={info['nu']} Nw={info['nw']} P={info['planes_per_batch']}", flush=True)
    assert info["nw"] > 2 * info["planes_per_batch"]          # several batches, both plane buffers
    assert plan.workspace_bytes <= _lib.WG_SCRATCH_BYTES
    rdt, cdt = plan.real_dtype, plan.complex_dtype
    dirty = torch.from_numpy(rng.standard_normal((npix, npix))).to(dev, rdt)
    vis = torch.from_numpy(synth.complex_gaussian(rng, (uvw_h.shape[0], len(freq_h)))).to(dev, cdt)
    wgt = torch.from_numpy(rng.uniform(0.5, 1.5, (uvw_h.shape[0], len(freq_h)))).to(dev, rdt)
    eager_v = plan.degrid(dirty, wgt=wgt)
    eager_i = plan.grid(vis, wgt=wgt)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    outs = [torch.empty_like(eager_v), torch.empty_like(eager_i), torch.empty_like(eager_v),
            torch.empty_like(eager_i)]
    torch.cuda.synchronize()
    # warm-up on a side stream before the capture
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.degrid(dirty, wgt=wgt, out=outs[0], workspace=ws)
        plan.grid(vis, wgt=wgt, out=outs[1], workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.degrid(dirty, wgt=wgt, out=outs[0], workspace=ws)
        plan.grid(vis, wgt=wgt, out=outs[1], workspace=ws)
        rc_v = _noalloc(plan, 0, dirty, outs[2], wgt)
        rc_i = _noalloc(plan, 1, vis, outs[3], wgt)
    assert rc_v == _lib.WG_OK and rc_i == _lib.WG_OK
    for rep in range(3):
        for t in outs:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        print(f"   replay {rep}", flush=True)
        assert torch.equal(outs[0], eager_v) and torch.equal(outs[2], eager_v)
        assert torch.equal(outs[1], eager_i) and torch.equal(outs[3], eager_i)
    del g
    plan.close()


def test_concurrent_calls_on_one_plan(dev):
    """Two host threads apply one plan at once, each on its own stream with
    its own workspace and outputs.  The calls share the plan's second stream
    and its enqueue lock; every output must equal the single-stream result
    bit for bit."""
    import threading

    import paper_2010_10122_amd as wg
    rng = np.random.default_rng(23)
    ant = synth.antennas_disk(rng, 16, 3000.0)
    uvw_h = synth.earth_rotation_uvw(ant, 6.0, 30)[:3000]
    freq_h = synth.channels(0.9e9, 1.7e9, 6)
    npix = 192
    pix = 6.0 * np.pi / 180 / npix
    plan = wg.Plan(torch.from_numpy(uvw_h).to(dev), torch.from_numpy(freq_h).to(dev), npix, npix, pix, pix, 1e-5,
                   "f32")
    dirty = torch.from_numpy(rng.standard_normal((npix, npix))).to(dev, plan.real_dtype)
    vis = torch.from_numpy(synth.complex_gaussian(rng, (uvw_h.shape[0], len(freq_h)))).to(dev, plan.complex_dtype)
    ref_v = plan.degrid(dirty)
    ref_i = plan.grid(vis)
    torch.cuda.synchronize()
    results, errors = {}, []

    def worker(k):
        try:
            st = torch.cuda.Stream()
            ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
            outs = []
            for _ in range(3):
                ov = torch.empty_like(ref_v)
                oi = torch.empty_like(ref_i)
                plan.degrid(dirty, out=ov, workspace=ws, stream=st)
                plan.grid(vis, out=oi, workspace=ws, stream=st)
                outs.append((ov, oi))
            st.synchronize()
            results[k] = outs
        except Exception as e:          # reported by the main thread
            errors.append(repr(e))

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for k in range(2):
        for ov, oi in results[k]:
            assert torch.equal(ov, ref_v) and torch.equal(oi, ref_i)
    print(f"[concurrent] {sum(len(r) for r in results.values())} call pairs equal", flush=True)
    plan.close()
