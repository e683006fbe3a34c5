"""GPU tests of plan memory ownership (the boundary's allocation contract):

* a plan returns every device byte it holds when destroyed, through
  hipMalloc/hipFree and through PyTorch's caching allocator (the C ABI's
  allocator callbacks), also over many create/destroy cycles;
* wg_plan_estimate bounds the plan's resident bytes and the workspace
  before the plan exists.
"""
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


@pytest.fixture(scope="module")
def wide_coords(dev):
    c = synth.wide_field(with_vis=False)
    uvw = torch.from_numpy(c["uvw"]).to(dev)
    freq = torch.from_numpy(c["freq"]).to(dev)
    torch.cuda.synchronize()
    return c, uvw, freq


@pytest.mark.parametrize("torch_allocator", [False, True])
def test_create_destroy_returns_memory(dev, wide_coords, torch_allocator):
    """Ten wide-field plans (92.9M visibilities, 2048^2, FP32 eps 1e-5: about
    2.8 GB each) created and destroyed: device memory is back at its
    starting level."""
    import paper_2010_10122_amd as wg
    c, uvw, freq = wide_coords
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0, _ = torch.cuda.mem_get_info(dev)
    alloc0 = torch.cuda.memory_allocated(dev)
    held = []
    for i in range(10):
        plan = wg.Plan(uvw, freq, c["npix_x"], c["npix_y"], c["pixsize_x"], c["pixsize_y"], 1e-5, "f32",
                       torch_allocator=torch_allocator)
        held.append(plan.info["plan_bytes"])
        if torch_allocator:
            # the plan's blocks are the caching allocator's
            assert torch.cuda.memory_allocated(dev) - alloc0 >= plan.info["plan_bytes"]
        plan.close()
        if torch_allocator:
            assert torch.cuda.memory_allocated(dev) == alloc0, i
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free1, _ = torch.cuda.mem_get_info(dev)
    print(f"[memory] torch_allocator={torch_allocator}: plan {held[0] / 2**30:.2f} GiB, free before "
          f"{free0 / 2**30:.2f} GiB, after {free1 / 2**30:.2f} GiB", flush=True)
    assert min(held) > 1 << 30
    assert abs(free1 - free0) <= 64 << 20


@pytest.mark.parametrize("prec,eps,mask_frac", [("f32", 1e-5, 0.0), ("f64", 1e-10, 0.3)])
def test_estimate_bounds_plan(dev, prec, eps, mask_frac):
    """wg_plan_estimate, called before the plan exists, bounds the built
    plan's resident bytes and workspace (the serving loop admits plan builds
    by it)."""
    import paper_2010_10122_amd as wg
    rng = np.random.default_rng(17)
    ant = synth.antennas_disk(rng, 32, 4000.0)
    uvw_h = synth.earth_rotation_uvw(ant, 6.0, 200)
    freq_h = synth.channels(0.9e9, 1.7e9, 8)
    uvw = torch.from_numpy(uvw_h).to(dev)
    freq = torch.from_numpy(freq_h).to(dev)
    mask = None
    if mask_frac > 0:
        mask = torch.from_numpy((rng.random((uvw_h.shape[0], 8)) > mask_frac).astype(np.uint8)).to(dev)
    pix = 8.0 * np.pi / 180 / 512
    est = wg.Plan.estimate(uvw, freq, 512, 512, pix, pix, eps, prec, mask=mask)
    plan = wg.Plan(uvw, freq, 512, 512, pix, pix, eps, prec, mask=mask)
    info = plan.info
    print(f"[estimate] {prec}: plan {info['plan_bytes']} <= {est['plan_bytes']}, peak {est['peak_bytes']}, "
          f"workspace {info['workspace_bytes']} <= {est['workspace_bytes']}", flush=True)
    assert info["plan_bytes"] <= est["plan_bytes"] <= 1.25 * info["plan_bytes"] + (1 << 20)
    assert est["peak_bytes"] >= est["plan_bytes"]
    assert info["workspace_bytes"] <= est["workspace_bytes"]
    plan.close()
