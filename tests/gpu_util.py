"""Helpers for the GPU tests: run the product through its Python binding (the
C ABI) and compare with the oracle."""
import numpy as np


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def eps_adj(d_img, vis, img, i_vis):
    """eq. (adjointness) criterion of Sect. 5.1."""
    lhs = np.vdot(d_img, vis).real
    rhs = np.vdot(img, i_vis)
    den = min(np.linalg.norm(vis) * np.linalg.norm(d_img), np.linalg.norm(img) * np.linalg.norm(i_vis))
    return abs(lhs - rhs) / den


def to_dev(case, torch, dev, mask=None):
    uvw = torch.from_numpy(np.ascontiguousarray(case["uvw"])).to(dev)
    freq = torch.from_numpy(np.ascontiguousarray(case["freq"])).to(dev)
    m = None if mask is None else torch.from_numpy(np.ascontiguousarray(mask, dtype=np.uint8)).to(dev)
    return uvw, freq, m


def run_product(case, eps, prec, torch, dev, dirty=None, vis=None, wgt=None, mask=None, **plan_kw):
    import paper_2010_10122_amd as wg
    uvw, freq, m = to_dev(case, torch, dev, mask)
    plan = wg.Plan(uvw, freq, case["npix_x"], case["npix_y"], case["pixsize_x"], case["pixsize_y"], eps, prec,
                   mask=m, **plan_kw)
    rdt = plan.real_dtype
    cdt = plan.complex_dtype
    w = None if wgt is None else torch.from_numpy(np.ascontiguousarray(wgt)).to(dev, rdt)
    out = {"plan": plan, "info": plan.info}
    if dirty is not None:
        out["vis"] = plan.degrid(torch.from_numpy(np.ascontiguousarray(dirty)).to(dev, rdt), wgt=w).cpu().numpy()
    if vis is not None:
        out["img"] = plan.grid(torch.from_numpy(np.ascontiguousarray(vis)).to(dev, cdt), wgt=w).cpu().numpy()
    torch.cuda.synchronize()
    return out


def oracle_plan_from(info, case, mask=None):
    from oracle import plan as P
    return P.make_plan(case["uvw"], case["freq"], case["npix_x"], case["npix_y"], case["pixsize_x"],
                       case["pixsize_y"], info["alpha"], info["sigma"], do_wgridding=bool(info["do_wgridding"]),
                       mask=mask)
