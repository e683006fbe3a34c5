#!/usr/bin/env python
"""Benchmark: w-gridding grid & degrid throughput on one MI355X.

Workload (wide field): 2048^2 image over 10 deg, 64 antennas in a 5 km disk,
8 h at 10 s dumps (5,806,080 rows) x 16 channels over 0.9-1.7 GHz =
92,897,280 visibilities, 500 point sources; synthetic, seeded.

One step = one forward (degrid) plus one adjoint (grid) application of the
operator with the plan (kernel choice, corrections, visibility index)
resident on the device; plan construction is timed separately (cold).
value = visibilities / mean time of one operator application, FP32 at
epsilon = 1e-5; the plain FP64 form at the same epsilon is timed beside it.

Further legs after the headline (each can be switched off; --quick runs the
headline alone): FP64 at eps 1e-5 and 1e-10, differentiation, a serving
load sweep, run time against epsilon (Sect. 6.3), the Sect. 6 benchmark
shape (Sect. 6.1 FP32 eps 1e-4; Sect. 6.2 FP64 eps 1e-10 without w, multi-
channel and flattened), the large workload, and last the CPU leg: the
oracle timed on a bounded slice (cpu_baseline) and the sampled accuracy of
every leg's outputs against the oracle's direct sum.

Prints one JSON line.  --gpus N with N > 1 is refused: the operator runs on
one GPU (sharding over GPUs is not implemented).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mvis/s grid & degrid at ε=1e-5 FP32 vs plain FP64; p50/p99 serve latency"
HBM_PEAK_GBS = 8000.0


def kernel_bytes(info, kind, n_launch_planes, precision):
    """Algorithmic HBM bytes of one launch of a kernel kind covering
    ``n_launch_planes`` w-planes (average batch), from the data each kernel
    must read and write at least once."""
    sc = 8.0 if precision == "f32" else 16.0
    sr = sc / 2
    nu, nv, nx, ny = info["nu"], info["nv"], info["npix_x"], info["npix_y"]
    P = n_launch_planes
    nbatch = math.ceil(info["nw"] / info["planes_per_batch"])
    f_batch = (info["planes_per_batch"] + info["alpha"] - 1) / info["planes_per_batch"]
    vis_per_launch = info["n_vis"] * f_batch / nbatch
    if kind == "grid":           # visibilities + index in, P full grid planes out
        return P * nu * nv * sc + vis_per_launch * (sc + 4)
    if kind == "degrid":         # P grid planes in, visibility accumulators updated
        return P * nu * nv * sc + vis_per_launch * (4 + 2 * sc)
    if kind == "fft_rows_grid":  # P grid planes in, pruned rows out
        return P * nu * nv * sc + P * nu * ny * sc
    if kind == "fft_cols_grid":  # pruned rows in, n-1 in, image accumulator read+write
        return P * nu * ny * sc + nx * ny * 8 + 2 * nx * ny * sr
    if kind == "fft_rows_degrid":  # corrected image + n-1 in, P padded rows out
        return nx * ny * (sr + 8) + P * nx * nv * sc
    if kind == "fft_cols_degrid":  # P padded rows in, P grid planes out
        return P * nx * nv * sc + P * nu * nv * sc
    return float("nan")


def profiled_traffic(kind):
    """HBM bytes per dispatch of ``kind`` from the committed rocprofv3 counter
    summary of this workload (2 x FETCH_SIZE + WRITE_SIZE, see the profile
    file), or None when the kernel sources changed since it was taken."""
    import glob
    import hashlib
    path = os.path.join(ROOT, "profiles", "wide_field_f32_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) == 2 and not line.startswith("#"):
                vals[parts[0]] = parts[1]
    src = sorted(glob.glob(os.path.join(ROOT, "paper_2010_10122_amd", "csrc", "*")))
    h = hashlib.sha1(b"".join(open(q, "rb").read() for q in src)).hexdigest()
    if vals.get("source_sha1") != h or kind not in vals:
        return None
    return float(vals[kind])


def _cpu_info():
    """(threads the oracle may use, CPU model) of this host."""
    cores = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        cores = min(cores, int(os.environ["OMP_NUM_THREADS"]))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, model


def cpu_baseline(case, info, n_vis, sample_rows=800_000, seed=99):
    """The oracle O2 (plain FP64 w-gridder: exact kernel, numpy FFTs, its own
    binning) at the same plan as the timed FP32 run, on a slice of the
    workload, extrapolated to the whole operator.

    A full O2 application of this workload runs every one of its N_w planes
    (minutes each way), so it is timed on a slice: the alpha + 1 planes
    around the median first plane of a row sample, with the visibilities of
    that sample whose alpha planes lie in the slice (run A), and again with
    an eighth of them (run B).  O2's cost per call is modelled as
    T = F + a N_w + b n_v: F (the correction 1/(n Psi), recomputed by every
    call) is timed on its own, b comes from A - B, a from A; the whole
    operator is then F + a N_w + b n_v per direction.  value =
    n_v / mean(T_degrid, T_grid) in Mvis/s, labelled extrapolated.  The
    direct sum O1 is timed beside it on spot visibilities (ns per term)."""
    import numpy as np
    from oracle import o1, o2
    from oracle import plan as P
    uvw, freq = case["uvw"], case["freq"]
    nrow = uvw.shape[0]
    alpha, sigma = info["alpha"], info["sigma"]
    pl = P.make_plan(uvw, freq, case["npix_x"], case["npix_y"], case["pixsize_x"], case["pixsize_y"], alpha, sigma)
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(nrow, size=min(nrow, sample_rows), replace=False))
    b = P.bin_visibilities(uvw[rows], freq, pl)
    S = alpha + 1
    j0 = int(np.median(b["iw"]))
    in_slice = b["idx"][(b["iw"] >= j0) & (b["iw"] <= j0 + S - alpha)]
    sub_uvw = np.ascontiguousarray(uvw[rows])
    sub_vis = case["vis"][rows].astype(np.complex128)
    masks = {}
    for name, sel in (("A", in_slice), ("B", in_slice[::8])):
        m = np.zeros((len(rows), len(freq)), np.uint8)
        m.reshape(-1)[sel] = 1
        masks[name] = (m, len(sel))
    t0 = time.perf_counter()
    o2.correction(pl)
    t_corr = time.perf_counter() - t0
    t = {}
    for d in ("degrid", "grid"):
        for name, (m, _) in masks.items():
            t0 = time.perf_counter()
            if d == "degrid":
                o2.degrid(sub_uvw, freq, case["dirty"], pl, mask=m)
            else:
                o2.grid(sub_uvw, freq, sub_vis, pl, mask=m)
            t[d, name] = time.perf_counter() - t0
    n_a, n_b = masks["A"][1], masks["B"][1]
    full = {}
    coef = {}
    for d in ("degrid", "grid"):
        bv = max(0.0, (t[d, "A"] - t[d, "B"]) / max(1, n_a - n_b))
        av = max(0.0, (t[d, "A"] - t_corr - bv * n_a) / S)
        full[d] = t_corr + av * pl["nw"] + bv * n_vis
        coef[d] = {"a_s_per_plane": av, "b_us_per_vis": bv * 1e6,
                   "slice_A_s": round(t[d, "A"], 3), "slice_B_s": round(t[d, "B"], 3)}
    # O1 on spot visibilities of the point-source image (ns per term)
    nsrc = int(np.count_nonzero(case["dirty"]))
    idx = rng.choice(n_vis, size=20000, replace=False)
    t0 = time.perf_counter()
    o1.forward(uvw, freq, case["dirty"], case["pixsize_x"], case["pixsize_y"], vis_idx=idx)
    o1_ns = (time.perf_counter() - t0) / (len(idx) * nsrc) * 1e9
    cores, model = _cpu_info()
    return {
        "value": n_vis / (0.5 * (full["degrid"] + full["grid"])) / 1e6,
        "unit": "Mvis/s",
        "cores": 1,                  # numpy's FFT and elementwise kernels run on one thread
        "host_threads": cores,
        "cpu_model": model,
        "kind": "oracle",
        "oracle": "O2 same plan",
        "extrapolated": True,
        "sample": (f"O2 (FP64, numpy) at the FP32 plan alpha={alpha} sigma={sigma} N={pl['nu']} N_w={pl['nw']}: "
                   f"{S} planes from plane {j0} with {n_a} visibilities (run A) and {n_b} (run B) of a "
                   f"{len(rows)}-row sample, correction timed alone ({t_corr:.1f} s); T = F + a N_w + b n_v "
                   f"extrapolated to N_w={pl['nw']}, n_v={n_vis}"),
        "degrid_s_extrapolated": round(full["degrid"], 1),
        "grid_s_extrapolated": round(full["grid"], 1),
        "model": coef,
        "o1_ns_per_term": round(o1_ns, 3),
        "o1_threads": cores,
    }


def serving(case, count, dev, checks, loads=(0.5, 0.8, 0.95), seed=4, n_configs=12):
    """Serving workload: ``count`` degrid/grid requests over ``n_configs``
    operator configurations (image sizes 512^2 to 4096^2, 1e5 to 2e7
    visibilities drawn from the wide-field array, epsilon 1e-4 to 1e-9, FP32
    for eps >= 1e-5 else FP64), each request with its own seeded data.

    * closed loop with plans built on demand (cold), then again with the
      plans resident (warm): the saturated request rate;
    * Poisson arrivals at each offered load rho times the saturated rate,
      with p50/p99 latency; every output there must equal the warm output of
      the same request bit for bit (the apply path is deterministic);
    * every warm output is checked against the direct sum on 4 sampled
      entries in the accuracy leg at the end (``checks``)."""
    import numpy as np
    import torch

    import synth
    from paper_2010_10122_amd.serve import Request, Server, summarize

    _, configs, specs = synth.serving_requests(seed=seed, count=count, n_configs=n_configs, base=case)
    coords = {}
    for c in configs:
        r0, r1 = c["rows"]
        key = (r0, r1, c["nchan"])
        if key not in coords:
            coords[key] = (torch.from_numpy(np.ascontiguousarray(case["uvw"][r0:r1])).to(dev),
                           torch.from_numpy(np.ascontiguousarray(case["freq"][:c["nchan"]])).to(dev))
    reqs = []
    for sp in specs:
        r0, r1 = sp["rows"]
        key = (r0, r1, sp["nchan"])
        uvw, freq = coords[key]
        g = torch.Generator(device=dev).manual_seed(sp["seed"])
        if sp["direction"] == "degrid":
            data = torch.randn((sp["npix"], sp["npix"]), generator=g, device=dev,
                               dtype=torch.float32 if sp["precision"] == "f32" else torch.float64)
        else:
            data = torch.randn((r1 - r0, sp["nchan"]), generator=g, device=dev,
                               dtype=torch.complex64 if sp["precision"] == "f32" else torch.complex128)
        reqs.append(Request(sp["rid"], sp["direction"], key, uvw, freq, sp["npix"], sp["pixsize"],
                            sp["epsilon"], sp["precision"], data))
    torch.cuda.synchronize()

    def digest(res):
        # exact fingerprint of each output: its words summed as int64
        out = {}
        for r in res:
            o = r.output.reshape(-1)
            o = torch.view_as_real(o) if o.is_complex() else o
            w = o.contiguous().view(torch.int64 if o.element_size() == 8 else torch.int32)
            out[r.rid] = int(w.to(torch.int64).sum())
        return out

    srv = Server(dev, n_slots=4)
    res, makespan = srv.run(reqs, realtime=False)
    cold = summarize(res, makespan)
    print(f"[bench] serving closed loop, plans built on demand: {cold}", file=sys.stderr, flush=True)
    del res
    res, makespan = srv.run(reqs, realtime=False)
    warm = summarize(res, makespan)
    print(f"[bench] serving closed loop, plans resident: {warm}", file=sys.stderr, flush=True)
    ref_digest = digest(res)
    warm_out = {r.rid: r.output for r in res}
    del res
    rate = len(reqs) / makespan
    points = []
    mismatches = 0
    for k, rho in enumerate(loads):
        arr = np.cumsum(np.random.default_rng(seed + 1 + k).exponential(1.0 / (rho * rate), len(reqs)))
        for r, t in zip(reqs, arr):
            r.arrival = float(t)
        res, makespan = srv.run(reqs, realtime=True)
        s = summarize(res, makespan)
        s["offered_load"] = rho
        s["offered_rate_per_s"] = rho * rate
        d = digest(res)
        s["outputs_equal_to_warm"] = sum(d[rid] == ref_digest[rid] for rid in d)
        mismatches += len(d) - s["outputs_equal_to_warm"]
        points.append(s)
        print(f"[bench] serving Poisson rho={rho}: {s}", file=sys.stderr, flush=True)
        del res
    stats = {str(k): v for k, v in srv.stats.items()}
    srv.close()
    out = {"requests": len(reqs), "configs": len(configs), "slots": 4, "closed_loop_cold": cold,
           "closed_loop_warm": warm, "saturated_rate_per_s": rate, "poisson": points,
           "bitwise_mismatches_vs_warm": mismatches, "server_stats": stats,
           "mix": (f"{len(configs)} configurations: image 512^2-4096^2, 1e5-2e7 vis (log-uniform), eps "
                   "1e-4/1e-5 FP32, 1e-7/1e-9 FP64; requests uniform over them, degrid/grid 50/50")}

    def check():
        import numpy as np

        from oracle import o1
        rng = np.random.default_rng(9)
        worst = 0.0
        for req in reqs:
            r0, r1, nch = req.coord_key
            o = warm_out[req.rid]
            if req.direction == "degrid":
                idx = rng.choice(req.n_vis, size=4, replace=False)
                got = o.reshape(-1)[torch.from_numpy(idx).to(o.device)].cpu().numpy()
                ref = o1.forward(case["uvw"][r0:r1], case["freq"][:nch], req.data.cpu().numpy(), req.pixsize,
                                 req.pixsize, vis_idx=idx)
            else:
                pp = rng.integers(0, req.npix, 4)
                qq = rng.integers(0, req.npix, 4)
                got = o[torch.from_numpy(pp).to(o.device), torch.from_numpy(qq).to(o.device)].cpu().numpy()
                ref = o1.adjoint(case["uvw"][r0:r1], case["freq"][:nch], req.data.cpu().numpy(), req.npix,
                                 req.npix, req.pixsize, req.pixsize, pixels=(pp, qq))
            worst = max(worst, float(np.linalg.norm(got - ref) / np.linalg.norm(ref)) / req.epsilon)
        out["oracle_check"] = {"requests_checked": len(reqs), "samples_each": 4, "max_rel_err_over_eps": worst}

    checks.append(("serving", check))
    return out


def eps_sweep(case, dev, uvw, freq, n_vis, checks):
    """Run time against requested accuracy (Sect. 6.3) on the wide-field
    workload: for each epsilon the planner's kernel choice, then one degrid
    and one grid timed after a warm-up of each.  FP32 where epsilon >= 1e-5,
    FP64 from 1e-4 to 1e-12 (the paper runs both types).  The degridding
    error against the direct sum on 1000 random visibilities is taken in the
    accuracy leg at the end (``checks``)."""
    import numpy as np
    import torch

    import paper_2010_10122_amd as wg
    idx = np.random.default_rng(71).choice(n_vis, size=1000, replace=False)
    idx_t = torch.from_numpy(idx).to(dev)
    rows, samples = [], []
    for prec, epss in (("f32", (1e-4, 3e-5, 1e-5)),
                       ("f64", (1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9, 1e-10, 1e-11, 1e-12))):
        rdt = torch.float32 if prec == "f32" else torch.float64
        cdt = torch.complex64 if prec == "f32" else torch.complex128
        dirty = torch.from_numpy(case["dirty"]).to(dev, rdt)
        vis = torch.from_numpy(case["vis"]).to(dev, cdt)
        for eps in epss:
            plan = wg.Plan(uvw, freq, case["npix_x"], case["npix_y"], case["pixsize_x"], case["pixsize_y"], eps,
                           prec)
            ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
            # outputs allocated before the timed calls
            out_v = plan.degrid(dirty, workspace=ws)
            out_i = plan.grid(vis, workspace=ws)
            t = {}
            for name in ("degrid", "grid"):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if name == "degrid":
                    plan.degrid(dirty, out=out_v, workspace=ws)
                else:
                    plan.grid(vis, out=out_i, workspace=ws)
                torch.cuda.synchronize()
                t[name] = time.perf_counter() - t0
            samples.append(out_v.reshape(-1)[idx_t].cpu().numpy())
            info = plan.info
            rows.append({"precision": prec, "epsilon": eps, "alpha": info["alpha"], "sigma": info["sigma"],
                         "nu": info["nu"], "nw": info["nw"], "degrid_ms": round(t["degrid"] * 1e3, 1),
                         "grid_ms": round(t["grid"] * 1e3, 1),
                         "mvis_s": round(n_vis / (0.5 * (t["degrid"] + t["grid"])) / 1e6, 1),
                         "whole_apply_hbm_frac": round(info["bytes_grid"] / (0.5 * (t["degrid"] + t["grid"])) /
                                                       1e9 / HBM_PEAK_GBS, 4)})
            print(f"[bench] eps sweep {prec} {eps:g}: {rows[-1]}", file=sys.stderr, flush=True)
            plan.close()
            del ws, out_v, out_i
        del dirty, vis
        torch.cuda.empty_cache()

    def check():
        import numpy as np

        from oracle import o1
        ref = o1.forward(case["uvw"], case["freq"], case["dirty"], case["pixsize_x"], case["pixsize_y"], vis_idx=idx,
                          pixels=np.nonzero(case["dirty"]))
        for r, got in zip(rows, samples):
            r["degrid_rel_err_vs_oracle"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))

    checks.append(("eps sweep", check))
    return {"workload": "wide field (as the headline), one degrid + one grid per epsilon", "rows": rows}


def paper_shape(dev, checks, steps=2):
    """The benchmark set-up of Sect. 6 (synthetic stand-in for its MeerKAT
    L-band set: 61 antennas, 824,476 rows x 2048 channels, flagged down to
    about 470 million visibilities, 4096^2 over 1.6 deg):

    * Sect. 6.1: FP32, eps = 1e-4, degrid and grid (plan build timed cold);
    * Sect. 6.2: gridding and degridding without the w term, FP64,
      eps = 1e-10, on the multi-channel set and on its flattened form (one
      channel, one row per selected visibility).

    Visibilities of the gridding legs are drawn on the device (seeded).  The
    degridding error of each leg against the direct sum on 64 random
    selected visibilities is taken in the accuracy leg (``checks``)."""
    import numpy as np
    import torch

    import paper_2010_10122_amd as wg
    import synth
    t0 = time.perf_counter()
    c = synth.meerkat_like()
    n_vis = int(c["mask"].sum())
    uvw = torch.from_numpy(c["uvw"]).to(dev)
    freq = torch.from_numpy(c["freq"]).to(dev)
    mask = torch.from_numpy(c["mask"]).to(dev)
    print(f"[bench] paper shape: {c['uvw'].shape[0]} rows x {len(c['freq'])} ch, {n_vis} selected, "
          f"generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    gen = torch.Generator(device=dev).manual_seed(61)
    out = {"workload": (f"paper shape (Sect. 6): {c['uvw'].shape[0]} rows x {len(c['freq'])} ch, "
                        f"{n_vis} selected vis, {c['npix_x']}^2 over 1.6 deg")}
    sel = np.flatnonzero(c["mask"].reshape(-1))
    pick = np.sort(np.random.default_rng(62).choice(sel, 64, replace=False))
    samples = {}

    def leg(name, uvw_, freq_, mask_, eps, prec, do_w, nv, idx):
        rdt = torch.float32 if prec == "f32" else torch.float64
        cdt = torch.complex64 if prec == "f32" else torch.complex128
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = wg.Plan(uvw_, freq_, c["npix_x"], c["npix_y"], c["pixsize_x"], c["pixsize_y"], eps, prec,
                       do_wgridding=do_w, mask=mask_)
        torch.cuda.synchronize()
        plan_s = time.perf_counter() - t0
        info = plan.info
        dirty = torch.from_numpy(c["dirty"]).to(dev, rdt)
        vis = torch.randn((plan.n_rows, plan.n_chan), dtype=cdt, device=dev, generator=gen)
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
        # outputs allocated before the timed calls (the visibilities of the
        # multichannel FP64 leg alone are 27 GB)
        out_v = plan.degrid(dirty, workspace=ws)
        out_i = plan.grid(vis, workspace=ws)
        t = {"degrid": 0.0, "grid": 0.0}
        for _ in range(steps):
            for d in ("degrid", "grid"):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if d == "degrid":
                    plan.degrid(dirty, out=out_v, workspace=ws)
                else:
                    plan.grid(vis, out=out_i, workspace=ws)
                torch.cuda.synchronize()
                t[d] += (time.perf_counter() - t0) / steps
        samples[name] = out_v.reshape(-1)[torch.from_numpy(idx).to(dev)].cpu().numpy()
        r = {"precision": prec, "epsilon": eps, "w_gridding": do_w, "n_vis": nv, "alpha": info["alpha"],
             "sigma": info["sigma"], "nu": info["nu"], "nw": info["nw"], "plan_ms": round(plan_s * 1e3, 1),
             "degrid_ms": round(t["degrid"] * 1e3, 1), "grid_ms": round(t["grid"] * 1e3, 1),
             "degrid_mvis_s": round(nv / t["degrid"] / 1e6, 1), "grid_mvis_s": round(nv / t["grid"] / 1e6, 1),
             "mvis_s": round(nv / (0.5 * (t["degrid"] + t["grid"])) / 1e6, 1),
             "degrid_over_grid": round(t["degrid"] / t["grid"], 3),
             "whole_apply_hbm_frac": round(info["bytes_grid"] / (0.5 * (t["degrid"] + t["grid"])) / 1e9 /
                                           HBM_PEAK_GBS, 4)}
        print(f"[bench] {name}: {r}", file=sys.stderr, flush=True)
        plan.close()
        del vis, ws, dirty, out_v, out_i
        torch.cuda.empty_cache()
        return r

    out["sect61_f32_eps1e-4"] = leg("sect61_f32_eps1e-4", uvw, freq, mask, 1e-4, "f32", True, n_vis, pick)
    out["sect62_f64_eps1e-10_no_w"] = leg("sect62_f64_eps1e-10_no_w", uvw, freq, mask, 1e-10, "f64", False,
                                          n_vis, pick)
    # flattened: one row per selected visibility, uvw scaled to the first
    # channel; the picked visibilities are rows searchsorted(sel, pick)
    sel_t = torch.from_numpy(sel).to(dev)
    rr = torch.div(sel_t, len(c["freq"]), rounding_mode="floor")
    ch = sel_t - rr * len(c["freq"])
    uvw_f = (uvw[rr] * (freq[ch] / freq[0])[:, None]).contiguous()
    del sel_t, rr, ch
    out["sect62_f64_eps1e-10_no_w_flat"] = leg("sect62_f64_eps1e-10_no_w_flat", uvw_f, freq[:1].contiguous(), None,
                                               1e-10, "f64", False, n_vis, np.searchsorted(sel, pick))
    del uvw_f, uvw, mask
    torch.cuda.empty_cache()

    def check():
        import numpy as np

        from oracle import o1
        nz = np.nonzero(c["dirty"])
        ref_w = o1.forward(c["uvw"], c["freq"], c["dirty"], c["pixsize_x"], c["pixsize_y"], vis_idx=pick, pixels=nz)
        ref_nw = o1.forward(c["uvw"], c["freq"], c["dirty"], c["pixsize_x"], c["pixsize_y"], do_wgridding=False,
                            vis_idx=pick, pixels=nz)
        for name, ref in (("sect61_f32_eps1e-4", ref_w), ("sect62_f64_eps1e-10_no_w", ref_nw),
                          ("sect62_f64_eps1e-10_no_w_flat", ref_nw)):
            got = samples[name]
            out[name]["degrid_rel_err_vs_oracle"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))

    checks.append(("paper shape", check))
    return out


def differentiation(dev, gd_steps=50, seed=5):
    """Differentiation workload: 1024^2 FP32 image (pixel 10 deg / 2048),
    64 antennas, 2 h, 4 channels (4,999,680 visibilities); data d = R(sky) +
    10% Gaussian noise from a 100-source sky (synthesised with an FP64 plan
    at eps 1e-10); loss 0.5 ||R x - d||^2 with R = degrid as an autograd
    Function whose backward is the gridder.  Reports the relative difference
    between the autograd gradient and central differences on 32 random
    pixels, then times ``gd_steps`` steps of gradient descent end to end."""
    import numpy as np
    import torch

    import paper_2010_10122_amd as wg
    import synth
    from paper_2010_10122_amd import autograd as ag

    case = synth.differentiation(seed=seed)
    rng = case["rng"]
    n = case["npix_x"]
    uvw = torch.from_numpy(case["uvw"]).to(dev)
    freq = torch.from_numpy(case["freq"]).to(dev)
    px = case["pixsize_x"]
    p64 = wg.Plan(uvw, freq, n, n, px, px, 1e-10, "f64")
    d_true = p64.degrid(torch.from_numpy(case["sky"]).to(dev))
    p64.close()
    noise = torch.from_numpy(synth.complex_gaussian(rng, tuple(d_true.shape))).to(dev)
    data = (d_true + case["noise_frac"] * torch.std(d_true.abs()) * noise).to(torch.complex64)
    del d_true, noise
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = wg.Plan(uvw, freq, n, n, px, px, 1e-5, "f32")
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    x = torch.from_numpy(rng.standard_normal((n, n))).to(dev, torch.float32).requires_grad_(True)

    def loss_fn(img):
        r = ag.degrid(img, plan) - data
        return 0.5 * torch.sum(r.real.double() ** 2 + r.imag.double() ** 2)

    (g,) = torch.autograd.grad(loss_fn(x), x)
    pix = rng.choice(n * n, 32, replace=False)
    fd = []
    with torch.no_grad():
        for p in pix:
            e = torch.zeros(n * n, dtype=torch.float32, device=dev)
            e[int(p)] = 16.0          # the loss is quadratic: no truncation error at any step
            e = e.view(n, n)
            fd.append(float(loss_fn(x + e) - loss_fn(x - e)) / 32.0)
    gp = g.view(-1)[torch.from_numpy(pix).to(dev)].double().cpu().numpy()
    fd_err = float(np.linalg.norm(np.array(fd) - gp) / np.linalg.norm(gp))
    lam = ag.lipschitz_estimate(plan, iters=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, losses = ag.gradient_descent(plan, data, steps=gd_steps, step_size=1.0 / lam)
    torch.cuda.synchronize()
    t_gd = time.perf_counter() - t0
    n_vis = plan.n_rows * plan.n_chan
    plan.close()
    out = {"workload": f"{n}^2 FP32 image, {n_vis} vis, eps=1e-5, loss 0.5||R x - d||^2",
           "fd_rel_err_32px": fd_err, "gd_steps": gd_steps, "gd_s": round(t_gd, 4),
           "gd_ms_per_step": round(t_gd / gd_steps * 1e3, 3),
           "loss_first": losses[0], "loss_last": losses[-1], "plan_ms": round(plan_s * 1e3, 1),
           "mvis_s": round(2 * n_vis * gd_steps / t_gd / 1e6, 2)}
    print(f"[bench] differentiation: {out}", file=sys.stderr, flush=True)
    return out


def large_workload(dev):
    """Large workload: 8192^2 image over 30 deg, 256 antennas (log-radial to
    10 km), 4 h in 1000 dumps x 8 channels = 261,120,000 visibilities, FP32 at
    eps = 1e-5 (about 12,500 w-planes).  One degrid and one grid after a
    warm-up of each; Mvis/s and the whole-apply fraction of the HBM roofline
    (algorithmic bytes of the plan / time / 8 TB/s)."""
    import torch

    import paper_2010_10122_amd as wg
    import synth

    t0 = time.perf_counter()
    c = synth.large()
    print(f"[bench] large workload generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    uvw = torch.from_numpy(c["uvw"]).to(dev)
    freq = torch.from_numpy(c["freq"]).to(dev)
    dirty = torch.from_numpy(c["dirty"]).to(dev)
    vis = torch.from_numpy(c["vis"]).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = wg.Plan(uvw, freq, c["npix_x"], c["npix_y"], c["pixsize_x"], c["pixsize_y"], 1e-5, "f32")
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = plan.info
    print(f"[bench] large plan alpha={info['alpha']} sigma={info['sigma']} N={info['nu']} Nw={info['nw']} "
          f"in {plan_s:.1f} s", file=sys.stderr, flush=True)
    # one timed application per direction (each runs tens of seconds)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    out_v = torch.empty((plan.n_rows, plan.n_chan), dtype=plan.complex_dtype, device=dev)
    out_i = torch.empty((plan.npix_x, plan.npix_y), dtype=plan.real_dtype, device=dev)
    t_op = {}
    for name in ("degrid", "grid"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if name == "degrid":
            plan.degrid(dirty, out=out_v, workspace=ws)
        else:
            plan.grid(vis, out=out_i, workspace=ws)
        torch.cuda.synchronize()
        t_op[name] = time.perf_counter() - t0
        print(f"[bench] large {name}: {t_op[name]:.2f} s", file=sys.stderr, flush=True)
    t_deg, t_grid = t_op["degrid"], t_op["grid"]
    n_vis = info["n_vis"]
    plan.close()
    out = {"workload": f"large: 8192^2 image, 30 deg, {c['uvw'].shape[0]} rows x {len(c['freq'])} ch = {n_vis} vis, "
                       "eps=1e-5 FP32",
           "alpha": info["alpha"], "sigma": info["sigma"], "nu": info["nu"], "nw": info["nw"],
           "plan_ms": round(plan_s * 1e3, 1), "degrid_ms": round(t_deg * 1e3, 1), "grid_ms": round(t_grid * 1e3, 1),
           "degrid_mvis_s": round(n_vis / t_deg / 1e6, 2), "grid_mvis_s": round(n_vis / t_grid / 1e6, 2),
           "degrid_hbm_frac": round(info["bytes_degrid"] / t_deg / 1e9 / HBM_PEAK_GBS, 4),
           "grid_hbm_frac": round(info["bytes_grid"] / t_grid / 1e9 / HBM_PEAK_GBS, 4)}
    print(f"[bench] large: {out}", file=sys.stderr, flush=True)
    return out


def time_operator(plan, dirty, vis, steps, warmup, prof=None):
    import torch
    for _ in range(warmup):
        plan.degrid(dirty)
        plan.grid(vis)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_deg = t_grid = 0.0
    out_v = torch.empty((plan.n_rows, plan.n_chan), dtype=plan.complex_dtype, device=dirty.device)
    out_i = torch.empty((plan.npix_x, plan.npix_y), dtype=plan.real_dtype, device=dirty.device)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dirty.device)
    if prof is not None:
        prof.reset()
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for _ in range(steps):
        ev[0].record()
        plan.degrid(dirty, out=out_v, workspace=ws)
        ev[1].record()
        plan.grid(vis, out=out_i, workspace=ws)
        ev[2].record()
        torch.cuda.synchronize()
        t_deg += ev[0].elapsed_time(ev[1]) / 1e3
        t_grid += ev[1].elapsed_time(ev[2]) / 1e3
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    return t_deg / steps, t_grid / steps, wall, out_v


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--dumps", type=int, default=2880, help="time dumps (2880 = the full 8 h workload)")
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiation workload")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the large workload (8192^2, 261M visibilities; about two minutes)")
    ap.add_argument("--no-eps-sweep", action="store_true", help="skip the run time against epsilon sweep")
    ap.add_argument("--no-paper-shape", action="store_true", help="skip the Sect. 6 benchmark shape")
    ap.add_argument("--serve-requests", type=int, default=60,
                    help="requests of the serving workload, per load point (0 = skip)")
    ap.add_argument("--quick", action="store_true",
                    help="the FP32 headline only (no FP64, differentiation, serving, sweeps, large or CPU legs)")
    args = ap.parse_args()
    if args.quick:
        args.no_fp64 = args.no_diff = args.no_large = args.no_eps_sweep = args.no_paper_shape = True
        args.no_cpu_baseline = True
        args.serve_requests = 0
    if args.gpus != 1:
        print(f"bench.py: the operator runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2010_10122_amd as wg
    import synth

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    case = synth.wide_field(n_dumps=args.dumps)
    n_vis = case["uvw"].shape[0] * len(case["freq"])
    print(f"[bench] workload {case['name']}: {n_vis} visibilities, generated in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    uvw = torch.from_numpy(case["uvw"]).to(dev)
    freq = torch.from_numpy(case["freq"]).to(dev)
    # a plain streaming kernel of known size (512 MiB read + 512 MiB write),
    # run once outside the timed region: it calibrates the HBM byte counters
    # of a profiler run of this script
    calib = torch.ones(128 * 2 ** 20, dtype=torch.float32, device=dev)
    calib_out = torch.mul(calib, 2.0)
    del calib, calib_out
    res = {}
    prof = wg.Profiler()
    legs = [("f32", "f32", 1e-5, args.steps)]
    if not args.no_fp64:
        legs += [("f64", "f64", 1e-5, args.fp64_steps), ("f64_1e-10", "f64", 1e-10, 1)]
    for key, prec, eps, steps in legs:
        rdt = torch.float32 if prec == "f32" else torch.float64
        cdt = torch.complex64 if prec == "f32" else torch.complex128
        dirty = torch.from_numpy(case["dirty"]).to(dev, rdt)
        vis = torch.from_numpy(case["vis"]).to(dev, cdt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = wg.Plan(uvw, freq, case["npix_x"], case["npix_y"], case["pixsize_x"], case["pixsize_y"], eps, prec)
        torch.cuda.synchronize()
        plan_s = time.perf_counter() - t0
        info = plan.info
        print(f"[bench] {prec} plan alpha={info['alpha']} sigma={info['sigma']} N={info['nu']} Nw={info['nw']} "
              f"P={info['planes_per_batch']} in {plan_s:.2f} s", file=sys.stderr, flush=True)
        # headline: the timed steps run without instrumentation; the
        # per-kernel breakdown comes from the same number of steps run
        # again with the event profiler attached
        t_deg, t_grid, wall, out_v = time_operator(plan, dirty, vis, steps, args.warmup)
        with prof:
            t_deg_i, t_grid_i, _, _ = time_operator(plan, dirty, vis, steps, 0, prof)
        kern = prof.read()
        print(f"[bench] {key}: degrid {t_deg * 1e3:.1f} ms, grid {t_grid * 1e3:.1f} ms", file=sys.stderr, flush=True)
        # keep a sample of this very output for the accuracy check of the
        # CPU-baseline leg (degrid of 2000 random visibilities)
        idx = np.random.default_rng(7).choice(n_vis, size=2000, replace=False)
        sample = out_v.reshape(-1)[torch.from_numpy(idx).to(dev)].cpu().numpy()
        res[key] = dict(info=info, t_deg=t_deg, t_grid=t_grid, wall=wall, steps=steps, plan_s=plan_s,
                        kernels=kern, sample_idx=idx, sample=sample, t_instr=t_deg_i + t_grid_i)
        plan.close()
        del dirty, vis
        torch.cuda.empty_cache()

    r = res["f32"]
    t_op = 0.5 * (r["t_deg"] + r["t_grid"])
    value = n_vis / t_op / 1e6
    # dominant kernel: largest total time in the timed region
    kern = r["kernels"]
    dom = max((k for k in kern if kern[k][1] > 0 and k not in ("image", "vis")), key=lambda k: kern[k][0])
    tot_ms, nl = kern[dom]
    avg_s = tot_ms / nl / 1e3
    info = r["info"]
    planes_per_launch = info["nw"] / math.ceil(info["nw"] / info["planes_per_batch"])
    bytes_launch = kernel_bytes(info, dom, planes_per_launch, "f32")
    achieved = bytes_launch / avg_s / 1e9
    traffic = profiled_traffic(dom) if args.dumps == 2880 else None
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "avg_launch_ms": round(avg_s * 1e3, 4), "bytes_per_launch": bytes_launch, "launches": nl}
    per_kernel = {k: {"total_ms": round(v[0], 3), "launches": v[1],
                      "avg_ms": round(v[0] / v[1], 4) if v[1] else None,
                      "gbs": (round(kernel_bytes(info, k, planes_per_launch, "f32") / (v[0] / v[1] / 1e3) / 1e9, 1)
                              if v[1] and k not in ("image", "vis") else None)}
                  for k, v in kern.items()}
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mvis/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round((r["t_deg"] + r["t_grid"]) * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"wide field: {case['npix_x']}^2 image, 10 deg, {case['uvw'].shape[0]} rows x "
                         f"{len(case['freq'])} ch = {n_vis} vis, eps=1e-5 FP32"),
            "npix": case["npix_x"], "n_vis": n_vis, "epsilon": 1e-5,
            "alpha": info["alpha"], "sigma": info["sigma"], "nu": info["nu"], "nw": info["nw"],
            "planes_per_batch": info["planes_per_batch"],
        },
        "grid_mvis_s": round(n_vis / r["t_grid"] / 1e6, 2),
        "degrid_mvis_s": round(n_vis / r["t_deg"] / 1e6, 2),
        "plan_ms": round(r["plan_s"] * 1e3, 1),
        "whole_apply_hbm_frac": round(info["bytes_grid"] / t_op / 1e9 / HBM_PEAK_GBS, 4),
        "ms_per_step_instrumented": round(r["t_instr"] * 1e3, 3),
        "kernels": per_kernel,
        "roofline": roof,
    }
    for key, name in (("f64", "fp64"), ("f64_1e-10", "fp64_eps1e-10")):
        if key not in res:
            continue
        f = res[key]
        out[name] = {"epsilon": 1e-5 if key == "f64" else 1e-10,
                     "grid_mvis_s": round(n_vis / f["t_grid"] / 1e6, 2),
                     "degrid_mvis_s": round(n_vis / f["t_deg"] / 1e6, 2),
                     "value": round(n_vis / (0.5 * (f["t_deg"] + f["t_grid"])) / 1e6, 2),
                     "alpha": f["info"]["alpha"], "sigma": f["info"]["sigma"], "nu": f["info"]["nu"],
                     "nw": f["info"]["nw"], "plan_ms": round(f["plan_s"] * 1e3, 1), "steps": f["steps"]}
    if "fp64" in out:
        out["fp32_over_fp64"] = round(value / out["fp64"]["value"], 3)
    checks = []
    if not args.no_diff:
        out["differentiation"] = differentiation(dev)
    if args.serve_requests > 0:
        out["serving"] = serving(case, args.serve_requests, dev, checks)
        p08 = next(p for p in out["serving"]["poisson"] if p["offered_load"] == 0.8)
        out["serve_p50_ms"] = p08["p50_ms"]
        out["serve_p99_ms"] = p08["p99_ms"]
    if not args.no_eps_sweep:
        out["eps_sweep"] = eps_sweep(case, dev, uvw, freq, n_vis, checks)
    if not args.no_paper_shape:
        out["paper_shape"] = paper_shape(dev, checks)
    if not args.no_large:
        out["large"] = large_workload(dev)
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(case, r["info"], n_vis)
        # accuracy of the timed outputs against the oracle (same leg)
        from oracle import o1
        for prec, rr in res.items():
            ref = o1.forward(case["uvw"], case["freq"], case["dirty"], case["pixsize_x"], case["pixsize_y"],
                             vis_idx=rr["sample_idx"], pixels=np.nonzero(case["dirty"]))
            err = float(np.linalg.norm(rr["sample"] - ref) / np.linalg.norm(ref))
            (out if prec == "f32" else out["fp64" if prec == "f64" else "fp64_eps1e-10"])[
                "degrid_rel_err_vs_oracle"] = err
        # the other legs' outputs against the oracle
        for name, check in checks:
            t1 = time.perf_counter()
            check()
            print(f"[bench] oracle check of {name} in {time.perf_counter() - t1:.1f} s", file=sys.stderr,
                  flush=True)
        print(f"[bench] cpu baseline and oracle checks in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    prof.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
