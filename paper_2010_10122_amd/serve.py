"""Serving loop: continuous batching of operator applications on one GPU.

Requests (degrid or grid, any image size, visibility count, epsilon and
precision) arrive over time.  The loop admits a waiting request as soon as a
slot (HIP stream) is free and its HBM footprint (plan if not cached, apply
workspace, output) fits the budget, so requests that arrive while others run
join the work already on the device and overlap with it.  Plans (kernel
choice, corrections, visibility index) are cached by coordinate set and
operator parameters and stay resident until the cache must make room.

Every kernel of the apply path is deterministic (no atomics, fixed
summation orders), so a request's result is bitwise the same alone and in
any mix.
"""
import collections
import dataclasses
import time

import numpy as np
import torch

from .plan import Plan


@dataclasses.dataclass
class Request:
    rid: int
    direction: str                 # "degrid" (image -> vis) or "grid" (vis -> image)
    coord_key: object              # identifies (uvw, freq) for the plan cache
    uvw: torch.Tensor              # device [n_rows, 3] float64
    freq: torch.Tensor             # device [n_chan] float64
    npix: int
    pixsize: float
    epsilon: float
    precision: str                 # "f32" / "f64"
    data: torch.Tensor             # device input (image or visibilities)
    arrival: float = 0.0           # seconds after the start of the run
    do_wgridding: bool = True

    @property
    def n_vis(self):
        return int(self.uvw.shape[0] * self.freq.shape[0])


@dataclasses.dataclass
class Result:
    rid: int
    output: torch.Tensor
    arrival: float
    admitted: float
    finished: float
    n_vis: int
    plan_key: tuple
    plan_cached: bool

    @property
    def latency(self):
        return self.finished - self.arrival


class _Job:
    __slots__ = ("req", "plan", "key", "out", "ws", "done", "admitted", "bytes", "cached")


class Server:
    def __init__(self, device=None, n_slots=4, hbm_budget=None, plan_cache_bytes=None, poll_s=50e-6):
        self.device = torch.device(device or "cuda:0")
        self.streams = [torch.cuda.Stream(self.device) for _ in range(n_slots)]   # default priority
        total = torch.cuda.get_device_properties(self.device).total_memory
        self.budget = int(hbm_budget if hbm_budget is not None else 0.6 * total)
        self.plan_cache_bytes = int(plan_cache_bytes if plan_cache_bytes is not None else 0.25 * self.budget)
        self.cache = collections.OrderedDict()      # key -> Plan (LRU order)
        self.in_use = collections.Counter()         # key -> running jobs
        self.poll_s = poll_s
        self.used = 0                               # bytes held by in-flight jobs
        self.stats = collections.Counter()

    # ---- plan cache -----------------------------------------------------------
    @staticmethod
    def plan_key(req):
        return (req.coord_key, req.npix, float(req.pixsize), float(req.epsilon), req.precision,
                bool(req.do_wgridding))

    def _cache_bytes(self):
        return sum(p.info["plan_bytes"] for p in self.cache.values())

    def _evict(self, need):
        for key in list(self.cache.keys()):
            if self._cache_bytes() + need <= self.plan_cache_bytes:
                return
            if self.in_use[key] == 0:
                self.cache.pop(key).close()
                self.stats["plan_evictions"] += 1

    def _plan(self, req, stream):
        key = self.plan_key(req)
        if key in self.cache:
            self.cache.move_to_end(key)
            return key, self.cache[key], True
        with torch.cuda.stream(stream):
            plan = Plan(req.uvw, req.freq, req.npix, req.npix, req.pixsize, req.pixsize, req.epsilon,
                        req.precision, do_wgridding=req.do_wgridding, stream=stream)
        self._evict(plan.info["plan_bytes"])
        self.cache[key] = plan
        self.stats["plans_created"] += 1
        return key, plan, False

    # ---- footprint ------------------------------------------------------------
    @staticmethod
    def _out_bytes(req, plan):
        if req.direction == "degrid":
            return plan.n_rows * plan.n_chan * (8 if req.precision == "f32" else 16)
        return plan.npix_x * plan.npix_y * (4 if req.precision == "f32" else 8)

    # ---- main loop --------------------------------------------------------------
    def run(self, requests, realtime=True):
        """Serve ``requests`` (sorted by arrival).  With realtime=True arrivals
        are honoured on the wall clock; otherwise all are present at t=0."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = collections.deque()
        free = list(range(len(self.streams)))
        running = {}
        results = []
        t0 = time.perf_counter()
        while pending or waiting or running:
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                waiting.append(pending.popleft())
            # completions
            for slot in list(running):
                job = running[slot]
                if job.done.query():
                    t = time.perf_counter() - t0
                    results.append(Result(job.req.rid, job.out, job.req.arrival if realtime else 0.0,
                                          job.admitted, t, job.req.n_vis, job.key, job.cached))
                    self.used -= job.bytes
                    self.in_use[job.key] -= 1
                    job.ws = None
                    del running[slot]
                    free.append(slot)
            # admissions: first come, first served, while a slot and memory are free
            while waiting and free:
                req = waiting[0]
                slot = free[-1]
                stream = self.streams[slot]
                key, plan, cached = self._plan(req, stream)
                need = plan.workspace_bytes + self._out_bytes(req, plan)
                if running and self.used + need > self.budget:
                    break                                 # wait for memory to free up
                waiting.popleft()
                free.pop()
                job = _Job()
                job.req, job.plan, job.key, job.cached = req, plan, key, cached
                job.bytes = need
                job.admitted = time.perf_counter() - t0
                self.used += need
                self.in_use[key] += 1
                with torch.cuda.stream(stream):
                    job.ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device=self.device)
                    req.data.record_stream(stream)
                    if req.direction == "degrid":
                        job.out = plan.degrid(req.data, workspace=job.ws, stream=stream)
                    else:
                        job.out = plan.grid(req.data, workspace=job.ws, stream=stream)
                    job.done = torch.cuda.Event()
                    job.done.record(stream)
                running[slot] = job
                self.stats["admitted"] += 1
            if not (running or waiting) and pending and realtime:
                time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 0.01)))
            elif running:
                time.sleep(self.poll_s)
        makespan = time.perf_counter() - t0
        return results, makespan

    def close(self):
        torch.cuda.synchronize(self.device)
        for p in self.cache.values():
            p.close()
        self.cache.clear()


def summarize(results, makespan):
    lat = np.array([r.latency for r in results])
    nvis = sum(r.n_vis for r in results)
    return {
        "requests": len(results),
        "p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
        "p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
        "mean_ms": float(lat.mean() * 1e3) if len(lat) else None,
        "makespan_s": makespan,
        "mvis_s": nvis / makespan / 1e6 if makespan > 0 else None,
        "plans_cached_hits": int(sum(r.plan_cached for r in results)),
    }
