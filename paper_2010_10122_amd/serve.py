"""Serving loop: continuous batching of operator applications on one GPU.

Requests (degrid or grid, any image size, visibility count, epsilon and
precision) arrive over time.  A waiting request is admitted as soon as its
plan is resident, a slot (HIP stream) is free and its apply footprint
(workspace and output) fits the HBM budget, so requests that arrive while
others run join the work already on the device and overlap with it.

Plans (kernel choice, corrections, visibility index) are cached by
coordinate set and operator parameters.  A missing plan is built off the
admission path, on a planner thread with a stream of its own: the thread
first sizes it (``wg_plan_estimate``), the loop reserves the build's peak
footprint in the budget (evicting unused cached plans if needed) and only
then lets the thread build it.  Plan memory comes from PyTorch's caching
allocator, so building and evicting plans does not synchronise the device.

Every kernel of the apply path is deterministic (no atomics, fixed
summation orders), so a request's result is bitwise the same alone and in
any mix.
"""
import collections
import concurrent.futures
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


class _Build:
    """A plan on its way into the cache: sizing, then (once reserved) building."""
    __slots__ = ("req", "future", "peak", "plan_bytes", "state")


class Server:
    """Continuous-batching server of w-gridding operator applications.

    n_slots: concurrent apply streams; hbm_budget: bytes for resident plans,
    builds in progress and in-flight applications together (default 60 % of
    the device); plan_cache_bytes: soft cap of the resident plans."""

    def __init__(self, device=None, n_slots=4, hbm_budget=None, plan_cache_bytes=None, poll_s=50e-6):
        self.device = torch.device(device or "cuda:0")
        self.streams = [torch.cuda.Stream(self.device) for _ in range(n_slots)]   # default priority
        self.plan_stream = torch.cuda.Stream(self.device)
        self.planner = concurrent.futures.ThreadPoolExecutor(max_workers=1, thread_name_prefix="wg-planner")
        total = torch.cuda.get_device_properties(self.device).total_memory
        self.budget = int(hbm_budget if hbm_budget is not None else 0.6 * total)
        self.plan_cache_bytes = int(plan_cache_bytes if plan_cache_bytes is not None else 0.5 * self.budget)
        self.cache = collections.OrderedDict()      # key -> Plan (LRU order)
        self.in_use = collections.Counter()         # key -> admitted jobs not yet finished
        self.poll_s = poll_s
        self.jobs_bytes = 0                         # workspace + output of in-flight jobs
        self.reserved = 0                           # peak footprint of builds in progress
        self.stats = collections.Counter()

    # ---- plan cache -----------------------------------------------------------
    @staticmethod
    def plan_key(req):
        return (req.coord_key, req.npix, float(req.pixsize), float(req.epsilon), req.precision,
                bool(req.do_wgridding))

    def _cache_bytes(self):
        return sum(p.info["plan_bytes"] for p in self.cache.values())

    def _avail(self):
        return self.budget - self.jobs_bytes - self.reserved - self._cache_bytes()

    def _evict_for(self, need, keep=()):
        """Destroy least recently used plans with no job in flight until
        ``need`` bytes are available (or nothing more can go)."""
        for key in list(self.cache.keys()):
            if self._avail() >= need:
                return True
            if self.in_use[key] == 0 and key not in keep:
                self.cache.pop(key).close()          # its jobs are done: no device work uses it
                self.stats["plan_evictions"] += 1
        return self._avail() >= need

    def _trim_cache(self, keep=()):
        for key in list(self.cache.keys()):
            if self._cache_bytes() <= self.plan_cache_bytes:
                return
            if self.in_use[key] == 0 and key not in keep:
                self.cache.pop(key).close()
                self.stats["plan_evictions"] += 1

    # planner thread: both steps run on the planner stream, which first waits
    # for the work that produced the request's coordinates
    def _size_plan(self, req, ready):
        with torch.cuda.device(self.device):
            self.plan_stream.wait_event(ready)
            return Plan.estimate(req.uvw, req.freq, req.npix, req.npix, req.pixsize, req.pixsize, req.epsilon,
                                 req.precision, do_wgridding=req.do_wgridding, stream=self.plan_stream)

    def _build_plan(self, req, ready):
        with torch.cuda.device(self.device):
            self.plan_stream.wait_event(ready)
            return Plan(req.uvw, req.freq, req.npix, req.npix, req.pixsize, req.pixsize, req.epsilon,
                        req.precision, do_wgridding=req.do_wgridding, stream=self.plan_stream)

    # ---- footprint ------------------------------------------------------------
    @staticmethod
    def _out_bytes(req, plan):
        if req.direction == "degrid":
            return plan.n_rows * plan.n_chan * (8 if req.precision == "f32" else 16)
        return plan.npix_x * plan.npix_y * (4 if req.precision == "f32" else 8)

    # ---- main loop --------------------------------------------------------------
    def run(self, requests, realtime=True):
        """Serve ``requests`` (sorted by arrival).  With realtime=True arrivals
        are honoured on the wall clock; otherwise all are present at t=0.
        The requests' tensors must have been produced on the stream that is
        current when ``run`` is called (or be complete)."""
        ready = torch.cuda.Event()
        ready.record(torch.cuda.current_stream(self.device))
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = collections.deque()
        free = list(range(len(self.streams)))
        running = {}
        builds = {}                                   # key -> _Build
        results = []
        cached_on_arrival = {}                        # rid -> plan resident when the request arrived
        t0 = time.perf_counter()
        while pending or waiting or running or builds:
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                req = pending.popleft()
                cached_on_arrival[req.rid] = self.plan_key(req) in self.cache
                waiting.append(req)
            progressed = False
            # completions
            for slot in list(running):
                job = running[slot]
                if job.done.query():
                    t = time.perf_counter() - t0
                    results.append(Result(job.req.rid, job.out, job.req.arrival if realtime else 0.0,
                                          job.admitted, t, job.req.n_vis, job.key, job.cached))
                    self.jobs_bytes -= job.bytes
                    self.in_use[job.key] -= 1
                    job.ws = None
                    del running[slot]
                    free.append(slot)
                    progressed = True
            # plan sizing / building
            for key, b in list(builds.items()):
                if not b.future.done():
                    continue
                progressed = True
                if b.state == "sizing":
                    est = b.future.result()
                    b.peak, b.plan_bytes, b.state, b.future = est["peak_bytes"], est["plan_bytes"], "sized", None
                else:                                 # built
                    plan = b.future.result()
                    self.reserved -= b.peak
                    self.cache[key] = plan
                    self.stats["plans_created"] += 1
                    del builds[key]
            for key, b in builds.items():
                if b.state != "sized":
                    continue
                busy = running or any(o.state == "building" for o in builds.values())
                if self._avail() < b.peak and not self._evict_for(b.peak, keep=self._wanted(waiting)) and busy:
                    continue                          # wait for memory
                self.reserved += b.peak
                b.state = "building"
                b.future = self.planner.submit(self._build_plan, b.req, ready)
            # admissions: first come, first served among requests whose plan is resident
            for req in list(waiting):
                if not free:
                    break
                key = self.plan_key(req)
                if key not in self.cache:
                    if key not in builds:
                        b = _Build()
                        b.req, b.state, b.peak, b.plan_bytes = req, "sizing", 0, 0
                        b.future = self.planner.submit(self._size_plan, req, ready)
                        builds[key] = b
                    continue
                plan = self.cache[key]
                self.cache.move_to_end(key)
                need = plan.workspace_bytes + self._out_bytes(req, plan)
                if self._avail() < need and not self._evict_for(need, keep={key} | self._wanted(waiting)) \
                        and running:
                    break                             # wait for memory to free up
                waiting.remove(req)
                slot = free.pop()
                stream = self.streams[slot]
                job = _Job()
                job.req, job.plan, job.key = req, plan, key
                job.cached = cached_on_arrival[req.rid]
                job.bytes = need
                job.admitted = time.perf_counter() - t0
                self.jobs_bytes += need
                self.in_use[key] += 1
                stream.wait_event(ready)             # inputs produced on the submitter's stream
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
                progressed = True
            self._trim_cache(keep={self.plan_key(r) for r in waiting} | set(builds))
            if progressed:
                continue
            if not (running or waiting or builds) and pending and realtime:
                time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 0.01)))
            else:
                time.sleep(self.poll_s)
        makespan = time.perf_counter() - t0
        return results, makespan

    def _wanted(self, waiting):
        return {self.plan_key(r) for r in waiting}

    def close(self):
        torch.cuda.synchronize(self.device)
        self.planner.shutdown(wait=True)
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
