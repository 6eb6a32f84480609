"""Continuous-batching request loop for AIM solves on one GPU.

Requests (a contour, a frequency, 1..16 plane-wave incidences, a precision)
arrive over time.  The scheduler admits them first-come first-served into a
fixed number of slots whenever a slot is free and the request's device
footprint fits the remaining HBM budget; an admitted request runs on its own
HIP stream from its own worker thread (set-up, right-hand sides, GMRES solve
of all its incidences as one batch, monostatic RCS, release), so requests
that arrive while others are on the GPU overlap with them on the device.
Grid-kernel spectra are shared through the library's resident cache, so
requests with the same grid and k*eps do not recompute them.

Each solve depends only on its own request: a result is the same alone and
in any mix (tests check this bitwise).  The executor is injectable so the
admission logic can be exercised without a device.
"""
from __future__ import annotations

import math
import queue
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class ServeResult:
    rid: int
    arrival: float
    admit: float = math.nan
    finish: float = math.nan
    status: str = "pending"
    n: int = 0
    m: int = 0
    nrhs: int = 0
    precision: int = 0
    iterations: int = 0
    matvecs: int = 0
    resid: float = math.nan
    sigma: np.ndarray | None = None
    x: np.ndarray | None = None
    footprint: int = 0

    @property
    def latency(self):
        return self.finish - self.arrival


def gpu_footprint(req, restart):
    from . import aim
    return aim.aim_footprint_bytes(req.xy, req.k, req.eta, req.basis, req.m, req.eps,
                                   precision=aim.AIM_MIXED if req.precision else aim.AIM_FP64,
                                   max_rhs=len(req.phis), restart=restart)


class GpuExecutor:
    """Runs one request on the calling thread's own stream."""

    def __init__(self, restart=1000, maxit=4000, keep_solution=False):
        self.restart = restart
        self.maxit = maxit
        self.keep = keep_solution
        self._tls = threading.local()

    def footprint(self, req):
        return gpu_footprint(req, self.restart)

    def _stream(self):
        import torch
        s = getattr(self._tls, "stream", None)
        if s is None:
            s = torch.cuda.Stream()          # default priority
            self._tls.stream = s
        return s

    def __call__(self, req, res: ServeResult):
        import torch
        from . import aim
        stream = self._stream()
        with torch.cuda.stream(stream):
            prec = aim.AIM_MIXED if req.precision else aim.AIM_FP64
            ctx = aim.Context(req.xy, req.k, req.eta, req.basis, req.m, req.eps, precision=prec,
                              max_rhs=len(req.phis), stream=stream)
            try:
                b = ctx.rhs_planewave(np.asarray(req.phis, dtype=float))
                x, info = ctx.solve("TM", b, tol=req.tol, maxit=self.maxit, restart=self.restart,
                                    precision=prec)
                res.sigma = ctx.rcs(x, req.phis)
                res.iterations = max(d["iterations"] for d in info)
                res.matvecs = max(d["matvecs"] for d in info)
                res.resid = max(d["resid_true"] for d in info)
                res.status = "ok" if all(d["converged"] for d in info) else "noconv"
                if self.keep:
                    res.x = x.cpu().numpy()
            finally:
                stream.synchronize()
                ctx.close()
        res.n, res.m, res.nrhs, res.precision = len(req.xy), req.m, len(req.phis), req.precision


class Server:
    def __init__(self, executor, hbm_budget: int, slots: int = 4):
        self.exe = executor
        self.budget = int(hbm_budget)
        self.slots = int(slots)
        self.max_reserved = 0
        self.max_active = 0

    def run(self, requests, realtime: bool = True):
        reqs = sorted(requests, key=lambda r: r.arrival)
        results = {r.rid: ServeResult(r.rid, r.arrival) for r in reqs}
        work = queue.Queue()
        done = queue.Queue()

        def worker():
            while True:
                item = work.get()
                if item is None:
                    return
                req, res = item
                try:
                    self.exe(req, res)
                except Exception as e:               # failure is recorded, the loop goes on
                    res.status = f"error: {e}"
                res.finish = time.perf_counter() - t0
                done.put(req.rid)

        threads = [threading.Thread(target=worker, daemon=True) for _ in range(self.slots)]
        for t in threads:
            t.start()
        pending = deque()
        fp = {}
        active = 0
        reserved = 0
        nxt = 0
        finished = 0
        t0 = time.perf_counter()
        offset = 0.0 if realtime else None
        while finished < len(reqs):
            now = time.perf_counter() - t0
            if not realtime and nxt < len(reqs) and not pending and active == 0:
                offset = reqs[nxt].arrival - now        # skip idle gaps in simulated time
            eff = now + (offset or 0.0)
            while nxt < len(reqs) and reqs[nxt].arrival <= eff:
                r = reqs[nxt]
                fp[r.rid] = self.exe.footprint(r)
                results[r.rid].footprint = fp[r.rid]
                if fp[r.rid] > self.budget:
                    results[r.rid].status = "rejected"
                    results[r.rid].finish = now
                    finished += 1
                else:
                    pending.append(r)
                nxt += 1
            while pending and active < self.slots and reserved + fp[pending[0].rid] <= self.budget:
                r = pending.popleft()
                reserved += fp[r.rid]
                active += 1
                self.max_reserved = max(self.max_reserved, reserved)
                self.max_active = max(self.max_active, active)
                results[r.rid].admit = time.perf_counter() - t0
                work.put((r, results[r.rid]))
            wait = 0.002
            if nxt < len(reqs) and realtime:
                wait = max(0.0, min(wait, reqs[nxt].arrival - (time.perf_counter() - t0)))
            try:
                rid = done.get(timeout=wait if wait > 0 else 1e-4)
                active -= 1
                reserved -= fp[rid]
                finished += 1
                while True:
                    rid = done.get_nowait()
                    active -= 1
                    reserved -= fp[rid]
                    finished += 1
            except queue.Empty:
                pass
        for _ in threads:
            work.put(None)
        for t in threads:
            t.join()
        self.wall = time.perf_counter() - t0
        return [results[r.rid] for r in reqs]


def summarize(results, wall):
    ok = [r for r in results if r.status == "ok"]
    lat = sorted(r.latency for r in ok)

    def pct(p):
        if not lat:
            return math.nan
        return lat[min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))]

    return {
        "requests": len(results),
        "completed": len(ok),
        "rejected": sum(r.status == "rejected" for r in results),
        "failed": sum(r.status not in ("ok", "rejected") for r in results),
        "wall_s": wall,
        "requests_per_s": len(ok) / wall if wall > 0 else math.nan,
        "solves_per_s": sum(r.nrhs for r in ok) / wall if wall > 0 else math.nan,
        "matvecs_per_s": sum(r.matvecs * r.nrhs for r in ok) / wall if wall > 0 else math.nan,
        "latency_s": {"p50": pct(50), "p99": pct(99), "max": lat[-1] if lat else math.nan},
        "max_resid": max((r.resid for r in ok), default=math.nan),
    }
