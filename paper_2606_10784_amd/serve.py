"""Continuous-batching request loop for AIM solves on one GPU.

Requests (a contour, a frequency, 1..16 plane-wave incidences, a precision)
arrive over time.  The scheduler admits them first-come first-served into a
fixed number of slots whenever a slot is free and the request's device
footprint fits the remaining HBM budget; an admitted request runs on its own
HIP stream from its own worker thread (set-up, right-hand sides, GMRES solve
of all its incidences as one batch, monostatic RCS, release), so requests
that arrive while others are on the GPU overlap with them on the device.
Grid-kernel spectra are shared through the library's resident cache, so
requests with the same grid and k*eps do not recompute them.  The budget
counts each admitted request's footprint (its tables, Krylov space, spectrum
and the largest set-up temporary) and the cached spectra no request uses; the
latter are dropped when a request would not fit beside them.

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


def describe(res: ServeResult, req):
    """Sizes of the request, recorded at arrival."""
    res.n, res.m, res.nrhs, res.precision = len(req.xy), req.m, len(req.phis), req.precision


def log_line(res: ServeResult):
    """One JSON line per finished request: times in seconds from the start
    of the run, sizes, precision and solver counts."""
    import json
    f = lambda v: None if (isinstance(v, float) and math.isnan(v)) else v
    return json.dumps({"rid": res.rid, "arrival": f(res.arrival), "admit": f(res.admit), "finish": f(res.finish),
                       "latency": f(res.latency), "status": res.status, "N": res.n, "m": res.m, "R": res.nrhs,
                       "precision": "mixed" if res.precision else "fp64", "iterations": res.iterations,
                       "matvecs": res.matvecs, "resid": f(res.resid)})


class RequestLog:
    """Appends log_line of each finished request to a JSONL file (thread-safe)."""

    def __init__(self, path):
        self.path = path
        self.lock = threading.Lock()
        self.n = 0
        if path:
            open(path, "w").close()

    def write(self, res: ServeResult):
        if not self.path:
            return
        with self.lock, open(self.path, "a") as fh:
            fh.write(log_line(res) + "\n")
            self.n += 1


def gpu_footprint(req, restart):
    from . import aim
    return aim.aim_footprint_bytes(req.xy, req.k, req.eta, req.basis, req.m, req.eps,
                                   precision=aim.AIM_MIXED if req.precision else aim.AIM_FP64,
                                   max_rhs=len(req.phis), restart=restart)


class GpuCache:
    """The library's spectrum cache as seen by admission: the spectra no
    context uses stay resident outside every footprint, so a server counts
    them against its budget and drops them when they stand in the way."""

    def cache_idle_bytes(self):
        from . import aim
        return aim.aim_cache_idle_bytes()

    def cache_clear(self):
        from . import aim
        aim.aim_cache_clear()


def admit_fits(exe, reserved, need, budget):
    """A request of footprint `need` fits beside `reserved` bytes if the two
    fit the budget once the idle cached spectra (if the executor has a
    cache) are dropped; they are dropped only then."""
    if reserved + need > budget:
        return False
    idle = getattr(exe, "cache_idle_bytes", None)
    if idle is not None and reserved + need + idle() > budget:
        exe.cache_clear()
    return True


class GpuExecutor(GpuCache):
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
                              max_rhs=len(req.phis), stream=stream, max_restart=self.restart)
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
    def __init__(self, executor, hbm_budget: int, slots: int = 4, log_path=None):
        self.exe = executor
        self.budget = int(hbm_budget)
        self.slots = int(slots)
        self.max_reserved = 0
        self.max_active = 0
        self.log = RequestLog(log_path)

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
                self.log.write(res)
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
                describe(results[r.rid], r)
                if fp[r.rid] > self.budget:
                    results[r.rid].status = "rejected"
                    results[r.rid].finish = now
                    self.log.write(results[r.rid])
                    finished += 1
                else:
                    pending.append(r)
                nxt += 1
            while pending and active < self.slots and admit_fits(self.exe, reserved, fp[pending[0].rid], self.budget):
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


class GpuStepEngine(GpuCache):
    """Step-wise requests for StepServer: set-up (context, right-hand sides,
    aim solver with its caller-owned Krylov workspace) on the request's own
    stream, one Arnoldi step per round for every running solver, retirement
    (monostatic RCS, release).  group=True steps all running solvers in one
    aim_solver_step call, which runs the column passes of requests that share
    a grid-kernel spectrum (same grid, k eps and precision) as one launch;
    group=False steps them one call each (no shared launches)."""

    def __init__(self, restart=1000, maxit=4000, keep_solution=False, group=True):
        self.restart = restart
        self.maxit = maxit
        self.keep = keep_solution
        self.group = group

    def footprint(self, req):
        return gpu_footprint(req, self.restart)

    def prepare(self, req):
        import torch
        from . import aim
        stream = torch.cuda.Stream()            # default priority
        prec = aim.AIM_MIXED if req.precision else aim.AIM_FP64
        ctx = aim.Context(req.xy, req.k, req.eta, req.basis, req.m, req.eps, precision=prec,
                          max_rhs=len(req.phis), stream=stream, max_restart=0)
        try:
            # b and the initial guess are queued on the request's stream, the
            # one the library's work runs on
            with torch.cuda.stream(stream):
                b = ctx.rhs_planewave(np.asarray(req.phis, dtype=float))
                solver = aim.Solver(ctx, "TM", b, tol=req.tol, maxit=self.maxit, restart=self.restart,
                                    precision=prec)
        except Exception:
            stream.synchronize()
            ctx.close()
            raise
        return {"ctx": ctx, "stream": stream, "solver": solver}

    def step(self, jobs):
        from . import aim
        if self.group:
            aim.aim_solver_step([j["solver"] for j in jobs])
        else:
            for j in jobs:
                aim.aim_solver_step([j["solver"]])

    def done(self, job):
        from . import aim
        return job["solver"].poll()[0] != aim.AIM_PENDING

    def finish(self, req, job, res: ServeResult):
        from . import aim
        import torch
        ctx, solver = job["ctx"], job["solver"]
        try:
            st, info = solver.poll()
            solver.end()                         # the stream has drained
            if st not in (aim.AIM_OK, aim.AIM_E_NOCONV):
                raise aim.AimError(st, "solver")
            with torch.cuda.stream(job["stream"]):
                res.sigma = ctx.rcs(solver.x, req.phis)
            res.iterations = max(d["iterations"] for d in info)
            res.matvecs = max(d["matvecs"] for d in info)
            res.resid = max(d["resid_true"] for d in info)
            res.status = "ok" if st == aim.AIM_OK else "noconv"
            if self.keep:
                res.x = solver.x.cpu().numpy()
        finally:
            job["stream"].synchronize()
            ctx.close()
        res.n, res.m, res.nrhs, res.precision = len(req.xy), req.m, len(req.phis), req.precision

    def discard(self, job):
        job["solver"].end()
        job["stream"].synchronize()
        job["ctx"].close()


class StepServer:
    """Iteration-level continuous batching on one host thread.  Requests are
    admitted first-come first-served while a slot is free and their footprint
    fits the HBM budget; a small pool of set-up threads prepares each admitted
    request; every round gives each prepared, unfinished request one Arnoldi
    step, then retires the finished ones, so a request that arrives while
    others run starts stepping with them at the next round."""

    def __init__(self, engine, hbm_budget: int, slots: int = 8, setup_workers: int = 2, log_path=None):
        self.eng = engine
        self.budget = int(hbm_budget)
        self.slots = int(slots)
        self.setup_workers = int(setup_workers)
        self.max_reserved = 0
        self.max_active = 0
        self.rounds = 0
        self.log = RequestLog(log_path)

    def run(self, requests, realtime: bool = True):
        from concurrent.futures import ThreadPoolExecutor
        reqs = sorted(requests, key=lambda r: r.arrival)
        byid = {r.rid: r for r in reqs}
        results = {r.rid: ServeResult(r.rid, r.arrival) for r in reqs}
        pool = ThreadPoolExecutor(max_workers=self.setup_workers)
        pending = deque()
        setting_up = {}                      # rid -> future
        running = {}                         # rid -> job
        fp = {}
        reserved = 0
        nxt = 0
        finished = 0
        t0 = time.perf_counter()
        offset = 0.0 if realtime else None

        def release(rid, status=None):
            nonlocal reserved, finished
            reserved -= fp[rid]
            finished += 1
            if status is not None:
                results[rid].status = status
            results[rid].finish = time.perf_counter() - t0
            self.log.write(results[rid])

        try:
            while finished < len(reqs):
                now = time.perf_counter() - t0
                idle = not pending and not setting_up and not running
                if not realtime and nxt < len(reqs) and idle:
                    offset = reqs[nxt].arrival - now     # skip idle gaps in simulated time
                eff = now + (offset or 0.0)
                while nxt < len(reqs) and reqs[nxt].arrival <= eff:
                    r = reqs[nxt]
                    fp[r.rid] = self.eng.footprint(r)
                    results[r.rid].footprint = fp[r.rid]
                    describe(results[r.rid], r)
                    if fp[r.rid] > self.budget:
                        results[r.rid].status = "rejected"
                        results[r.rid].finish = now
                        self.log.write(results[r.rid])
                        finished += 1
                    else:
                        pending.append(r)
                    nxt += 1
                while pending and len(setting_up) + len(running) < self.slots and \
                        admit_fits(self.eng, reserved, fp[pending[0].rid], self.budget):
                    r = pending.popleft()
                    reserved += fp[r.rid]
                    results[r.rid].admit = time.perf_counter() - t0
                    setting_up[r.rid] = pool.submit(self.eng.prepare, r)
                    self.max_reserved = max(self.max_reserved, reserved)
                    self.max_active = max(self.max_active, len(setting_up) + len(running))
                for rid in [rid for rid, f in setting_up.items() if f.done()]:
                    f = setting_up.pop(rid)
                    try:
                        running[rid] = f.result()
                    except Exception as e:               # failure is recorded, the loop goes on
                        release(rid, f"error: {e}")
                if running:
                    rids = list(running)
                    self.eng.step([running[rid] for rid in rids])
                    self.rounds += 1
                    for rid in rids:
                        if self.eng.done(running[rid]):
                            job = running.pop(rid)
                            try:
                                self.eng.finish(byid[rid], job, results[rid])
                            except Exception as e:
                                results[rid].status = f"error: {e}"
                            release(rid)
                else:
                    wait = 0.001
                    if nxt < len(reqs) and realtime:
                        wait = max(0.0, min(wait, reqs[nxt].arrival - (time.perf_counter() - t0)))
                    time.sleep(wait)
        finally:
            for f in setting_up.values():
                try:
                    self.eng.discard(f.result())
                except Exception:
                    pass
            for job in running.values():
                self.eng.discard(job)
            pool.shutdown(wait=True)
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
