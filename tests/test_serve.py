"""Continuous-batching server: admission logic on the CPU with a stand-in
executor (never a product path), and on the GPU that each request's result
is identical alone and inside a concurrent mix."""
import threading
import time

import numpy as np
import pytest

from paper_2606_10784_amd import serve
from paper_2606_10784_amd import workloads as wl


class FakeExecutor:
    """Sleeps for a request-dependent time and tracks concurrency."""

    def __init__(self, fps, durations):
        self.fps = fps
        self.dur = durations
        self.lock = threading.Lock()
        self.running = 0
        self.peak = 0
        self.log = []

    def footprint(self, req):
        return self.fps[req.rid]

    def __call__(self, req, res):
        with self.lock:
            self.running += 1
            self.peak = max(self.peak, self.running)
            self.log.append(("start", req.rid, time.perf_counter()))
        time.sleep(self.dur[req.rid])
        with self.lock:
            self.running -= 1
        res.status = "ok"
        res.nrhs = len(req.phis)
        res.matvecs = 10


def _reqs(arrivals):
    return [wl.ServeRequest(i, a, np.zeros((8, 2)), 1.0, 1.0, 16, 0.1, np.zeros(2), 0)
            for i, a in enumerate(arrivals)]


class CachedExecutor(FakeExecutor):
    """A stand-in with a spectrum cache: finished requests leave `idle` bytes
    of cached spectra until the server clears them."""

    def __init__(self, fps, durations, idle_per_request):
        super().__init__(fps, durations)
        self.idle = 0
        self.per = idle_per_request
        self.clears = 0

    def __call__(self, req, res):
        super().__call__(req, res)
        with self.lock:
            self.idle += self.per

    def cache_idle_bytes(self):
        with self.lock:
            return self.idle

    def cache_clear(self):
        with self.lock:
            self.idle = 0
            self.clears += 1


@pytest.mark.parametrize("stepwise", [False, True])
def test_admission_counts_idle_cached_spectra(stepwise):
    """Idle cached spectra count against the budget: a request that fits
    beside the reserved footprints but not beside the idle cache gets the
    cache dropped first; with a budget that holds both, nothing is dropped."""
    reqs = _reqs([0.0, 0.001, 0.002, 0.003])
    fps = {0: 60, 1: 60, 2: 60, 3: 60}
    dur = {i: 0.01 for i in fps}
    for budget, expect_clear in ((100, True), (1000, False)):
        if stepwise:
            exe = CachedStepEngine(fps, {i: 3 for i in fps}, idle_per_request=50)
            srv = serve.StepServer(exe, hbm_budget=budget, slots=2)
        else:
            exe = CachedExecutor(fps, dur, idle_per_request=50)
            srv = serve.Server(exe, hbm_budget=budget, slots=2)
        res = srv.run(reqs)
        assert all(r.status == "ok" for r in res)
        assert srv.max_reserved <= budget
        assert (exe.clears > 0) == expect_clear


def test_admission_respects_budget_slots_and_fifo():
    reqs = _reqs([0.0, 0.001, 0.002, 0.003, 0.004, 0.005, 0.006])
    fps = {0: 40, 1: 40, 2: 40, 3: 10, 4: 90, 5: 10, 6: 200}
    dur = {i: 0.03 for i in fps}
    exe = FakeExecutor(fps, dur)
    srv = serve.Server(exe, hbm_budget=100, slots=3)
    res = srv.run(reqs)
    st = {r.rid: r.status for r in res}
    assert st[6] == "rejected"                     # larger than the whole budget
    assert all(st[i] == "ok" for i in range(6))
    assert srv.max_reserved <= 100
    assert exe.peak <= 3 and srv.max_active <= 3
    # first come, first served: admission order follows arrival order
    admits = [r.admit for r in res if r.status == "ok"]
    assert admits == sorted(admits)
    # request 2 (40) had to wait for 0 or 1 to release memory (budget 100)
    r = {x.rid: x for x in res}
    assert r[2].admit >= min(r[0].finish, r[1].finish) - 1e-3
    s = serve.summarize(res, srv.wall)
    assert s["completed"] == 6 and s["rejected"] == 1
    assert s["latency_s"]["p50"] <= s["latency_s"]["p99"]


def test_requests_arriving_while_busy_overlap():
    reqs = _reqs([0.0, 0.01, 0.02, 0.03])
    exe = FakeExecutor({i: 1 for i in range(4)}, {i: 0.1 for i in range(4)})
    srv = serve.Server(exe, hbm_budget=10, slots=4)
    res = srv.run(reqs)
    assert exe.peak == 4                           # later arrivals joined running work
    assert srv.wall < 0.35


def test_failure_in_one_request_does_not_stop_the_loop():
    class Boom(FakeExecutor):
        def __call__(self, req, res):
            if req.rid == 1:
                raise RuntimeError("boom")
            super().__call__(req, res)
    reqs = _reqs([0.0, 0.0, 0.0])
    exe = Boom({i: 1 for i in range(3)}, {i: 0.01 for i in range(3)})
    res = serve.Server(exe, hbm_budget=10, slots=2).run(reqs)
    assert [r.status.startswith("error") for r in res] == [False, True, False]


@pytest.mark.gpu
def test_result_identical_alone_and_in_mix():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    reqs = wl.serving_stream(4, rate=0.0, seed=7, ka_range=(10.0, 40.0), max_rhs=3)
    exe = serve.GpuExecutor(restart=200, keep_solution=True)
    alone = {}
    for r in reqs:
        out = serve.Server(exe, hbm_budget=64 << 30, slots=1).run([r])[0]
        assert out.status == "ok", out.status
        alone[r.rid] = out
    srv = serve.Server(exe, hbm_budget=64 << 30, slots=4)
    mix = srv.run(reqs)
    assert srv.max_active >= 2
    for out in mix:
        assert out.status == "ok"
        a = alone[out.rid]
        assert np.array_equal(out.x, a.x), out.rid
        assert np.array_equal(out.sigma, a.sigma)
        assert out.resid <= 1.0000001 * reqs[out.rid].tol


class FakeStepEngine:
    """Step-wise stand-in: request rid needs steps[rid] rounds."""

    def __init__(self, fps, steps, fail_prepare=(), fail_finish=()):
        self.fps = fps
        self.steps = steps
        self.fail_prepare = set(fail_prepare)
        self.fail_finish = set(fail_finish)
        self.order = []
        self.peak = 0
        self.discarded = 0

    def footprint(self, req):
        return self.fps[req.rid]

    def prepare(self, req):
        if req.rid in self.fail_prepare:
            raise RuntimeError("setup failed")
        return {"rid": req.rid, "left": self.steps[req.rid]}

    def step(self, jobs):
        self.peak = max(self.peak, len(jobs))
        for j in jobs:
            j["left"] -= 1
        time.sleep(2e-4)      # a device step takes time and releases the GIL

    def done(self, job):
        return job["left"] <= 0

    def finish(self, req, job, res):
        if req.rid in self.fail_finish:
            raise RuntimeError("retire failed")
        self.order.append(req.rid)
        res.status = "ok"
        res.nrhs = len(req.phis)
        res.matvecs = self.steps[req.rid]

    def discard(self, job):
        self.discarded += 1


class CachedStepEngine(FakeStepEngine):
    """Step-wise stand-in with a spectrum cache (see CachedExecutor)."""

    def __init__(self, fps, steps, idle_per_request):
        super().__init__(fps, steps)
        self.lock = threading.Lock()
        self.idle = 0
        self.per = idle_per_request
        self.clears = 0

    def finish(self, req, job, res):
        super().finish(req, job, res)
        with self.lock:
            self.idle += self.per

    def cache_idle_bytes(self):
        with self.lock:
            return self.idle

    def cache_clear(self):
        with self.lock:
            self.idle = 0
            self.clears += 1


def test_step_server_admission_budget_slots_fifo():
    reqs = _reqs([0.0] * 7)
    fps = {0: 40, 1: 40, 2: 40, 3: 10, 4: 90, 5: 10, 6: 200}
    eng = FakeStepEngine(fps, {i: 20 for i in fps})
    srv = serve.StepServer(eng, hbm_budget=100, slots=3, setup_workers=2)
    res = srv.run(reqs, realtime=False)
    st = {r.rid: r.status for r in res}
    assert st[6] == "rejected" and all(st[i] == "ok" for i in range(6))
    assert srv.max_reserved <= 100 and srv.max_active <= 3 and eng.peak <= 3
    admits = [r.admit for r in res if r.status == "ok"]
    assert admits == sorted(admits)


def test_step_server_short_request_overtakes_long_one():
    """Interleaving at step granularity: a short request admitted after a long
    one finishes first, and the long one keeps stepping meanwhile."""
    reqs = _reqs([0.0, 0.0])
    eng = FakeStepEngine({0: 1, 1: 1}, {0: 400, 1: 5})
    srv = serve.StepServer(eng, hbm_budget=10, slots=2, setup_workers=1)
    res = srv.run(reqs, realtime=False)
    assert all(r.status == "ok" for r in res)
    assert eng.order == [1, 0] and eng.peak == 2
    assert srv.rounds >= 400


def test_step_server_failures_recorded():
    reqs = _reqs([0.0, 0.0, 0.0, 0.0])
    eng = FakeStepEngine({i: 1 for i in range(4)}, {i: 3 for i in range(4)}, fail_prepare={1}, fail_finish={2})
    res = serve.StepServer(eng, hbm_budget=10, slots=4).run(reqs, realtime=False)
    st = [r.status for r in res]
    assert st[0] == "ok" and st[3] == "ok"
    assert st[1].startswith("error: setup") and st[2].startswith("error: retire")


@pytest.mark.gpu
def test_step_server_results_identical_alone_in_mix_and_threaded():
    """Each request's result is bitwise the same solved alone, interleaved
    step by step with the others, and by the thread-per-request server."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    reqs = wl.serving_stream(5, rate=0.0, seed=11, ka_range=(10.0, 40.0), max_rhs=3)
    eng = serve.GpuStepEngine(restart=200, keep_solution=True)
    alone = {}
    for r in reqs:
        out = serve.StepServer(eng, hbm_budget=64 << 30, slots=1).run([r], realtime=False)[0]
        assert out.status == "ok", out.status
        alone[r.rid] = out
    srv = serve.StepServer(eng, hbm_budget=64 << 30, slots=8)
    mix = srv.run(reqs, realtime=False)
    assert srv.max_active >= 2
    threaded = serve.Server(serve.GpuExecutor(restart=200, keep_solution=True), hbm_budget=64 << 30,
                            slots=4).run(reqs, realtime=False)
    th = {o.rid: o for o in threaded}
    for out in mix:
        assert out.status == "ok"
        a = alone[out.rid]
        assert np.array_equal(out.x, a.x), out.rid
        assert np.array_equal(out.sigma, a.sigma)
        assert np.array_equal(th[out.rid].x, a.x) and np.array_equal(th[out.rid].sigma, a.sigma)
        assert out.resid <= 1.0000001 * reqs[out.rid].tol


def test_request_log_has_one_line_per_request(tmp_path):
    """The JSONL request log: one line per request (completed, rejected or
    failed) with its times and sizes."""
    import json
    reqs = _reqs([0.0, 0.001, 0.002, 0.003])
    fps = {0: 10, 1: 10, 2: 500, 3: 10}
    exe = FakeExecutor(fps, {i: 0.01 for i in fps})
    path = tmp_path / "req.jsonl"
    res = serve.Server(exe, hbm_budget=100, slots=2, log_path=str(path)).run(reqs)
    lines = [json.loads(l) for l in open(path)]
    assert sorted(d["rid"] for d in lines) == [0, 1, 2, 3]
    by = {d["rid"]: d for d in lines}
    assert by[2]["status"] == "rejected"
    for r in res:
        d = by[r.rid]
        assert d["N"] == 8 and d["m"] == 16 and d["R"] == 2 and d["precision"] == "fp64"
        assert d["arrival"] == r.arrival and d["finish"] == r.finish
        if r.status == "ok":
            assert d["admit"] <= d["finish"] and d["matvecs"] == 10
