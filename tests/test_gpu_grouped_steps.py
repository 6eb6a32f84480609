"""Grouped steps of aim_solver_step: solvers on different contexts that
share a grid-kernel spectrum (same grid size, k eps and precision) run the
column pass of each Arnoldi step as one launch over all their tiles, on one
stream or across streams.  Each solver still ends bitwise at its aim_solve
result, alone or in any group (the grouped launch computes every tile as a
solo one), and with the FP32 grid of the mixed refinement too."""
import numpy as np
import pytest

from paper_2606_10784_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2606_10784_amd import aim  # noqa: E402

K = wl.K0
ETA = wl.ETA0


def _contexts(shared_stream):
    """Three contours on the same 64-point grid at eps = 0.1 (one spectrum)
    and one on a 128-point grid (a spectrum of its own)."""
    rng = np.random.default_rng(31)
    s0 = torch.cuda.Stream()
    shapes = [wl.circle(1.0, 500), wl.random_star(rng, 0.9, 420), wl.star5(0.8, 384), wl.circle(2.0, 640)]
    grids = [64, 64, 64, 128]
    out = []
    for xy, m in zip(shapes, grids):
        s = s0 if shared_stream else torch.cuda.Stream()
        out.append(aim.Context(xy, K, ETA, 0, m, 0.1, max_rhs=2, precision=aim.AIM_MIXED, stream=s,
                               max_restart=30))
    return out


@pytest.mark.parametrize("shared_stream", [False, True])
@pytest.mark.parametrize("precision", [aim.AIM_FP64, aim.AIM_MIXED])
def test_grouped_steps_equal_solo_solves(shared_stream, precision):
    ctxs = _contexts(shared_stream)
    print(f"[grouped] shared_stream={shared_stream} precision={precision}", flush=True)
    kw = dict(tol=1e-8, restart=30, maxit=3000, precision=precision)
    bs = [c.rhs_planewave(np.array([0.3, 2.0])[: 1 + i % 2]) for i, c in enumerate(ctxs)]
    refs = []
    for c, b in zip(ctxs, bs):
        x, info = c.solve("TM", b, **kw)
        refs.append((x.clone(), info))
    torch.cuda.synchronize()
    solvers = [aim.Solver(c, "TM", b, **kw) for c, b in zip(ctxs, bs)]
    rounds = 0
    while any(s.poll()[0] == aim.AIM_PENDING for s in solvers):
        assert aim.aim_solver_step(solvers) == aim.AIM_OK
        rounds += 1
        assert rounds < 20000
    torch.cuda.synchronize()
    for s, (x, info) in zip(solvers, refs):
        st, inf = s.poll()
        assert st == aim.AIM_OK
        assert torch.equal(s.x, x)
        assert [d["iterations"] for d in inf] == [d["iterations"] for d in info]
        s.end()
    print(f"[grouped] rounds {rounds}, iterations", [r[1][0]["iterations"] for r in refs])
    for c in ctxs:
        c.close()
