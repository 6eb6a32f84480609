"""Step-wise solving (aim_solver_begin / step / poll / end), the serving
extension of the solve: a solver advanced by single Arnoldi steps, alone or
interleaved with others on the same and on other contexts, FP64 or mixed
refinement, ends bitwise at the result of aim_solve (aim_solve runs the same
state machine to the end; each solver has its own Krylov workspace); poll
reports AIM_PENDING until the end and then the status aim_solve returns."""
import math

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


@pytest.fixture(scope="module")
def ctxs():
    cyl = aim.Context(wl.circle(1.0, 500), K, ETA, 0, 64, 0.1, max_rhs=2, precision=aim.AIM_MIXED)
    cyl.filter(wl.alpha_half_bins(0.1))
    star = aim.Context(wl.star5(0.6, 256), K, ETA, 1, 64, 0.05, max_rhs=1)
    star.filter(wl.alpha_half_bins(0.05))
    return cyl, star


def _run(solvers, limit=100000):
    steps = 0
    while any(s.poll()[0] == aim.AIM_PENDING for s in solvers):
        st = aim.aim_solver_step(solvers)
        assert st == aim.AIM_OK
        steps += 1
        assert steps < limit
    return steps


def test_stepwise_solve_equals_aim_solve(ctxs):
    cyl, _ = ctxs
    b = cyl.rhs_planewave([0.0, 1.0])
    kw = dict(tol=1e-8, restart=16, maxit=2000)
    x_ref, info_ref = cyl.solve("TM", b, **kw)
    sv = aim.Solver(cyl, "TM", b, **kw)
    st, info0 = sv.poll()
    assert st == aim.AIM_PENDING and info0[0]["resid_true"] == -1.0
    steps = _run([sv])
    st, info = sv.poll()
    print("steps", steps, "iterations", [d["iterations"] for d in info], "restarts", info[0]["restarts"])
    assert st == aim.AIM_OK
    assert info[0]["restarts"] >= 2                      # several cycles were stepped through
    assert torch.equal(sv.x, x_ref)
    for d, e in zip(info, info_ref):
        assert (d["iterations"], d["matvecs"], d["restarts"], d["converged"]) == \
            (e["iterations"], e["matvecs"], e["restarts"], e["converged"])
        assert d["resid_true"] == e["resid_true"] and d["resid_est"] == e["resid_est"]
    assert sv.step() == aim.AIM_OK                       # a finished solver is skipped
    sv.end()


def test_interleaved_group_each_equals_its_solo_solve(ctxs):
    cyl, star = ctxs
    b1 = cyl.rhs_planewave(0.3)
    b2 = cyl.rhs_planewave([2.0, 4.0])
    b3 = star.rhs_planewave(0.7)
    jobs = [(cyl, "TM", b1, dict(tol=1e-7, restart=24, precision=aim.AIM_MIXED)),
            (cyl, "TM", b2, dict(tol=1e-9, restart=40)),
            (star, "TE_CP_UNF", b3, dict(tol=1e-8, restart=30))]
    refs = [c.solve(f, b, **kw) for c, f, b, kw in jobs]
    solvers = [aim.Solver(c, f, b, **kw) for c, f, b, kw in jobs]
    _run(solvers)
    for sv, (x_ref, info_ref) in zip(solvers, refs):
        st, info = sv.poll()
        assert st == aim.AIM_OK
        assert torch.equal(sv.x, x_ref)
        assert [d["iterations"] for d in info] == [d["iterations"] for d in info_ref]
        sv.end()


def test_stepwise_mixed_refinement_equals_aim_solve(ctxs):
    cyl, _ = ctxs
    b = cyl.rhs_planewave([0.5, 2.5])
    kw = dict(tol=1e-8, restart=20, maxit=2000, precision=aim.AIM_MIXED)
    x_ref, info_ref = cyl.solve("TM", b, **kw)
    sv = aim.Solver(cyl, "TM", b, **kw)
    _run([sv])
    st, info = sv.poll()
    print("mixed: outer", info[0]["outer"], "inner steps", [d["iterations"] for d in info])
    assert st == aim.AIM_OK and info[0]["outer"] >= 2
    assert torch.equal(sv.x, x_ref)
    for d, e in zip(info, info_ref):
        assert (d["iterations"], d["matvecs"], d["outer"], d["resid_true"]) == \
            (e["iterations"], e["matvecs"], e["outer"], e["resid_true"])
    sv.end()


def test_maxit_reports_noconv_like_aim_solve(ctxs):
    cyl, _ = ctxs
    b = cyl.rhs_planewave(0.0)
    x_ref, info_ref = cyl.solve("TM", b, tol=1e-12, restart=8, maxit=12)
    assert info_ref[0].get("status") == "noconv"
    sv = aim.Solver(cyl, "TM", b, tol=1e-12, restart=8, maxit=12)
    _run([sv])
    st, info = sv.poll()
    assert st == aim.AIM_E_NOCONV and info[0]["converged"] == 0
    assert torch.equal(sv.x, x_ref) and info[0]["resid_true"] == info_ref[0]["resid_true"]
    sv.end()


def test_solver_arguments_rejected(ctxs):
    cyl, star = ctxs
    b = cyl.rhs_planewave(0.0)
    for kw in (dict(restart=0), dict(restart=1001), dict(tol=0.0), dict(maxit=0)):
        with pytest.raises(aim.AimError):
            aim.Solver(cyl, "TM", b, **kw)
    with pytest.raises(aim.AimError):
        aim.Solver(cyl, "TE_CP", b)                      # hat form on a pulse context
    with pytest.raises(aim.AimError):
        aim.Solver(star, "TM", star.rhs_planewave(0.0))  # pulse form on a hat context


def test_closing_a_context_ends_its_solvers():
    ctx = aim.Context(wl.circle(1.0, 200), K, ETA, 0, 64, 0.1, max_rhs=1)
    b = ctx.rhs_planewave(0.0)
    sv = aim.Solver(ctx, "TM", b, tol=1e-8, restart=20)
    for _ in range(5):
        sv.step()
    ctx.close()                                      # ends the running solver first
    assert sv.handle is None
    sv.end()                                         # a second end is a no-op


def test_stepwise_tm_calderon_equals_aim_solve():
    """The TM Calderon form (dual hat space, preconditioned right-hand side
    formed at begin), FP64 and mixed."""
    ctx = aim.Context(wl.circle(1.0, 96), K, ETA, 0, 64, 0.1, max_rhs=1, precision=aim.AIM_MIXED, dual=1)
    try:
        b = ctx.rhs_planewave(0.4)
        for prec in (aim.AIM_FP64, aim.AIM_MIXED):
            kw = dict(tol=1e-8, restart=16, maxit=500, precision=prec)
            x_ref, info_ref = ctx.solve("TM_CP_UNF", b, **kw)
            sv = aim.Solver(ctx, "TM_CP_UNF", b, **kw)
            _run([sv])
            st, info = sv.poll()
            assert st == aim.AIM_OK
            assert torch.equal(sv.x, x_ref)
            assert info[0]["iterations"] == info_ref[0]["iterations"]
            sv.end()
    finally:
        ctx.close()
