"""GPU GMRES solves checked with the oracle's FP64 operators and the Mie
series.  Several solutions meet a tolerance, so parity is on the residual
(evaluated with the oracle operator) and on the current within the
condition-number bound."""
import math

import numpy as np
import pytest

from oracle import aim as oaim
from oracle import excitation, mie
from oracle.solver import gmres as ogmres
from paper_2606_10784_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2606_10784_amd import aim  # noqa: E402

K = wl.K0
ETA = wl.ETA0


def _t(x):
    x = np.asarray(x)
    if x.ndim == 2:
        x = x.T
    return torch.from_numpy(np.ascontiguousarray(x.astype(np.complex128))).cuda()


def _n(t):
    a = t.cpu().numpy()
    return a.T if a.ndim == 2 else a


@pytest.fixture(scope="module")
def tm():
    """Circle a = 1 (ka = 2 pi), N = 512 pulses, grid 64 at lambda/10."""
    w = wl.cylinder_small()
    orc = oaim.AimOracle(w.xy, K, ETA, 0, w.m, w.eps, alpha=w.alpha)
    ctx = aim.Context(w.xy, K, ETA, 0, w.m, w.eps, max_rhs=4, precision=aim.AIM_MIXED, max_restart=200)
    ctx.filter(w.alpha)
    b = excitation.rhs_tm(w.xy, 0, K, 0.0)
    x_or, inf = ogmres(lambda v: orc.apply('TM', v), b, tol=1e-11, restart=200)
    assert inf['converged']
    return w, orc, ctx, b, x_or


def test_tm_solve_fp64_residual_and_current(tm):
    w, orc, ctx, b, x_or = tm
    x, info = ctx.solve("TM", _t(b), tol=1e-8, restart=100)
    xs = _n(x)
    res = np.linalg.norm(b - orc.apply('TM', xs)) / np.linalg.norm(b)
    print("tm fp64 iters", info[0]['iterations'], "resid(oracle op)", res, "gpu true", info[0]['resid_true'])
    assert info[0]['converged'] == 1
    assert res < 1.5e-8
    assert np.linalg.norm(xs - x_or) / np.linalg.norm(x_or) < 1e-5
    # physics: Mie current at the segment midpoints; at a lambda/10 grid the
    # AIM far-interaction error (~2e-3 on the operator) dominates
    phm = 2 * math.pi * (np.arange(512) + 0.5) / 512
    jm = mie.mie_tm_current(phm, K, 1.0, ETA)
    assert np.linalg.norm(xs - jm) / np.linalg.norm(jm) < 3e-2


def test_tm_solve_mixed_precision(tm):
    w, orc, ctx, b, x_or = tm
    x, info = ctx.solve("TM", _t(b), tol=1e-8, restart=100, precision=aim.AIM_MIXED)
    xs = _n(x)
    res = np.linalg.norm(b - orc.apply('TM', xs)) / np.linalg.norm(b)
    print("tm mixed iters", info[0]['iterations'], "outer", info[0]['outer'], "resid", res)
    assert info[0]['converged'] == 1
    assert res < 1.05e-8
    assert np.linalg.norm(xs - x_or) / np.linalg.norm(x_or) < 1e-4


def test_tm_multi_rhs_equals_single(tm):
    w, orc, ctx, b, x_or = tm
    ph = [0.0, 1.1, 2.9]
    B = ctx.rhs_planewave(ph)
    X, infos = ctx.solve("TM", B, tol=1e-6)
    for r, p in enumerate(ph):
        xr, _ = ctx.solve("TM", B[r].contiguous(), tol=1e-6)
        assert torch.equal(X[r], xr)
    sig = ctx.rcs(X, ph)
    ex = mie.mie_tm_backscatter(K, 1.0)
    assert np.all(np.abs(sig - ex) / ex < 2e-2)        # circle: every angle alike


def test_initial_guess_resume(tm):
    w, orc, ctx, b, x_or = tm
    x1, i1 = ctx.solve("TM", _t(b), tol=1e-4)
    x2, i2 = ctx.solve("TM", _t(b), x0=x1, tol=1e-8)
    assert i2[0]['converged'] == 1
    res = np.linalg.norm(b - orc.apply('TM', _n(x2))) / np.linalg.norm(b)
    assert res < 1.5e-8


@pytest.fixture(scope="module")
def te():
    xy = wl.star5(0.8, 300)
    eps = 0.05
    m = wl.grid_side_for(xy, eps)
    alpha = wl.alpha_half_bins(eps)
    orc = oaim.AimOracle(xy, K, ETA, 1, m, eps, alpha=alpha)
    ctx = aim.Context(xy, K, ETA, 1, m, eps, max_rhs=1, precision=aim.AIM_MIXED)
    ctx.filter(alpha)
    return xy, orc, ctx


@pytest.mark.parametrize("form,op", [("TE_CP", "TE_CP"), ("TE_CP_UNF", "TE_CP_UNF")])
def test_te_calderon_solve(te, form, op):
    xy, orc, ctx = te
    b = excitation.rhs_te(xy, 1, K, ETA, 0.7)
    Sop = (lambda v: orc.apply('S_ALPHA', v)) if op == "TE_CP" else (lambda v: orc.apply('S', v))
    bp = orc.gram_inv(Sop(orc.gram_inv(b)))
    x, info = ctx.solve(form, _t(b), tol=1e-8)
    xs = _n(x)
    res = np.linalg.norm(bp - orc.apply(op, xs)) / np.linalg.norm(bp)
    print(form, "iters", info[0]['iterations'], "resid", res)
    assert info[0]['converged'] == 1
    assert res < 1.5e-8


def test_te_calderon_mixed(te):
    xy, orc, ctx = te
    b = excitation.rhs_te(xy, 1, K, ETA, 0.7)
    bp = orc.gram_inv(orc.apply('S_ALPHA', orc.gram_inv(b)))
    x, info = ctx.solve("TE_CP", _t(b), tol=1e-7, precision=aim.AIM_MIXED)
    res = np.linalg.norm(bp - orc.apply('TE_CP', _n(x))) / np.linalg.norm(bp)
    print("te mixed", info[0], res)
    assert res < 1.05e-7


@pytest.mark.parametrize("restart", [7, 23])
def test_tm_short_restart_cycles(tm, restart):
    """Restart lengths that do not divide the residual-check batch: every
    cycle ends by finalising its last Hessenberg column on its own."""
    w, orc, ctx, b, x_or = tm
    x, info = ctx.solve("TM", _t(b), tol=1e-8, restart=restart, maxit=20000)
    res = np.linalg.norm(b - orc.apply('TM', _n(x))) / np.linalg.norm(b)
    print("restart", restart, "iters", info[0]['iterations'], "restarts", info[0]['restarts'], "resid", res)
    assert info[0]['converged'] == 1
    assert info[0]['restarts'] > 1
    assert res < 1.5e-8


def test_tm_maxit_mid_cycle(tm):
    w, orc, ctx, b, x_or = tm
    x, info = ctx.solve("TM", _t(b), tol=1e-12, restart=10, maxit=13)
    assert info[0]['converged'] == 0
    assert info[0]['iterations'] == 13
    res = np.linalg.norm(b - orc.apply('TM', _n(x))) / np.linalg.norm(b)
    assert abs(res - info[0]['resid_true']) < 1e-8 * max(res, 1e-300) + 1e-12
    assert res < 1.0


def test_tm_solve_deterministic(tm):
    w, orc, ctx, b, x_or = tm
    x1, _ = ctx.solve("TM", _t(b), tol=1e-6, restart=50)
    x2, _ = ctx.solve("TM", _t(b), tol=1e-6, restart=50)
    assert torch.equal(x1, x2)


def test_longest_restart_on_a_large_star():
    """restart = 1000 (the largest allowed): the Givens batches past ~600
    columns exceed one block's LDS and are split; the solve converges to the
    same current as a short-restart solve, in fewer steps."""
    rq = wl.serving_stream(24, 0.0)[9]          # star, ka ~ 320, N = 6400, m = 1024
    print(f"long restart N={len(rq.xy)} m={rq.m}", flush=True)
    ctx = aim.Context(rq.xy, rq.k, rq.eta, 0, rq.m, rq.eps, max_rhs=1, max_restart=1000)
    b = ctx.rhs_planewave(float(rq.phis[0]))
    x1, i1 = ctx.solve("TM", b, tol=1e-6, restart=1000, maxit=4000)
    x3, i3 = ctx.solve("TM", b, tol=1e-6, restart=300, maxit=6000)
    print("iterations restart 1000:", i1[0]["iterations"], " restart 300:", i3[0]["iterations"])
    assert i1[0]["converged"] == 1 and i3[0]["converged"] == 1
    assert i1[0]["iterations"] > 620                  # reached the split batches
    assert i1[0]["iterations"] < i3[0]["iterations"]
    a, c = x1.cpu().numpy(), x3.cpu().numpy()
    assert np.linalg.norm(a - c) / np.linalg.norm(c) < 1e-3


def test_degenerate_right_hand_sides():
    """A zero column beside a nonzero one: x = 0 for it, converged, no NaN;
    and an exact initial guess: returned after the first residual check."""
    n = 64
    xy = wl.circle(1.0, n)
    ctx = aim.Context(xy, K, ETA, 0, 64, 0.1, max_rhs=2)
    b1 = ctx.rhs_planewave(0.7).cpu().numpy()
    B = torch.from_numpy(np.stack([np.zeros(n, complex), b1])).cuda()
    X, info = ctx.solve("TM", B, tol=1e-10, restart=40, maxit=200)
    Xs = X.cpu().numpy()
    print([(d["iterations"], d["converged"], d["resid_true"]) for d in info])
    assert np.all(np.isfinite(Xs))
    assert np.all(Xs[0] == 0) and info[0]["converged"] == 1 and info[0]["iterations"] == 0
    assert info[1]["converged"] == 1 and info[1]["resid_true"] <= 1e-10
    x0 = torch.from_numpy(Xs[1]).cuda()
    x2, i2 = ctx.solve("TM", torch.from_numpy(b1).cuda(), x0=x0, tol=1e-8, restart=40, maxit=200)
    assert i2[0]["converged"] == 1 and i2[0]["iterations"] == 0
    assert np.array_equal(x2.cpu().numpy(), Xs[1])
