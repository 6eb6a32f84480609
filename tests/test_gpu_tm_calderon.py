"""TM Calderon operators (dual hats on the barycentric refinement): parity
with oracle.dual, solves equal to the TM EFIE's, the Fourier spectrum of the
preconditioned operator on the circle (plateau 1/4 unfiltered, the low
modes kept and the high modes compressed by N^alpha)."""
import math

import numpy as np
import pytest

from oracle import dual as odual
from oracle import mie
from paper_2606_10784_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2606_10784_amd import aim  # noqa: E402

K = 2 * math.pi


def _setup(xy, eps, alpha, precision=aim.AIM_FP64, max_rhs=2, oracle=True):
    m = wl.grid_side_for(odual.refined_polygon(xy), eps)
    ctx = aim.Context(xy, K, wl.ETA0, 0, m, eps, precision=precision, max_rhs=max_rhs, dual=1, max_restart=200)
    ctx.filter(alpha)
    orc = odual.TMCalderonOracle(xy, K, wl.ETA0, m, eps, alpha=alpha) if oracle else None
    return ctx, orc


def _cols(x):
    return torch.from_numpy(np.ascontiguousarray(x.T)).cuda()


CASES = [("circle40", wl.circle(0.5, 40), 0.05),       # T^-1 over all N offsets
         ("star96", wl.star5(1.0, 96), 0.08),          # banded T^-1
         # unequal segments (ratios up to ~4) on a non-convex contour
         ("irregular48", wl.irregular_polygon(np.random.default_rng(48), 0.5, 48, depth=0.2, jitter=0.25), 0.05)]


@pytest.mark.parametrize("name,xy,eps", CASES, ids=[c[0] for c in CASES])
def test_tm_calderon_operators_match_oracle(name, xy, eps):
    alpha = math.sqrt(2 * math.pi) / eps
    print(f"tm calderon parity {name}", flush=True)
    ctx, orc = _setup(xy, eps, alpha, precision=aim.AIM_MIXED)
    n = xy.shape[0]
    assert ctx.info()["dual_unknowns"] == 2 * n
    rng = np.random.default_rng(7)
    x = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    for op in ("TM_PC", "TM_PC_UNF", "TM_CP", "TM_CP_UNF"):
        ref = orc.apply(op, x)
        y = ctx.matvec(op, _cols(x)).cpu().numpy().T
        err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
        yf = ctx.matvec(aim.OPS[op] | aim.AIM_OP_GRID_FP32, _cols(x)).cpu().numpy().T
        errf = np.max(np.abs(yf - ref)) / np.max(np.abs(ref))
        print(op, "fp64", err, "fp32 grid", errf)
        assert err < 1e-12
        assert errf < 1e-5


def test_tm_calderon_on_a_grid_side_not_a_power_of_two():
    """The pulse space and its dual hats share a 40-point grid side (FFT
    length 128): the preconditioned operators equal the oracle's with the
    same embedding length."""
    xy, eps = wl.circle(0.5, 40), 0.05
    alpha = math.sqrt(2 * math.pi) / eps
    ctx = aim.Context(xy, K, wl.ETA0, 0, 40, eps, precision=aim.AIM_MIXED, max_rhs=2, dual=1, max_restart=0)
    assert ctx.info()["n_pad"] == 128
    ctx.filter(alpha)
    orc = odual.TMCalderonOracle(xy, K, wl.ETA0, 40, eps, alpha=alpha, n=128)
    x = np.random.default_rng(11).standard_normal((40, 2)) + 1j * np.random.default_rng(12).standard_normal((40, 2))
    for op in ("TM_PC", "TM_CP", "TM_CP_UNF"):
        ref = orc.apply(op, x)
        y = ctx.matvec(op, _cols(x)).cpu().numpy().T
        err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
        print(op, "m=40", err)
        assert err < 1e-12


def test_n_alpha_matches_oracle():
    xy = wl.star5(1.0, 64)
    eps = 0.08
    alpha = math.sqrt(2 * math.pi) / eps
    from oracle import aim as oaim
    m = wl.grid_side_for(xy, eps)
    ctx = aim.Context(xy, K, wl.ETA0, 1, m, eps, max_rhs=1)
    ctx.filter(alpha)
    orc = oaim.AimOracle(xy, K, wl.ETA0, 1, m, eps, alpha=alpha, near=False)
    x = np.random.default_rng(3).standard_normal(64) + 0j
    y = ctx.matvec("N_ALPHA", torch.from_numpy(x).cuda()).cpu().numpy()
    ref = orc.apply("N_ALPHA", x)
    err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
    print("N_ALPHA", err)
    assert err < 1e-12


def test_tm_calderon_needs_the_dual_space():
    xy = wl.circle(0.5, 40)
    ctx = aim.Context(xy, K, wl.ETA0, 0, wl.grid_side_for(xy, 0.05), 0.05)
    x = torch.ones(40, dtype=torch.complex128, device="cuda")
    with pytest.raises(aim.AimError) as e:
        ctx.matvec("TM_CP", x)
    assert e.value.status == aim.AIM_E_STATE


def test_tm_calderon_solve_equals_tm_efie():
    """The preconditioner changes the iteration, not the solution: the TM
    EFIE and the unfiltered TM Calderon form reach the same current (which
    matches the Mie series), the Calderon form in fewer steps.  The filtered
    form, where it converges, reaches it too."""
    a, n, eps = 1.0, 192, 1.0 / 15
    xy = wl.circle(a, n)
    ctx, _ = _setup(xy, eps, math.sqrt(2 * math.pi) / eps, max_rhs=1, oracle=False)
    b = ctx.rhs_planewave(0.0)
    sols, its = {}, {}
    for form in ("TM", "TM_CP_UNF"):
        x, info = ctx.solve(form, b, tol=1e-9, restart=200, maxit=2000)
        sols[form] = x.cpu().numpy()
        its[form] = info[0]["iterations"]
    try:
        x, info = ctx.solve("TM_CP", b, tol=1e-6, restart=200, maxit=1000)
        sols["TM_CP"] = x.cpu().numpy()
        its["TM_CP"] = info[0]["iterations"]
    except aim.AimError as e:
        assert e.status == aim.AIM_E_NOCONV
        its["TM_CP"] = None
    print("iterations", its)
    ref = sols["TM"]
    d = np.linalg.norm(sols["TM_CP_UNF"] - ref) / np.linalg.norm(ref)
    print("TM_CP_UNF vs TM EFIE", d)
    assert d < 1e-6
    if "TM_CP" in sols:
        # the filtered preconditioner compresses the modes past its cutoff, so
        # its residual test does not see them: the current agrees to the
        # discretisation level, not to the solver tolerance
        d = np.linalg.norm(sols["TM_CP"] - ref) / np.linalg.norm(ref)
        print("TM_CP vs TM EFIE", d)
        assert d < 2e-2
    phi = 2 * math.pi * (np.arange(n) + 0.5) / n
    jm = mie.mie_tm_current(phi, K, a, wl.ETA0)
    assert np.linalg.norm(ref - jm) / np.linalg.norm(jm) < 3e-2
    assert its["TM_CP_UNF"] < its["TM"]


def test_tm_calderon_mixed_precision_solve():
    """FP64 refinement around an inner GMRES whose grid parts (S and the
    dual N) are FP32: the FP64 residual of the preconditioned system meets the
    tolerance and the current equals the FP64 solve's."""
    a, n, eps = 1.0, 192, 1.0 / 15
    xy = wl.circle(a, n)
    ctx, _ = _setup(xy, eps, math.sqrt(2 * math.pi) / eps, precision=aim.AIM_MIXED, max_rhs=1, oracle=False)
    b = ctx.rhs_planewave(0.0)
    x64, i64 = ctx.solve("TM_CP_UNF", b, tol=1e-8, restart=200, maxit=2000)
    xm, im = ctx.solve("TM_CP_UNF", b, tol=1e-8, restart=200, maxit=2000, precision=aim.AIM_MIXED)
    print("fp64", i64[0]["iterations"], i64[0]["resid_true"], " mixed", im[0]["iterations"], im[0]["outer"],
          im[0]["resid_true"])
    assert im[0]["converged"] == 1 and im[0]["resid_true"] <= 1e-8
    d = np.linalg.norm(xm.cpu().numpy() - x64.cpu().numpy()) / np.linalg.norm(x64.cpu().numpy())
    print("mixed vs fp64 current", d)
    assert d < 1e-6


def test_tm_calderon_spectrum_on_the_circle():
    """Fourier quotients of the preconditioned TM operator (divided by
    jk eta): unfiltered, the product lambda^N lambda^S of the circle (plateau
    1/4); filtered at the paper's alpha = 8k, lambda^S times the analytic
    lambda^{N^alpha} below the cutoff and compressed past it (the TM
    counterpart of Fig. 3).  On the circle the Maue form gives
    lambda^{N^alpha}_n = (n/a)^2 lambda^{S^alpha}_n
                         - k^2 (lambda^{S^alpha}_{n+1} + lambda^{S^alpha}_{n-1}) / 2."""
    # the numerical filter approaches the analytic one as alpha eps / pi -> 0
    # (eq. (12)); at alpha = 8k the oracle's N^alpha is 50 % / 15 % / 4.3 %
    # off below the cutoff at eps = lambda/30, /60, /120: the test uses /120
    a, n, eps = 1.0, 160, 1.0 / 120
    xy = wl.circle(a, n)
    alpha = 8 * K
    ctx, orc = _setup(xy, eps, alpha, max_rhs=32)
    nus = np.arange(0, n // 2 + 1)
    lU = ctx.fourier_spectrum("TM_CP_UNF", nus) / (1j * K * wl.ETA0)
    lF = ctx.fourier_spectrum("TM_CP", nus) / (1j * K * wl.ETA0)
    th = 2 * math.pi * np.arange(n) / n
    sel = np.array([0, 5, 30, 60, 80])
    E = np.exp(1j * np.outer(th, sel))
    ref = np.einsum('jm,jm->m', E.conj(), orc.apply("TM_CP", E)) / n / (1j * K * wl.ETA0)
    err = np.max(np.abs(lF[sel] - ref)) / np.max(np.abs(ref))
    print("filtered spectrum vs oracle", err)
    assert err < 1e-10
    lS = mie.circle_eig_S(nus, K, a)
    ex = lS * mie.circle_eig_N(nus, K, a)
    lSa = mie.circle_eig_S_alpha(np.arange(0, n // 2 + 2), K, a, alpha)
    lNa = np.array([(v / a) ** 2 * lSa[v] - K ** 2 * (lSa[v + 1] + lSa[abs(v - 1)]) / 2 for v in nus])
    exF = lS * lNa
    low = nus <= 2 * K * a
    mid = (nus > 3 * K * a) & (nus <= n // 4)
    print("unfiltered vs lambda^N lambda^S (low)", np.max(np.abs(lU[low] - ex[low])),
          " plateau", np.abs(lU[mid]).min(), np.abs(lU[mid]).max(), " top", np.abs(lU[nus > n // 4]).max())
    assert np.max(np.abs(lU[low] - ex[low])) < 0.02
    # the plateau 1/4, up to the O((nu h)^2) discretisation drift near Nyquist
    assert np.all(np.abs(lU[mid] - 0.25) < 0.03)
    assert np.all(np.abs(lU[nus > n // 4] - 0.25) < 0.08)

    def rel(x, y):   # modes near a zero of J_n(ka) or J_n'(ka) measured against 0.2 max|y|
        return np.abs(x - y) / np.maximum(np.abs(y), 0.2 * np.max(np.abs(y)))
    below = nus <= 0.45 * alpha * a
    above = nus >= 1.2 * alpha * a
    gap = rel(lF[below], exF[below])
    tail = np.max(np.abs(lF[above])) / np.max(np.abs(lU))
    print("filtered vs lambda^S lambda^{N^alpha} below the cutoff", gap.max(),
          " filtered past 1.2 alpha a", tail)
    assert gap.max() < 0.08
    assert tail < 1e-3
