"""aim_footprint_bytes, the host-only estimate the serving loop admits
requests by, bounds what a context then holds on the device: its tables,
buffers (aim_get_info's device_bytes after a solve), the caller-owned
Krylov workspace of that restart length and its grid-kernel spectrum in the
shared cache.  It is also not wastefully loose (at most 2.5x)."""
import math

import numpy as np
import pytest

from paper_2606_10784_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2606_10784_amd import aim  # noqa: E402


def _spectrum_bytes(m, mixed):
    n = 32
    while n < 2 * m:
        n *= 2
    rl = n
    while rl > 16:
        rl >>= 4
    return (n // 2 + 1) * (n // rl // 2 + 1) * rl * (24 if mixed else 16)


def _cases():
    out = []
    for r in wl.serving_stream(2, rate=0.0, seed=3, ka_range=(10.0, 60.0), max_rhs=8):
        out.append((r.xy, r.k, r.eta, 0, r.m, r.eps, r.precision, len(r.phis), 0))
    out.append((wl.circle(2.0, 4096), wl.K0, wl.ETA0, 0, 256, 1 / 40, 1, 1, 1))
    out.append((wl.star5(2.0, 2048), wl.K0, wl.ETA0, 1, 256, 1 / 40, 0, 2, 0))
    # non-convex contours with unequal segments: near pairs per basis vary
    # along the contour (55 on average, up to 79, against the bound's 74)
    irr = wl.irregular_polygon(np.random.default_rng(7), 2.0, 2048)
    out.append((irr, wl.K0, wl.ETA0, 0, 256, 1 / 40, 0, 1, 0))
    out.append((wl.irregular_polygon(np.random.default_rng(9), 2.0, 4096, depth=0.2), wl.K0, wl.ETA0, 1, 256,
                1 / 40, 1, 3, 0))
    return out


@pytest.mark.parametrize("case", range(6))
def test_footprint_bounds_device_bytes(case):
    xy, k, eta, basis, m, eps, prec, R, dual = _cases()[case]
    restart = 120
    p = aim.AIM_MIXED if prec else aim.AIM_FP64
    est = aim.aim_footprint_bytes(xy, k, eta, basis, m, eps, precision=p, max_rhs=R, restart=restart, dual=dual)
    ctx = aim.Context(xy, k, eta, basis, m, eps, precision=p, max_rhs=R, dual=dual, max_restart=restart)
    try:
        b = ctx.rhs_planewave(np.linspace(0.0, 1.0, R))
        ctx.solve("TM" if basis == 0 else "TE_CP_UNF", b, tol=1e-3, restart=restart, maxit=2)
        held = ctx.info()["device_bytes"] + _spectrum_bytes(m, prec) + aim.aim_workspace_bytes(len(xy), R, restart)
        print(f"case {case}: N={len(xy)} m={m} rhs={R} dual={dual} estimate {est / 1e6:.1f} MB, "
              f"held {held / 1e6:.1f} MB, ratio {est / held:.2f}")
        assert held <= est <= 2.5 * held
    finally:
        ctx.close()
