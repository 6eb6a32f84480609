"""GPU parity of the near-field singular quadrature over the whole range
aim_setup accepts.

Two polygons on grids so coarse that every segment pair lies in the near
zone, so the correction holds the exact Galerkin entries of eq. (4) and of
the Maue form of eq. (2) for every pair (self, vertex-sharing, disjoint) and
S_AIM equals the dense Galerkin matrix:
  * a 12-gon whose segments are 0.98 wavelengths long (k h = 6.16, next to
    the limit k h <= 2 pi);
  * a wedge with an acute tip (0.26 rad between its segments) and a
    0.02-wavelength segment between two long ones (disjoint neighbours
    1/18 of their length apart).
The oracle's moments are pinned against adaptive QUADPACK with a
log-weighted rule over this range (tests/test_oracle_galerkin.py).  Bound:
|C_gpu - C_oracle| <= 1e-12 max|C_oracle| per entry; matvecs 1e-12."""
import math

import numpy as np
import pytest

from oracle import aim as oaim
from paper_2606_10784_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2606_10784_amd import aim  # noqa: E402

K = wl.K0
ETA = wl.ETA0

WEDGE = np.array([[0.0, 0.0], [0.75, 0.05], [1.5, 0.1], [1.0, 0.2], [0.5, 0.3], [0.0, 0.4],
                  [-0.3, 0.2], [-0.3, 0.18], [-0.2, 0.0]])
GON12 = wl.circle(0.98 / (2.0 * math.sin(math.pi / 12)), 12)
CASES = {"wedge": (WEDGE, 0.8), "12gon": (GON12, 1.2)}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("basis", [0, 1])
def test_near_entries_all_pairs(name, basis):
    xy, eps = CASES[name]
    N = xy.shape[0]
    m = wl.grid_side_for(xy, eps)
    orc = oaim.AimOracle(xy, K, ETA, basis, m, eps)
    pairs = orc.near_sel_pairs
    assert pairs.shape[0] == N * N          # every pair corrected
    print(f"[near] {name} basis={basis} N={N} m={m}", flush=True)
    ctx = aim.Context(xy, K, ETA, basis, m, eps)
    ops = ("S",) if basis == 0 else ("S", "N")
    for op in ops:
        C = orc.Cnear[op]
        scale = np.max(np.abs(C))
        worst = 0.0
        for row in range(N):
            cols, vals = ctx.near_row(op, row)
            sel = pairs[:, 0] == row
            assert np.array_equal(cols, pairs[sel, 1])
            worst = max(worst, float(np.max(np.abs(vals - C[sel]))) / scale)
        print(f"[near] {name} basis={basis} {op}: entries rel err {worst:.2e}")
        assert worst < 1e-12
        x = wl.probe_vector(N, seed=21)
        y = ctx.matvec(op, torch.from_numpy(x).cuda()).cpu().numpy()
        ref = orc.apply(op, x)
        err = float(np.max(np.abs(y - ref)) / np.max(np.abs(ref)))
        print(f"[near] {name} basis={basis} {op}: matvec rel err {err:.2e}")
        assert err < 1e-12
    ctx.close()
