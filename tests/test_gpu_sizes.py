"""Every grid size the library supports (m = 16 .. 1024, FFT lengths n =
32 .. 2048; n = 4096 is covered by the full-size star; grid sides that are
not powers of two take the next power-of-two FFT length), each with its own
radix split and folded spectrum layout, against the oracle: a circle filling
most of the grid with an odd number of segments (ragged against every lane
group and tile), pulses and hats, two right-hand sides, FP64 to 1e-12 and
the FP32 grid to 1e-5 of max|y|.  Also: zero in, zero out."""
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

K, ETA, EPS = wl.K0, wl.ETA0, 0.1


def _case(m, basis):
    a = 0.35 * (m - 1) * EPS
    n = int(2 * math.pi * a / (0.8 * EPS)) | 1          # odd, h ~ 0.8 eps
    return wl.circle(a, max(n, 9)), a


SIZES = [(16, 0), (32, 0), (64, 1), (128, 0), (256, 1), (512, 0), (1024, 0)]


@pytest.mark.parametrize("m,basis", SIZES, ids=[f"m{m}_{'hat' if b else 'pulse'}" for m, b in SIZES])
def test_every_grid_size_matches_oracle(m, basis):
    xy, _ = _case(m, basis)
    n = xy.shape[0]
    alpha = wl.alpha_half_bins(EPS)
    print(f"size sweep m={m} basis={basis} N={n}", flush=True)
    ctx = aim.Context(xy, K, ETA, basis, m, EPS, max_rhs=2, precision=aim.AIM_MIXED)
    ctx.filter(alpha)
    orc = oaim.AimOracle(xy, K, ETA, basis, m, EPS, alpha=alpha)
    rng = np.random.default_rng(m)
    x = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    xt = torch.from_numpy(x).cuda()
    for op in (("S", "S_ALPHA", "TM") if basis == 0 else ("S_ALPHA", "N", "TE_CP")):
        ref = orc.apply(op, x.T).T
        y = ctx.matvec(op, xt).cpu().numpy()
        yf = ctx.matvec(aim.OPS[op] | aim.AIM_OP_GRID_FP32, xt).cpu().numpy()
        e64 = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
        e32 = np.max(np.abs(yf - ref)) / np.max(np.abs(ref))
        print(op, e64, e32)
        # TE_CP: G^-1 S^alpha G^-1 N, where N x is ~1e3 larger than the product
        assert e64 < (1e-10 if op == "TE_CP" else 1e-12)
        assert e32 < 1e-5
    z = torch.zeros_like(xt)
    assert torch.count_nonzero(ctx.matvec("S_ALPHA", z)).item() == 0


# (m, basis, FFT length, circle sized for grid side m_case): 1500 keeps the
# m = 600 circle on a 4096-point embedding
ODD_SIZES = [(17, 1, 64, 17), (48, 1, 128, 48), (600, 0, 2048, 600), (1500, 0, 4096, 600)]


@pytest.mark.parametrize("m,basis,n_fft,m_case", ODD_SIZES,
                         ids=[f"m{m}_{'hat' if b else 'pulse'}" for m, b, _, _ in ODD_SIZES])
def test_grid_side_not_a_power_of_two(m, basis, n_fft, m_case):
    """A grid side that is not a power of two (17, 48, the paper's Sec. IV
    grid of 600 points, 1500) runs on the FFT length n = the smallest power
    of two >= 2m: the oracle with the same embedding length gives the same
    operators, filtered ones included (the numerical filter's DFT bins
    follow n)."""
    xy, _ = _case(m_case, basis)
    n = xy.shape[0]
    alpha = wl.alpha_half_bins(EPS)
    print(f"odd grid side m={m} basis={basis} N={n}", flush=True)
    ctx = aim.Context(xy, K, ETA, basis, m, EPS, max_rhs=2, precision=aim.AIM_MIXED)
    assert ctx.info()["n_pad"] == n_fft
    ctx.filter(alpha)
    orc = oaim.AimOracle(xy, K, ETA, basis, m, EPS, alpha=alpha, n=n_fft)
    rng = np.random.default_rng(m)
    x = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    xt = torch.from_numpy(x).cuda()
    for op in (("S", "S_ALPHA", "TM") if basis == 0 else ("S_ALPHA", "N", "TE_CP")):
        ref = orc.apply(op, x.T).T
        y = ctx.matvec(op, xt).cpu().numpy()
        yf = ctx.matvec(aim.OPS[op] | aim.AIM_OP_GRID_FP32, xt).cpu().numpy()
        e64 = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
        e32 = np.max(np.abs(yf - ref)) / np.max(np.abs(ref))
        print(op, e64, e32)
        assert e64 < (1e-10 if op == "TE_CP" else 1e-12)
        assert e32 < 1e-5


@pytest.mark.parametrize("basis", [0, 1])
def test_smallest_polygon_and_grid(basis):
    """The smallest accepted inputs: an octagon (N = 8, every pair in the near
    zone) on the 16 x 16 grid, one rhs."""
    xy = wl.circle(0.45, 8)
    print(f"octagon basis={basis}", flush=True)
    alpha = wl.alpha_half_bins(EPS)
    ctx = aim.Context(xy, K, ETA, basis, 16, EPS, max_rhs=1)
    ctx.filter(alpha)
    orc = oaim.AimOracle(xy, K, ETA, basis, 16, EPS, alpha=alpha)
    x = np.random.default_rng(8).standard_normal(8) + 1j * np.random.default_rng(9).standard_normal(8)
    for op in (("S", "S_ALPHA", "TM") if basis == 0 else ("S_ALPHA", "N", "GRAM_INV", "TE_CP")):
        ref = orc.apply(op, x)
        y = ctx.matvec(op, torch.from_numpy(x).cuda()).cpu().numpy()
        err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
        print(op, err)
        assert err < 1e-12
