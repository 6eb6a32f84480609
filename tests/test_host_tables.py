"""Host tier: the library's host set-up (build_host_tables in
csrc/host_setup.cpp), built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, host code only, no device), against the
oracle's tables: anchor cells, the 4 x 4 stencil weights of every channel
and their grid points, the per-node map of Sec. III-A, the near-zone pattern
and the argument / geometry errors.  Any sanitizer report fails the run."""
import math
import os
import subprocess

import numpy as np
import pytest

from oracle import aim as oaim
from paper_2606_10784_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
AIM_OK, AIM_E_ARG, AIM_E_GEOM = 0, 1, 2
CHANNELS = {0: ("phi",), 1: ("phi", "dphi", "tx", "ty")}


@pytest.fixture(scope="module")
def dumper(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("host") / "host_tables_dump")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host", "host_tables_dump.cpp"),
           os.path.join(ROOT, "paper_2606_10784_amd", "csrc", "host_setup.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("host toolchain unavailable: " + r.stderr[-500:])
    return exe


def _run(exe, tmp, xy, k, basis, m, eps, quad=10, near_radius=6, node_order=0, eta=wl.ETA0):
    xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64).reshape(-1, 2))
    N = xy.shape[0]
    fin, fout = os.path.join(tmp, "in.bin"), os.path.join(tmp, "out.bin")
    with open(fin, "wb") as f:
        np.array([N, basis, m, quad, near_radius, node_order], dtype=np.int32).tofile(f)
        np.array([k, eta, eps], dtype=np.float64).tofile(f)
        xy.tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, fin, fout], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    raw = open(fout, "rb").read()
    head = np.frombuffer(raw[:28], dtype=np.int32)
    st, Nn, S, n_act, nr, band_w, nnz = (int(v) for v in head)
    out = {"status": st}
    if st != AIM_OK:
        return out
    off = 28
    def take(dtype, count):
        nonlocal off
        a = np.frombuffer(raw[off:off + count * np.dtype(dtype).itemsize], dtype=dtype)
        off += count * np.dtype(dtype).itemsize
        return a
    out.update(S=S, n_act=n_act, nr=nr, band_w=band_w)
    out["anc"] = np.stack([take(np.int32, N), take(np.int32, N)], axis=1)
    out["lin"] = take(np.int64, N * S).reshape(N, S)
    out["W"] = {ch: take(np.float64, N * S).reshape(N, S) for ch in CHANNELS[basis]}
    ptr = take(np.int32, N + 1)
    col = take(np.int32, nnz)
    out["pairs"] = np.stack([np.repeat(np.arange(N), np.diff(ptr)), col], axis=1)
    assert off == len(raw)
    return out


CASES = {
    "circle_pulse": (wl.circle(1.0, 500), wl.K0, 0, 64, 0.1),
    "star_hat": (wl.star5(0.6, 256), wl.K0, 1, 64, 0.05),
    "irregular_pulse": (wl.irregular_polygon(np.random.default_rng(7), 2.0, 300), wl.K0, 0, 128, 1 / 25),
    "irregular_hat": (wl.irregular_polygon(np.random.default_rng(9), 1.5, 160, depth=0.2), 3 * wl.K0, 1, 64, 0.06),
    "circle_pulse_m48": (wl.circle(1.8, 300), wl.K0, 0, 48, 0.1),       # a grid side that is not a power of two
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_host_tables_match_oracle(dumper, tmp_path, name):
    xy, k, basis, m, eps = CASES[name]
    out = _run(dumper, str(tmp_path), xy, k, basis, m, eps)
    assert out["status"] == AIM_OK
    grid = oaim.Grid(m, eps)
    assert np.array_equal(out["anc"], oaim.anchors(xy, basis, grid))
    assert out["S"] == 16
    for ch in CHANNELS[basis]:
        W, G = oaim.stencil_weights(xy, basis, grid, 10, ch)
        assert np.array_equal(out["lin"], G), ch
        assert np.max(np.abs(out["W"][ch] - W)) <= 1e-14 * np.max(np.abs(W)), ch
    orc = oaim.AimOracle(xy, k, wl.ETA0, basis, m, eps, near=False)
    assert np.array_equal(out["pairs"], orc._near_pairs())
    # active rows: the span of the stencils' rows
    assert out["nr"] == int(G.max() // m - G.min() // m + 1)


@pytest.mark.parametrize("order,basis", [(4, 0), (6, 1), (10, 0)])
def test_host_node_map_matches_oracle(dumper, tmp_path, order, basis):
    """Per-node order-P map (Sec. III-A read literally) at h / eps = 6.24."""
    k = wl.K0
    xy = wl.circle(0.5, 40)
    h = 2 * 0.5 * math.sin(math.pi / 40)
    eps = h / 6.24
    m = wl.grid_side_for(xy, eps, margin_cells=8)
    out = _run(dumper, str(tmp_path), xy, k, basis, m, eps, node_order=order)
    assert out["status"] == AIM_OK
    grid = oaim.Grid(m, eps)
    for ch in CHANNELS[basis]:
        W, G = oaim.stencil_weights_node(xy, basis, grid, 10, ch, order)
        assert out["S"] == W.shape[1]
        assert np.array_equal(out["lin"], G), ch
        assert np.max(np.abs(out["W"][ch] - W)) <= 1e-13 * np.max(np.abs(W)), ch
    assert out["pairs"].shape[0] == 0


def test_host_errors(dumper, tmp_path):
    t = str(tmp_path)
    xy = wl.circle(1.0, 64)
    for bad_m in (15, 2049):                                                        # m outside 16..2048
        assert _run(dumper, t, xy, wl.K0, 0, bad_m, 0.1)["status"] == AIM_E_ARG
    assert _run(dumper, t, xy, wl.K0, 0, 16, 0.1)["status"] == AIM_E_GEOM         # contour leaves the grid
    assert _run(dumper, t, wl.circle(0.4, 8), 4 * wl.K0, 0, 16, 0.1)["status"] == AIM_E_ARG   # k h > 2 pi
    assert _run(dumper, t, wl.circle(0.4, 7), wl.K0, 0, 16, 0.1)["status"] == AIM_E_ARG      # < 8 vertices
    assert _run(dumper, t, xy, wl.K0, 0, 64, 0.05, near_radius=2)["status"] == AIM_E_ARG
    assert _run(dumper, t, xy, wl.K0, 0, 64, 0.05, node_order=3)["status"] == AIM_E_ARG
    assert _run(dumper, t, wl.circle(0.5, 40), wl.K0, 0, 16, 0.07, node_order=10)["status"] == AIM_E_GEOM
    bad = xy.copy()
    bad[5] = bad[4]                                                                  # zero-length segment
    assert _run(dumper, t, bad, wl.K0, 0, 64, 0.1)["status"] == AIM_E_ARG
    bad[5, 0] = np.nan
    assert _run(dumper, t, bad, wl.K0, 0, 64, 0.1)["status"] == AIM_E_ARG
