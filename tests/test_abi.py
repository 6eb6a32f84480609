"""C-ABI library: loads and exports every function include/aim.h declares
(no compute calls; runs without a GPU)."""
import ctypes
import os

import pytest

from paper_2606_10784_amd import aim
from paper_2606_10784_amd import workloads as wl


def test_library_exports_every_declared_function():
    lib = aim._lib()
    names = aim.header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(aim.EXPORTS)


def test_strerror_and_footprint_are_host_only():
    lib = aim._lib()
    assert lib.aim_strerror(aim.AIM_E_GEOM) == b"stencil leaves the grid"
    w = wl.cylinder_large()
    fp = aim.aim_footprint_bytes(w.xy, w.k, w.eta, 0, w.m, w.eps, max_rhs=1)
    # T intermediate alone: nr x n x 16 bytes, nr <= m
    assert 1024 * 2048 * 16 < fp < 2e9
    # affine in the batch size: per-rhs buffers (intermediates, Krylov space)
    # on top of the per-context tables
    fp2 = aim.aim_footprint_bytes(w.xy, w.k, w.eta, 0, w.m, w.eps, max_rhs=2)
    fp8 = aim.aim_footprint_bytes(w.xy, w.k, w.eta, 0, w.m, w.eps, max_rhs=8)
    # (up to the 256-byte alignment of the 18 workspace buffers)
    assert fp2 > fp and abs((fp8 - fp) - 7 * (fp2 - fp)) <= 7 * 18 * 256
    # the Krylov space grows with the restart length, its Hessenberg part
    # quadratically
    f100 = aim.aim_footprint_bytes(w.xy, w.k, w.eta, 0, w.m, w.eps, restart=100)
    f1000 = aim.aim_footprint_bytes(w.xy, w.k, w.eta, 0, w.m, w.eps, restart=1000)
    assert f1000 - f100 > 900 * 16384 * 16 + (1001 ** 2 - 101 ** 2) * 16


def test_setup_rejects_bad_arguments_without_device():
    lib = aim._lib()
    h = ctypes.c_void_p()
    assert lib.aim_setup(None, ctypes.byref(h)) == aim.AIM_E_ARG
    for bad_m in (15, 2049):                                                      # m outside 16..2048
        p, _keep = aim.make_params(wl.circle(1.0, 64), wl.K0, wl.ETA0, 0, bad_m, 0.1)
        assert lib.aim_setup(ctypes.byref(p), ctypes.byref(h)) == aim.AIM_E_ARG
    p, _keep = aim.make_params(wl.circle(1.0, 64), wl.K0, wl.ETA0, 0, 16, 0.1)   # contour leaves grid
    assert lib.aim_setup(ctypes.byref(p), ctypes.byref(h)) == aim.AIM_E_GEOM
    p, _keep = aim.make_params(wl.circle(0.4, 8), 4 * wl.K0, wl.ETA0, 0, 16, 0.1)  # k h > 2 pi
    assert lib.aim_setup(ctypes.byref(p), ctypes.byref(h)) == aim.AIM_E_ARG
    p, _keep = aim.make_params(wl.circle(0.4, 7), wl.K0, wl.ETA0, 0, 16, 0.1)    # fewer than 8 vertices
    assert lib.aim_setup(ctypes.byref(p), ctypes.byref(h)) == aim.AIM_E_ARG
    for bad in (2, 61):                                                           # near_radius outside 3..m-4
        p, _keep = aim.make_params(wl.circle(1.0, 64), wl.K0, wl.ETA0, 0, 64, 0.05, near_radius=bad)
        assert lib.aim_setup(ctypes.byref(p), ctypes.byref(h)) == aim.AIM_E_ARG
    assert lib.aim_filter(None, 1.0) == aim.AIM_E_ARG
    assert lib.aim_matvec(None, 0, 1, None, None) == aim.AIM_E_ARG


def test_node_map_parameters_checked_on_the_host():
    """node_order: 0 or even in 2..12 (AIM_E_ARG), every node stencil inside
    the grid (AIM_E_GEOM); both decided before any device call."""
    lib = aim._lib()
    h = ctypes.c_void_p()
    xy = wl.circle(0.5, 40)
    for bad in (3, 14, -2):
        p, _keep = aim.make_params(xy, wl.K0, wl.ETA0, 0, 256, 0.0126, node_order=bad)
        assert lib.aim_setup(ctypes.byref(p), ctypes.byref(h)) == aim.AIM_E_ARG
    p, _keep = aim.make_params(xy, wl.K0, wl.ETA0, 0, 16, 0.07, node_order=10)   # stencils leave the grid
    assert lib.aim_setup(ctypes.byref(p), ctypes.byref(h)) == aim.AIM_E_GEOM
    fb = aim.aim_footprint_bytes(xy, wl.K0, wl.ETA0, 0, 128, 0.0126)
    fn = aim.aim_footprint_bytes(xy, wl.K0, wl.ETA0, 0, 128, 0.0126, node_order=10)
    assert fn > fb


def test_dual_space_parameters_checked_on_the_host():
    lib = aim._lib()
    h = ctypes.c_void_p()
    xy = wl.circle(0.5, 40)
    for basis, dual in ((1, 1), (0, 2)):      # dual hats only for pulses; dual is 0 or 1
        p, _keep = aim.make_params(xy, wl.K0, wl.ETA0, basis, 64, 0.05, dual=dual)
        assert lib.aim_setup(ctypes.byref(p), ctypes.byref(h)) == aim.AIM_E_ARG
    f0 = aim.aim_footprint_bytes(xy, wl.K0, wl.ETA0, 0, 64, 0.05)
    f1 = aim.aim_footprint_bytes(xy, wl.K0, wl.ETA0, 0, 64, 0.05, dual=1)
    assert f1 > f0


def test_batch_size_bounded_on_the_host():
    """max_rhs in 1..AIM_MAX_RHS (the launch grids hold one block row per rhs
    and channel), decided before any device call; the binding's constant is
    the header's."""
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "aim.h")).read()
    assert int(re.search(r"#define AIM_MAX_RHS (\d+)", hdr).group(1)) == aim.AIM_MAX_RHS
    lib = aim._lib()
    h = ctypes.c_void_p()
    xy = wl.circle(0.5, 40)
    for bad in (0, aim.AIM_MAX_RHS + 1):
        p, _keep = aim.make_params(xy, wl.K0, wl.ETA0, 0, 64, 0.05, max_rhs=bad)
        assert lib.aim_setup(ctypes.byref(p), ctypes.byref(h)) == aim.AIM_E_ARG


def test_solver_calls_checked_on_the_host():
    """The step-wise solver's host-side argument checks (no device needed)."""
    lib = aim._lib()
    assert lib.aim_strerror(aim.AIM_PENDING) == b"solve not finished"
    assert lib.aim_solver_step(None, 0) == aim.AIM_OK
    assert lib.aim_solver_step(None, 1) == aim.AIM_E_ARG
    assert lib.aim_solver_step(None, -1) == aim.AIM_E_ARG
    assert lib.aim_solver_poll(None, None) == aim.AIM_E_ARG
    assert lib.aim_solver_end(None) == aim.AIM_E_ARG
    h = ctypes.c_void_p()
    assert lib.aim_solver_begin(None, 0, 0, 1, None, None, 1e-6, 10, 10, None, 0, ctypes.byref(h)) == aim.AIM_E_ARG


def test_workspace_size_and_checks_on_the_host():
    """aim_workspace_bytes is host-only and holds the Krylov space (restart + 1
    vectors per rhs) plus the quadratic Hessenberg part; aim_setup rejects a
    misaligned or short caller workspace and max_restart outside 0..1000
    before any device call."""
    N = 16384
    w100, w400 = aim.aim_workspace_bytes(N, 1, 100), aim.aim_workspace_bytes(N, 1, 400)
    assert w100 >= 101 * N * 16 and w400 - w100 >= 300 * N * 16 + (401 ** 2 - 101 ** 2) * 16
    assert aim.aim_workspace_bytes(N, 3, 100) > 3 * w100 - 3 * 4096
    for bad in ((0, 1, 10), (N, 0, 10), (N, 1, 0), (N, 1, 1001), (N, aim.AIM_MAX_RHS + 1, 10)):
        assert aim.aim_workspace_bytes(*bad) == 0
    lib = aim._lib()
    h = ctypes.c_void_p()
    xy = wl.circle(0.5, 40)
    need = aim.aim_workspace_bytes(40, 1, 20)
    for kw in (dict(max_restart=-1), dict(max_restart=1001),
               dict(max_restart=20, workspace=256 * 1024 + 8, workspace_bytes=need),      # misaligned
               dict(max_restart=20, workspace=256 * 1024, workspace_bytes=need - 1),      # short
               dict(max_restart=0, workspace=256 * 1024, workspace_bytes=need)):          # no restart
        p, _keep = aim.make_params(xy, wl.K0, wl.ETA0, 0, 64, 0.05, **kw)
        assert lib.aim_setup(ctypes.byref(p), ctypes.byref(h)) == aim.AIM_E_ARG, kw
    # the admission estimate counts the longer of the two workspaces
    f0 = aim.aim_footprint_bytes(xy, wl.K0, wl.ETA0, 0, 64, 0.05, restart=0, max_restart=0)
    f20 = aim.aim_footprint_bytes(xy, wl.K0, wl.ETA0, 0, 64, 0.05, restart=0, max_restart=20)
    assert f20 - f0 == need
    assert aim.aim_footprint_bytes(xy, wl.K0, wl.ETA0, 0, 64, 0.05, restart=20, max_restart=20) == f20


def test_one_hip_runtime_whatever_the_import_order():
    """Loading the library before torch must not map a second HIP / HSA
    runtime: torch ships its own copies (same sonames), and two HSA runtimes
    on one device crash the process at the first device work."""
    import subprocess
    import sys
    code = ("from paper_2606_10784_amd import aim; aim._lib(); import torch; "
            "maps = open('/proc/self/maps').read(); "
            "print(len({l.split()[-1] for l in maps.splitlines() if 'amdhip64' in l}), "
            "len({l.split()[-1] for l in maps.splitlines() if 'hsa-runtime64' in l}))")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=root, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.split() == ["1", "1"], r.stdout
