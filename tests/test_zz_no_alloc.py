"""aim_rcs_monostatic_noalloc (the allocation-free entry point) against
aim_rcs_monostatic, through the C ABI: two calls in a row, the second with
a smaller input (fewer angles on a context with fewer unknowns), each
bitwise equal to the existing entry point's values (both run the same
kernels in the same order, only the buffers differ), and the device's free
memory unchanged across them.  A call beyond the fixed array's size is
refused on the host."""
import ctypes

import numpy as np
import pytest

from paper_2606_10784_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2606_10784_amd import aim  # noqa: E402


def _sig(lib_fn, ctx, J, phis):
    ph = np.ascontiguousarray(phis, dtype=np.float64)
    sig = np.full(ph.size, np.nan)
    st = lib_fn(ctx.handle, ph.size, ctypes.c_void_p(J.data_ptr()), ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return st, sig


def test_noalloc_rcs_equals_rcs_two_calls():
    lib = aim._lib()
    cases = [(wl.circle(1.0, 500), 8, 0), (wl.circle(0.8, 300), 3, 1)]
    ctxs = []
    for xy, R, seed in cases:
        print(f"[noalloc] N={xy.shape[0]} nrhs={R}", flush=True)
        ctx = aim.Context(xy, wl.K0, wl.ETA0, 0, 64, 0.1, max_rhs=R, max_restart=40)
        ctxs.append(ctx)
        phis = np.linspace(0.0, 2.0 * np.pi, R, endpoint=False) + 0.1 * seed
        b = ctx.rhs_planewave(phis)
        J, _ = ctx.solve("TM", b, tol=1e-8, restart=40)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        st1, s_ref = _sig(lib.aim_rcs_monostatic, ctx, J, phis)
        st2, s_new = _sig(lib.aim_rcs_monostatic_noalloc, ctx, J, phis)
        assert st1 == aim.AIM_OK and st2 == aim.AIM_OK
        assert torch.cuda.mem_get_info()[0] == free0
        print(f"[noalloc] sigma range {s_ref.min():.6g} .. {s_ref.max():.6g}")
        assert np.all(np.isfinite(s_new)) and np.array_equal(s_new, s_ref)
    # beyond the array: refused on the host, nothing launched
    big = aim.Context(wl.circle(3.0, 16384), wl.K0, wl.ETA0, 0, 128, 0.1, max_rhs=1, max_restart=0)
    ctxs.append(big)
    Jb = torch.zeros((32, 16384), dtype=torch.complex128, device="cuda")
    st, _ = _sig(lib.aim_rcs_monostatic_noalloc, big, Jb, np.zeros(32))
    assert st == aim.AIM_E_ARG
    st, s31 = _sig(lib.aim_rcs_monostatic_noalloc, big, Jb[:31].contiguous(), np.zeros(31))
    assert st == aim.AIM_OK and np.all(s31 == 0.0)
    for c in ctxs:
        c.close()
