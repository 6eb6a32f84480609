"""The solve paths allocate no device memory: with the context's Krylov
workspace bound at set-up and a caller-owned workspace for the step-wise
solver, aim_rhs_planewave, aim_solve, aim_solver_begin / step / poll / end
and aim_rcs_monostatic leave the device's free memory (hipMemGetInfo)
unchanged (after one warm-up pass).  The calls go straight through the C ABI on buffers allocated
beforehand, so the caching allocator does not take part."""
import ctypes

import numpy as np
import pytest

from paper_2606_10784_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2606_10784_amd import aim  # noqa: E402


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("precision", [aim.AIM_FP64, aim.AIM_MIXED])
def test_free_memory_flat_across_solve_paths(precision):
    N, R, restart = 400, 3, 30
    lib = aim._lib()
    ctx = aim.Context(wl.circle(1.0, N), wl.K0, wl.ETA0, 0, 64, 0.1, max_rhs=R, precision=aim.AIM_MIXED,
                      max_restart=restart)
    phis = np.ascontiguousarray(np.array([0.0, 0.7, 2.1]))
    php = phis.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    b = torch.empty((R, N), dtype=torch.complex128, device="cuda")
    x = torch.zeros_like(b)
    xs = torch.zeros_like(b)
    ws_bytes = aim.aim_workspace_bytes(N, R, restart)
    ws, ws_ptr = aim._workspace(ws_bytes)
    infos = (aim.AimSolveInfo * R)()
    sig = np.zeros(R)
    sgp = sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    h = ctypes.c_void_p()
    torch.cuda.synchronize()
    free0 = None
    seen = []
    for it in range(3):
        if it == 1:       # after one warm-up pass (runtime code loading)
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            seen = []
        assert lib.aim_rhs_planewave(ctx.handle, R, php, 1.0, _p(b)) == aim.AIM_OK
        seen.append(torch.cuda.mem_get_info()[0])
        x.zero_()
        torch.cuda.synchronize()
        st = lib.aim_solve(ctx.handle, aim.AIM_TM_EFIE, precision, R, _p(b), _p(x), 1e-8, 2000, restart, infos)
        assert st == aim.AIM_OK
        seen.append(torch.cuda.mem_get_info()[0])
        xs.zero_()
        torch.cuda.synchronize()
        assert lib.aim_solver_begin(ctx.handle, aim.AIM_TM_EFIE, precision, R, _p(b), _p(xs), 1e-8, 2000, restart,
                                    ctypes.c_void_p(ws_ptr), ctypes.c_size_t(ws_bytes), ctypes.byref(h)) == aim.AIM_OK
        while lib.aim_solver_poll(h, None) == aim.AIM_PENDING:
            assert lib.aim_solver_step(ctypes.byref(h), 1) == aim.AIM_OK
        seen.append(torch.cuda.mem_get_info()[0])
        assert lib.aim_solver_end(h) == aim.AIM_OK
        assert lib.aim_rcs_monostatic(ctx.handle, R, _p(x), php, sgp) == aim.AIM_OK
        seen.append(torch.cuda.mem_get_info()[0])
        torch.cuda.synchronize()
        # the step-wise solve is aim_solve's, bit for bit
        assert torch.equal(x, xs)
    print("free bytes before", free0, "after each call", sorted(set(seen)))
    assert all(f == free0 for f in seen)
    assert np.all(sig > 0)
    ctx.close()
