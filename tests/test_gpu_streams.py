"""The binding orders the library's work after the caller's: a context set
up on its own stream reads inputs that the caller queued on torch's current
stream only once they are written, and the caller's later work sees the
library's outputs.  The input here is written after a 20 ms device sleep on
the current stream; without the join the library would read stale memory."""
import numpy as np
import pytest

from paper_2606_10784_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2606_10784_amd import aim  # noqa: E402


@pytest.fixture(scope="module")
def ctx_own_stream():
    xy = wl.circle(1.0, 300)
    s = torch.cuda.Stream()
    ctx = aim.Context(xy, wl.K0, wl.ETA0, 0, 64, 0.1, stream=s, max_rhs=2)
    yield ctx
    ctx.close()


def _late(src):
    """A copy of src written on the current stream after a device sleep."""
    dst = torch.zeros_like(src)
    torch.cuda._sleep(50_000_000)
    dst.copy_(src)
    return dst


def test_matvec_reads_late_input(ctx_own_stream):
    ctx = ctx_own_stream
    x = torch.from_numpy(wl.probe_vector(ctx.N, seed=4)).cuda()
    ref = ctx.matvec("S", x).clone()
    torch.cuda.synchronize()
    for _ in range(3):
        y = ctx.matvec("S", _late(x))
        assert torch.equal(y.cpu(), ref.cpu())


def test_solve_and_solver_see_late_rhs(ctx_own_stream):
    ctx = ctx_own_stream
    b = ctx.rhs_planewave(np.array([0.0, 1.0]))
    xr, _ = ctx.solve("TM", b, tol=1e-8)
    torch.cuda.synchronize()
    x, _ = ctx.solve("TM", _late(b), tol=1e-8)
    assert torch.equal(x.cpu(), xr.cpu())
    sv = aim.Solver(ctx, "TM", _late(b), x0=_late(torch.zeros_like(b)), tol=1e-8)
    while sv.poll()[0] == aim.AIM_PENDING:
        sv.step()
    assert torch.equal(sv.x.cpu(), xr.cpu())
    sv.end()
