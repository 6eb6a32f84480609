"""Python binding of libaim (ctypes; argument marshalling only).

Every computation runs in the HIP library; PyTorch provides device memory
and the stream.  Vectors are complex128 CUDA tensors of shape (N,) or
(nrhs, N) -- one right-hand side per row, i.e. the column-major N x nrhs
layout of the C ABI.

The names follow the C ABI (aim_setup, aim_filter, aim_matvec, aim_solve,
...); `Context` wraps the opaque handle.
"""
from __future__ import annotations

import ctypes
import math
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaim.so")

AIM_OK, AIM_E_ARG, AIM_E_GEOM, AIM_E_OOM, AIM_E_HIP, AIM_E_STATE, AIM_E_NOCONV, AIM_E_NUMERIC, AIM_PENDING = range(9)
AIM_PULSE, AIM_HAT = 0, 1
(AIM_OP_S, AIM_OP_S_ALPHA, AIM_OP_N, AIM_OP_GRAM_INV, AIM_OP_TM, AIM_OP_TE_CP, AIM_OP_TE_CP_UNF, AIM_OP_N_ALPHA,
 AIM_OP_TM_PC, AIM_OP_TM_PC_UNF, AIM_OP_TM_CP, AIM_OP_TM_CP_UNF) = range(12)
AIM_OP_GRID_FP32 = 0x100
AIM_TM_EFIE, AIM_TE_CALDERON, AIM_TE_CALDERON_UNFILTERED, AIM_TM_CALDERON, AIM_TM_CALDERON_UNFILTERED = range(5)
AIM_FP64, AIM_MIXED = 0, 1
AIM_MAX_RHS = 4096
AIM_K_ANTERP, AIM_K_ROWS_FWD, AIM_K_COLS, AIM_K_ROWS_INV, AIM_K_INTERP = range(5)

OPS = {'S': AIM_OP_S, 'S_ALPHA': AIM_OP_S_ALPHA, 'N': AIM_OP_N, 'GRAM_INV': AIM_OP_GRAM_INV,
       'TM': AIM_OP_TM, 'TE_CP': AIM_OP_TE_CP, 'TE_CP_UNF': AIM_OP_TE_CP_UNF, 'N_ALPHA': AIM_OP_N_ALPHA,
       'TM_PC': AIM_OP_TM_PC, 'TM_PC_UNF': AIM_OP_TM_PC_UNF, 'TM_CP': AIM_OP_TM_CP, 'TM_CP_UNF': AIM_OP_TM_CP_UNF}
FORMS = {'TM': AIM_TM_EFIE, 'TE_CP': AIM_TE_CALDERON, 'TE_CP_UNF': AIM_TE_CALDERON_UNFILTERED,
         'TM_CP': AIM_TM_CALDERON, 'TM_CP_UNF': AIM_TM_CALDERON_UNFILTERED}


class AimError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {_lib().aim_strerror(status).decode()} (status {status})")


class AimParams(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int32), ("xy", ctypes.POINTER(ctypes.c_double)),
                ("k", ctypes.c_double), ("eta", ctypes.c_double), ("basis", ctypes.c_int32),
                ("m", ctypes.c_int32), ("eps", ctypes.c_double), ("quad", ctypes.c_int32),
                ("near_radius", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_rhs", ctypes.c_int32), ("stream", ctypes.c_void_p), ("node_order", ctypes.c_int32),
                ("dual", ctypes.c_int32), ("max_restart", ctypes.c_int32), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


class AimCtxInfo(ctypes.Structure):
    _fields_ = [("n_unknowns", ctypes.c_int32), ("m", ctypes.c_int32), ("n_pad", ctypes.c_int32),
                ("n_active", ctypes.c_int32), ("active_rows", ctypes.c_int32), ("basis", ctypes.c_int32),
                ("near_nnz_s", ctypes.c_int64), ("near_nnz_n", ctypes.c_int64), ("k", ctypes.c_double),
                ("eps", ctypes.c_double), ("alpha", ctypes.c_double), ("device_bytes", ctypes.c_size_t),
                ("near_band", ctypes.c_int32), ("node_order", ctypes.c_int32), ("map_points", ctypes.c_int32),
                ("dual_unknowns", ctypes.c_int32)]


class AimSolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("matvecs", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("outer", ctypes.c_int32), ("converged", ctypes.c_int32), ("resid_est", ctypes.c_double),
                ("resid_true", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_LIB = None

EXPORTS = {
    "aim_footprint_bytes": (ctypes.c_size_t, [ctypes.POINTER(AimParams), ctypes.c_int32]),
    "aim_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "aim_setup": (ctypes.c_int, [ctypes.POINTER(AimParams), ctypes.POINTER(ctypes.c_void_p)]),
    "aim_filter": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "aim_filter_analytic": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "aim_matvec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "aim_rhs_planewave": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.c_double, ctypes.c_void_p]),
    "aim_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.POINTER(AimSolveInfo)]),
    "aim_rcs_monostatic": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "aim_rcs_monostatic_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "aim_fourier_spectrum": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "aim_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(AimCtxInfo)]),
    "aim_eval_green": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "aim_near_row": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int32)]),
    "aim_profile_start": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "aim_profile_stop": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "aim_solver_begin": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "aim_solver_step": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32]),
    "aim_solver_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(AimSolveInfo)]),
    "aim_solver_end": (ctypes.c_int, [ctypes.c_void_p]),
    "aim_cache_clear": (ctypes.c_size_t, []),
    "aim_cache_idle_bytes": (ctypes.c_size_t, []),
    "aim_destroy": (None, [ctypes.c_void_p]),
    "aim_strerror": (ctypes.c_char_p, [ctypes.c_int]),
}


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libaim.so not built ({LIB_PATH}); run paper_2606_10784_amd/build.py")
        # torch first: its HIP and HSA runtimes are then the ones the library
        # binds to (same sonames).  Loaded the other way round, torch maps its
        # own copies beside the system ones and the process holds two HSA
        # runtimes on one device, which crashes at the first device work.
        _torch()
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def _check(st, what):
    if st != AIM_OK:
        raise AimError(st, what)


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _join_in_stream(s):
    torch = _torch()
    cur = torch.cuda.current_stream()
    if s.cuda_stream != cur.cuda_stream:
        s.wait_stream(cur)
    return cur, s


def _join_in(ctx):
    """Orders the library's work after the caller's: the context's stream
    waits for torch's current stream, where the caller (and this binding)
    queued the inputs.  Returns (current stream, context stream)."""
    return _join_in_stream(ctx._stream_obj)


def _join_out(streams, *tensors):
    """The caller's current stream waits for the library's asynchronous
    work; tensors used on the context's stream are recorded there so the
    caching allocator does not hand their memory out before it finished."""
    cur, s = streams
    if s.cuda_stream != cur.cuda_stream:
        cur.wait_stream(s)
        for t in tensors:
            t.record_stream(s)


def _as_cols(x, N):
    """(N,) or (nrhs, N) complex128 CUDA tensor -> (tensor, nrhs)."""
    torch = _torch()
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.complex128):
        raise TypeError("expected a complex128 CUDA tensor")
    if not x.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if x.dim() == 1:
        if x.shape[0] != N:
            raise ValueError("length mismatch")
        return x, 1
    if x.dim() != 2 or x.shape[1] != N:
        raise ValueError("expected shape (nrhs, N)")
    return x, x.shape[0]


def aim_workspace_bytes(n_unknowns, nrhs, restart):
    return int(_lib().aim_workspace_bytes(int(n_unknowns), int(nrhs), int(restart)))


def _workspace(nbytes):
    """Caller-owned device memory for a Krylov workspace (a torch tensor,
    256-byte aligned)."""
    torch = _torch()
    if nbytes <= 0:
        raise ValueError("invalid workspace size")
    t = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-t.data_ptr()) % 256
    return t, t.data_ptr() + off


def make_params(xy, k, eta, basis, m, eps, quad=10, near_radius=6, precision=AIM_FP64, max_rhs=1, stream=None,
                node_order=0, dual=0, max_restart=0, workspace=None, workspace_bytes=0):
    arr = np.ascontiguousarray(np.asarray(xy, dtype=np.float64).reshape(-1, 2))
    p = AimParams()
    p.n_vertices = arr.shape[0]
    p.xy = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.k, p.eta, p.basis, p.m, p.eps = float(k), float(eta), int(basis), int(m), float(eps)
    p.quad, p.near_radius, p.precision, p.max_rhs = int(quad), int(near_radius), int(precision), int(max_rhs)
    p.stream = stream
    p.node_order = int(node_order)
    p.dual = int(dual)
    p.max_restart = int(max_restart)
    p.workspace = workspace
    p.workspace_bytes = int(workspace_bytes)
    return p, arr


def aim_footprint_bytes(xy, k, eta, basis, m, eps, quad=10, near_radius=6, precision=AIM_FP64, max_rhs=1,
                        restart=100, node_order=0, dual=0, max_restart=0):
    p, _keep = make_params(xy, k, eta, basis, m, eps, quad, near_radius, precision, max_rhs, None, node_order, dual,
                           max_restart)
    return int(_lib().aim_footprint_bytes(ctypes.byref(p), int(restart)))


class Context:
    """Owns one aim_ctx (geometry, grid tables, spectra, near field) and the
    torch tensor that holds aim_solve's Krylov workspace (GMRES restarts up to
    max_restart for max_rhs right-hand sides; max_restart = 0 leaves solves
    to step-wise solvers)."""

    def __init__(self, xy, k, eta, basis, m, eps, quad=10, near_radius=6, precision=AIM_FP64, max_rhs=1,
                 stream=None, node_order=0, dual=0, max_restart=100):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("libaim needs a HIP device")
        self._stream_obj = stream if stream is not None else torch.cuda.current_stream()
        N = np.asarray(xy).reshape(-1, 2).shape[0]
        if node_order != 0:
            max_restart = 0                     # no solves on a per-node context
        self._ws, ws_ptr, ws_bytes = None, None, 0
        if max_restart > 0:
            ws_bytes = aim_workspace_bytes(N, max_rhs, max_restart)
            self._ws, ws_ptr = _workspace(ws_bytes)
        p, self._xy = make_params(xy, k, eta, basis, m, eps, quad, near_radius, precision, max_rhs,
                                  _stream_handle(self._stream_obj), node_order, dual, max_restart, ws_ptr, ws_bytes)
        self.max_restart = max_restart
        h = ctypes.c_void_p()
        # the workspace tensor is filled on the context's stream (set-up)
        _join_in_stream(self._stream_obj)
        _check(_lib().aim_setup(ctypes.byref(p), ctypes.byref(h)), "aim_setup")
        if self._ws is not None and self._stream_obj.cuda_stream != torch.cuda.current_stream().cuda_stream:
            self._ws.record_stream(self._stream_obj)
        self._h = h
        self.N = p.n_vertices
        self.basis = basis
        self.max_rhs = max_rhs
        self.precision = precision
        self._solvers = weakref.WeakSet()      # live step-wise solvers on this context

    @property
    def handle(self):
        return self._h

    def close(self):
        """Ends the context's live solvers (the library requires it), then
        destroys the context."""
        if getattr(self, "_h", None):
            for sv in list(getattr(self, "_solvers", ())):
                sv.end()
            _lib().aim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        inf = AimCtxInfo()
        _check(_lib().aim_get_info(self._h, ctypes.byref(inf)), "aim_get_info")
        return {f: getattr(inf, f) for f, _ in inf._fields_}

    def filter(self, alpha):
        return aim_filter(self, alpha)

    def filter_analytic(self, alpha):
        return aim_filter_analytic(self, alpha)

    def matvec(self, op, x, y=None):
        return aim_matvec(self, op, x, y)

    def solve(self, form, b, x0=None, tol=1e-6, maxit=5000, restart=100, precision=AIM_FP64):
        return aim_solve(self, form, b, x0, tol, maxit, restart, precision)

    def rhs_planewave(self, phis, amp=1.0):
        return aim_rhs_planewave(self, phis, amp)

    def rcs(self, J, phis):
        return aim_rcs_monostatic(self, J, phis)

    def eval_green(self, R):
        return aim_eval_green(self, R)

    def fourier_spectrum(self, op, nus):
        return aim_fourier_spectrum(self, op, nus)

    def near_row(self, op, row):
        return aim_near_row(self, op, row)


def aim_setup(xy, k, eta, basis, m, eps, **kw):
    return Context(xy, k, eta, basis, m, eps, **kw)


def aim_filter(ctx, alpha):
    _check(_lib().aim_filter(ctx.handle, float(alpha)), "aim_filter")


def aim_filter_analytic(ctx, alpha):
    _check(_lib().aim_filter_analytic(ctx.handle, float(alpha)), "aim_filter_analytic")


def aim_matvec(ctx, op, x, y=None):
    torch = _torch()
    opc = OPS[op] if isinstance(op, str) else int(op)
    x, nrhs = _as_cols(x, ctx.N)
    if y is None:
        y = torch.empty_like(x)
    _as_cols(y, ctx.N)
    ss = _join_in(ctx)
    st = _lib().aim_matvec(ctx.handle, opc, nrhs, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()))
    _join_out(ss, x, y)
    _check(st, "aim_matvec")
    return y


def aim_rhs_planewave(ctx, phis, amp=1.0):
    torch = _torch()
    ph = np.ascontiguousarray(np.atleast_1d(np.asarray(phis, dtype=np.float64)))
    b = torch.empty((ph.size, ctx.N), dtype=torch.complex128, device="cuda")
    ss = _join_in(ctx)
    st = _lib().aim_rhs_planewave(ctx.handle, ph.size, ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  float(amp), ctypes.c_void_p(b.data_ptr()))
    _join_out(ss, b)
    _check(st, "aim_rhs_planewave")
    return b[0] if np.ndim(phis) == 0 else b


def aim_solve(ctx, form, b, x0=None, tol=1e-6, maxit=5000, restart=100, precision=AIM_FP64):
    """Returns (x, [info dict per rhs]); raises AimError unless converged."""
    torch = _torch()
    fc = FORMS[form] if isinstance(form, str) else int(form)
    b, nrhs = _as_cols(b, ctx.N)
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    infos = (AimSolveInfo * nrhs)()
    ss = _join_in(ctx)                      # x0 is queued on the current stream
    st = _lib().aim_solve(ctx.handle, fc, int(precision), nrhs, ctypes.c_void_p(b.data_ptr()),
                          ctypes.c_void_p(x.data_ptr()), float(tol), int(maxit), int(restart), infos)
    _join_out(ss, b, x)
    out = [infos[i].as_dict() for i in range(nrhs)]
    if st not in (AIM_OK, AIM_E_NOCONV):
        raise AimError(st, "aim_solve")
    if st == AIM_E_NOCONV:
        for d in out:
            d['status'] = 'noconv'
    return x, out


class Solver:
    """A step-wise solve (aim_solver_begin): step() advances it by one Arnoldi
    step, poll() reports (status, [info per rhs]).  Keeps b and the context
    alive until end()."""

    def __init__(self, ctx, form, b, x0=None, tol=1e-6, maxit=5000, restart=100, precision=AIM_FP64):
        torch = _torch()
        fc = FORMS[form] if isinstance(form, str) else int(form)
        self.ctx = ctx
        self.b, self.nrhs = _as_cols(b, ctx.N)
        self.x = torch.zeros_like(self.b) if x0 is None else x0.clone()
        # the solver's Krylov workspace: caller-owned device memory
        ws_bytes = aim_workspace_bytes(ctx.N, self.nrhs, restart) if 1 <= int(restart) <= 1000 else 0
        self._ws, ws_ptr = _workspace(ws_bytes) if ws_bytes > 0 else (None, None)
        h = ctypes.c_void_p()
        ss = _join_in(ctx)                  # b and x0 are queued on the current stream
        st = _lib().aim_solver_begin(ctx.handle, fc, int(precision), self.nrhs, ctypes.c_void_p(self.b.data_ptr()),
                                     ctypes.c_void_p(self.x.data_ptr()), float(tol), int(maxit), int(restart),
                                     ctypes.c_void_p(ws_ptr), ctypes.c_size_t(ws_bytes), ctypes.byref(h))
        _join_out(ss, self.b, self.x, *([self._ws] if self._ws is not None else []))
        _check(st, "aim_solver_begin")
        self.handle = h.value
        ctx._solvers.add(self)

    def step(self):
        return aim_solver_step([self])

    def poll(self):
        infos = (AimSolveInfo * self.nrhs)()
        st = _lib().aim_solver_poll(self.handle, infos)
        return st, [infos[i].as_dict() for i in range(self.nrhs)]

    def end(self):
        if self.handle:
            st = _lib().aim_solver_end(self.handle)
            self.handle = None
            _check(st, "aim_solver_end")

    def __del__(self):
        try:
            self.end()
        except Exception:
            pass


def aim_solver_step(solvers):
    """One Arnoldi step for each unfinished solver of the group; returns the
    status (the first error any solver met)."""
    arr = (ctypes.c_void_p * len(solvers))(*[s.handle for s in solvers])
    return _lib().aim_solver_step(arr, len(solvers))


def aim_rcs_monostatic(ctx, J, phis):
    J, nrhs = _as_cols(J, ctx.N)
    ph = np.ascontiguousarray(np.atleast_1d(np.asarray(phis, dtype=np.float64)))
    if ph.size != nrhs:
        raise ValueError("one angle per current column")
    sig = np.zeros(nrhs)
    _join_in(ctx)                            # synchronous: nothing to join afterwards
    _check(_lib().aim_rcs_monostatic(ctx.handle, nrhs, ctypes.c_void_p(J.data_ptr()),
                                     ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "aim_rcs_monostatic")
    return sig


def aim_rcs_monostatic_noalloc(ctx, J, phis):
    """aim_rcs_monostatic with every buffer of the call in the library's
    fixed per-device array (no device allocation; see include/aim.h)."""
    J, nrhs = _as_cols(J, ctx.N)
    ph = np.ascontiguousarray(np.atleast_1d(np.asarray(phis, dtype=np.float64)))
    if ph.size != nrhs:
        raise ValueError("one angle per current column")
    sig = np.zeros(nrhs)
    _join_in(ctx)
    _check(_lib().aim_rcs_monostatic_noalloc(ctx.handle, nrhs, ctypes.c_void_p(J.data_ptr()),
                                             ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "aim_rcs_monostatic_noalloc")
    return sig


def aim_fourier_spectrum(ctx, op, nus):
    """lambda_nu of `op` in the contour's Fourier basis (see include/aim.h)."""
    op = OPS[op] if isinstance(op, str) else int(op)
    nu = np.ascontiguousarray(np.atleast_1d(np.asarray(nus)).astype(np.int32))
    out = np.zeros(2 * nu.size)
    _check(_lib().aim_fourier_spectrum(ctx.handle, op, nu.size, nu.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "aim_fourier_spectrum")
    return out[0::2] + 1j * out[1::2]


def aim_eval_green(ctx, R):
    torch = _torch()
    R = R.contiguous()
    out = torch.empty(R.shape, dtype=torch.complex128, device="cuda")
    ss = _join_in(ctx)
    st = _lib().aim_eval_green(ctx.handle, R.numel(), ctypes.c_void_p(R.data_ptr()), ctypes.c_void_p(out.data_ptr()))
    _join_out(ss, R, out)
    _check(st, "aim_eval_green")
    return out


def aim_near_row(ctx, op, row):
    opc = OPS[op] if isinstance(op, str) else int(op)
    n = ctypes.c_int32()
    _check(_lib().aim_near_row(ctx.handle, opc, int(row), 0, None, None, ctypes.byref(n)), "aim_near_row")
    cols = np.zeros(n.value, dtype=np.int32)
    vals = np.zeros(2 * n.value, dtype=np.float64)
    _check(_lib().aim_near_row(ctx.handle, opc, int(row), n.value,
                               cols.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               vals.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(n)),
           "aim_near_row")
    return cols, vals[0::2] + 1j * vals[1::2]


def aim_profile_start(ctx, kernel, every=1, max_samples=4096):
    _check(_lib().aim_profile_start(ctx.handle, int(kernel), int(every), int(max_samples)), "aim_profile_start")


def aim_profile_stop(ctx):
    """(mean ms of the sampled launches, samples, launches seen)"""
    ms = ctypes.c_double()
    ns = ctypes.c_int64()
    nl = ctypes.c_int64()
    _check(_lib().aim_profile_stop(ctx.handle, ctypes.byref(ms), ctypes.byref(ns), ctypes.byref(nl)),
           "aim_profile_stop")
    return ms.value, ns.value, nl.value


def aim_cache_clear():
    return int(_lib().aim_cache_clear())


def aim_cache_idle_bytes():
    return int(_lib().aim_cache_idle_bytes())


def header_functions(path=None):
    """Function names declared in include/aim.h (for export checks)."""
    import re
    path = path or os.path.join(os.path.dirname(_HERE), "include", "aim.h")
    txt = open(path).read()
    decl = r"^(?:aim_status|size_t|void|const\s+char\s*\*)\s*(aim_[a-z_]+)\s*\("
    return sorted(set(re.findall(decl, txt, flags=re.M)))
