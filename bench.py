#!/usr/bin/env python3
"""Benchmark of the filtered-AIM EFIE hot path on one MI355X.

One step = one full TM-EFIE GMRES solve (plain FP64, restart 400)
to a 1e-6 relative residual on the PEC cylinder with ka = 200
(N = 16384 pulse segments, AIM grid 1024 x 1024 at lambda/15 padded to
2048 x 2048, half of the spectrum kept by the filter), plane wave at 0 deg.
Inputs (geometry, right-hand side, spectra, near field) are resident in HBM
before the timed region.  `value` is AIM matvecs/s over the timed solves;
solves/s, solve latency percentiles, matvec-only throughput and the
mixed-precision (FP32 grid + FP64 refinement) solve are reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cylinder_ka200",
                    choices=["cylinder_ka200", "cylinder_ka2pi", "star_te", "cylinder_ka200_360rhs", "spectrum",
                             "tm_calderon"],
                    help="cylinder_ka200: the benchmark line; the others are separate measurements")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--restart", type=int, default=400)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="with --mode matvec: also run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--matvecs", type=int, default=50, help="matvec-only timing loop length")
    ap.add_argument("--mode", default="solve", choices=["solve", "matvec"],
                    help="matvec: set-up plus --matvecs FP64 matvecs only (short runs for counters)")
    ap.add_argument("--serve-requests", type=int, default=24,
                    help="requests of the serving stream (0: skip the serving measurement)")
    ap.add_argument("--serve-log-dir", default=None, help="directory of the per-request JSONL logs")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the star TE Calderon and 360-incidence measurements of the default line")
    return ap.parse_args()


PROF_EVERY = 16
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic_cols_conv.json")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current source of the FFT kernels."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
        src = os.path.join(os.path.dirname(TRAFFIC_FILE), "..", "paper_2606_10784_amd", "csrc", "fft.hip")
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except Exception:
        return None
    if rec.get("kernel") != kernel or rec.get("source_sha256") != sha:
        return None
    return rec.get("bytes_per_launch")


def serving(n_req, slots=4, budget=96 << 30, log_dir=None):
    """The serving stream through three schedulers: iteration-level batching
    with grouped column passes (StepServer, aim_solver_step over all running
    requests: requests that share a grid-kernel spectrum run their column
    pass as one launch), the same without grouping (one aim_solver_step call
    per request) and a thread per request (Server).  Each: closed-loop
    capacity, then Poisson arrivals at fractions of that capacity (0.5, 0.7,
    0.9 for the grouped scheduler, 0.7 for the others).  Every run writes a
    JSONL line per request to log_dir."""
    from paper_2606_10784_amd import serve
    from paper_2606_10784_amd import workloads as wl
    import tempfile
    log_dir = log_dir or tempfile.gettempdir()

    def done(what, summ):
        print(f"[bench] serving {what}: {summ['completed']}/{summ['requests']} in {summ['wall_s']:.1f} s, "
              f"p50 {summ['latency_s']['p50']:.3f} s p99 {summ['latency_s']['p99']:.3f} s",
              file=sys.stderr, flush=True)
        return summ

    def run(name, make, rate):
        path = os.path.join(log_dir, f"serve_{name}.jsonl")
        srv = make(path)
        reqs = wl.serving_stream(n_req, rate=rate)
        summ = serve.summarize(srv.run(reqs, realtime=rate > 0), srv.wall)
        summ["log"] = path
        if hasattr(srv, "rounds"):
            summ["rounds"] = srv.rounds
        return done(name, summ)

    out = {"stream": f"{n_req} TM requests, random stars ka~logU[10,400], 1-16 rhs, FP64/mixed, "
                     f"HBM budget {budget >> 30} GiB"}
    grp = serve.GpuStepEngine(restart=1000, group=True)
    mk = lambda path: serve.StepServer(grp, hbm_budget=budget, slots=2 * slots, log_path=path)
    cap = run("steps_grouped_closed", mk, 0.0)
    out["steps_grouped"] = {"slots": 2 * slots, "closed_loop": cap}
    for f in (0.5, 0.7, 0.9):
        rate = f * cap["requests_per_s"]
        out["steps_grouped"][f"poisson_{f}"] = dict(run(f"steps_grouped_poisson_{f}", mk, rate), rate_per_s=rate)
    solo = serve.GpuStepEngine(restart=1000, group=False)
    mk = lambda path: serve.StepServer(solo, hbm_budget=budget, slots=2 * slots, log_path=path)
    cap2 = run("steps_ungrouped_closed", mk, 0.0)
    rate = 0.7 * cap2["requests_per_s"]
    out["steps_ungrouped"] = {"slots": 2 * slots, "closed_loop": cap2,
                              "poisson_0.7": dict(run("steps_ungrouped_poisson_0.7", mk, rate), rate_per_s=rate)}
    exe = serve.GpuExecutor(restart=1000)
    mk = lambda path: serve.Server(exe, hbm_budget=budget, slots=slots, log_path=path)
    cap3 = run("threads_closed", mk, 0.0)
    rate = 0.7 * cap3["requests_per_s"]
    out["threads"] = {"slots": slots, "closed_loop": cap3,
                      "poisson_0.7": dict(run("threads_poisson_0.7", mk, rate), rate_per_s=rate)}
    return out


def kernel_bytes(kid, inf, nch=1, nrhs=1, b=16):
    """Algorithmic HBM bytes of one launch of pipeline kernel `kid`."""
    N, n, nr, nact = inf["n_unknowns"], inf["n_pad"], inf["active_rows"], inf["n_active"]
    H = n // 2 + 1
    nnz = inf["near_nnz_s"]
    p = nch * nrhs
    if kid == 0:   # anterpolation: x, transposed stencils, U
        return N * 16 * nrhs + N * 16 * (4 + 8) + (nact + 1) * 4 + p * nact * b
    if kid == 1:   # row FFTs: U in, T out
        return p * nact * b + nact * 4 + p * nr * n * b
    if kid == 2:   # column FFT . spectrum . inverse: T in and out, quarter spectrum once
        return 2 * p * nr * n * b + H * H * b
    if kid == 3:   # inverse row FFTs: T in, V out
        return p * nr * n * b + p * nact * b + nact * 4
    if kid == 4:   # interpolation + near field: stencils, V, near CSR, x, y
        return N * 16 * (8 + 4) + p * nact * b + nnz * (16 + 4) + (N + 1) * 4 + 2 * N * 16 * nrhs
    raise ValueError(kid)


def kernel_flops(kid, inf):
    n, nr = inf["n_pad"], inf["active_rows"]
    lg = math.log2(n)
    if kid == 1 or kid == 3:
        return nr * 5 * n * lg
    if kid == 2:
        return n * (2 * 5 * n * lg + 6 * n)
    return 0.0


def _host_threads():
    """Threads the oracle's numpy/scipy calls use."""
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(w, sample_every=64, reps=2):
    """Oracle AIM matvec on the host: full direct-Toeplitz grid product plus
    the near-field product of every `sample_every`-th row (scaled)."""
    import numpy as np
    from oracle import aim as oaim
    from paper_2606_10784_amd import workloads as wl
    threads = _host_threads()
    A = oaim.AimOracle(w.xy, w.k, w.eta, w.basis, w.m, w.eps, alpha=w.alpha, near=False)
    rows = np.arange(0, w.n_unknowns, sample_every)
    A.near_pairs = A._near_pairs()
    A._build_near(("S",), rows)
    x = wl.probe_vector(w.n_unknowns, seed=1)
    t0 = time.perf_counter()
    for _ in range(reps):
        A.op_S(x, near=False)
    t_grid = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        A.near_apply("S", x)
    t_near = (time.perf_counter() - t0) / reps * (w.n_unknowns / rows.size)
    per = t_grid + t_near
    return {"value": 1.0 / per, "unit": "AIM matvecs/s", "cores": int(threads), "kind": "oracle",
            "sample": (f"{reps} oracle S_AIM matvecs at {w.name}: direct Toeplitz sum over all "
                       f"{A.act.size} active grid points (measured) + near-field product of "
                       f"{rows.size} of {w.n_unknowns} rows scaled to all rows; {per:.2f} s per matvec")}


def alpha_sweep(ctx, b, alphas, tol, maxit=3000, restart=300):
    """Filtered TE Calderon solves (G^-1 S^alpha G^-1 N, FP64) over cutoffs:
    iterations to tol (or maxit), the unpreconditioned residual
    ||N j - b|| / ||b|| and the current's distance from the unfiltered
    solution (G^-1 S G^-1 N, near field included)."""
    import torch
    from paper_2606_10784_amd import aim
    t0 = time.perf_counter()
    xu, iu = ctx.solve("TE_CP_UNF", b, tol=tol, restart=restart, maxit=maxit)
    t_unf = time.perf_counter() - t0
    nb = float(torch.linalg.norm(b))
    ru = float(torch.linalg.norm(ctx.matvec("N", xu) - b)) / nb
    out = {"unfiltered": {"iterations": iu[0]["iterations"], "converged": iu[0]["converged"], "seconds": t_unf,
                          "resid_unpreconditioned": ru}, "filtered": []}
    for a in alphas:
        ctx.filter(a)
        t0 = time.perf_counter()
        x, info = ctx.solve("TE_CP", b, tol=tol, restart=restart, maxit=maxit)
        dt = time.perf_counter() - t0
        rn = float(torch.linalg.norm(ctx.matvec("N", x) - b)) / nb
        dx = float(torch.linalg.norm(x - xu) / torch.linalg.norm(xu))
        out["filtered"].append({"alpha": a, "alpha_eps_over_pi": a * ctx_eps(ctx) / math.pi,
                                "iterations": info[0]["iterations"], "converged": info[0]["converged"],
                                "resid_preconditioned": info[0]["resid_true"], "resid_unpreconditioned": rn,
                                "rel_diff_vs_unfiltered": dx, "seconds": dt})
        print(f"[bench] TE_CP alpha={a:.1f} its={info[0]['iterations']} conv={info[0]['converged']} "
              f"unprec={rn:.2e} diff={dx:.2e} {dt:.2f}s", file=sys.stderr, flush=True)
    return out


def ctx_eps(ctx):
    return ctx.info()["eps"]


def star_alphas(eps):
    """Cutoffs from the 50 %-bin one (the configurations' filter) to the
    largest grid frequency sqrt(2) pi / eps (every bin kept)."""
    a50 = math.sqrt(2.0 * math.pi) / eps
    return [a50, 0.9 * math.pi / eps, math.pi / eps, 1.2 * math.pi / eps, math.sqrt(2.0) * math.pi / eps]


def c2_star(args, sweep=True):
    """Star N = 65536 hats, grid 2048 -> 4096 at lambda/30: Calderon-
    preconditioned TE solves, unfiltered (FP64 and mixed) and filtered over
    the cutoff sweep; operator timings."""
    import torch
    from paper_2606_10784_amd import aim
    from paper_2606_10784_amd import workloads as wl
    w = wl.star_large()
    t0 = time.perf_counter()
    ctx = aim.Context(w.xy, w.k, w.eta, w.basis, w.m, w.eps, precision=aim.AIM_MIXED, max_rhs=1, max_restart=300)
    ctx.filter(w.alpha)
    torch.cuda.synchronize()
    inf = ctx.info()
    out = {"workload": w.name, "N": inf["n_unknowns"], "grid": f"{w.m}x{w.m} pad {inf['n_pad']}",
           "near_nnz": inf["near_nnz_s"], "alpha_50pct": w.alpha, "setup_s": time.perf_counter() - t0, "solves": {}}
    b = ctx.rhs_planewave(0.0)
    for lab, op in (("N", "N"), ("S_ALPHA", "S_ALPHA"), ("TE_CP", "TE_CP"), ("TE_CP_UNF", "TE_CP_UNF")):
        for prec in (0, aim.AIM_OP_GRID_FP32):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            y = ctx.matvec(aim.OPS[op] | prec, b)
            e0.record()
            for _ in range(10):
                ctx.matvec(aim.OPS[op] | prec, b, y)
            e1.record()
            torch.cuda.synchronize()
            out.setdefault("matvec_ms", {})[lab + ("_fp32grid" if prec else "")] = e0.elapsed_time(e1) / 10
    for prec in (aim.AIM_FP64, aim.AIM_MIXED):
        t0 = time.perf_counter()
        x, info = ctx.solve("TE_CP_UNF", b, tol=args.tol, restart=300, maxit=3000, precision=prec)
        dt = time.perf_counter() - t0
        out["solves"][f"TE_CP_UNF_{'fp64' if prec == 0 else 'mixed'}"] = {
            "seconds": dt, "iterations": info[0]["iterations"], "outer": info[0]["outer"],
            "converged": info[0]["converged"], "resid_true": info[0]["resid_true"]}
        print(f"[bench] TE_CP_UNF prec={prec} its={info[0]['iterations']} {dt:.2f}s", file=sys.stderr, flush=True)
    if sweep:
        out["alpha_sweep"] = alpha_sweep(ctx, b, star_alphas(w.eps), args.tol)
    ctx.close()
    return out


def star_te(args):
    print(json.dumps(c2_star(args)), flush=True)


def tm_calderon(args):
    """Cylinder ka = 200 (N = 16384 pulses) with its dual hat space (32768
    refined hats): the TM EFIE against the TM Calderon forms, unfiltered and
    with N^alpha at the 50 % cutoff; operator timings and solves."""
    import numpy as np
    import torch
    from paper_2606_10784_amd import aim
    from paper_2606_10784_amd import workloads as wl
    w = wl.cylinder_large()
    t0 = time.perf_counter()
    ctx = aim.Context(w.xy, w.k, w.eta, w.basis, w.m, w.eps, precision=aim.AIM_MIXED, max_rhs=1, dual=1,
                      max_restart=args.restart)
    ctx.filter(w.alpha)
    torch.cuda.synchronize()
    inf = ctx.info()
    out = {"workload": w.name + "_tm_calderon", "N": inf["n_unknowns"], "dual_unknowns": inf["dual_unknowns"],
           "grid": f"{w.m}x{w.m} pad {inf['n_pad']}", "alpha": w.alpha, "setup_s": time.perf_counter() - t0,
           "matvec_ms": {}, "solves": {}}
    b = ctx.rhs_planewave(0.0)
    for op in ("TM", "TM_PC", "TM_PC_UNF", "TM_CP", "TM_CP_UNF"):
        y = ctx.matvec(op, b)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            ctx.matvec(op, b, y)
        e1.record()
        torch.cuda.synchronize()
        out["matvec_ms"][op] = e0.elapsed_time(e1) / 20
    ref = None
    for form in ("TM", "TM_CP_UNF", "TM_CP"):
        for prec in (aim.AIM_FP64, aim.AIM_MIXED):
            ctx.solve(form, b, tol=args.tol, restart=args.restart, maxit=3000, precision=prec)   # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = ctx.solve(form, b, tol=args.tol, restart=args.restart, maxit=3000, precision=prec)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            xs = x.cpu().numpy()
            if ref is None:
                ref = xs
            key = f"{form}_{'fp64' if prec == aim.AIM_FP64 else 'mixed'}"
            out["solves"][key] = {"seconds": dt, "iterations": info[0]["iterations"], "outer": info[0]["outer"],
                                  "converged": info[0]["converged"], "resid_true": info[0]["resid_true"],
                                  "rel_diff_vs_tm_efie": float(np.linalg.norm(xs - ref) / np.linalg.norm(ref))}
            print(f"[bench] {key} its={info[0]['iterations']} {dt * 1e3:.1f} ms", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)
    ctx.close()


def mie_backscatter_tm(k, a):
    """Monostatic scattering width of a PEC circular cylinder, TM (the Mie
    series): sigma = (4 / k) |sum_n (-1)^n J_n(ka) / H_n^(2)(ka)|^2."""
    from scipy import special
    x = k * a
    nmax = int(x + 10 * x ** (1.0 / 3.0) + 20)
    s = 0.0 + 0.0j
    for n in range(-nmax, nmax + 1):
        m = abs(n)
        s += (-1) ** n * special.jv(m, x) / (special.jv(m, x) - 1j * special.yv(m, x))
    return 4.0 / k * abs(s) ** 2


def c3_batched(args):
    """Cylinder ka = 200 with 360 plane waves (1 degree steps) in one batched
    solve: FP32-grid GMRES inside FP64 refinement and plain FP64, monostatic
    RCS against the Mie series."""
    import numpy as np
    import torch
    from paper_2606_10784_amd import aim
    from paper_2606_10784_amd import workloads as wl
    w = wl.cylinder_large()
    R = 360
    phis = np.deg2rad(np.arange(R))
    ctx = aim.Context(w.xy, w.k, w.eta, w.basis, w.m, w.eps, precision=aim.AIM_MIXED, max_rhs=R,
                      max_restart=args.restart)
    B = ctx.rhs_planewave(phis)
    out = {"workload": w.name + "_360rhs", "nrhs": R, "restart": args.restart, "solves": {}}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for prec, lab in ((0, "fp64"), (aim.AIM_OP_GRID_FP32, "fp32grid")):
        Y = ctx.matvec(aim.AIM_OP_TM | prec, B)
        e0.record()
        for _ in range(3):
            ctx.matvec(aim.AIM_OP_TM | prec, B, Y)
        e1.record()
        torch.cuda.synchronize()
        out[f"batched_matvec_ms_{lab}"] = e0.elapsed_time(e1) / 3
    sig_mie = mie_backscatter_tm(w.k, 200.0 / w.k)
    for prec, lab in ((aim.AIM_MIXED, "mixed"), (aim.AIM_FP64, "fp64")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, infos = ctx.solve("TM", B, tol=args.tol, restart=args.restart, precision=prec)
        dt = time.perf_counter() - t0
        sig = ctx.rcs(X, phis)
        out["solves"][lab] = {"seconds": dt, "rhs_solves_per_s": R / dt,
                              "iterations_max": max(d["iterations"] for d in infos),
                              "converged": sum(d["converged"] for d in infos),
                              "resid_true_max": max(d["resid_true"] for d in infos),
                              "rcs_min": float(sig.min()), "rcs_max": float(sig.max()),
                              "rcs_max_rel_dev_vs_mie": float(np.max(np.abs(sig - sig_mie)) / sig_mie)}
        print(f"[bench] 360 rhs {lab}: {dt:.2f}s", file=sys.stderr, flush=True)
    out["mixed_speedup_vs_fp64"] = out["solves"]["fp64"]["seconds"] / out["solves"]["mixed"]["seconds"]
    ctx.close()
    return out


def batched_360(args):
    print(json.dumps(c3_batched(args)), flush=True)


def spectrum(args):
    """The paper's Sec. IV spectra at its parameters: every Fourier mode
    0..N/2 of S and S^alpha (pulses, Fig. 2), of G^-1 S G^-1 N and
    G^-1 S^alpha G^-1 N (hats, Fig. 3) and of the TM Calderon products (pulses
    with the dual hats) through aim_fourier_spectrum, modes/s, and the
    oracle's quotient for a few modes timed on the host."""
    import numpy as np
    import torch
    from paper_2606_10784_amd import aim
    from paper_2606_10784_amd import workloads as wl
    out = {"workload": "paper_circle_spectrum", "spectra": {}}
    nmax = None
    for basis, ops, dual in ((wl.PULSE, ("S", "S_ALPHA"), 0), (wl.HAT, ("TE_CP_UNF", "TE_CP"), 0),
                             (wl.PULSE, ("TM_CP_UNF", "TM_CP"), 1)):
        w = wl.paper_circle(basis)
        N = w.n_unknowns
        nus = np.arange(0, N // 2 + 1)
        nmax = N // 2
        t0 = time.perf_counter()
        ctx = aim.Context(w.xy, w.k, w.eta, basis, w.m, w.eps, quad=w.quad, max_rhs=64, dual=dual, max_restart=0)
        ctx.filter(w.alpha)
        t_setup = time.perf_counter() - t0
        for op in ops:
            ctx.fourier_spectrum(op, nus[:8])   # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lam = ctx.fourier_spectrum(op, nus)
            dt = time.perf_counter() - t0
            mag = np.abs(lam)
            aa = w.alpha * 1.0   # radius 1 m
            sel = lambda lo, hi: mag[(nus >= lo) & (nus <= hi)]
            out["spectra"][op] = {
                "N": N, "modes": int(nus.size), "seconds": dt, "modes_per_s": nus.size / dt,
                "abs_lambda_at": {str(int(v)): float(mag[int(v)]) for v in (0, round(aa / 2), round(aa), nmax)},
                "max_abs_past_1.2_alpha_a_over_abs_lambda0": float(sel(1.2 * aa, nmax).max() / mag[0]),
                "setup_s": t_setup}
            print(f"[bench] spectrum {op}: {nus.size} modes in {dt*1e3:.1f} ms", file=sys.stderr, flush=True)
        ctx.close()
    # the paper's own map (per-node order-10 Lambda) for S^alpha
    w = wl.paper_circle(wl.PULSE)
    N = w.n_unknowns
    nus = np.arange(0, N // 2 + 1)
    t0 = time.perf_counter()
    ctx = aim.Context(w.xy, w.k, w.eta, wl.PULSE, w.m, w.eps, quad=w.quad, max_rhs=64, node_order=10,
                      max_restart=0)
    ctx.filter(w.alpha)
    t_setup = time.perf_counter() - t0
    inf = ctx.info()
    ctx.fourier_spectrum("S_ALPHA", nus[:8])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam = ctx.fourier_spectrum("S_ALPHA", nus)
    dt = time.perf_counter() - t0
    out["spectra"]["S_ALPHA_node_order_10"] = {
        "N": N, "modes": int(nus.size), "seconds": dt, "modes_per_s": nus.size / dt, "setup_s": t_setup,
        "map_points": inf["map_points"], "n_active": inf["n_active"],
        "max_abs_past_1.2_alpha_a_over_abs_lambda0": float(np.abs(lam[nus >= 1.2 * w.alpha]).max() / abs(lam[0]))}
    print(f"[bench] spectrum S_ALPHA per-node P=10: {nus.size} modes in {dt*1e3:.1f} ms", file=sys.stderr, flush=True)
    ctx.close()
    if not args.no_cpu_baseline:
        # the oracle's quotient of S^alpha for 4 modes on the host
        from oracle import aim as oaim
        w = wl.paper_circle(wl.PULSE)
        N = w.n_unknowns
        # n: the library's FFT length for the 600-point side (its numerical filter's DFT bins)
        A = oaim.AimOracle(w.xy, w.k, w.eta, wl.PULSE, w.m, w.eps, alpha=w.alpha, near=False, n=2048)
        th = 2 * math.pi * np.arange(N) / N
        t0 = time.perf_counter()
        for nu in (0, 17, 45, 90):
            e = np.exp(1j * nu * th)
            np.vdot(e, A.gram_inv(A.op_S_alpha(e))) / N
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 4 / dt, "unit": "modes/s (S_ALPHA)", "cores": _host_threads(),
                               "kind": "oracle", "sample": "4 Fourier modes of S^alpha at the paper's parameters"}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2606_10784_amd import aim
    from paper_2606_10784_amd import workloads as wl

    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    if args.workload == "spectrum":
        return spectrum(args)
    if args.workload == "tm_calderon":
        return tm_calderon(args)
    if args.workload == "star_te":
        return star_te(args)
    if args.workload == "cylinder_ka200_360rhs":
        return batched_360(args)
    w = wl.cylinder_large() if args.workload == "cylinder_ka200" else wl.cylinder_small()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    t_setup = time.perf_counter()
    ctx = aim.Context(w.xy, w.k, w.eta, w.basis, w.m, w.eps, quad=w.quad, near_radius=w.near_radius,
                      precision=aim.AIM_MIXED, max_rhs=1, stream=stream, max_restart=args.restart)
    ctx.filter(w.alpha)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    inf = ctx.info()
    b = ctx.rhs_planewave(0.0)
    print(f"[bench] setup {t_setup:.2f} s  N={inf['n_unknowns']} n={inf['n_pad']} active={inf['n_active']} "
          f"rows={inf['active_rows']} near={inf['near_nnz_s']}", file=sys.stderr, flush=True)
    if args.mode == "matvec":
        xprobe = torch.from_numpy(wl.probe_vector(w.n_unknowns, seed=3)).to(dev)
        yprobe = torch.empty_like(xprobe)
        for _ in range(args.matvecs):
            ctx.matvec("TM", xprobe, yprobe)
        if args.copy_calibration:
            src = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
            dst = torch.empty_like(src)
            src.fill_(1.0)
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "matvec", "matvecs": args.matvecs, "workload": w.name,
                          "alg_bytes_cols_conv": kernel_bytes(2, inf)}), flush=True)
        ctx.close()
        return

    # warm-up solves
    for i in range(args.warmup):
        x, info = ctx.solve("TM", b, tol=args.tol, restart=args.restart)
        print(f"[bench] warmup {i} iters={info[0]['iterations']} resid={info[0]['resid_true']:.2e}",
              file=sys.stderr, flush=True)

    # rank the pipeline kernels on a short matvec loop (event-timed)
    xprobe = torch.from_numpy(wl.probe_vector(w.n_unknowns, seed=3)).to(dev)
    yprobe = torch.empty_like(xprobe)
    ktimes = {}
    for kid in range(5):
        aim.aim_profile_start(ctx, kid, 1, 64)
        for _ in range(10):
            ctx.matvec("TM", xprobe, yprobe)
        ms, ns, nl = aim.aim_profile_stop(ctx)
        ktimes[kid] = ms
    dom = max(ktimes, key=ktimes.get)
    names = ["anterp", "rows_fwd", "cols_conv", "rows_inv", "interp_near"]

    # ---------------- timed region: K FP64 solves ----------------
    # every PROF_EVERY-th launch of the dominant kernel is bracketed by HIP
    # events on the context's stream (an event pair around every launch would
    # itself slow the solve by several per cent)
    aim.aim_profile_start(ctx, dom, PROF_EVERY, 100000)
    torch.cuda.synchronize()
    lat, mv, its, res = [], 0, [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        x, info = ctx.solve("TM", b, tol=args.tol, restart=args.restart)
        lat.append(time.perf_counter() - ts)
        mv += info[0]["matvecs"]
        its.append(info[0]["iterations"])
        res.append(info[0]["resid_true"])
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    dom_ms, dom_samples, dom_launches = aim.aim_profile_stop(ctx)
    # -------------------------------------------------------------
    print(f"[bench] timed {args.steps} solves in {t_total:.3f} s", file=sys.stderr, flush=True)

    # matvec-only throughput (events around a back-to-back loop)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(5):
        ctx.matvec("TM", xprobe, yprobe)
    e0.record()
    for _ in range(args.matvecs):
        ctx.matvec("TM", xprobe, yprobe)
    e1.record()
    torch.cuda.synchronize()
    mv_ms = e0.elapsed_time(e1) / args.matvecs
    e0.record()
    for _ in range(args.matvecs):
        ctx.matvec(aim.AIM_OP_TM | aim.AIM_OP_GRID_FP32, xprobe, yprobe)
    e1.record()
    torch.cuda.synchronize()
    mv32_ms = e0.elapsed_time(e1) / args.matvecs
    # per-matvec distribution: 100 matvecs, each between its own event pair
    def spread(op):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(100)]
        for a, z in evs:
            a.record()
            ctx.matvec(op, xprobe, yprobe)
            z.record()
        torch.cuda.synchronize()
        t = np.sort([a.elapsed_time(z) for a, z in evs])
        return {"p10": float(t[9]), "p50": float(np.median(t)), "p90": float(t[89])}
    mv_spread = {"fp64": spread("TM"), "fp32_grid": spread(aim.AIM_OP_TM | aim.AIM_OP_GRID_FP32)}

    # mixed-precision solve at the same accuracy (reported beside value)
    tm0 = time.perf_counter()
    xm, infm = ctx.solve("TM", b, tol=args.tol, restart=args.restart, precision=aim.AIM_MIXED)
    t_mixed = time.perf_counter() - tm0
    dx = float(torch.linalg.norm(xm - x) / torch.linalg.norm(x))

    # achievable HBM rate: a plain 1 GiB device-to-device copy (read + write)
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    for _ in range(3):
        dst.copy_(src)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst

    alg_b = kernel_bytes(dom, inf)
    achieved = alg_b / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else 0.0
    value = mv / t_total
    lat_ms = sorted(1e3 * v for v in lat)

    def pct(p):
        return lat_ms[min(len(lat_ms) - 1, int(math.ceil(p / 100.0 * len(lat_ms))) - 1)]

    out = {
        "metric": "AIM matvecs/s + solves/s at 1e-6 residual vs FP64 plain; p50/p99 latency",
        "value": value,
        "unit": "AIM matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": w.name, "form": "TM-EFIE", "solver": f"GMRES({args.restart}) FP64",
                   "tol": args.tol, "N": inf["n_unknowns"], "grid": f"{w.m}x{w.m} pad {inf['n_pad']}",
                   "eps_over_lambda": w.eps, "filter_alpha": w.alpha},
        "solves_per_s": args.steps / t_total,
        "latency_ms": {"p50": pct(50), "p99": pct(99)},
        "iterations": its,
        "resid_true": max(res),
        "matvec_only": {"fp64_ms": mv_ms, "fp64_per_s": 1e3 / mv_ms, "fp32_grid_ms": mv32_ms,
                        "fp32_grid_per_s": 1e3 / mv32_ms, "each_ms": mv_spread},
        "mixed_solve": {"seconds": t_mixed, "iterations": infm[0]["iterations"], "outer": infm[0]["outer"],
                        "resid_true": infm[0]["resid_true"], "rel_diff_vs_fp64": dx,
                        "speedup_vs_fp64": (t_total / args.steps) / t_mixed},
        "kernel_ms": {names[k]: v for k, v in ktimes.items()},
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(names[dom]),
                     "alg_bytes_per_launch": alg_b, "avg_ms": dom_ms, "samples": dom_samples,
                     "sample_every": PROF_EVERY,
                     "flops_per_launch": kernel_flops(dom, inf),
                     "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "setup_s": t_setup,
    }
    ctx.close()
    if args.serve_requests > 0:
        print("[bench] serving stream ...", file=sys.stderr, flush=True)
        out["serving"] = serving(args.serve_requests, log_dir=args.serve_log_dir)
    if not args.no_configs:
        print("[bench] star N=65536 TE Calderon (filtered vs unfiltered) ...", file=sys.stderr, flush=True)
        out["c2_star_te"] = c2_star(args)
        print("[bench] cylinder ka=200, 360 incidences ...", file=sys.stderr, flush=True)
        out["c3_360_incidences"] = c3_batched(args)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
