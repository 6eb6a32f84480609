"""Restarted GMRES (oracle; test infrastructure).

The paper names iterative solvers only in general terms (abstract, Sec. I);
the solver here is the textbook GMRES(r) of Saad and Schultz with modified
Gram-Schmidt Arnoldi and Givens rotations, x0 given (default 0), stopping
when the Arnoldi residual estimate |g_{j+1}| <= tol * ||b||.  The true
residual ||b - A x|| / ||b|| is recomputed at every restart and on exit.

Pinned by: tests/test_oracle_solver.py (dense systems against
numpy.linalg.solve, the error within cond(A) * tol).
"""
from __future__ import annotations

import numpy as np


def gmres(apply_A, b, x0=None, tol=1e-6, restart=100, maxit=5000):
    b = np.asarray(b, dtype=complex)
    n = b.size
    x = np.zeros(n, dtype=complex) if x0 is None else np.array(x0, dtype=complex)
    bnorm = np.linalg.norm(b)
    info = {'iterations': 0, 'matvecs': 0, 'converged': False, 'history': []}
    if bnorm == 0.0:
        info['converged'] = True
        return np.zeros(n, dtype=complex), info
    it = 0
    while it < maxit:
        r = b - apply_A(x)
        info['matvecs'] += 1
        beta = np.linalg.norm(r)
        info['history'].append(beta / bnorm)
        if beta <= tol * bnorm:
            info['converged'] = True
            break
        V = np.zeros((n, restart + 1), dtype=complex)
        H = np.zeros((restart + 1, restart), dtype=complex)
        cs = np.zeros(restart, dtype=complex)
        sn = np.zeros(restart, dtype=complex)
        g = np.zeros(restart + 1, dtype=complex)
        g[0] = beta
        V[:, 0] = r / beta
        j_done = 0
        for j in range(restart):
            w = apply_A(V[:, j])
            info['matvecs'] += 1
            for i in range(j + 1):
                H[i, j] = np.vdot(V[:, i], w)
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
                H[i, j] = t
            # complex Givens rotation [c s; -conj(s) c], c real, zeroing H[j+1, j]
            a, bb = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if a == 0:
                cs[j], sn[j] = 0.0, 1.0
            else:
                cs[j] = abs(a) / den
                sn[j] = (a / abs(a)) * np.conj(bb) / den
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            info['history'].append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or it >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x = x + V[:, :j_done] @ y
        if abs(g[j_done]) <= tol * bnorm:
            r = b - apply_A(x)
            info['matvecs'] += 1
            if np.linalg.norm(r) <= tol * bnorm * 1.0000001 or it >= maxit:
                info['converged'] = np.linalg.norm(r) <= tol * bnorm * 1.0000001
                info['true_residual'] = np.linalg.norm(r) / bnorm
                break
    info['iterations'] = it
    if 'true_residual' not in info:
        info['true_residual'] = np.linalg.norm(b - apply_A(x)) / bnorm
    return x, info
