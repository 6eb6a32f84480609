"""Dual (barycentric) basis and the TM Calderon form (oracle; test
infrastructure).

The paper filters the single layer and preconditions the TE equation with it
(Sec. IV: G^-1 S^alpha G^-1 N).  Its TM counterpart preconditions the TM
single layer S (pulses) with the hypersingular N, filtered the same way
(N^alpha: the Maue channels of eq. (2) through the filtered grid kernel of
eq. (10), no near-field correction).  N needs a continuous basis whose mixed
Gram matrix with the pulses is invertible; the primal hats fail for even N
(the pulse/hat Gram is singular at the alternating mode), so the dual hats
of the barycentric refinement are used:

  * refined polygon: 2N vertices r_2j = v_j, r_2j+1 = midpoint M_j of
    segment j (the same curve, every segment halved);
  * dual hat psi_j, centred at M_j: 1 at M_j, 1/2 at v_j and v_j+1, 0 at
    M_j-1 and M_j+1, linear on each refined segment, i.e.
    psi_j = h'_2j / 2 + h'_2j+1 + h'_2j+2 / 2 in the refined hats h';
  * mixed Gram G_pd[i][j] = <pulse_i, psi_j>: 3 h_i / 4 on the diagonal,
    h_i / 8 for j = i +- 1 (cyclic);
  * TM Calderon operator
      A = G_pd^-T  R N'^(alpha) R^T  G_pd^-1  (jk eta S),   R = psi in h',
    for the system A j = G_pd^-T R N'^(alpha) R^T G_pd^-1 b, whose solution is
    that of the TM EFIE jk eta S j = b.

Everything here is dense linear algebra on the oracle's own operators (AIM
oracles of oracle.aim on the primal pulses and the refined hats).

Pinned by: tests/test_oracle_dual.py (mixed Gram against quadrature of the
dual hats' pointwise definition; R reproduces psi at the refined vertices;
the dense Galerkin Calderon product G_pd^-T R N' R^T G_pd^-1 S on a circle
against lambda^N lambda^S of the closed-form circle eigenvalues and the
plateau 1/4).
"""
from __future__ import annotations

import numpy as np

from .aim import AimOracle
from .geometry import segments


def refined_polygon(xy):
    """2N vertices: v_j at 2j, the midpoint of segment j at 2j+1."""
    xy = np.asarray(xy, dtype=float)
    mid = 0.5 * (xy + np.roll(xy, -1, axis=0))
    out = np.empty((2 * xy.shape[0], 2))
    out[0::2] = xy
    out[1::2] = mid
    return out


def dual_combination(n):
    """R (n x 2n): psi_j = sum_k R[j, k] h'_k."""
    R = np.zeros((n, 2 * n))
    j = np.arange(n)
    R[j, 2 * j] = 0.5
    R[j, 2 * j + 1] = 1.0
    R[j, (2 * j + 2) % (2 * n)] = 0.5
    return R


def mixed_gram(xy):
    """G_pd[i][j] = <pulse_i, psi_j> (closed form, dense)."""
    _, _, h, _, _ = segments(xy)
    n = h.size
    G = np.zeros((n, n))
    for i in range(n):
        G[i, i] += 0.75 * h[i]
        G[i, (i - 1) % n] += h[i] / 8.0
        G[i, (i + 1) % n] += h[i] / 8.0
    return G


class TMCalderonOracle:
    """TM Calderon operators of one geometry / frequency / grid."""

    def __init__(self, xy, k, eta, m, eps, p=10, near_radius=6, alpha=np.inf, n=None):
        """n: length of the grid's circulant embedding (default 2m)."""
        self.xy = np.asarray(xy, dtype=float)
        self.k, self.eta = float(k), float(eta)
        self.N = self.xy.shape[0]
        self.primal = AimOracle(self.xy, k, eta, 0, m, eps, p=p, near_radius=near_radius, alpha=alpha, n=n)
        self.dual = AimOracle(refined_polygon(self.xy), k, eta, 1, m, eps, p=p, near_radius=near_radius,
                              alpha=alpha, n=n)
        self.R = dual_combination(self.N)
        self.G = mixed_gram(self.xy)

    def set_alpha(self, alpha):
        self.primal.set_alpha(alpha)
        self.dual.set_alpha(alpha)

    def precond(self, x, filtered=True):
        """G_pd^-T R N'^(alpha) R^T G_pd^-1 x (x: pulse-tested values)."""
        u = np.linalg.solve(self.G, x)
        w = self.dual.apply('N_ALPHA' if filtered else 'N', self.R.T @ u)
        return np.linalg.solve(self.G.T, self.R @ w)

    def apply(self, op, x):
        x = np.asarray(x, dtype=complex)
        if op == 'TM_PC':
            return self.precond(x, True)
        if op == 'TM_PC_UNF':
            return self.precond(x, False)
        if op == 'TM_CP':
            return self.precond(self.primal.apply('TM', x), True)
        if op == 'TM_CP_UNF':
            return self.precond(self.primal.apply('TM', x), False)
        return self.primal.apply(op, x)
