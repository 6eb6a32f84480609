"""Mesh geometry and Gauss-Legendre rules (oracle; test infrastructure).

Sec. II: the curve gamma is meshed by N straight segments; segment j runs
from vertex j to vertex j+1 (cyclic).  Eq. (7): integrals over a segment use
a p-node Gauss rule.

Pinned by: tests/test_oracle_geometry.py (perimeter of the inscribed polygon,
Gauss-Legendre exactness on polynomials of degree <= 2p-1, outward normals).
"""
from __future__ import annotations

import numpy as np


def segments(xy: np.ndarray):
    """Return (start, end, h, t, nrm) per segment of the closed polygon xy.

    t is the unit tangent (direction of increasing vertex index, i.e. CCW for a
    CCW polygon) and nrm = (t_y, -t_x) the outward normal for a CCW polygon.
    """
    xy = np.asarray(xy, dtype=float)
    a = xy
    b = np.roll(xy, -1, axis=0)
    d = b - a
    h = np.hypot(d[:, 0], d[:, 1])
    t = d / h[:, None]
    nrm = np.stack([t[:, 1], -t[:, 0]], axis=1)
    return a, b, h, t, nrm


def gauss_legendre01(p: int):
    """p-node Gauss-Legendre rule on [0, 1]: nodes, weights (sum = 1)."""
    x, w = np.polynomial.legendre.leggauss(p)
    return 0.5 * (x + 1.0), 0.5 * w


def segment_nodes(xy: np.ndarray, p: int):
    """Quadrature nodes on every segment.

    Returns (tau (p,), pts (N, p, 2), wts (N, p)) with pts = a + tau h t and
    wts = w h (physical arc-length weights)."""
    a, b, h, t, _ = segments(xy)
    tau, w = gauss_legendre01(p)
    pts = a[:, None, :] + (b - a)[:, None, :] * tau[None, :, None]
    wts = h[:, None] * w[None, :]
    return tau, pts, wts


def basis_pieces(nseg: int, basis: int):
    """Support of each basis function as a list of (segment, c0, c1, dphi)
    pieces, where on that segment phi(tau) = c0 + c1 tau (tau in [0,1] from the
    segment start) and dphi is the arc-length derivative times h (= c1).

    basis 0 (pulse): basis j = 1 on segment j.
    basis 1 (hat): piecewise-linear Lagrange function of Sec. II, equal to 1 at
    vertex j; it rises on segment j-1 and falls on segment j.
    """
    pieces = []
    for j in range(nseg):
        if basis == 0:
            pieces.append([(j, 1.0, 0.0)])
        else:
            pieces.append([((j - 1) % nseg, 0.0, 1.0), (j, 1.0, -1.0)])
    return pieces
