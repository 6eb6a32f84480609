"""Pins of oracle.galerkin: singular moments, circle spectra, symmetry, Gram."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import galerkin, mie
from oracle.geometry import gauss_legendre01, segments
from paper_2606_10784_amd import workloads as wl

K = 2 * math.pi


def _g(R):
    return -0.25j * special.hankel2(0, K * R)


def _brute_pair(A0, A1, B0, B1, u, v, split_inner=None):
    """Nested adaptive QUADPACK integration of g tau^u sigma^v h_a h_b."""
    A0, A1, B0, B1 = (np.asarray(p, float) for p in (A0, A1, B0, B1))
    ha = np.linalg.norm(A1 - A0)
    hb = np.linalg.norm(B1 - B0)

    def inner(t, part):
        ra = A0 + (A1 - A0) * t

        def f(s):
            R = np.linalg.norm(ra - (B0 + (B1 - B0) * s))
            val = _g(R) if R > 0 else 0.0
            return (val.real if part == 0 else val.imag) * t ** u * s ** v * ha * hb
        pts = [t] if split_inner else None
        return integrate.quad(f, 0.0, 1.0, points=pts, epsabs=1e-15, epsrel=1e-13, limit=200)[0]

    re = integrate.quad(lambda t: inner(t, 0), 0, 1, epsabs=1e-15, epsrel=1e-13, limit=200)[0]
    im = integrate.quad(lambda t: inner(t, 1), 0, 1, epsabs=1e-15, epsrel=1e-13, limit=200)[0]
    return re + 1j * im


@pytest.mark.parametrize("uv", [(0, 0), (1, 1), (1, 0)])
def test_self_moments_vs_adaptive_quadrature(uv):
    h = 0.07
    M = galerkin.moments_self(h, K)
    ref = _brute_pair([0, 0], [h, 0], [0, 0], [h, 0], *uv, split_inner=True)
    assert abs(M[uv] - ref) / abs(ref) < 1e-10


@pytest.mark.parametrize("uv", [(0, 0), (0, 1), (1, 1)])
def test_adjacent_moments_vs_adaptive_quadrature(uv):
    A0, A1 = [0.0, 0.0], [0.05, 0.0]
    B1 = [0.05 + 0.04 * math.cos(0.4), 0.04 * math.sin(0.4)]
    M = galerkin.moments_adjacent(A0, A1, A1, B1, K)
    ref = _brute_pair(A0, A1, A1, B1, *uv)
    assert abs(M[uv] - ref) / abs(ref) < 1e-10
    # orientation swap is the transpose
    Mt = galerkin.moments_adjacent(A1, B1, A0, A1, K)
    assert np.max(np.abs(Mt - M.T)) < 1e-15 * np.max(np.abs(M)) * 10


def _circle_eigs(N, basis, op, ns, a=1.0):
    xy = wl.circle(a, N)
    pairs = np.stack([np.zeros(N, int), np.arange(N)], 1)
    row = galerkin.assemble_entries(xy, basis, K, pairs, op)
    h = 2 * a * math.sin(math.pi / N)
    den = np.array([h if basis == 0 else h * (4 + 2 * math.cos(2 * math.pi * n / N)) / 6 for n in ns])
    return np.array([np.sum(row * np.exp(2j * math.pi * n * np.arange(N) / N)) for n in ns]) / den


@pytest.mark.parametrize("basis,op", [(0, 'S'), (1, 'S'), (1, 'N')])
def test_circle_eigenvalues_second_order(basis, op):
    """The N-gon Galerkin matrices are circulant; their Fourier eigenvalues
    (divided by the Gram eigenvalue) converge at O(h^2) to the closed forms
    lambda_n^S = -(j pi a/2) J_n H_n^(2), lambda_n^N = (j pi a k^2/2) J_n' H_n^(2)'.
    Richardson extrapolation removes the h^2 term."""
    ns = np.array([0, 1, 3, 5, 9])
    ex = mie.circle_eig_S(ns, K, 1.0) if op == 'S' else mie.circle_eig_N(ns, K, 1.0)
    l1 = _circle_eigs(256, basis, op, ns)
    l2 = _circle_eigs(512, basis, op, ns)
    e1 = np.abs(l1 - ex) / np.abs(ex)
    e2 = np.abs(l2 - ex) / np.abs(ex)
    assert np.all(e2 < 5e-3)
    ratio = e1[:2] / e2[:2]
    assert np.all((ratio > 3.5) & (ratio < 4.5))
    rich = (4 * l2 - l1) / 3
    er = np.abs(rich - ex) / np.abs(ex)
    assert np.all(er < 1e-4)
    assert np.all(er[:2] < 1e-6)


def test_calderon_identity_high_modes():
    """S N -> 1/4 for n >> ka (Calderon identity on the circle)."""
    ns = np.array([20, 24, 28])
    pS = _circle_eigs(512, 1, 'S', ns)
    pN = _circle_eigs(512, 1, 'N', ns)
    assert np.all(np.abs(pS * pN - 0.25) < 2e-3)


def test_complex_symmetry_on_star():
    xy = wl.star5(0.8, 40)
    for basis, op in ((0, 'S'), (1, 'S'), (1, 'N')):
        A = galerkin.dense_matrix(xy, basis, K, op)
        assert np.max(np.abs(A - A.T)) < 1e-13 * np.max(np.abs(A))


def test_gram_closed_form_and_solve():
    xy = wl.star5(1.0, 37)
    A0, A1, h, _, _ = segments(xy)
    x, w = gauss_legendre01(4)
    Gq = np.zeros((37, 37))
    # quadrature of phi_i phi_j for hats
    for s in range(37):
        fall, rise = 1 - x, x              # hat s falls, hat s+1 rises on segment s
        i, j = s, (s + 1) % 37
        Gq[i, i] += h[s] * np.sum(w * fall * fall)
        Gq[j, j] += h[s] * np.sum(w * rise * rise)
        Gq[i, j] += h[s] * np.sum(w * fall * rise)
        Gq[j, i] += h[s] * np.sum(w * fall * rise)
    G = galerkin.gram(xy, 1)
    assert np.max(np.abs(G - Gq)) < 1e-16 * 10
    rng = np.random.default_rng(3)
    b = rng.standard_normal((37, 3)) + 1j * rng.standard_normal((37, 3))
    assert np.max(np.abs(galerkin.gram_solve(xy, 1, b) - np.linalg.solve(G, b))) < 1e-12
    assert np.max(np.abs(galerkin.gram_solve(xy, 1, b[:, 0]) - np.linalg.solve(G, b[:, 0]))) < 1e-12
    assert np.allclose(galerkin.gram(xy, 0), np.diag(h))
