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


# --------------------------------------------------------------------------
# references with the logarithm taken by QUADPACK's log-weighted rule (QAWS),
# the Bessel functions by SciPy: valid over the whole accepted range k h <= 2 pi
# --------------------------------------------------------------------------
_EG = 0.57721566490153286060651209


def _F(R):
    """g(R) + (1/2 pi) J0(kR) ln R from SciPy's Hankel function."""
    if R == 0.0:
        return -0.25j - (math.log(K / 2.0) + _EG) / (2.0 * math.pi)
    return _g(R) + special.j0(K * R) * math.log(R) / (2.0 * math.pi)


def _q(f, a, b, **kw):
    return integrate.quad(f, a, b, epsabs=1e-17, epsrel=2e-14, limit=400, **kw)[0]


def _cq(f, a, b, **kw):
    return _q(lambda x: f(x).real, a, b, **kw) + 1j * _q(lambda x: f(x).imag, a, b, **kw)


def _self_ref(h, u, v):
    """h^2 int_0^1 tau^u int_0^1 g(h |tau - sigma|) sigma^v dsigma dtau, the
    inner integral split at sigma = tau with ln|tau - sigma| as the weight."""
    def inner(t):
        flog = lambda s: -special.j0(K * h * abs(t - s)) / (2.0 * math.pi) * s ** v
        r = 0.0
        if t < 1.0:
            r += _q(flog, t, 1.0, weight='alg-loga', wvar=(0, 0))
        if t > 0.0:
            r += _q(flog, 0.0, t, weight='alg-logb', wvar=(0, 0))
        rest = lambda s: (-special.j0(K * h * abs(t - s)) * math.log(h) / (2.0 * math.pi)
                          + _F(h * abs(t - s))) * s ** v
        return (r + _cq(rest, 0.0, 1.0, points=[t])) * t ** u
    return h * h * _cq(inner, 0.0, 1.0)


def _adjacent_ref(A0, V, B1, u, v):
    """Moments of segments A0 -> V and V -> B1 (tau along the first, sigma
    along the second) in polar coordinates about V: s = rho cos psi along the
    first segment, s' = rho sin psi along the second, R = rho r(psi); the
    rho integral with ln rho as the weight, psi adaptive."""
    A0, V, B1 = (np.asarray(p, float) for p in (A0, V, B1))
    ha, hb = np.linalg.norm(A0 - V), np.linalg.norm(B1 - V)
    cab = float((A0 - V) @ (B1 - V)) / (ha * hb)
    psid = math.atan2(hb, ha)

    def radial(ps):
        c, s = math.cos(ps), math.sin(ps)
        r = math.sqrt(1.0 - 2.0 * c * s * cab)
        pm = min(ha / c if c > 0 else np.inf, hb / s if s > 0 else np.inf)
        poly = lambda rho: (1.0 - rho * c / ha) ** u * (rho * s / hb) ** v * rho
        flog = lambda rho: -special.j0(K * rho * r) / (2.0 * math.pi) * poly(rho)
        rest = lambda rho: (-special.j0(K * rho * r) * math.log(r) / (2.0 * math.pi) + _F(rho * r)) * poly(rho)
        return _q(flog, 0.0, pm, weight='alg-loga', wvar=(0, 0)) + _cq(rest, 0.0, pm)
    pts = [0.25 * math.pi] if 0.0 < 0.25 * math.pi < psid else None
    pts2 = [0.25 * math.pi] if psid < 0.25 * math.pi else None
    return _cq(radial, 0.0, psid, points=pts) + _cq(radial, psid, 0.5 * math.pi, points=pts2)


@pytest.mark.parametrize("kh", [math.pi, 2.0 * math.pi])
@pytest.mark.parametrize("uv", [(0, 0), (1, 0), (1, 1)])
def test_self_moments_full_range(kh, uv):
    """Self moments up to the longest segment aim_setup accepts (k h = 2 pi)."""
    h = kh / K
    M = galerkin.moments_self(h, K)
    assert abs(M[uv] - _self_ref(h, *uv)) < 1e-12 * np.max(np.abs(M))


def _ray(V, L, ang):
    return [V[0] + L * math.cos(ang), V[1] + L * math.sin(ang)]


# (length of the first segment, length of the second, direction of the second
# segment relative to the continuation of the first): straight-ish, unequal
# lengths at the longest accepted segment, acute vertices down to 0.05 rad
_ADJ_CASES = [
    (1.0, 0.5, 0.4),                  # k h = 2 pi and pi, gentle bend
    (1.0, 0.05, 1.2),                 # length ratio 20
    (0.5, 0.1, math.pi - 0.2),        # acute vertex: 0.2 rad between the segments
    (1.0, 1.0, math.pi - 0.05),       # k h = 2 pi, 0.05 rad between the segments
    (0.05, 0.5, -(math.pi - 0.3)),    # acute, clockwise, short first segment
]


@pytest.mark.parametrize("case", range(len(_ADJ_CASES)))
def test_adjacent_moments_full_range(case):
    ha, hb, turn = _ADJ_CASES[case]
    A0, V = [0.0, 0.0], [ha, 0.0]
    B1 = _ray(V, hb, turn)
    M = galerkin.moments_adjacent(A0, V, V, B1, K)
    for uv in ((0, 0), (0, 1), (1, 0), (1, 1)):
        assert abs(M[uv] - _adjacent_ref(A0, V, B1, *uv)) < 1e-12 * np.max(np.abs(M)), uv


@pytest.mark.parametrize("gap,turn", [(0.1, 0.0), (0.02, 0.0), (0.02, 0.6)])
def test_close_disjoint_moments(gap, turn):
    """Segments a and a+2 around a short middle segment (gap / h down to
    1/50): the nearly singular kernel needs the recursive subdivision."""
    A0, A1 = np.array([-1.0, 0.0]), np.array([0.0, 0.0])
    B0 = A1 + gap * np.array([math.cos(turn), math.sin(turn)])
    B1 = B0 + np.array([math.cos(2 * turn), math.sin(2 * turn)])
    pairs = np.array([[0, 2]])
    xy = np.array([A0, A1, B0, B1, [0.0, -1.0]])
    M = galerkin.segment_pair_moments(xy, pairs, K)[0]
    assert len(galerkin.disjoint_pieces(A0, A1, B0, B1)) > 1
    for u in (0, 1):
        for v in (0, 1):
            ref = _brute_pair(A0, A1, B0, B1, u, v)
            assert abs(M[u, v] - ref) < 1e-12 * np.max(np.abs(M)), (u, v)


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
