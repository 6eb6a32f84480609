"""Pins of oracle.green: g, its log/regular split, and g^alpha of eq. (6)."""
import math

import numpy as np
from scipy import special

from oracle import green as G

K = 2 * math.pi


def test_regular_part_series_matches_scipy_bessel():
    # F = g + (1/2pi) J0(kR) ln R, series branch (kR < 2) vs SciPy H0^(2)
    R = np.linspace(0.003, 1.9 / K, 50)
    F = G.green_regular(R, K)
    ref = G.green(R, K) + special.j0(K * R) * np.log(R) / (2 * math.pi)
    assert np.max(np.abs(F - ref) / np.abs(ref)) < 1e-12


def test_small_argument_asymptote():
    # g(R) = -(1/2pi)(ln(kR/2) + gamma) - j/4 + O(R^2 ln R)
    for R in (1e-5, 1e-7):
        asym = -(math.log(K * R / 2) + G.EULER_GAMMA) / (2 * math.pi) - 0.25j
        assert abs(G.green(R, K) - asym) < 1e-8
    F0 = G.green_regular(np.array([0.0]), K)[0]
    assert abs(F0 - (-(math.log(K / 2) + G.EULER_GAMMA) / (2 * math.pi) - 0.25j)) < 1e-15


def test_filtered_kernel_origin_closed_form():
    # (1/2pi) PV int_0^alpha s/(s^2-k^2) ds - j/4 = ln(alpha^2/k^2 - 1)/(4 pi) - j/4
    for alpha in (2 * K, 8 * K):
        lp = G.green_alpha_lowpass(0.0, K, alpha)[0]
        assert abs(lp - G.green_alpha_origin(K, alpha)) < 1e-12


def test_filtered_kernel_two_forms_agree():
    # low-pass principal-value form vs eq. (6) tail form
    alpha = 8 * K
    R = np.array([0.05, 0.3, 1.0, 2.5])
    lp = G.green_alpha_lowpass(R, K, alpha)
    tl = G.green_alpha_tail(R, K, alpha)
    assert np.max(np.abs(lp - tl)) < 1e-7


def test_filtered_kernel_is_regular_and_tends_to_g():
    # g^alpha is bounded at the origin while g is not; the gap to g shrinks
    # as alpha grows (the removed spectral tail vanishes)
    R = 0.3
    g = G.green(R, K)
    gaps = [abs(G.green_alpha_lowpass(R, K, f * K)[0] - g) for f in (4, 16, 64)]
    assert gaps[0] > gaps[1] > gaps[2]
    assert gaps[2] < 3e-2 * gaps[0]      # tail ~ (alpha R)^(-3/2)
    # imaginary part is untouched by the filter (only the real PV part moves)
    assert abs(G.green_alpha_lowpass(R, K, 8 * K)[0].imag - g.imag) < 1e-12


def test_green_matches_amos_hankel():
    # g from Cephes J0/Y0 against the independent AMOS Hankel routine
    R = np.geomspace(1e-4, 30.0, 200)
    ref = -0.25j * special.hankel2(0, K * R)
    assert np.max(np.abs(G.green(R, K) - ref) / np.abs(ref)) < 1e-13


def test_filtered_circle_eigenvalue_by_addition_theorem():
    """lambda_n^{S,alpha} = int_0^{2pi} g^alpha(2a sin(t/2)) e^{jnt} a dt: the
    filtered kernel is entire in R^2, so the periodic trapezoid rule of the
    low-pass form pins the oracle's Bessel-product closed form."""
    from oracle import mie
    a, alpha = 1.0, 3 * K
    M = 160
    t = 2 * math.pi * np.arange(M) / M
    ga = G.green_alpha_lowpass(2 * a * np.abs(np.sin(t / 2)), K, alpha)
    for n in (0, 4, 11, 17):
        lam = np.sum(ga * np.exp(1j * n * t)) * a * 2 * math.pi / M
        ref = mie.circle_eig_S_alpha([n], K, a, alpha)[0]
        assert abs(lam - ref) < 1e-9 * abs(mie.circle_eig_S_alpha([0], K, a, alpha)[0])
    # alpha -> infinity recovers the unfiltered eigenvalue
    big = mie.circle_eig_S_alpha([2], K, a, 400 * K)[0]
    assert abs(big - mie.circle_eig_S(2, K, a)) < 2e-3 * abs(big)
