"""2D Helmholtz Green's function and its analytically filtered form (oracle).

Test infrastructure.  Definitions followed:
  * g(r, r') = -(j/4) H0^(2)(k|r - r'|), time convention e^{jwt}   (Sec. II)
  * g^alpha = g - (1/2pi) int_alpha^inf J0(s R) s/(s^2 - k^2) ds     (eq. (6))

Besides g itself this module provides the split used by the singular
quadrature of the near field:
      g(R) = -(1/2pi) J0(kR) ln R + F(R),
where F is an entire function of R^2 (from the ascending series of Y0), and
two independent evaluations of g^alpha: the low-pass principal-value form
      g^alpha(R) = (1/2pi) PV int_0^alpha J0(sR) s/(s^2-k^2) ds - (j/4) J0(kR)
and the tail form of eq. (6).

Pinned by: tests/test_oracle_green.py (series vs SciPy Hankel, small-R
asymptote, low-pass vs tail form, alpha -> inf limit, closed form at R = 0).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

EULER_GAMMA = 0.57721566490153286060651209


def green(R, k):
    """g(R) = -(j/4) H0^(2)(k R) = -(1/4) Y0(kR) - (j/4) J0(kR) for R > 0."""
    x = k * np.asarray(R, dtype=float)
    return -0.25 * special.y0(x) - 0.25j * special.j0(x)


def j0_series_coeffs(k, nterms=24):
    """c_m with J0(kR) = sum_m c_m R^(2m): c_m = (-1)^m (k/2)^(2m) / (m!)^2."""
    m = np.arange(nterms)
    lg = special.gammaln(m + 1.0)
    mag = np.exp(2.0 * m * math.log(k / 2.0) - 2.0 * lg)
    return np.where(m % 2 == 0, 1.0, -1.0) * mag


def _y0_series_tail(x, nterms=40):
    """S(x) = sum_{m>=1} (-1)^(m+1) H_m (x/2)^(2m) / (m!)^2  (ascending series
    of Y0:  Y0(x) = (2/pi)[(ln(x/2) + gamma) J0(x) + S(x)])."""
    x = np.asarray(x, dtype=float)
    q = (x / 2.0) ** 2
    out = np.zeros_like(x)
    term = np.ones_like(x)
    hm = 0.0
    for m in range(1, nterms):
        term = term * q / (m * m)
        hm += 1.0 / m
        out = out + (1.0 if m % 2 == 1 else -1.0) * hm * term
    return out


def green_regular(R, k):
    """F(R) = g(R) + (1/2pi) J0(kR) ln R, an entire function of R^2.

    For kR < 2 it is summed from the ascending series (no cancellation);
    otherwise it is formed from SciPy's Bessel functions."""
    R = np.asarray(R, dtype=float)
    x = k * R
    out = np.empty(R.shape, dtype=complex)
    small = x < 2.0
    xs = x[small]
    j0s = special.j0(xs)
    out[small] = -0.25j * j0s - (1.0 / (2.0 * math.pi)) * (
        j0s * (math.log(k / 2.0) + EULER_GAMMA) + _y0_series_tail(xs))
    Rb = R[~small]
    out[~small] = green(Rb, k) + (1.0 / (2.0 * math.pi)) * special.j0(k * Rb) * np.log(Rb)
    return out


# --------------------------------------------------------------------------
# analytically filtered kernel, eq. (6)
# --------------------------------------------------------------------------
def _gl_panels(a, b, npanel, p):
    x, w = np.polynomial.legendre.leggauss(p)
    edges = np.linspace(a, b, npanel + 1)
    lo, hi = edges[:-1, None], edges[1:, None]
    s = 0.5 * (hi - lo) * (x[None, :] + 1.0) + lo
    ws = 0.5 * (hi - lo) * w[None, :]
    return s.ravel(), ws.ravel()


def green_alpha_lowpass(R, k, alpha, panels_per_unit=4.0, p=24):
    """g^alpha(R) from the low-pass principal-value form.

    PV int_0^alpha f(s)/(s-k) ds with f(s) = s J0(sR)/(s+k) is written as
    int_0^alpha (f(s)-f(k))/(s-k) ds + f(k) ln((alpha-k)/k); the Gauss panels
    have a break point at s = k.  Valid for alpha > k and any R >= 0."""
    assert alpha > k
    R = np.atleast_1d(np.asarray(R, dtype=float))
    out = np.empty(R.shape, dtype=complex)
    for i, r in enumerate(R):
        osc = max(1.0, r)  # oscillation scale of J0(s r)
        n1 = max(4, int(math.ceil(k * osc * panels_per_unit / math.pi)))
        n2 = max(4, int(math.ceil((alpha - k) * osc * panels_per_unit / math.pi)))
        s1, w1 = _gl_panels(0.0, k, n1, p)
        s2, w2 = _gl_panels(k, alpha, n2, p)
        s = np.concatenate([s1, s2])
        w = np.concatenate([w1, w2])
        f = s * special.j0(s * r) / (s + k)
        fk = 0.5 * special.j0(k * r)
        pv = np.sum(w * (f - fk) / (s - k)) + fk * math.log((alpha - k) / k)
        out[i] = pv / (2.0 * math.pi) - 0.25j * special.j0(k * r)
    return out


def green_alpha_tail(R, k, alpha, smax_factor=400.0, p=24):
    """g^alpha(R) from eq. (6): g minus the spectral tail above alpha, R > 0.

    s/(s^2-k^2) = 1/s + k^2/(s(s^2-k^2)).  The first part integrates in
    closed form: int_{alpha R}^inf J0(t)/t dt = -gamma - ln(alpha R/2) +
    int_0^{alpha R} (1-J0(t))/t dt (SciPy it2j0y0).  The second part decays
    like s^-3.5 and is integrated by Gauss panels up to smax_factor*alpha."""
    R = np.atleast_1d(np.asarray(R, dtype=float))
    out = np.empty(R.shape, dtype=complex)
    for i, r in enumerate(R):
        x = alpha * r
        e1 = -EULER_GAMMA - math.log(x / 2.0) + special.it2j0y0(x)[0]
        smax = smax_factor * alpha
        npan = max(64, int(math.ceil((smax - alpha) * r / math.pi * 2.0)))
        # geometric-ish panelling: dense near alpha where the integrand is largest
        s, w = _gl_panels(0.0, 1.0, npan, p)
        # map u in [0,1] -> s = alpha * (smax/alpha)^u (log spacing)
        lr = math.log(smax / alpha)
        ss = alpha * np.exp(lr * s)
        ww = w * lr * ss
        e2 = np.sum(ww * special.j0(ss * r) * k * k / (ss * (ss * ss - k * k)))
        out[i] = green(r, k) - (e1 + e2) / (2.0 * math.pi)
    return out


def green_alpha_origin(k, alpha):
    """Closed form g^alpha(0) = (1/4pi) ln(alpha^2/k^2 - 1) - j/4."""
    return math.log(alpha * alpha / (k * k) - 1.0) / (4.0 * math.pi) - 0.25j
