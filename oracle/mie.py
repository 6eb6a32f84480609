"""Closed forms for the PEC circular cylinder (oracle; test infrastructure).

These are textbook results used as pins; none of them is the method.

  * eigenvalues of the single-layer operator on the circle of radius a
    (addition theorem of H0^(2)):  lambda_n^S = -(j pi a / 2) J_n(ka) H_n^(2)(ka)
  * hypersingular operator of eq. (2):
        lambda_n^N = (j pi a k^2 / 2) J_n'(ka) H_n^(2)'(ka)
  * analytically filtered single layer (eq. (5)-(6)) on the circle:
        lambda_n^{S,alpha} = a PV int_0^alpha J_n(sa)^2 s/(s^2-k^2) ds
                             - (j pi a / 2) J_n(ka)^2
  * Mie currents for a plane wave along +x (E0 = H0 = 1):
        TM  J_z(phi)   = 2 E0 / (pi k a eta) sum_n j^-n e^{jn phi} / H_n^(2)(ka)
        TE  J_phi(phi) = 2 j H0 / (pi k a)   sum_n j^-n e^{jn phi} / H_n^(2)'(ka)
  * TM backscatter width: sigma = (4/k) |sum_n (-1)^n J_n(ka)/H_n^(2)(ka)|^2
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def _hn2(n, x):
    return special.hankel2(n, x)


def circle_eig_S(n, k, a):
    n = np.abs(np.asarray(n))
    return -0.5j * math.pi * a * special.jv(n, k * a) * _hn2(n, k * a)


def circle_eig_N(n, k, a):
    n = np.abs(np.asarray(n))
    return 0.5j * math.pi * a * k * k * special.jvp(n, k * a) * special.h2vp(n, k * a)


def circle_eig_S_alpha(n, k, a, alpha, p=32):
    """PV integral by subtraction at s = k and Gauss panels on [0,k], [k,alpha]."""
    out = []
    x, w = np.polynomial.legendre.leggauss(p)
    for nn in np.atleast_1d(np.abs(n)):
        def panels(lo, hi, npan):
            e = np.linspace(lo, hi, npan + 1)
            s = (0.5 * (e[1:, None] - e[:-1, None]) * (x[None] + 1) + e[:-1, None]).ravel()
            ww = (0.5 * (e[1:, None] - e[:-1, None]) * w[None]).ravel()
            return s, ww
        npan = max(8, int(alpha * a / 2))
        s1, w1 = panels(0.0, k, max(8, int(k * a / 2)))
        s2, w2 = panels(k, alpha, npan)
        s = np.concatenate([s1, s2])
        ww = np.concatenate([w1, w2])
        f = special.jv(nn, s * a) ** 2 * s / (s + k)
        fk = special.jv(nn, k * a) ** 2 * 0.5
        pv = np.sum(ww * (f - fk) / (s - k)) + fk * math.log((alpha - k) / k)
        out.append(a * pv - 0.5j * math.pi * a * special.jv(nn, k * a) ** 2)
    return np.array(out)


def mie_tm_current(phi, k, a, eta, E0=1.0, nmax=None):
    x = k * a
    if nmax is None:
        nmax = int(x + 10 * x ** (1 / 3) + 20)
    phi = np.asarray(phi, dtype=float)
    out = np.zeros(phi.shape, dtype=complex)
    for n in range(-nmax, nmax + 1):
        hn = _hn2(abs(n), x) * (1.0 if n >= 0 or n % 2 == 0 else -1.0)
        out += (1j) ** (-n) * np.exp(1j * n * phi) / hn
    return 2.0 * E0 / (math.pi * x * eta) * out


def mie_te_current(phi, k, a, H0=1.0, nmax=None):
    x = k * a
    if nmax is None:
        nmax = int(x + 10 * x ** (1 / 3) + 20)
    phi = np.asarray(phi, dtype=float)
    out = np.zeros(phi.shape, dtype=complex)
    for n in range(-nmax, nmax + 1):
        hp = special.h2vp(abs(n), x) * (1.0 if n >= 0 or n % 2 == 0 else -1.0)
        out += (1j) ** (-n) * np.exp(1j * n * phi) / hp
    return 2.0j * H0 / (math.pi * x) * out


def mie_tm_backscatter(k, a, nmax=None):
    x = k * a
    if nmax is None:
        nmax = int(x + 10 * x ** (1 / 3) + 20)
    s = 0.0 + 0.0j
    for n in range(-nmax, nmax + 1):
        s += (-1) ** n * special.jv(abs(n), x) / _hn2(abs(n), x)
    return 4.0 / k * abs(s) ** 2
