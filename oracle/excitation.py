"""Plane-wave right-hand sides and monostatic RCS (oracle; test infrastructure).

Sec. II: the TE excitation vector is E_t = <phi_i, (jk/eta) E_t>.  The TM
system (not in the paper; derived from the same g) is jk eta S j = b with
b_i = <phi_i, E_z^inc>.  A plane wave propagating along khat =
(cos phi_inc, sin phi_inc) has E_z^inc = E0 exp(-jk khat.r) (TM) and
E^inc = eta H0 (z x khat) exp(-jk khat.r) (TE).

Monostatic 2D scattering width (TM):
    sigma(phi_inc) = (k eta^2 / 4) |int J_z exp(-jk khat.r') dl'|^2,
the far-field integral taken in the backscatter direction -khat.

Pinned by: tests/test_oracle_mie.py (TM/TE currents and backscatter of the
circle against the Mie series).
"""
from __future__ import annotations

import numpy as np

from .geometry import gauss_legendre01, segments


def _basis_integrals(xy, basis, p, fn):
    """b_i = int phi_i(r) fn(r, seg) dl over the support of basis i."""
    xy = np.asarray(xy, dtype=float)
    nb = xy.shape[0]
    A0, A1, h, t, _ = segments(xy)
    tau, w = gauss_legendre01(p)
    pts = A0[:, None, :] + (A1 - A0)[:, None, :] * tau[None, :, None]
    f = fn(pts, t)                                 # (nseg, p, ...)
    wk = h[:, None] * w[None, :]
    if basis == 0:
        return np.einsum('sp,sp...->s...', wk, f)
    rise = np.einsum('sp,sp...->s...', wk * tau[None, :], f)        # on segment s, hat s+1
    fall = np.einsum('sp,sp...->s...', wk * (1.0 - tau[None, :]), f)  # on segment s, hat s
    return fall + np.roll(rise, 1, axis=0)


def rhs_tm(xy, basis, k, phi_inc, E0=1.0, p=10):
    phi_inc = np.atleast_1d(np.asarray(phi_inc, dtype=float))
    kh = np.stack([np.cos(phi_inc), np.sin(phi_inc)], axis=1)   # (R,2)

    def fn(pts, t):
        return E0 * np.exp(-1j * k * np.einsum('spd,rd->spr', pts, kh))
    b = _basis_integrals(xy, basis, p, fn)
    return b[:, 0] if b.shape[1] == 1 else b


def rhs_te(xy, basis, k, eta, phi_inc, H0=1.0, p=10):
    phi_inc = np.atleast_1d(np.asarray(phi_inc, dtype=float))
    kh = np.stack([np.cos(phi_inc), np.sin(phi_inc)], axis=1)
    pol = np.stack([-kh[:, 1], kh[:, 0]], axis=1)                 # z x khat

    def fn(pts, t):
        ph = np.exp(-1j * k * np.einsum('spd,rd->spr', pts, kh))
        tdot = np.einsum('sd,rd->sr', t, pol)[:, None, :]
        return eta * H0 * tdot * ph
    b = (1j * k / eta) * _basis_integrals(xy, basis, p, fn)
    return b[:, 0] if b.shape[1] == 1 else b


def rcs_monostatic_tm(xy, basis, k, eta, J, phi_inc, p=10):
    """sigma(phi_inc) for currents J (N,) or (N, R) solved at those angles."""
    b = rhs_tm(xy, basis, k, phi_inc, 1.0, p)
    b = b.reshape(b.shape[0], -1)
    J = np.asarray(J).reshape(b.shape[0], -1)
    s = np.sum(b * J, axis=0)
    return k * eta * eta / 4.0 * np.abs(s) ** 2
