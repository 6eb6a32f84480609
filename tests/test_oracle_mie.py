"""Pins of oracle.excitation + Galerkin solves against the Mie series."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import excitation, galerkin, mie
from paper_2606_10784_amd import workloads as wl

K = 2 * math.pi
ETA = wl.ETA0


def test_mie_current_integrates_to_closed_form_backscatter():
    """sigma from the far-field integral of the Mie TM current equals the
    closed-form backscatter width (two independent series)."""
    a = 1.0
    phi = 2 * math.pi * np.arange(4096) / 4096
    J = mie.mie_tm_current(phi, K, a, ETA)
    # monostatic, incidence along +x: integrate J exp(-jk x) a dphi
    s = np.sum(J * np.exp(-1j * K * a * np.cos(phi))) * a * 2 * math.pi / 4096
    sig = K * ETA ** 2 / 4 * abs(s) ** 2
    assert abs(sig - mie.mie_tm_backscatter(K, a)) < 1e-9 * sig


def _tm_solve(N, a=1.0):
    xy = wl.circle(a, N)
    S = galerkin.dense_matrix(xy, 0, K, 'S')
    b = excitation.rhs_tm(xy, 0, K, 0.0)
    j = np.linalg.solve(1j * K * ETA * S, b)
    return xy, j


def test_tm_current_converges_to_mie():
    errs = []
    for N in (64, 128):
        xy, j = _tm_solve(N)
        phm = 2 * math.pi * (np.arange(N) + 0.5) / N
        ref = mie.mie_tm_current(phm, K, 1.0, ETA)
        errs.append(np.linalg.norm(j - ref) / np.linalg.norm(ref))
    assert errs[1] < 2e-2
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_tm_backscatter_converges_to_mie():
    xy, j = _tm_solve(128)
    sig = excitation.rcs_monostatic_tm(xy, 0, K, ETA, j, 0.0)[0]
    ex = mie.mie_tm_backscatter(K, 1.0)
    assert abs(sig - ex) / ex < 1e-2


def test_te_current_converges_to_mie():
    errs = []
    for N in (64, 128):
        xy = wl.circle(1.0, N)
        Nm = galerkin.dense_matrix(xy, 1, K, 'N')
        b = excitation.rhs_te(xy, 1, K, ETA, 0.0)
        j = np.linalg.solve(Nm, b)
        phv = 2 * math.pi * np.arange(N) / N
        ref = mie.mie_te_current(phv, K, 1.0)
        errs.append(np.linalg.norm(j - ref) / np.linalg.norm(ref))
    assert errs[1] < 2e-2
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_rhs_is_basis_projection_of_plane_wave():
    """Multi-angle RHS columns equal single-angle calls; pulse RHS against an
    adaptive quadrature of exp(-jk x) on one segment."""
    xy = wl.star5(1.0, 50)
    angs = [0.0, 0.7, 2.0]
    B = excitation.rhs_tm(xy, 1, K, angs)
    for i, ph in enumerate(angs):
        assert np.allclose(B[:, i], excitation.rhs_tm(xy, 1, K, ph), rtol=0, atol=1e-15)
    b = excitation.rhs_tm(xy, 0, K, 0.0)
    A0, A1 = xy[3], xy[4]
    h = np.linalg.norm(A1 - A0)
    re = integrate.quad(lambda t: math.cos(K * (A0[0] + t * (A1[0] - A0[0]))), 0, 1, epsabs=1e-17, epsrel=1e-13)[0]
    im = integrate.quad(lambda t: -math.sin(K * (A0[0] + t * (A1[0] - A0[0]))), 0, 1, epsabs=1e-17, epsrel=1e-13)[0]
    assert abs(b[3] - h * (re + 1j * im)) < 1e-15
