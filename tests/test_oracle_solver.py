"""Pins of oracle.solver (restarted GMRES) against a direct dense solve."""
import math

import numpy as np

from oracle import excitation, galerkin
from oracle.solver import gmres
from paper_2606_10784_amd import workloads as wl

K = 2 * math.pi


def test_gmres_matches_direct_solve_within_condition_bound():
    xy = wl.circle(1.0, 96)
    A = 1j * K * wl.ETA0 * galerkin.dense_matrix(xy, 0, K, 'S')
    b = excitation.rhs_tm(xy, 0, K, 0.3)
    xd = np.linalg.solve(A, b)
    kappa = np.linalg.cond(A)
    for restart in (100, 8):
        x, info = gmres(lambda v: A @ v, b, tol=1e-8, restart=restart, maxit=3000)
        assert info['converged']
        assert np.linalg.norm(b - A @ x) <= 1.0000001e-8 * np.linalg.norm(b)
        assert np.linalg.norm(x - xd) <= kappa * 1e-8 * np.linalg.norm(xd)


def test_gmres_exact_in_n_steps_and_zero_rhs():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12)) + 8 * np.eye(12)
    b = rng.standard_normal(12) + 0j
    x, info = gmres(lambda v: A @ v, b, tol=1e-13, restart=12)
    assert info['iterations'] <= 12
    assert np.linalg.norm(A @ x - b) < 1e-12 * np.linalg.norm(b)
    x0, info0 = gmres(lambda v: A @ v, np.zeros(12), tol=1e-6)
    assert info0['converged'] and np.all(x0 == 0)
