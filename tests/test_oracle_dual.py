"""Pins of oracle.dual: the dual (barycentric) hats, the mixed Gram matrix
and the TM Calderon product."""
import math

import numpy as np

from oracle import dual, galerkin, mie
from oracle.geometry import gauss_legendre01, segments
from paper_2606_10784_amd import workloads as wl


def _psi_at_refined_vertex(j, q, n):
    """Pointwise definition of psi_j at refined vertex q (2n of them): 1 at
    the midpoint 2j+1, 1/2 at the vertices 2j and 2j+2, else 0."""
    q %= 2 * n
    if q == 2 * j + 1:
        return 1.0
    if q == 2 * j or q == (2 * j + 2) % (2 * n):
        return 0.5
    return 0.0


def test_mixed_gram_matches_quadrature_of_the_dual_hats():
    xy = wl.star5(1.0, 30)                   # unequal segments
    n = xy.shape[0]
    rf = dual.refined_polygon(xy)
    A0, A1, hr, _, _ = segments(rf)
    tau, w = gauss_legendre01(4)             # psi is linear on each refined segment
    G = dual.mixed_gram(xy)
    for i in range(n):                       # pulse i covers refined segments 2i, 2i+1
        for j in range(n):
            val = 0.0
            for s in (2 * i, 2 * i + 1):
                a, b = _psi_at_refined_vertex(j, s, n), _psi_at_refined_vertex(j, s + 1, n)
                val += np.sum(w * hr[s] * ((1 - tau) * a + tau * b))
            assert abs(val - G[i, j]) < 1e-15, (i, j)
    # refined polygon: the same curve, every segment halved
    _, _, h, _, _ = segments(xy)
    assert np.allclose(hr[0::2], 0.5 * h) and np.allclose(hr[1::2], 0.5 * h)


def test_combination_reproduces_the_dual_hats_at_the_refined_vertices():
    n = 11
    R = dual.dual_combination(n)
    for j in range(n):
        for q in range(2 * n):
            assert R[j, q] == _psi_at_refined_vertex(j, q, n)


def test_mixed_gram_invertible_where_the_primal_pairing_is_not():
    """Even N: the pulse/primal-hat pairing is singular at the alternating
    mode; the pulse/dual-hat pairing has eigenvalues in [h/2, h]."""
    xy = wl.circle(1.0, 32)
    _, _, h, _, _ = segments(xy)
    Gph = np.zeros((32, 32))
    for i in range(32):                      # <pulse_i, hat_j>: h/2 for j = i, i+1
        Gph[i, i] = Gph[i, (i + 1) % 32] = h[i] / 2
    alt = (-1.0) ** np.arange(32)
    assert np.linalg.norm(Gph @ alt) < 1e-12
    ev = np.linalg.eigvals(dual.mixed_gram(xy))
    assert np.all(np.abs(ev) > 0.49 * h[0]) and np.all(np.abs(ev) < 1.01 * h[0])


def test_dense_tm_calderon_product_on_a_circle():
    """A = G_pd^-T R N' R^T G_pd^-1 S with dense Galerkin S (pulses) and N'
    (refined hats) is circulant on a regular polygon; its Fourier
    eigenvalues converge (second order in h) to lambda^N lambda^S of the
    circle and level off at 1/4 (Calderon identity N S = 1/4 + compact, with
    this sign of N)."""
    a, k = 0.5, 2 * math.pi
    nus = np.arange(0, 13)
    ex = mie.circle_eig_S(nus, k, a) * mie.circle_eig_N(nus, k, a)
    err = {}
    for n in (40, 80):
        xy = wl.circle(a, n)
        S = galerkin.dense_matrix(xy, 0, k, 'S', p_far=12, p_near=16)
        Nr = galerkin.dense_matrix(dual.refined_polygon(xy), 1, k, 'N', p_far=12, p_near=16)
        R, G = dual.dual_combination(n), dual.mixed_gram(xy)
        A = np.linalg.solve(G.T, R @ Nr @ R.T @ np.linalg.solve(G, S))
        th = 2 * math.pi * np.arange(n) / n
        q = np.array([np.vdot(np.exp(1j * v * th), A @ np.exp(1j * v * th)) / n for v in nus])
        err[n] = np.abs(q - ex)
        print(n, "max |q - lambda^N lambda^S| for nu <= 12:", err[n].max())
    assert err[80].max() < 0.005
    assert err[80][:7].max() < 0.35 * err[40][:7].max()
    assert np.all(np.abs(q[7:] - 0.25) < 0.005)


def test_aim_tm_calderon_unfiltered_close_to_dense():
    """The AIM form (4 x 4 stencils with the near-field correction on both
    meshes) of the unfiltered operator approximates the dense Galerkin one."""
    n, a, k, eps = 40, 0.5, 2 * math.pi, 0.05
    xy = wl.circle(a, n)
    orc = dual.TMCalderonOracle(xy, k, wl.ETA0, wl.grid_side_for(dual.refined_polygon(xy), eps), eps)
    S = galerkin.dense_matrix(xy, 0, k, 'S', p_far=12, p_near=16)
    Nr = galerkin.dense_matrix(dual.refined_polygon(xy), 1, k, 'N', p_far=12, p_near=16)
    R, G = dual.dual_combination(n), dual.mixed_gram(xy)
    Ad = np.linalg.solve(G.T, R @ Nr @ R.T @ np.linalg.solve(G, 1j * k * wl.ETA0 * S))
    rng = np.random.default_rng(4)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = orc.apply('TM_CP_UNF', x)
    err = np.linalg.norm(y - Ad @ x) / np.linalg.norm(Ad @ x)
    print("AIM vs dense TM Calderon", err)
    assert err < 2e-3
