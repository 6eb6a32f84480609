"""Pins of oracle.geometry and the shared contour generators."""
import math

import numpy as np

from oracle.geometry import gauss_legendre01, segments
from paper_2606_10784_amd import workloads as wl


def test_inscribed_polygon_perimeter_closed_form():
    a, n = 1.7, 97
    _, _, h, _, _ = segments(wl.circle(a, n))
    assert abs(h.sum() - 2 * n * a * math.sin(math.pi / n)) < 1e-13


def test_normals_point_outward_and_tangents_ccw():
    xy = wl.circle(2.0, 64)
    a, b, h, t, nrm = segments(xy)
    mid = 0.5 * (a + b)
    assert np.all(np.sum(nrm * mid, axis=1) > 0)
    # CCW: z-component of mid x t is positive
    assert np.all(mid[:, 0] * t[:, 1] - mid[:, 1] * t[:, 0] > 0)


def test_gauss_legendre_exactness():
    for p in (1, 4, 10, 16):
        x, w = gauss_legendre01(p)
        for deg in range(2 * p):
            assert abs(np.sum(w * x ** deg) - 1.0 / (deg + 1)) < 1e-14
        if p <= 4:   # degree 2p is not integrated exactly
            assert abs(np.sum(w * x ** (2 * p)) - 1.0 / (2 * p + 1)) > 1e-6


def test_star_equal_arc_and_on_curve():
    from scipy.integrate import quad
    a = 2.0
    xy = wl.star5(a, 400)
    # arc length between consecutive nodes, integrated independently
    th_n = np.unwrap(np.arctan2(xy[:, 1], xy[:, 0]))
    dens = lambda t: math.hypot(a * (1 + 0.3 * math.cos(5 * t)), -1.5 * a * math.sin(5 * t))
    arcs = [quad(dens, th_n[i], th_n[i + 1], epsabs=1e-16, epsrel=1e-13)[0] for i in range(0, 399, 7)]
    assert (max(arcs) - min(arcs)) / np.mean(arcs) < 1e-9
    # at a fine mesh the chords are uniform too
    _, _, h, _, _ = segments(wl.star5(a, 4000))
    assert (h.max() - h.min()) / h.mean() < 1e-4
    th = np.arctan2(xy[:, 1], xy[:, 0])
    r = np.hypot(xy[:, 0], xy[:, 1])
    assert np.max(np.abs(r - a * (1 + 0.3 * np.cos(5 * th)))) < 1e-12
    # counter-clockwise ordering: positive signed area
    area = 0.5 * np.sum(xy[:, 0] * np.roll(xy[:, 1], -1) - np.roll(xy[:, 0], -1) * xy[:, 1])
    assert area > 0
