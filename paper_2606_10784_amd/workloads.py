"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds only input generation: closed contours (the scatterer
curve gamma of Sec. II), grid parameters, incidence angles and seeded probe
vectors.  It contains none of the method's arithmetic (no Green's function,
no quadrature of the operators, no grid maps) and imports neither the HIP
binding nor the oracle.

Units: wavelength lambda = 1, so k = 2*pi; eta is the free-space impedance.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ETA0 = 376.730313668
LAMBDA = 1.0
K0 = 2.0 * math.pi / LAMBDA

PULSE = 0
HAT = 1


# --------------------------------------------------------------------------
# contours (closed, counter-clockwise polygons)
# --------------------------------------------------------------------------
def circle(a: float, n: int) -> np.ndarray:
    """n vertices of a regular polygon inscribed in the circle of radius a,
    counter-clockwise, first vertex on the +x axis."""
    th = 2.0 * np.pi * np.arange(n) / n
    return np.stack([a * np.cos(th), a * np.sin(th)], axis=1)


def _fourier_curve(a, coef, phase):
    """r(theta) = a * (1 + sum_m coef[m] cos(m theta + phase[m])), m = 1.."""
    coef = np.asarray(coef, dtype=float)
    phase = np.asarray(phase, dtype=float)
    ms = np.arange(1, len(coef) + 1)

    def r(th):
        th = np.asarray(th, dtype=float)[..., None]
        return a * (1.0 + np.sum(coef * np.cos(ms * th + phase), axis=-1))

    def dr(th):
        th = np.asarray(th, dtype=float)[..., None]
        return a * np.sum(-coef * ms * np.sin(ms * th + phase), axis=-1)

    return r, dr


def equal_arc_polygon(r, dr, n: int, modes: int = 512) -> np.ndarray:
    """n vertices at equal arc length along the smooth star-shaped curve
    (r(theta) cos theta, r(theta) sin theta), counter-clockwise.

    The arc-length density f(theta) = sqrt(r^2 + r'^2) is periodic and smooth,
    so its Fourier series (from equispaced samples) integrates exactly term by
    term; Newton's method then inverts the cumulative arc length.
    """
    m = 2 * modes
    tg = 2.0 * np.pi * np.arange(m) / m
    f = np.sqrt(r(tg) ** 2 + dr(tg) ** 2)
    fh = np.fft.rfft(f) / m
    total = 2.0 * np.pi * fh[0].real
    kk = np.arange(1, len(fh))

    def s_of(th):
        # s(theta) = f0*theta + 2 Re sum_k fh_k (e^{ik theta} - 1) / (ik)
        out = fh[0].real * th
        chunk = 4096
        for i0 in range(0, th.size, chunk):
            t = th[i0:i0 + chunk, None]
            e = (np.exp(1j * kk * t) - 1.0) / (1j * kk)
            out[i0:i0 + chunk] += 2.0 * np.real(e @ fh[1:])
        return out

    target = total * np.arange(n) / n
    th = 2.0 * np.pi * np.arange(n) / n
    for _ in range(30):
        ds = s_of(th) - target
        th = th - ds / np.sqrt(r(th) ** 2 + dr(th) ** 2)
        if np.max(np.abs(ds)) < 1e-14 * total:
            break
    rr = r(th)
    return np.stack([rr * np.cos(th), rr * np.sin(th)], axis=1)


def star5(a: float, n: int, amp: float = 0.3, lobes: int = 5) -> np.ndarray:
    """Star r = a(1 + amp cos(lobes*theta)) meshed at equal arc length."""
    coef = np.zeros(lobes)
    coef[lobes - 1] = amp
    r, dr = _fourier_curve(a, coef, np.zeros(lobes))
    return equal_arc_polygon(r, dr, n)


def random_star(rng: np.random.Generator, a: float, n: int, mmax: int = 8,
                cmax: float = 0.05) -> np.ndarray:
    """r = a(1 + sum_{m<=mmax} c_m cos(m theta + phi_m)), c_m ~ U(0, cmax),
    phi_m ~ U(0, 2 pi), meshed at equal arc length."""
    c = rng.uniform(0.0, cmax, size=mmax)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=mmax)
    r, dr = _fourier_curve(a, c, ph)
    return equal_arc_polygon(r, dr, n)


def irregular_polygon(rng: np.random.Generator, a: float, n: int, depth: float = 0.35,
                      modes: int = 5, jitter: float = 0.45) -> np.ndarray:
    """A simple, star-shaped, generally non-convex CCW polygon with unequal
    segments: vertex angles theta_i = 2 pi (i + u_i) / n with u_i ~ U(-jitter,
    jitter), radii r = a (1 + sum_m c_m cos(m theta + phi_m)) with
    sum |c_m| <= depth < 1, so r > 0 and the sorted angles give a simple polygon."""
    th = 2.0 * np.pi * (np.arange(n) + rng.uniform(-jitter, jitter, size=n)) / n
    c = rng.uniform(0.0, 1.0, size=modes)
    c *= depth / max(c.sum(), 1e-300)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=modes)
    mm = np.arange(1, modes + 1)[:, None]
    r = a * (1.0 + np.sum(c[:, None] * np.cos(mm * th[None, :] + ph[:, None]), axis=0))
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


# --------------------------------------------------------------------------
# workload configurations
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    xy: np.ndarray            # (N, 2) vertices, CCW
    k: float
    eta: float
    basis: int                # PULSE (TM) or HAT (TE)
    m: int                    # grid points per side
    eps: float                # grid step
    quad: int = 10            # Gauss-Legendre nodes per segment
    near_radius: int = 6      # anchor Chebyshev radius of the near zone
    stencil: int = 4
    alpha: float = math.inf   # spectral cutoff of the filtered kernel
    phi_inc: list = field(default_factory=lambda: [0.0])
    tol: float = 1e-6

    @property
    def n_unknowns(self) -> int:
        return self.xy.shape[0]


def alpha_half_bins(eps: float) -> float:
    """Cutoff that keeps half of the DFT bins of the padded grid: the disc
    pi alpha^2 equals half the square (2 pi / eps)^2."""
    return math.sqrt(2.0 * math.pi) / eps


def cylinder_small(n: int = 512) -> Workload:
    """PEC circular cylinder of radius 1 lambda (ka = 2 pi), N pulse segments,
    grid 64 x 64 at lambda/10 (padded 128 x 128)."""
    eps = 0.1
    return Workload("cylinder_ka2pi_N512", circle(1.0, n), K0, ETA0, PULSE, 64, eps,
                    alpha=alpha_half_bins(eps))


def cylinder_large(n: int = 16384) -> Workload:
    """PEC circular cylinder ka = 200 (radius 31.83 lambda), N = 16384 pulse
    segments, grid 1024 x 1024 at lambda/15 (padded 2048 x 2048)."""
    a = 200.0 / K0
    eps = 1.0 / 15.0
    return Workload("cylinder_ka200_N16384", circle(a, n), K0, ETA0, PULSE, 1024, eps,
                    alpha=alpha_half_bins(eps))


def star_large(n: int = 65536, basis: int = HAT) -> Workload:
    """Star r = 20 lambda (1 + 0.3 cos 5 theta), N equal-arc unknowns,
    grid 2048 x 2048 at lambda/30 (padded 4096 x 4096)."""
    eps = 1.0 / 30.0
    return Workload("star_a20_N65536", star5(20.0, n), K0, ETA0, basis, 2048, eps,
                    alpha=alpha_half_bins(eps))


def paper_circle(basis: int = PULSE) -> Workload:
    """The paper's Sec. IV spectral experiment at its parameters (SI units):
    f = 0.4 GHz, mesh size h = pi/(15 k) (lambda/30), p = 10, grid step
    2.4 m / 599, cutoff alpha = 8 k.  The mesh of its figures is not given; a
    circle of radius 1 m (inside the paper's L = 1.2 m grid) with N = 30 k a
    segments.  The grid is the paper's, 600 points per side (L = 1.2 m); the
    library embeds it in FFTs of length 2048 (the paper's embedding has
    2m - 1 = 1199): the unfiltered products are the same, the numerical
    filter's DFT bins are finer."""
    c0 = 299792458.0
    k = 2.0 * math.pi * 0.4e9 / c0
    a = 1.0
    n = int(round(30.0 * k * a))
    return Workload(f"paper_circle_f0.4GHz_N{n}" + ("_hat" if basis == HAT else ""), circle(a, n), k, ETA0, basis,
                    600, 2.4 / 599.0, alpha=8.0 * k)


def scaled_cylinder(n: int, a: float, m: int, eps: float, basis: int = PULSE) -> Workload:
    """Small circular cylinders for parity tests spanning several tiles."""
    return Workload(f"cylinder_a{a:g}_N{n}_m{m}", circle(a, n), K0, ETA0, basis, m, eps,
                    alpha=alpha_half_bins(eps))


def probe_vector(n: int, nrhs: int = 1, seed: int = 0) -> np.ndarray:
    """Seeded complex normal probe x ~ CN(0, 1), column-major (n, nrhs)."""
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))) / math.sqrt(2.0)
    return np.ascontiguousarray(x.T) if nrhs > 1 else x[0]


def grid_side_for(xy: np.ndarray, eps: float, margin_cells: int = 4) -> int:
    """Smallest power of two m whose grid (m-1) eps covers the contour plus a
    stencil margin on each side."""
    rmax = float(np.max(np.abs(xy)))
    need = (2.0 * rmax + 2.0 * margin_cells * eps) / eps + 1.0
    m = 16
    while m < need:
        m *= 2
    return m


# --------------------------------------------------------------------------
# serving stream: random star contours at random frequencies
# --------------------------------------------------------------------------
@dataclass
class ServeRequest:
    rid: int
    arrival: float            # seconds after the stream starts
    xy: np.ndarray
    k: float
    eta: float
    m: int
    eps: float
    phis: np.ndarray          # incidence angles (one right-hand side each)
    precision: int            # 0 FP64, 1 mixed
    tol: float = 1e-6
    basis: int = PULSE


def serving_stream(n_req: int, rate: float, seed: int = 20261203, ka_range=(10.0, 400.0),
                   pts_per_lambda: float = 20.0, eps_lambda: float = 0.1, max_rhs: int = 16):
    """Poisson arrivals at `rate` per second of TM requests on seeded random
    stars r = a(1 + sum_{m<=8} c_m cos(m theta + phi_m)), a = 1,
    c_m ~ U(0, 0.05), ka ~ logU(ka_range), eps = eps_lambda * lambda (so
    k eps is the same for every request), N = pts_per_lambda points per
    wavelength of perimeter rounded up to a multiple of 256 (at least 1024),
    1..max_rhs incidence angles ~ U[0, 2 pi), precision FP64 or mixed with
    probability 1/2."""
    rng = np.random.default_rng(seed)
    rng_arr = np.random.default_rng([seed, 1])    # arrivals drawn apart: same requests at any rate
    t = 0.0
    out = []
    for i in range(n_req):
        t += rng_arr.exponential(1.0 / rate) if rate > 0 else 0.0
        ka = float(np.exp(rng.uniform(np.log(ka_range[0]), np.log(ka_range[1]))))
        k = ka                      # a = 1
        lam = 2.0 * np.pi / k
        c = rng.uniform(0.0, 0.05, size=8)
        ph = rng.uniform(0.0, 2.0 * np.pi, size=8)
        r, dr = _fourier_curve(1.0, c, ph)
        tg = 2.0 * np.pi * np.arange(4096) / 4096
        perim = float(np.mean(np.sqrt(r(tg) ** 2 + dr(tg) ** 2)) * 2.0 * np.pi)
        n = int(max(1024, 256 * int(np.ceil(pts_per_lambda * perim / lam / 256.0))))
        xy = equal_arc_polygon(r, dr, n)
        eps = eps_lambda * lam
        m = grid_side_for(xy, eps)
        nr = int(rng.integers(1, max_rhs + 1))
        phis = rng.uniform(0.0, 2.0 * np.pi, size=nr)
        prec = int(rng.integers(0, 2))
        out.append(ServeRequest(i, t, xy, k, ETA0, m, eps, phis, prec))
    return out
