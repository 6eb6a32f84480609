"""Dense Galerkin matrices S (eq. (4)), N (eq. (2)) and Gram G (Sec. II).

Test infrastructure.  Everything reduces to segment-pair moments

    M_uv(a, b) = int_a int_b g(|r - r'|) tau^u sigma^v ds ds',  u, v in {0, 1},

where tau (sigma) runs from 0 to 1 along segment a (b) from its first vertex
and ds is arc length.  A basis function restricted to a segment is
c0 + c1 tau (pulse: 1; hat: tau rising, 1 - tau falling), so

  [S]_ij = sum_{a in supp i, b in supp j} sum_uv p_u^i p_v^j M_uv(a, b)
  [N]_ij = sum_{a,b} [ phi_i'|_a phi_j'|_b M_00 - k^2 (t_a . t_b) (phi_i phi_j moments) ]

The N entry is the Maue (integrated-by-parts) form of the hypersingular
operator of eq. (2); its sign is fixed by the circle eigenvalue
(j pi a k^2 / 2) J_n'(ka) H_n^(2)'(ka) of -d/dn int d/dn' g.

Quadrature (eq. (7) is "to be understood in a formal sense" for the singular
entries; here they are integrated properly):
  * disjoint segments: tensor Gauss-Legendre with p points per segment; a
    pair closer than half its longer length is first split recursively (the
    longer piece halved) until every piece pair is at least half its longer
    piece length apart, so the nearly singular kernel stays resolved next to
    a short segment;
  * identical segments: with delta = |tau - sigma| the double integral
    collapses to int_0^1 g(h delta) Q_uv(delta) d delta, Q_uv a polynomial.
    g = -(1/2pi) J0(kR) ln R + F(R); the J0 ln part is integrated exactly
    term by term of the J0 power series, F by Gauss-Legendre (24 series
    terms: accurate to FP64 rounding for k h up to one wavelength per
    segment, k h <= 2 pi; past a few wavelengths the terms cancel);
  * segments sharing a vertex: polar coordinates (rho, psi) about the shared
    vertex; the rho integral of rho^q (ln rho + ln r(psi)) is exact term by
    term, psi by Gauss-Legendre on the two sub-ranges split at the rectangle
    diagonal; F by tensor Gauss-Legendre.  At an acute vertex the two
    segments fold towards each other and ln r(psi) is nearly singular at
    psi = pi/4 (r^2 = 1 - c + 2 c t^2 + ..., t = psi - pi/4, c the cosine of
    the vertex angle), with complex poles at t = +-i delta,
    delta = sqrt((1 - c) / (2 c)); the psi panels are then graded towards
    pi/4 at pi/4 +- delta 2^j.

Pinned by: tests/test_oracle_galerkin.py (self, adjacent and close disjoint
moments vs adaptive QUADPACK, with the logarithm taken by QUADPACK's
log-weighted rule, over k h up to 2 pi, unequal lengths, acute vertices and
gaps down to 1/50 of the segment length; circle eigenvalues of S and N,
Calderon S*N -> 1/4, symmetry S = S^T, N = N^T, Gram closed form vs
quadrature).
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import gauss_legendre01, segments
from .green import green, green_regular, j0_series_coeffs

TWO_PI = 2.0 * math.pi


# --------------------------------------------------------------------------
# segment-pair moments
# --------------------------------------------------------------------------
def _seg_dist(P0, P1, Q0, Q1):
    """Distance between two segments that do not cross: the smallest of the
    four endpoint-to-segment distances."""
    def pt(P, A, B):
        d = B - A
        L2 = float(d @ d)
        t = 0.0 if L2 == 0.0 else min(1.0, max(0.0, float((P - A) @ d) / L2))
        return float(np.hypot(*(P - (A + t * d))))
    return min(pt(P0, Q0, Q1), pt(P1, Q0, Q1), pt(Q0, P0, P1), pt(Q1, P0, P1))


def _seg_dist_arr(P0, P1, Q0, Q1):
    """_seg_dist for arrays of segment pairs, (P, 2) each."""
    def pt(P, A, B):
        d = B - A
        L2 = np.sum(d * d, axis=1)
        t = np.clip(np.sum((P - A) * d, axis=1) / np.where(L2 > 0, L2, 1.0), 0.0, 1.0)
        e = P - (A + t[:, None] * d)
        return np.hypot(e[:, 0], e[:, 1])
    return np.minimum(np.minimum(pt(P0, Q0, Q1), pt(P1, Q0, Q1)), np.minimum(pt(Q0, P0, P1), pt(Q1, P0, P1)))


def disjoint_pieces(A0, A1, B0, B1, eta=0.5, max_depth=40):
    """Parameter boxes (t0, t1, s0, s1) covering [0, 1]^2 for a pair of
    disjoint segments: a box whose pieces lie closer than eta times the
    longer piece length is split by halving its longer piece."""
    A0, A1, B0, B1 = (np.asarray(v, dtype=float) for v in (A0, A1, B0, B1))
    ha = float(np.hypot(*(A1 - A0)))
    hb = float(np.hypot(*(B1 - B0)))
    out = []
    stack = [(0.0, 1.0, 0.0, 1.0, 0)]
    while stack:
        t0, t1, s0, s1, dep = stack.pop()
        la, lb = ha * (t1 - t0), hb * (s1 - s0)
        d = _seg_dist(A0 + (A1 - A0) * t0, A0 + (A1 - A0) * t1, B0 + (B1 - B0) * s0, B0 + (B1 - B0) * s1)
        if d >= eta * max(la, lb) or dep >= max_depth:
            out.append((t0, t1, s0, s1))
        elif la >= lb:
            tm = 0.5 * (t0 + t1)
            stack += [(tm, t1, s0, s1, dep + 1), (t0, tm, s0, s1, dep + 1)]
        else:
            sm = 0.5 * (s0 + s1)
            stack += [(t0, t1, sm, s1, dep + 1), (t0, t1, s0, sm, dep + 1)]
    return out


def _moments_boxes(A0, A1, B0, B1, k, p, boxes):
    """Tensor Gauss-Legendre moments of one segment pair summed over
    parameter boxes (t0, t1, s0, s1), (2, 2) complex."""
    x, w = gauss_legendre01(p)
    bx = np.asarray(boxes, dtype=float)
    tau = bx[:, 0:1] + (bx[:, 1:2] - bx[:, 0:1]) * x[None, :]        # (nb, p)
    sig = bx[:, 2:3] + (bx[:, 3:4] - bx[:, 2:3]) * x[None, :]
    wt = (bx[:, 1:2] - bx[:, 0:1]) * w[None, :]
    ws = (bx[:, 3:4] - bx[:, 2:3]) * w[None, :]
    ra = A0[None, None, :] + (A1 - A0)[None, None, :] * tau[..., None]   # (nb, p, 2)
    rb = B0[None, None, :] + (B1 - B0)[None, None, :] * sig[..., None]
    d = ra[:, :, None, :] - rb[:, None, :, :]
    G = green(np.hypot(d[..., 0], d[..., 1]), k) * wt[:, :, None] * ws[:, None, :]
    f = float(np.hypot(*(A1 - A0)) * np.hypot(*(B1 - B0)))
    out = np.empty((2, 2), dtype=complex)
    out[0, 0] = G.sum() * f
    out[1, 0] = np.einsum('bij,bi->', G, tau) * f
    out[0, 1] = np.einsum('bij,bj->', G, sig) * f
    out[1, 1] = np.einsum('bij,bi,bj->', G, tau, sig) * f
    return out


def _moments_disjoint(A0, A1, B0, B1, k, p):
    """Tensor Gauss-Legendre moments for arrays of disjoint segment pairs.
    A0, A1, B0, B1: (P, 2).  Returns (P, 2, 2) complex.  Pairs closer than
    half their longer length are integrated over the boxes of
    disjoint_pieces."""
    tau, w = gauss_legendre01(p)
    ha = np.hypot(*(A1 - A0).T)
    hb = np.hypot(*(B1 - B0).T)
    out = np.empty((A0.shape[0], 2, 2), dtype=complex)
    chunk = max(1, 400000 // (p * p))
    for s in range(0, A0.shape[0], chunk):
        e = slice(s, s + chunk)
        ra = A0[e, None, :] + (A1 - A0)[e, None, :] * tau[None, :, None]   # (c,p,2)
        rb = B0[e, None, :] + (B1 - B0)[e, None, :] * tau[None, :, None]
        d = ra[:, :, None, :] - rb[:, None, :, :]
        R = np.hypot(d[..., 0], d[..., 1])                                # (c,p,p)
        G = green(R, k) * (w[:, None] * w[None, :])[None]
        f = (ha[e] * hb[e])[:, None, None]
        out[e, 0, 0] = (G.sum(axis=(1, 2))) * f[:, 0, 0]
        out[e, 1, 0] = np.einsum('cij,i->c', G, tau) * f[:, 0, 0]
        out[e, 0, 1] = np.einsum('cij,j->c', G, tau) * f[:, 0, 0]
        out[e, 1, 1] = np.einsum('cij,i,j->c', G, tau, tau) * f[:, 0, 0]
    for i in np.nonzero(_seg_dist_arr(A0, A1, B0, B1) < 0.5 * np.maximum(ha, hb))[0]:
        out[i] = _moments_boxes(A0[i], A1[i], B0[i], B1[i], k, p, disjoint_pieces(A0[i], A1[i], B0[i], B1[i]))
    return out


# Q_uv(delta) = int_0^{1-delta} [(s+delta)^u s^v + s^u (s+delta)^v] ds
_Q_SELF = {
    (0, 0): np.array([2.0, -2.0]),
    (1, 0): np.array([1.0, -1.0]),
    (0, 1): np.array([1.0, -1.0]),
    (1, 1): np.array([2.0 / 3.0, -1.0, 0.0, 1.0 / 3.0]),
}


def moments_self(h, k, nq=24, nterms=24):
    """Moments M_uv of a segment of length h with itself, (2, 2) complex."""
    cm = j0_series_coeffs(k, nterms)
    x, w = gauss_legendre01(nq)
    F = green_regular(h * x, k)
    out = np.empty((2, 2), dtype=complex)
    lnh = math.log(h)
    for (u, v), q in _Q_SELF.items():
        # log part: -(1/2pi) sum_m c_m h^{2m} int_0^1 delta^{2m} ln(h delta) Q(delta)
        acc = 0.0
        for m in range(nterms):
            sm = 0.0
            for pp, qc in enumerate(q):
                e = 2 * m + pp + 1
                sm += qc * (lnh / e - 1.0 / (e * e))
            acc += cm[m] * h ** (2 * m) * sm
        logpart = -acc / TWO_PI
        smooth = np.sum(w * F * np.polyval(q[::-1], x))
        out[u, v] = h * h * (logpart + smooth)
    return out


def psi_panels(psid, cab):
    """Panels of the polar angle psi in [0, pi/2] about a shared vertex:
    split at the rectangle diagonal psid = atan(h_b / h_a).  Beyond it the
    radial limit h_b / sin(psi) has its pole at psi = 0, before it h_a /
    cos(psi) at pi/2: for unequal lengths the panels are graded away from
    psid at psid 2^j and pi/2 - (pi/2 - psid) 2^j.  At an acute vertex
    (cab > 0, the cosine of the angle between the two segments) also at pi/4
    and at pi/4 +- delta 2^j, delta = sqrt((1 - cab) / (2 cab)), the distance
    of the complex poles of ln r(psi) from the real axis."""
    q = 0.25 * math.pi
    bps = {0.0, psid, 0.5 * math.pi}
    j = 1
    while psid * 2.0 ** j < 0.5 * math.pi and j < 48:
        bps.add(psid * 2.0 ** j)
        j += 1
    j = 1
    while 0.5 * math.pi - (0.5 * math.pi - psid) * 2.0 ** j > 0.0 and j < 48:
        bps.add(0.5 * math.pi - (0.5 * math.pi - psid) * 2.0 ** j)
        j += 1
    if cab > 0.0:
        delta = max(math.sqrt(max(1.0 - cab, 0.0) / (2.0 * cab)), 1e-12)
        bps.add(q)
        j = 0
        while delta * 2.0 ** j < q and j < 48:
            bps.add(q - delta * 2.0 ** j)
            bps.add(q + delta * 2.0 ** j)
            j += 1
    bps = sorted(bps)
    return [(a, b) for a, b in zip(bps[:-1], bps[1:]) if b > a]


def moments_adjacent(A0, A1, B0, B1, k, nq=32, nterms=24, pf=16):
    """Moments M_uv for two segments sharing exactly one vertex.

    tau runs A0 -> A1 and sigma runs B0 -> B1 (the segments' own orientation)."""
    A0, A1, B0, B1 = (np.asarray(v, dtype=float) for v in (A0, A1, B0, B1))
    if np.array_equal(A1, B0):
        V, Pa, Pb = A1, A0, B1
        a_from_v = False   # tau = 1 - s/ha
        b_from_v = True    # sigma = s'/hb
    elif np.array_equal(B1, A0):
        V, Pa, Pb = A0, A1, B0
        a_from_v = True
        b_from_v = False
    else:
        raise ValueError("segments do not share a vertex in chain order")
    ha = float(np.hypot(*(Pa - V)))
    hb = float(np.hypot(*(Pb - V)))
    ea = (Pa - V) / ha
    eb = (Pb - V) / hb
    cab = float(ea @ eb)
    # tau = t0 + t1 s ; sigma = s0 + s1 s'
    t0, t1 = (0.0, 1.0 / ha) if a_from_v else (1.0, -1.0 / ha)
    s0, s1 = (0.0, 1.0 / hb) if b_from_v else (1.0, -1.0 / hb)
    # polynomial weights in (s, s') of tau^u sigma^v: dict (i,j)->coef
    def poly(u, v):
        pa = {0: 1.0} if u == 0 else {0: t0, 1: t1}
        pb = {0: 1.0} if v == 0 else {0: s0, 1: s1}
        return {(i, j): ca * cb for i, ca in pa.items() for j, cb in pb.items()}

    cm = j0_series_coeffs(k, nterms)
    psid = math.atan2(hb, ha)
    out = np.empty((2, 2), dtype=complex)
    # psi quadrature on [0, psid] and [psid, pi/2], each graded towards
    # pi/4 at an acute vertex
    xg, wg = gauss_legendre01(nq)
    segs = [(lo, hi, (lambda ps: ha / np.cos(ps)) if hi <= psid else (lambda ps: hb / np.sin(ps)))
            for lo, hi in psi_panels(psid, cab)]
    # smooth part: tensor GL on the rectangle in (s, s')
    xs, ws = gauss_legendre01(pf)
    S, Sp = np.meshgrid(xs * ha, xs * hb, indexing='ij')
    Rr = np.sqrt(np.maximum(S * S + Sp * Sp - 2.0 * S * Sp * cab, 0.0))
    Fr = green_regular(Rr, k) * np.outer(ws * ha, ws * hb)
    for u in (0, 1):
        for v in (0, 1):
            P = poly(u, v)
            logacc = 0.0
            for lo, hi, rmax_fn in segs:
                ps = lo + (hi - lo) * xg
                wps = (hi - lo) * wg
                cps, sps = np.cos(ps), np.sin(ps)
                r2 = 1.0 - 2.0 * cps * sps * cab
                lnr = 0.5 * np.log(r2)
                Pm = rmax_fn(ps)
                lnP = np.log(Pm)
                tot = np.zeros_like(ps)
                for (i, j), c in P.items():
                    ang = c * cps ** i * sps ** j
                    for m in range(nterms):
                        q = 2 * m + i + j + 1          # power of rho incl. Jacobian
                        e = q + 1
                        rho_ln = Pm ** e * (lnP / e - 1.0 / (e * e))
                        rho_1 = Pm ** e / e
                        tot = tot + ang * cm[m] * r2 ** m * (rho_ln + lnr * rho_1)
                logacc += np.sum(wps * tot)
            smooth = np.sum(Fr * ((t0 + t1 * S) ** u) * ((s0 + s1 * Sp) ** v))
            out[u, v] = -logacc / TWO_PI + smooth
    return out


def segment_pair_moments(xy, pairs, k, p_far=10, p_near=16, near_factor=3.0):
    """Moments for an array of (a, b) segment index pairs, (P, 2, 2) complex.

    Identical and vertex-sharing pairs use the singular rules; other pairs
    use tensor Gauss-Legendre with p_near points when their midpoints are
    closer than near_factor * max(h_a, h_b), else p_far points."""
    xy = np.asarray(xy, dtype=float)
    A0s, A1s, h, _, _ = segments(xy)
    nseg = xy.shape[0]
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    a, b = pairs[:, 0], pairs[:, 1]
    out = np.empty((pairs.shape[0], 2, 2), dtype=complex)
    self_m = a == b
    adj = ((b - a) % nseg == 1) | ((a - b) % nseg == 1)
    adj &= ~self_m
    cache_self = {}
    for i in np.nonzero(self_m)[0]:
        hh = h[a[i]]
        key = round(hh, 15)
        if key not in cache_self:
            cache_self[key] = moments_self(hh, k)
        out[i] = cache_self[key]
    for i in np.nonzero(adj)[0]:
        out[i] = moments_adjacent(A0s[a[i]], A1s[a[i]], A0s[b[i]], A1s[b[i]], k)
    rest = ~(self_m | adj)
    if np.any(rest):
        ia = a[rest]
        ib = b[rest]
        mida = 0.5 * (A0s[ia] + A1s[ia])
        midb = 0.5 * (A0s[ib] + A1s[ib])
        dist = np.hypot(*(mida - midb).T)
        close = dist < near_factor * np.maximum(h[ia], h[ib])
        idx = np.nonzero(rest)[0]
        for flag, p in ((close, p_near), (~close, p_far)):
            if np.any(flag):
                sel = idx[flag]
                out[sel] = _moments_disjoint(A0s[a[sel]], A1s[a[sel]],
                                             A0s[b[sel]], A1s[b[sel]], k, p)
    return out


# --------------------------------------------------------------------------
# basis-pair assembly
# --------------------------------------------------------------------------
def _basis_piece_arrays(nseg, basis):
    """Per basis j and piece r: segment index, c0, c1 (phi = c0 + c1 tau)."""
    j = np.arange(nseg)
    if basis == 0:
        seg = j[:, None]
        c0 = np.ones((nseg, 1))
        c1 = np.zeros((nseg, 1))
    else:
        seg = np.stack([(j - 1) % nseg, j], axis=1)
        c0 = np.tile(np.array([0.0, 1.0]), (nseg, 1))
        c1 = np.tile(np.array([1.0, -1.0]), (nseg, 1))
    return seg, c0, c1


def assemble_entries(xy, basis, k, pairs, operator, p_far=10, p_near=16):
    """Entries [S]_ij or [N]_ij for an array of basis index pairs (i, j).

    operator: 'S' (single layer, eq. (4)) or 'N' (Maue form of eq. (2))."""
    xy = np.asarray(xy, dtype=float)
    nseg = xy.shape[0]
    _, _, h, t, _ = segments(xy)
    seg, c0, c1 = _basis_piece_arrays(nseg, basis)
    npc = seg.shape[1]
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    I, J = pairs[:, 0], pairs[:, 1]
    sp, owners, coefs = [], [], []
    for ra in range(npc):
        for rb in range(npc):
            sa = seg[I, ra]
            sb = seg[J, rb]
            pa = np.stack([c0[I, ra], c1[I, ra]], axis=1)     # (P, 2)
            pb = np.stack([c0[J, rb], c1[J, rb]], axis=1)
            w = (pa[:, :, None] * pb[:, None, :]).astype(complex)
            if operator == 'N':
                tt = np.sum(t[sa] * t[sb], axis=1)
                w *= -(k * k) * tt[:, None, None]
                w[:, 0, 0] += (c1[I, ra] / h[sa]) * (c1[J, rb] / h[sb])
            elif operator != 'S':
                raise ValueError(operator)
            sp.append(np.stack([sa, sb], axis=1))
            owners.append(np.arange(pairs.shape[0]))
            coefs.append(w)
    sp = np.concatenate(sp)
    owners = np.concatenate(owners)
    coefs = np.concatenate(coefs)
    uniq, inv = np.unique(sp, axis=0, return_inverse=True)
    M = segment_pair_moments(xy, uniq, k, p_far=p_far, p_near=p_near)
    vals = np.einsum('quv,quv->q', coefs, M[inv.ravel()])
    out = np.zeros(pairs.shape[0], dtype=complex)
    np.add.at(out, owners, vals)
    return out


def dense_matrix(xy, basis, k, operator, p_far=10, p_near=16):
    """Full N x N Galerkin matrix (small N only)."""
    n = np.asarray(xy).shape[0]
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing='ij')
    pairs = np.stack([ii.ravel(), jj.ravel()], axis=1)
    return assemble_entries(xy, basis, k, pairs, operator, p_far, p_near).reshape(n, n)


def gram(xy, basis):
    """Gram matrix [G]_ij = <phi_i, phi_j> as dense (closed form).

    Pulses: diag(h).  Hats: cyclic tridiagonal with (h_{i-1} + h_i)/3 on the
    diagonal, h_i/6 between hats i and i+1 (they share segment i)."""
    _, _, h, _, _ = segments(xy)
    n = h.size
    if basis == 0:
        return np.diag(h)
    G = np.zeros((n, n))
    for i in range(n):
        G[i, i] = (h[i - 1] + h[i]) / 3.0
        G[i, (i + 1) % n] += h[i] / 6.0
        G[(i + 1) % n, i] += h[i] / 6.0
    return G


def gram_solve(xy, basis, rhs):
    """G^{-1} rhs.  Hats: banded solve of the tridiagonal part plus a
    Sherman-Morrison correction for the two cyclic corner entries."""
    from scipy.linalg import solve_banded
    _, _, h, _, _ = segments(xy)
    rhs = np.asarray(rhs)
    if basis == 0:
        return rhs / (h[:, None] if rhs.ndim == 2 else h)
    n = h.size
    diag = (np.roll(h, 1) + h) / 3.0
    off = h[:-1] / 6.0               # G[i, i+1] for i < n-1
    corner = h[n - 1] / 6.0          # G[0, n-1] = G[n-1, 0]
    # G = T + u v^T with u = (gam, 0..0, corner), v = (1, 0..0, corner/gam)
    gam = -diag[0]
    d2 = diag.copy()
    d2[0] -= gam
    d2[-1] -= corner * corner / gam
    ab = np.zeros((3, n))
    ab[0, 1:] = off
    ab[1] = d2
    ab[2, :-1] = off
    u = np.zeros(n)
    u[0] = gam
    u[-1] = corner
    v = np.zeros(n)
    v[0] = 1.0
    v[-1] = corner / gam
    y = solve_banded((1, 1), ab, rhs)
    z = solve_banded((1, 1), ab, u)
    if rhs.ndim == 1:
        return y - z * (v @ y) / (1.0 + v @ z)
    return y - np.outer(z, v @ y) / (1.0 + v @ z)
