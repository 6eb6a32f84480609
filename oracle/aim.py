"""AIM operators with the numerically filtered grid kernel (oracle).

Test infrastructure.  Passages followed (Sec. III):
  * grid of m x m points with step eps, centred at the origin, side
    2L = (m-1) eps, point (ix, iy) at (-L + ix eps, -L + iy eps), row-major
    index iy*m + ix                                                (Sec. III-A)
  * G_nodes ~ Lambda^T G_grid Lambda with a sparse projection Lambda and a
    Toeplitz G_grid whose entries are g at grid offsets            (Sec. III-A)
  * the Toeplitz product through a zero-padded circulant embedding (eq. (8))
  * numerical filter: the DFT of the circulant kernel truncated to the disc
    |kappa| <= alpha                                               (Sec. III-B)
  * filtered operator S^alpha = Lambda^T [F^-1(F(c^alpha) F(b))]_restr
    Lambda                                                         (eq. (10))
  * the self-interaction of G_grid is set to zero                  (Sec. III-C)

Readings taken where the paper is silent:
  * Lambda is folded with the quadrature weights and basis values of eq. (7)
    into one 4 x 4 tensor-product cubic Lagrange stencil per basis function,
    anchored at the cell holding the basis centre (pulse: segment midpoint,
    hat: its vertex): W_j[t*4+s] = sum_k w_k v_j(r_k) l_s(x_k) l_t(y_k).
    The per-node form (stencil_weights_node) gives every quadrature node its
    own P x P stencil at its own cell (nodes -(P/2-1) .. P/2, so P = 4 is the
    same cubic stencil); the paper's Sec. IV uses order 10.
  * padding n = 2m (default) with the ring |d| = m of the kernel zero, the
    paper's n = 2m - 1, or any given n >= 2m - 1 (the GPU library's FFT length
    is the smallest power of two >= 2m): every such embedding gives the same
    Toeplitz product; the numerical filter depends on n through its DFT bins.
  * the cutoff keeps bins with qx^2 + qy^2 <= (alpha n eps / 2 pi)^2,
    inclusive, with q in FFT order.
  * the accurate operators S and N get a near-field correction
    C = (exact Galerkin - Lambda^T G_grid Lambda) on pairs whose anchors are
    within a Chebyshev distance R_near; S^alpha has none (eq. (10)).

The grid product is evaluated here by a direct sum over the active grid
points (the union of all stencils), which is the Toeplitz definition itself;
the filtered kernel values come from one inverse DFT of the masked spectrum
(the definition of c^alpha).  An FFT form of eq. (8) is kept only as a
cross-check.

The alternative of Fig. 1(a), a grid kernel sampled from the analytically
filtered g^alpha of eq. (6), is analytic_filtered_table.

Pinned by: tests/test_oracle_aim.py (moment reproduction of the stencil
weights, per-node weights to degree P-1 and equal to the per-basis stencil
where all nodes of a basis share its anchor cell, FFT = direct Toeplitz sum, alpha >= sqrt(2) pi/eps is the identity
filter, kept-bin fraction, symmetry x^T A y = y^T A x, S_AIM -> dense S,
circle spectrum of S^alpha_AIM vs the analytic filter, the analytic table
at the origin closed form and against the tail form of eq. (6)).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree

from . import galerkin
from .geometry import gauss_legendre01, segments
from .green import green, green_alpha_lowpass, green_alpha_origin

CHANNELS_S = ('phi',)
CHANNELS_N = ('dphi', 'tx', 'ty')


class GeometryError(ValueError):
    pass


class Grid:
    def __init__(self, m: int, eps: float, pad: int = 0, n: int | None = None):
        self.m = int(m)
        self.eps = float(eps)
        self.L = 0.5 * (self.m - 1) * self.eps
        self.n = 2 * self.m if pad == 0 else 2 * self.m - 1
        if n is not None:
            if int(n) < 2 * self.m - 1:
                raise ValueError("a circulant embedding needs n >= 2m - 1")
            self.n = int(n)
        self.pad = pad

    def coord(self, i):
        return -self.L + np.asarray(i) * self.eps


def lagrange_cubic(tt):
    """Cubic Lagrange basis on nodes -1, 0, 1, 2 evaluated at tt: (..., 4)."""
    tt = np.asarray(tt, dtype=float)
    l0 = -tt * (tt - 1.0) * (tt - 2.0) / 6.0
    l1 = (tt + 1.0) * (tt - 1.0) * (tt - 2.0) / 2.0
    l2 = -(tt + 1.0) * tt * (tt - 2.0) / 2.0
    l3 = (tt + 1.0) * tt * (tt - 1.0) / 6.0
    return np.stack([l0, l1, l2, l3], axis=-1)


def basis_centers(xy, basis):
    xy = np.asarray(xy, dtype=float)
    if basis == 0:
        return 0.5 * (xy + np.roll(xy, -1, axis=0))
    return xy.copy()


def anchors(xy, basis, grid: Grid):
    """Anchor cell (ix0, iy0) per basis: floor((c + L)/eps)."""
    c = basis_centers(xy, basis)
    a = np.floor((c + grid.L) / grid.eps).astype(np.int64)
    if a.min() - 1 < 0 or a.max() + 2 > grid.m - 1:
        raise GeometryError("stencil leaves the grid")
    return a


def stencil_weights(xy, basis, grid: Grid, p: int, channel: str):
    """Weights W (N, 16) and grid linear indices G (N, 16) of one channel.

    channel 'phi': v = phi_j; 'dphi': arc-length derivative; 'tx', 'ty':
    tangent component times phi_j.  Entry e = t*4 + s, stencil point
    (ix0 - 1 + s, iy0 - 1 + t)."""
    xy = np.asarray(xy, dtype=float)
    nb = xy.shape[0]
    A0, A1, h, t, _ = segments(xy)
    anc = anchors(xy, basis, grid)
    tau, w = gauss_legendre01(p)
    if basis == 0:
        pieces = [(np.arange(nb), np.ones(nb), np.zeros(nb))]
    else:
        j = np.arange(nb)
        pieces = [((j - 1) % nb, np.zeros(nb), np.ones(nb)),
                  (j, np.ones(nb), -np.ones(nb))]
    W = np.zeros((nb, 4, 4))
    for seg, c0, c1 in pieces:
        pts = A0[seg, None, :] + (A1 - A0)[seg, None, :] * tau[None, :, None]   # (nb,p,2)
        wk = h[seg, None] * w[None, :]
        phi = c0[:, None] + c1[:, None] * tau[None, :]
        if channel == 'phi':
            val = phi
        elif channel == 'dphi':
            val = np.broadcast_to((c1 / h[seg])[:, None], phi.shape)
        elif channel == 'tx':
            val = t[seg, 0][:, None] * phi
        elif channel == 'ty':
            val = t[seg, 1][:, None] * phi
        else:
            raise ValueError(channel)
        tx = (pts[..., 0] + grid.L) / grid.eps - anc[:, 0, None]
        ty = (pts[..., 1] + grid.L) / grid.eps - anc[:, 1, None]
        lx = lagrange_cubic(tx)          # (nb,p,4)
        ly = lagrange_cubic(ty)
        W += np.einsum('bk,bkt,bks->bts', wk * val, ly, lx)
    s = np.arange(4)
    ix = anc[:, 0, None, None] - 1 + s[None, None, :]
    iy = anc[:, 1, None, None] - 1 + s[None, :, None]
    G = iy * grid.m + ix
    return W.reshape(nb, 16), G.reshape(nb, 16)


def lagrange_nodes(order: int):
    """Interpolation nodes of an order-P stencil, in cells relative to the
    anchor cell: -(P/2 - 1), ..., P/2 (P even; P = 4 gives -1, 0, 1, 2)."""
    if order < 2 or order % 2:
        raise ValueError("stencil order must be even and >= 2")
    return np.arange(order) - (order // 2 - 1)


def lagrange_basis(tt, order: int):
    """All order-P Lagrange basis polynomials at tt: (..., P), by the product
    formula l_i(t) = prod_{j != i} (t - x_j) / (x_i - x_j)."""
    xs = lagrange_nodes(order).astype(float)
    tt = np.asarray(tt, dtype=float)[..., None]
    out = np.ones(tt.shape[:-1] + (order,))
    for i in range(order):
        for j in range(order):
            if j != i:
                out[..., i] *= (tt[..., 0] - xs[j]) / (xs[i] - xs[j])
    return out


def stencil_weights_node(xy, basis, grid: Grid, p: int, channel: str, order: int):
    """Lambda in its per-node form (Sec. III-A: Lambda maps every quadrature
    node to the grid): node r_k of basis j gets its own order x order
    tensor-product Lagrange stencil anchored at floor((r_k + L)/eps), and the
    basis row of Lambda Q collects w_k v_j(r_k) l_s(x_k) l_t(y_k) over its
    nodes.  Returns (W, G) of shape (N, S): the union of a basis's node
    stencils in ascending grid index, padded to the widest basis with weight
    0 at the basis's first point."""
    xy = np.asarray(xy, dtype=float)
    nb = xy.shape[0]
    A0, A1, h, t, _ = segments(xy)
    tau, w = gauss_legendre01(p)
    xs = lagrange_nodes(order)
    if basis == 0:
        pieces = [(np.arange(nb), np.ones(nb), np.zeros(nb))]
    else:
        j = np.arange(nb)
        pieces = [((j - 1) % nb, np.zeros(nb), np.ones(nb)),
                  (j, np.ones(nb), -np.ones(nb))]
    bid, lin, wt = [], [], []
    for seg, c0, c1 in pieces:
        pts = A0[seg, None, :] + (A1 - A0)[seg, None, :] * tau[None, :, None]   # (nb,p,2)
        wk = h[seg, None] * w[None, :]
        phi = c0[:, None] + c1[:, None] * tau[None, :]
        val = {'phi': phi,
               'dphi': np.broadcast_to((c1 / h[seg])[:, None], phi.shape),
               'tx': t[seg, 0][:, None] * phi,
               'ty': t[seg, 1][:, None] * phi}[channel]
        gx = (pts[..., 0] + grid.L) / grid.eps
        gy = (pts[..., 1] + grid.L) / grid.eps
        ax, ay = np.floor(gx).astype(np.int64), np.floor(gy).astype(np.int64)
        if min(ax.min(), ay.min()) + xs[0] < 0 or max(ax.max(), ay.max()) + xs[-1] > grid.m - 1:
            raise GeometryError("stencil leaves the grid")
        lx = lagrange_basis(gx - ax, order)      # (nb,p,P)
        ly = lagrange_basis(gy - ay, order)
        f = wk * val                             # (nb,p)
        ix = ax[..., None, None] + xs[None, None, None, :]         # (nb,p,1,P)
        iy = ay[..., None, None] + xs[None, None, :, None]         # (nb,p,P,1)
        lin.append(np.broadcast_to(iy * grid.m + ix, (nb, p, order, order)).reshape(-1))
        wt.append((f[..., None, None] * ly[..., :, None] * lx[..., None, :]).reshape(-1))
        bid.append(np.broadcast_to(np.arange(nb)[:, None, None, None], (nb, p, order, order)).reshape(-1))
    bid, lin, wt = np.concatenate(bid), np.concatenate(lin), np.concatenate(wt)
    key = bid * (grid.m * grid.m) + lin
    uk, inv = np.unique(key, return_inverse=True)
    acc = np.zeros(uk.size)
    np.add.at(acc, inv, wt)
    ub = uk // (grid.m * grid.m)
    counts = np.bincount(ub, minlength=nb)
    S = int(counts.max())
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    W = np.zeros((nb, S))
    G = np.repeat((uk[starts] % (grid.m * grid.m))[:, None], S, axis=1)
    pos = np.arange(uk.size) - starts[ub]
    W[ub, pos] = acc
    G[ub, pos] = uk % (grid.m * grid.m)
    return W, G


def kernel_table(grid: Grid, k: float):
    """T[dy, dx] = g(eps |d|) for 0 <= dx, dy <= m-1, T[0, 0] = 0 (Sec. III-C)."""
    d = np.arange(grid.m) * grid.eps
    R = np.hypot(d[:, None], d[None, :])
    T = np.zeros((grid.m, grid.m), dtype=complex)
    nz = R > 0
    T[nz] = green(R[nz], k)
    return T


def circulant_kernel(grid: Grid, T):
    """Circulant embedding c (n x n, FFT order) of the Toeplitz kernel."""
    n, m = grid.n, grid.m
    q = np.arange(n)
    d = np.where(q <= m - 1, q, q - n)
    valid = np.abs(d) <= m - 1
    ad = np.abs(d)
    c = np.zeros((n, n), dtype=complex)
    vy, vx = np.meshgrid(valid, valid, indexing='ij')
    ay, ax = np.meshgrid(ad, ad, indexing='ij')
    ok = vy & vx
    c[ok] = T[ay[ok], ax[ok]]
    return c


def cutoff_threshold(grid: Grid, alpha: float) -> float:
    """Integer-lattice form of |kappa| <= alpha with kappa = 2 pi q / (n eps)."""
    return ((alpha * grid.n) * grid.eps / (2.0 * math.pi)) ** 2


def filter_mask(grid: Grid, alpha: float):
    n = grid.n
    q = np.fft.fftfreq(n) * n
    q = np.rint(q)
    r2 = q[:, None] ** 2 + q[None, :] ** 2
    if not math.isfinite(alpha):
        return np.ones((n, n), dtype=bool)
    return r2 <= cutoff_threshold(grid, alpha)


def spectrum(grid: Grid, T):
    """F(c_grid): unnormalised 2D DFT of the circulant kernel (eq. (8))."""
    return np.fft.fft2(circulant_kernel(grid, T))


def filtered_table(grid: Grid, T, alpha):
    """Toeplitz table of c^alpha = F^-1(mask F(c_grid)) (Sec. III-B).

    c^alpha is even in each axis, so the table over 0 <= dx, dy <= m-1
    defines the whole restricted operator."""
    C = spectrum(grid, T)
    ca = np.fft.ifft2(C * filter_mask(grid, alpha))
    return ca[:grid.m, :grid.m].copy(), ca


def analytic_filtered_table(grid: Grid, k: float, alpha: float):
    """Toeplitz table of the grid kernel sampled from the analytically
    filtered Green's function, eq. (6): T[dy, dx] = g^alpha(eps |d|), the
    alternative to the numerical filter compared in Fig. 1(a).  g^alpha is
    regular, so the origin keeps its value (closed form g^alpha(0))."""
    d = np.arange(grid.m) * grid.eps
    T = np.zeros((grid.m, grid.m), dtype=complex)
    for iy in range(grid.m):
        for ix in range(iy + 1):
            r = math.hypot(d[iy], d[ix])
            v = green_alpha_origin(k, alpha) if r == 0.0 else green_alpha_lowpass(r, k, alpha)[0]
            T[iy, ix] = v
            T[ix, iy] = v
    return T


class AimOracle:
    """The discrete AIM operators of one geometry / frequency / grid."""

    def __init__(self, xy, k, eta, basis, m, eps, p=10, near_radius=6, pad=0,
                 alpha=math.inf, near=True, near_rows=None, node_order=0, n=None):
        """node_order = 0: one 4 x 4 stencil per basis (with the near-field
        correction); node_order = P: the per-node order-P Lambda, which has
        no near-field correction, so only S^alpha (and the Gram solve).
        n: length of the circulant embedding (>= 2m - 1), default from pad."""
        self.xy = np.asarray(xy, dtype=float)
        self.k, self.eta, self.basis = float(k), float(eta), int(basis)
        self.N = self.xy.shape[0]
        self.grid = Grid(m, eps, pad, n)
        self.p = p
        self.R = near_radius
        self.node_order = int(node_order)
        if self.node_order:
            near = False
            self.anc = np.floor((basis_centers(self.xy, basis) + self.grid.L) / self.grid.eps).astype(np.int64)
        else:
            self.anc = anchors(self.xy, basis, self.grid)
        chans = CHANNELS_S + (CHANNELS_N if basis == 1 else ())
        self.W, self.Gidx = {}, {}
        for ch in chans:
            if self.node_order:
                self.W[ch], self.Gidx[ch] = stencil_weights_node(self.xy, basis, self.grid, p, ch,
                                                                 self.node_order)
            else:
                self.W[ch], self.Gidx[ch] = stencil_weights(self.xy, basis, self.grid, p, ch)
        gidx = self.Gidx['phi']
        self.act = np.unique(gidx)                       # sorted linear indices
        self.aidx = np.searchsorted(self.act, gidx)      # (N, 16) active indices
        self.act_ix = self.act % m
        self.act_iy = self.act // m
        self.T = kernel_table(self.grid, self.k)
        self.Ta = None
        self.alpha = None
        self.set_alpha(alpha)
        self.near_pairs = self._near_pairs() if near else None
        self.Cnear = {}
        if near:
            rows = near_rows
            self._build_near(('S', 'N') if basis == 1 else ('S',), rows)

    # ------------------------------------------------------------------
    def set_alpha(self, alpha):
        self.alpha = alpha
        self.Ta, _ = filtered_table(self.grid, self.T, alpha)

    def set_alpha_analytic(self, alpha):
        """S^alpha from the analytically filtered grid kernel (Fig. 1(a))."""
        self.alpha = alpha
        self.Ta = analytic_filtered_table(self.grid, self.k, alpha)

    def _near_pairs(self):
        tree = cKDTree(self.anc.astype(float))
        pr = tree.query_pairs(r=self.R + 0.5, p=np.inf, output_type='ndarray')
        idx = np.arange(self.N)
        allp = np.concatenate([pr, pr[:, ::-1], np.stack([idx, idx], axis=1)])
        order = np.lexsort((allp[:, 1], allp[:, 0]))
        return allp[order]

    def grid_block(self, table, rows_act, cols_act):
        """Dense block K[a, b] = table[|dy|, |dx|] over active indices."""
        dx = np.abs(self.act_ix[rows_act, None] - self.act_ix[None, cols_act])
        dy = np.abs(self.act_iy[rows_act, None] - self.act_iy[None, cols_act])
        return table[dy, dx]

    def grid_pair_entries(self, table, pairs, ch_i, ch_j):
        """(Lambda_i^T G Lambda_j) for basis pairs, 16 x 16 stencil sums."""
        out = np.empty(pairs.shape[0], dtype=complex)
        gi = self.Gidx['phi']
        m = self.grid.m
        chunk = 20000
        for s in range(0, pairs.shape[0], chunk):
            pi = pairs[s:s + chunk, 0]
            pj = pairs[s:s + chunk, 1]
            a = gi[pi]
            b = gi[pj]
            dx = np.abs((a % m)[:, :, None] - (b % m)[:, None, :])
            dy = np.abs((a // m)[:, :, None] - (b // m)[:, None, :])
            K = table[dy, dx]
            out[s:s + chunk] = np.einsum('pe,pef,pf->p', self.W[ch_i][pi], K, self.W[ch_j][pj])
        return out

    def _build_near(self, ops, rows=None):
        pairs = self.near_pairs
        if rows is not None:
            sel = np.isin(pairs[:, 0], np.asarray(rows))
            pairs = pairs[sel]
        self.near_sel_pairs = pairs
        for op in ops:
            exact = galerkin.assemble_entries(self.xy, self.basis, self.k, pairs, op,
                                              p_far=16, p_near=16)
            if op == 'S':
                approx = self.grid_pair_entries(self.T, pairs, 'phi', 'phi')
            else:
                approx = self.grid_pair_entries(self.T, pairs, 'dphi', 'dphi') - self.k ** 2 * (
                    self.grid_pair_entries(self.T, pairs, 'tx', 'tx')
                    + self.grid_pair_entries(self.T, pairs, 'ty', 'ty'))
            self.Cnear[op] = exact - approx

    # ------------------------------------------------------------------
    def anterpolate(self, ch, x):
        """u_act = Lambda x for one channel (active grid points)."""
        u = np.zeros((self.act.size,) + x.shape[1:], dtype=complex)
        Wx = self.W[ch][..., None] * x[:, None, ...] if x.ndim == 2 else self.W[ch] * x[:, None]
        np.add.at(u, self.aidx.ravel(), Wx.reshape((-1,) + x.shape[1:]))
        return u

    def interpolate(self, ch, v):
        """y = Lambda^T v for one channel."""
        g = v[self.aidx]                                  # (N,16,...)
        if v.ndim == 2:
            return np.einsum('ne,ner->nr', self.W[ch], g)
        return np.einsum('ne,ne->n', self.W[ch], g)

    def grid_apply(self, table, u, block=4096):
        """v = K u over the active set by direct Toeplitz sums."""
        na = self.act.size
        v = np.zeros_like(u)
        for s in range(0, na, block):
            rows = np.arange(s, min(na, s + block))
            for t0 in range(0, na, block):
                cols = np.arange(t0, min(na, t0 + block))
                v[rows] += self.grid_block(table, rows, cols) @ u[cols]
        return v

    def near_apply(self, op, x):
        if self.near_pairs is None:
            raise ValueError("this operator has no near-field correction")
        pairs = self.near_sel_pairs
        C = self.Cnear[op]
        y = np.zeros((self.N,) + x.shape[1:], dtype=complex)
        contrib = C[:, None] * x[pairs[:, 1]] if x.ndim == 2 else C * x[pairs[:, 1]]
        np.add.at(y, pairs[:, 0], contrib)
        return y

    def op_S(self, x, near=True):
        y = self.interpolate('phi', self.grid_apply(self.T, self.anterpolate('phi', x)))
        return y + self.near_apply('S', x) if near else y

    def op_S_alpha(self, x):
        return self.interpolate('phi', self.grid_apply(self.Ta, self.anterpolate('phi', x)))

    def op_N(self, x, near=True):
        y = self.interpolate('dphi', self.grid_apply(self.T, self.anterpolate('dphi', x)))
        yt = (self.interpolate('tx', self.grid_apply(self.T, self.anterpolate('tx', x)))
              + self.interpolate('ty', self.grid_apply(self.T, self.anterpolate('ty', x))))
        y = y - self.k ** 2 * yt
        return y + self.near_apply('N', x) if near else y

    def op_N_alpha(self, x):
        """N through the filtered grid kernel, no near-field correction (the
        Maue channels of eq. (2) with the table of eq. (10))."""
        y = self.interpolate('dphi', self.grid_apply(self.Ta, self.anterpolate('dphi', x)))
        yt = (self.interpolate('tx', self.grid_apply(self.Ta, self.anterpolate('tx', x)))
              + self.interpolate('ty', self.grid_apply(self.Ta, self.anterpolate('ty', x))))
        return y - self.k ** 2 * yt

    def gram_inv(self, x):
        return galerkin.gram_solve(self.xy, self.basis, x)

    def op_TM(self, x):
        return 1j * self.k * self.eta * self.op_S(x)

    def op_TE_CP(self, x, filtered=True):
        z = self.gram_inv(self.op_N(x))
        z = self.op_S_alpha(z) if filtered else self.op_S(z)
        return self.gram_inv(z)

    def apply(self, op, x):
        x = np.asarray(x, dtype=complex)
        return {
            'S': self.op_S,
            'S_ALPHA': self.op_S_alpha,
            'N': self.op_N,
            'N_ALPHA': self.op_N_alpha,
            'GRAM_INV': self.gram_inv,
            'TM': self.op_TM,
            'TE_CP': lambda v: self.op_TE_CP(v, True),
            'TE_CP_UNF': lambda v: self.op_TE_CP(v, False),
        }[op](x)

    # ------------------------------------------------------------------
    def rows_apply(self, op, x, rows):
        """Selected output rows of S, S_ALPHA or N (near field restricted to
        the rows the oracle was built with)."""
        rows = np.asarray(rows)
        chans = {'S': ('phi',), 'S_ALPHA': ('phi',), 'N': CHANNELS_N}[op]
        table = self.Ta if op == 'S_ALPHA' else self.T
        need = np.unique(self.aidx[rows].ravel())
        y = np.zeros(rows.size, dtype=complex)
        allc = np.arange(self.act.size)
        for ch in chans:
            u = self.anterpolate(ch, x)
            v = np.zeros(self.act.size, dtype=complex)
            v[need] = self.grid_block(table, need, allc) @ u
            yc = np.einsum('ne,ne->n', self.W[ch][rows], v[self.aidx[rows]])
            y += yc if ch in ('phi', 'dphi') else -self.k ** 2 * yc
        if op in ('S', 'N'):
            full = self.near_apply(op, x)
            y += full[rows]
        return y

    # ------------------------------------------------------------------
    def grid_apply_fft(self, spectrum_full, u):
        """Cross-check of eq. (8): pad, FFT, multiply, inverse FFT, restrict."""
        n, m = self.grid.n, self.grid.m
        b = np.zeros((n, n), dtype=complex)
        b[self.act_iy, self.act_ix] = u
        r = np.fft.ifft2(spectrum_full * np.fft.fft2(b))
        return r[self.act_iy, self.act_ix]
