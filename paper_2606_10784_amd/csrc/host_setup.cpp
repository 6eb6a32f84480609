// Host-side set-up of libaim: mesh, quadrature, stencil weights, active grid
// points and the near-zone pattern.
//
// Sec. II: N straight segments, segment j from vertex j to vertex j+1.
// Eq. (7): p-node Gauss rule per segment.  Sec. III-A: m x m grid of step eps
// centred at the origin; Lambda projects quadrature nodes onto grid points.
// Lambda is folded with the quadrature weights and the basis values into one
// row of grid weights per basis function, in one of two forms:
//   * one 4 x 4 cubic-Lagrange stencil per basis (16 weights), anchored at
//     the cell that holds the basis centre (with the near-field correction);
//   * per node (Sec. III-A read literally): every quadrature node gets its
//     own P x P tensor-Lagrange stencil at its own cell, and the basis row is
//     the union of its nodes' stencils (no near-field correction: S^alpha).
#include <algorithm>
#include <cmath>
#include <numeric>

#include "aim_internal.h"

namespace aim {

void gauss_legendre01(int p, std::vector<double>& x, std::vector<double>& w) {
  // Newton iteration on the Legendre polynomial P_p in long double, roots
  // mapped from [-1, 1] to [0, 1].
  x.assign(p, 0.0);
  w.assign(p, 0.0);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < (p + 1) / 2; ++i) {
    long double z = std::cos(pi * (i + 0.75L) / (p + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1.0L, p1 = 0.0L;
      for (int j = 1; j <= p; ++j) {
        long double p2 = p1;
        p1 = p0;
        p0 = ((2.0L * j - 1.0L) * z * p1 - (j - 1.0L) * p2) / j;
      }
      dp = p * (z * p0 - p1) / (z * z - 1.0L);
      long double dz = p0 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    {
      long double p0 = 1.0L, p1 = 0.0L;
      for (int j = 1; j <= p; ++j) {
        long double p2 = p1;
        p1 = p0;
        p0 = ((2.0L * j - 1.0L) * z * p1 - (j - 1.0L) * p2) / j;
      }
      dp = p * (z * p0 - p1) / (z * z - 1.0L);
    }
    long double wt = 1.0L / ((1.0L - z * z) * dp * dp);   // half of 2/((1-z^2)P'^2)
    // z is the i-th largest root: nodes (1 -+ z)/2
    x[i] = (double)((1.0L - z) * 0.5L);
    x[p - 1 - i] = (double)((1.0L + z) * 0.5L);
    w[i] = (double)wt;
    w[p - 1 - i] = (double)wt;
  }
}

void twiddles(int n, std::vector<double>& tw) {
  tw.assign(2 * (size_t)n, 0.0);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < n; ++j) {
    long double a = 2.0L * pi * (long double)j / (long double)n;
    tw[2 * j] = (double)std::cos(a);
    tw[2 * j + 1] = (double)(-std::sin(a));
  }
  // exact values at the quarter points
  for (int q = 0; q < 4; ++q) {
    int j = q * n / 4;
    if ((int64_t)j * 4 != (int64_t)q * n) continue;
    static const double cre[4] = {1, 0, -1, 0}, cim[4] = {0, -1, 0, 1};
    tw[2 * j] = cre[q];
    tw[2 * j + 1] = cim[q];
  }
}

// order-P Lagrange basis on the nodes -(P/2 - 1), ..., P/2 at t
static void lagrangeP(int P, double t, double* l) {
  const int o = P / 2 - 1;
  for (int i = 0; i < P; ++i) {
    double v = 1.0;
    for (int j = 0; j < P; ++j)
      if (j != i) v *= (t - (double)(j - o)) / (double)(i - j);
    l[i] = v;
  }
}

static inline void lagrange4(double t, double l[4]) {
  // cubic Lagrange basis on nodes -1, 0, 1, 2
  l[0] = -t * (t - 1.0) * (t - 2.0) / 6.0;
  l[1] = (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0;
  l[2] = -(t + 1.0) * t * (t - 2.0) / 2.0;
  l[3] = (t + 1.0) * t * (t - 1.0) / 6.0;
}

aim_status build_host_tables(const aim_params* p, HostTables& t, std::string& err) {
  if (!p || !p->xy) { err = "null params"; return AIM_E_ARG; }
  const int N = p->n_vertices;
  const int m = p->m;
  if (N < 8) { err = "need at least 8 vertices"; return AIM_E_ARG; }
  if (m < 16 || m > 2048) { err = "m must be in [16, 2048]"; return AIM_E_ARG; }
  if (!(p->eps > 0) || !(p->k > 0) || !(p->eta > 0)) { err = "eps, k, eta must be positive"; return AIM_E_ARG; }
  if (p->quad < 1 || p->quad > 64) { err = "quad must be in [1, 64]"; return AIM_E_ARG; }
  if (p->near_radius < 3 || p->near_radius + 3 > m - 1) { err = "near_radius out of range"; return AIM_E_ARG; }
  if (p->basis != AIM_PULSE && p->basis != AIM_HAT) { err = "basis"; return AIM_E_ARG; }
  if (p->max_rhs < 1 || p->max_rhs > AIM_MAX_RHS) { err = "max_rhs"; return AIM_E_ARG; }
  const int P = p->node_order;
  if (P != 0 && (P < 2 || P > 12 || (P & 1))) { err = "node_order must be 0 or even in 2..12"; return AIM_E_ARG; }
  t.node_order = P;
  t.N = N;
  t.basis = p->basis;
  t.m = m;
  t.n = fft_length(m);
  t.p = p->quad;
  t.R = p->near_radius;
  t.k = p->k;
  t.eta = p->eta;
  t.eps = p->eps;
  t.L = 0.5 * (m - 1) * p->eps;
  t.nch = (p->basis == AIM_HAT) ? 4 : 1;
  t.vx.resize(N);
  t.vy.resize(N);
  for (int i = 0; i < N; ++i) {
    t.vx[i] = p->xy[2 * i];
    t.vy[i] = p->xy[2 * i + 1];
    if (!std::isfinite(t.vx[i]) || !std::isfinite(t.vy[i])) { err = "non-finite vertex"; return AIM_E_ARG; }
  }
  t.h.resize(N);
  t.tx.resize(N);
  t.ty.resize(N);
  for (int j = 0; j < N; ++j) {
    int j1 = (j + 1) % N;
    double dx = t.vx[j1] - t.vx[j], dy = t.vy[j1] - t.vy[j];
    double h = std::hypot(dx, dy);
    if (!(h > 0)) { err = "degenerate segment"; return AIM_E_ARG; }
    // The singular near-field moments sum the J0 power series in k h; past
    // one wavelength per segment its terms cancel beyond FP64 accuracy (and a
    // Galerkin mesh that coarse does not resolve the current anyway).
    if (!(p->k * h <= 2.0 * 3.141592653589793)) { err = "segment longer than a wavelength"; return AIM_E_ARG; }
    t.h[j] = h;
    t.tx[j] = dx / h;
    t.ty[j] = dy / h;
  }
  gauss_legendre01(t.p, t.gl_x, t.gl_w);

  // anchors: floor((c + L) / eps), c = segment midpoint (pulse) or vertex (hat)
  t.anc_x.resize(N);
  t.anc_y.resize(N);
  for (int j = 0; j < N; ++j) {
    double cx, cy;
    if (t.basis == AIM_PULSE) {
      int j1 = (j + 1) % N;
      cx = 0.5 * (t.vx[j] + t.vx[j1]);
      cy = 0.5 * (t.vy[j] + t.vy[j1]);
    } else {
      cx = t.vx[j];
      cy = t.vy[j];
    }
    double ax = std::floor((cx + t.L) / t.eps), ay = std::floor((cy + t.L) / t.eps);
    if (P == 0 && !(ax - 1 >= 0 && ax + 2 <= m - 1 && ay - 1 >= 0 && ay + 2 <= m - 1)) {
      err = "stencil leaves the grid";
      return AIM_E_GEOM;
    }
    t.anc_x[j] = (int32_t)ax;
    t.anc_y[j] = (int32_t)ay;
  }

  // grid weights per channel and the grid point of each (lin, row-major)
  const int nch = t.nch;
  std::vector<int64_t> lin;
  std::vector<int32_t> cnt(N, 16);     // real (unpadded) points per basis
  auto pieces = [&](int j, int q, int& s, double& c0, double& c1) {
    if (t.basis == AIM_PULSE) { s = j; c0 = 1.0; c1 = 0.0; }
    else if (q == 0) { s = (j - 1 + N) % N; c0 = 0.0; c1 = 1.0; }   // rising on segment j-1
    else { s = j; c0 = 1.0; c1 = -1.0; }                            // falling on segment j
  };
  const int nseg = (t.basis == AIM_PULSE) ? 1 : 2;
  if (P == 0) {
    t.S = 16;
    for (int c = 0; c < 4; ++c) t.W[c].assign(c < nch ? (size_t)N * 16 : 0, 0.0);
    for (int j = 0; j < N; ++j) {
      for (int q = 0; q < nseg; ++q) {
        int s;
        double c0, c1;
        pieces(j, q, s, c0, c1);
        int s1 = (s + 1) % N;
        double ax0 = t.vx[s], ay0 = t.vy[s];
        double ddx = t.vx[s1] - ax0, ddy = t.vy[s1] - ay0;
        for (int kq = 0; kq < t.p; ++kq) {
          double tau = t.gl_x[kq];
          double px = ax0 + ddx * tau, py = ay0 + ddy * tau;
          double wk = t.h[s] * t.gl_w[kq];
          double phi = c0 + c1 * tau;
          double val[4] = {phi, c1 / t.h[s], t.tx[s] * phi, t.ty[s] * phi};
          double lx[4], ly[4];
          lagrange4((px + t.L) / t.eps - t.anc_x[j], lx);
          lagrange4((py + t.L) / t.eps - t.anc_y[j], ly);
          for (int c = 0; c < nch; ++c) {
            double f = wk * val[c];
            double* Wj = &t.W[c][(size_t)j * 16];
            for (int tt = 0; tt < 4; ++tt)
              for (int ss = 0; ss < 4; ++ss) Wj[tt * 4 + ss] += f * lx[ss] * ly[tt];
          }
        }
      }
    }
    lin.resize((size_t)N * 16);
    for (int j = 0; j < N; ++j)
      for (int tt = 0; tt < 4; ++tt)
        for (int ss = 0; ss < 4; ++ss)
          lin[(size_t)j * 16 + tt * 4 + ss] = (int64_t)(t.anc_y[j] - 1 + tt) * m + (t.anc_x[j] - 1 + ss);
  } else {
    // per node: accumulate each basis's node stencils in a dense box over
    // its cells, then keep the touched cells in row-major order
    const int o = P / 2 - 1;
    std::vector<std::vector<int64_t>> blin(N);
    std::vector<std::vector<double>> bw(N);
    std::vector<double> box, lx(P), ly(P);
    std::vector<char> touched;
    std::vector<int> nax, nay;
    for (int j = 0; j < N; ++j) {
      nax.clear();
      nay.clear();
      int bx0 = m, by0 = m, bx1 = -1, by1 = -1;
      for (int q = 0; q < nseg; ++q) {
        int s;
        double c0, c1;
        pieces(j, q, s, c0, c1);
        const int s1 = (s + 1) % N;
        for (int kq = 0; kq < t.p; ++kq) {
          const double tau = t.gl_x[kq];
          const double px = t.vx[s] + (t.vx[s1] - t.vx[s]) * tau, py = t.vy[s] + (t.vy[s1] - t.vy[s]) * tau;
          const int ax = (int)std::floor((px + t.L) / t.eps), ay = (int)std::floor((py + t.L) / t.eps);
          if (ax - o < 0 || ax - o + P - 1 > m - 1 || ay - o < 0 || ay - o + P - 1 > m - 1) {
            err = "stencil leaves the grid";
            return AIM_E_GEOM;
          }
          nax.push_back(ax);
          nay.push_back(ay);
          bx0 = std::min(bx0, ax - o);
          by0 = std::min(by0, ay - o);
          bx1 = std::max(bx1, ax - o + P - 1);
          by1 = std::max(by1, ay - o + P - 1);
        }
      }
      const int BX = bx1 - bx0 + 1, BY = by1 - by0 + 1;
      box.assign((size_t)BX * BY * nch, 0.0);
      touched.assign((size_t)BX * BY, 0);
      int node = 0;
      for (int q = 0; q < nseg; ++q) {
        int s;
        double c0, c1;
        pieces(j, q, s, c0, c1);
        const int s1 = (s + 1) % N;
        for (int kq = 0; kq < t.p; ++kq, ++node) {
          const double tau = t.gl_x[kq];
          const double px = t.vx[s] + (t.vx[s1] - t.vx[s]) * tau, py = t.vy[s] + (t.vy[s1] - t.vy[s]) * tau;
          const double wk = t.h[s] * t.gl_w[kq];
          const double phi = c0 + c1 * tau;
          const double val[4] = {phi, c1 / t.h[s], t.tx[s] * phi, t.ty[s] * phi};
          const int ax = nax[node], ay = nay[node];
          lagrangeP(P, (px + t.L) / t.eps - ax, lx.data());
          lagrangeP(P, (py + t.L) / t.eps - ay, ly.data());
          for (int tt = 0; tt < P; ++tt)
            for (int ss = 0; ss < P; ++ss) {
              const size_t cell = (size_t)(ay - o + tt - by0) * BX + (ax - o + ss - bx0);
              touched[cell] = 1;
              for (int c = 0; c < nch; ++c) box[cell * nch + c] += wk * val[c] * lx[ss] * ly[tt];
            }
        }
      }
      for (int yy = 0; yy < BY; ++yy)
        for (int xx = 0; xx < BX; ++xx) {
          const size_t cell = (size_t)yy * BX + xx;
          if (!touched[cell]) continue;
          blin[j].push_back((int64_t)(by0 + yy) * m + (bx0 + xx));
          for (int c = 0; c < nch; ++c) bw[j].push_back(box[cell * nch + c]);
        }
      cnt[j] = (int)blin[j].size();
    }
    t.S = *std::max_element(cnt.begin(), cnt.end());
    const int S = t.S;
    for (int c = 0; c < 4; ++c) t.W[c].assign(c < nch ? (size_t)N * S : 0, 0.0);
    lin.resize((size_t)N * S);
    for (int j = 0; j < N; ++j)
      for (int e = 0; e < S; ++e) {
        const bool real = e < cnt[j];
        lin[(size_t)j * S + e] = blin[j][real ? e : 0];   // padding: the first point, weight 0
        for (int c = 0; c < nch; ++c) t.W[c][(size_t)j * S + e] = real ? bw[j][(size_t)e * nch + c] : 0.0;
      }
  }
  const int S = t.S;

  // active grid points: union of the map rows, sorted by row-major index
  std::vector<int64_t> act(lin);
  std::sort(act.begin(), act.end());
  act.erase(std::unique(act.begin(), act.end()), act.end());
  t.n_act = (int)act.size();
  t.act_ix.resize(t.n_act);
  t.act_iy.resize(t.n_act);
  for (int a = 0; a < t.n_act; ++a) {
    t.act_ix[a] = (int32_t)(act[a] % m);
    t.act_iy[a] = (int32_t)(act[a] / m);
  }
  t.aidx.resize((size_t)N * S);
  for (size_t q = 0; q < lin.size(); ++q)
    t.aidx[q] = (int32_t)(std::lower_bound(act.begin(), act.end(), lin[q]) - act.begin());
  t.y0 = t.act_iy.front();
  t.nr = t.act_iy.back() - t.y0 + 1;
  t.row_ptr.assign(t.nr + 1, 0);
  for (int a = 0; a < t.n_act; ++a) t.row_ptr[t.act_iy[a] - t.y0 + 1]++;
  for (int r = 0; r < t.nr; ++r) t.row_ptr[r + 1] += t.row_ptr[r];

  // transposed map rows (grid point -> contributing bases), for the gather;
  // padding entries are left out
  t.at_ptr.assign(t.n_act + 1, 0);
  size_t nent = 0;
  for (int j = 0; j < N; ++j)
    for (int e = 0; e < cnt[j]; ++e) t.at_ptr[t.aidx[(size_t)j * S + e] + 1]++, ++nent;
  for (int a = 0; a < t.n_act; ++a) t.at_ptr[a + 1] += t.at_ptr[a];
  t.at_basis.assign(nent, 0);
  for (int c = 0; c < 4; ++c) t.at_w[c].assign(c < nch ? nent : 0, 0.0);
  {
    std::vector<int32_t> fill(t.at_ptr.begin(), t.at_ptr.end() - 1);
    for (int j = 0; j < N; ++j)
      for (int e = 0; e < cnt[j]; ++e) {
        int a = t.aidx[(size_t)j * S + e];
        int pos = fill[a]++;
        t.at_basis[pos] = j;
        for (int c = 0; c < nch; ++c) t.at_w[c][pos] = t.W[c][(size_t)j * S + e];
      }
  }
  if (P != 0) {
    // the per-node map has no near-field correction
    t.nr_ptr.assign(N + 1, 0);
    t.nr_col.clear();
    t.band_w = -1;
    return AIM_OK;
  }

  // near zone: anchor Chebyshev distance <= R (CSR, sorted columns)
  std::vector<int64_t> key(N);
  std::vector<int32_t> ord(N);
  for (int j = 0; j < N; ++j) key[j] = (int64_t)t.anc_y[j] * m + t.anc_x[j];
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return key[a] < key[b] || (key[a] == key[b] && a < b); });
  std::vector<int64_t> skey(N);
  for (int q = 0; q < N; ++q) skey[q] = key[ord[q]];
  const int R = t.R;
  t.nr_ptr.assign(N + 1, 0);
  t.nr_col.clear();
  std::vector<int32_t> cols;
  for (int i = 0; i < N; ++i) {
    cols.clear();
    int ax = t.anc_x[i], ay = t.anc_y[i];
    for (int dy = -R; dy <= R; ++dy) {
      int y = ay + dy;
      if (y < 0 || y >= m) continue;
      int64_t lo = (int64_t)y * m + std::max(0, ax - R);
      int64_t hi = (int64_t)y * m + std::min(m - 1, ax + R);
      auto b = std::lower_bound(skey.begin(), skey.end(), lo);
      auto e = std::upper_bound(skey.begin(), skey.end(), hi);
      for (auto it = b; it != e; ++it) cols.push_back(ord[it - skey.begin()]);
    }
    std::sort(cols.begin(), cols.end());
    t.nr_col.insert(t.nr_col.end(), cols.begin(), cols.end());
    t.nr_ptr[i + 1] = (int32_t)t.nr_col.size();
  }
  // Banded symmetric storage of the near field when it pays: bases are
  // numbered along the contour, so near pairs have a small cyclic index
  // distance |i - j|_N <= w, and the near matrices are symmetric (Galerkin,
  // same test and trial functions; symmetric pattern).  Row i then keeps
  // only C(i, i + d), d = 0..w, and borrows C(i - d, i) for the other half.
  {
    int w = 0;
    for (int i = 0; i < N; ++i)
      for (int q = t.nr_ptr[i]; q < t.nr_ptr[i + 1]; ++q) {
        const int d = ((t.nr_col[q] - i) % N + N) % N;
        w = std::max(w, std::min(d, N - d));
      }
    const double dia_bytes = (double)(w + 1) * N * 16, csr_bytes = (double)t.nr_col.size() * 20;
    t.band_w = (2 * w + 1 < N && dia_bytes <= 0.75 * csr_bytes) ? w : -1;
  }
  return AIM_OK;
}

}  // namespace aim
