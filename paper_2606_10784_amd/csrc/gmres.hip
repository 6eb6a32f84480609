// Restarted GMRES on the device for the AIM systems (FP64 Krylov space).
//
// The paper applies its operators inside iterative solvers (abstract, Sec. I)
// without naming one; this is GMRES(restart) with complex Givens rotations,
// one independent Krylov space per right-hand side.  Orthogonalisation is
// classical Gram-Schmidt applied twice, with the second pass delayed by one
// step (the low-synchronisation "DCGS2" Arnoldi): step j runs one operator
// application, one reduction pass over the basis and one update pass, and the
// Hessenberg column of step j becomes final in step j + 1.  The only per-step
// device-to-host transfer is the residual estimate (8 bytes per right-hand
// side, every few steps).  Reductions use a fixed chunking and order, so
// results do not depend on which other right-hand sides share the batch.
//
// Delayed step j.  At its start Q_j = [q_0 .. q_{j-1}] is orthonormal, slot j
// holds u_j with A q_{j-1} = Q_j h + u_j (h: provisional column j-1), and
// w = A u_j has just been formed.  One pass gives s = Q_j^H u_j, alpha = |u_j|^2,
// z = Q_j^H w, zeta = u_j^H w.  Then
//   gamma = |u_j - Q_j s| = sqrt(alpha - |s|^2),  q_j = (u_j - Q_j s)/gamma,
//   column j-1 final: H[0:j, j-1] = h + s, H[j, j-1] = gamma,
//   d = q_j^H w = (zeta - s^H z)/gamma,  t = (z, d) = Q_{j+1}^H w,
//   A q_j = (w - A Q_j s)/gamma with A Q_j s = Q_{j+1} H s, hence
//   provisional column j: (t - H s)/gamma, and
//   u_{j+1} = (w - Q_{j+1} t)/gamma = (w - Q_j (z - e s) - e u_j)/gamma, e = d/gamma,
// so every basis vector is projected twice: once as u_{j+1} and once more in
// step j + 1 (s).  The second update pass writes q_j and u_{j+1} together.
//
// AIM_MIXED: iterative refinement  x <- x + d,  A_mixed d ~ b - A_64 x, where
// A_mixed runs the grid part in complex FP32 and everything else in FP64.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>
#include <memory>
#include <new>

#include "aim_internal.h"

namespace aim {

static constexpr int RED_CHUNK = 2048;
// Arnoldi steps enqueued between two host reads of the residual estimates
static constexpr int kCheckEvery = 8;
static_assert(kCheckEvery + 1 <= kResidPitch, "one check reads back at most kCheckEvery + 1 estimates per rhs");

// sum over a 256-thread block, same value in every thread, fixed order
// (butterfly within each wave, then the four waves in order).  red: 4*K doubles.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red) {
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o);
  const int wv = threadIdx.x >> 6;
  __syncthreads();   // red may still be read from a previous call
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) red[wv * K + k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = ((red[k] + red[K + k]) + red[2 * K + k]) + red[3 * K + k];
}

// partial |w|^2 over a chunk of rows
__global__ __launch_bounds__(256) void k_sqnorm(int N, const double2* __restrict__ w, int64_t ld_w,
                                                const int* __restrict__ active, double* __restrict__ part,
                                                int nchunk) {
  __shared__ double red[4];
  const int chunk = blockIdx.x, r = blockIdx.y;
  if (!active[r]) return;
  const double2* wr = w + (size_t)r * ld_w;
  double v[1] = {0.0};
  const int n0 = chunk * RED_CHUNK, n1 = min(N, n0 + RED_CHUNK);
  for (int n = n0 + threadIdx.x; n < n1; n += 256) {
    const double2 b = wr[n];
    v[0] += b.x * b.x + b.y * b.y;
  }
  block_sum<1>(v, red);
  if (threadIdx.x == 0) part[(size_t)r * nchunk + chunk] = v[0];
}

// out[r].x = sum of the chunk partials (fixed order)
__global__ void k_sqnorm_reduce(int nrhs, int nchunk, const double* part, const int* active, double2* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs || !active[r]) return;
  double t = 0.0;
  for (int c = 0; c < nchunk; ++c) t += part[(size_t)r * nchunk + c];
  out[r] = make_double2(t, 0.0);
}

constexpr int DOT_COLS = 1;   // basis slots per reduction block (4 sums each)
static inline int dot_groups(int j) { return (j + DOT_COLS) / DOT_COLS; }

// Reduction pass of delayed step j: partial sums over a chunk of rows of
// conj(V_i) . u and conj(V_i) . w for the basis slots i <= j, where slot j
// holds u (so i = j gives |u|^2 and u^H w).  w == nullptr: the u sums only.
// part layout [r][i][chunk][2].  Block (chunk, y) covers the slots
// DOT_COLS y .. DOT_COLS y + DOT_COLS - 1.
// Blocks with y >= dot_groups(j) form the provisional column j - 1 from the
// coefficients step j - 1 left in coef (s, z, then d, 1/gamma), one row i per
// block: ((z, d)_i - (H s)_i) / gamma over the final columns 0 .. j-2 of the
// row-major unrotated Hessenberg HuT; written to hp[(j - 1) & 1].
__global__ __launch_bounds__(256) void k_arnoldi_dots(int N, int j, const double2* __restrict__ V, int64_t ldv,
                                                      const double2* __restrict__ w, int64_t ld_w,
                                                      const int* __restrict__ active, double2* __restrict__ part,
                                                      int nchunk, int ldh, const double2* __restrict__ HuT,
                                                      const double2* __restrict__ coef, double2* __restrict__ hp) {
  __shared__ double red[16];
  const int chunk = blockIdx.x, i = blockIdx.y, r = blockIdx.z;
  if (!active[r]) return;
  if (i >= (j + DOT_COLS) / DOT_COLS) {
    // provisional column j - 1, row ih
    const int ih = (i - (j + DOT_COLS) / DOT_COLS) * nchunk + chunk;
    if (ih >= j) return;
    const double2* cf = coef + (size_t)r * (2 * ldh + 2);
    const double2* sj = cf;          // s of step j - 1 (j - 1 entries)
    const double2* row = HuT + (size_t)r * ldh * ldh + (size_t)ih * ldh;
    double a[2] = {0.0, 0.0};
    for (int k = max(0, ih - 1) + threadIdx.x; k < j - 1; k += 256) {
      const double2 h = row[k], c = sj[k];
      a[0] += h.x * c.x - h.y * c.y;
      a[1] += h.x * c.y + h.y * c.x;
    }
    block_sum<2>(a, red);
    if (threadIdx.x == 0) {
      const double2 t = ih < j - 1 ? cf[ldh + ih] : cf[2 * ldh];
      const double ig = cf[2 * ldh + 1].x;
      hp[((size_t)r * 2 + ((j - 1) & 1)) * ldh + ih] = make_double2((t.x - a[0]) * ig, (t.y - a[1]) * ig);
    }
    return;
  }
  // basis slots i0 .. i0+3 against u and w over one chunk of rows
  const int i0 = i * DOT_COLS;
  const double2* vb = V + (size_t)r * ldv;
  const double2* u = vb + (size_t)j * N;
  const double2* wr = w ? w + (size_t)r * ld_w : nullptr;
  const double2* vc[DOT_COLS];
#pragma unroll
  for (int q = 0; q < DOT_COLS; ++q) vc[q] = vb + (size_t)min(i0 + q, j) * N;   // clamped: unused sums
  double v[4 * DOT_COLS];
#pragma unroll
  for (int k = 0; k < 4 * DOT_COLS; ++k) v[k] = 0.0;
  const int n0 = chunk * RED_CHUNK, n1 = min(N, n0 + RED_CHUNK);
  constexpr int RU = DOT_COLS >= 4 ? 1 : 4 / DOT_COLS;   // rows per thread in flight
  for (int n = n0 + threadIdx.x; n < n1; n += RU * 256) {
    double2 bu[RU], bw[RU], a[RU][DOT_COLS];
#pragma unroll
    for (int m = 0; m < RU; ++m) {
      const int nn = min(n + m * 256, n1 - 1);   // clamped rows are loaded but not summed
      bu[m] = u[nn];
      bw[m] = wr ? wr[nn] : make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < DOT_COLS; ++q) a[m][q] = vc[q][nn];
    }
#pragma unroll
    for (int m = 0; m < RU; ++m) {
      if (n + m * 256 >= n1) break;
#pragma unroll
      for (int q = 0; q < DOT_COLS; ++q) {
        v[4 * q + 0] += a[m][q].x * bu[m].x + a[m][q].y * bu[m].y;
        v[4 * q + 1] += a[m][q].x * bu[m].y - a[m][q].y * bu[m].x;
        v[4 * q + 2] += a[m][q].x * bw[m].x + a[m][q].y * bw[m].y;
        v[4 * q + 3] += a[m][q].x * bw[m].y - a[m][q].y * bw[m].x;
      }
    }
  }
  // the 4 DOT_COLS sums over the block: halving exchanges within each wave
  // (each step keeps half of the sums, so lane groups end up with one sum
  // each), butterflies within the groups, then the four waves in order
  constexpr int NS = 4 * DOT_COLS;
  constexpr int H = NS == 16 ? 4 : (NS == 8 ? 3 : 2);   // log2 NS
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const int off = 32 >> h, keep = NS >> (h + 1);
    const bool hi = (lane & off) != 0;
#pragma unroll
    for (int k = 0; k < keep; ++k) {
      const double send = hi ? v[k] : v[k + keep];
      const double mine = hi ? v[k + keep] : v[k];
      v[k] = mine + __shfl_xor(send, off);
    }
  }
#pragma unroll
  for (int off = 32 >> H; off >= 1; off >>= 1) v[0] += __shfl_xor(v[0], off);
  // lane m << (6 - H) now holds sum number m
  __shared__ double wsum[4][NS];
  if ((lane & ((64 >> H) - 1)) == 0) wsum[wv][lane >> (6 - H)] = v[0];
  __syncthreads();
  if (threadIdx.x < 4 * DOT_COLS) {
    const int k = threadIdx.x, q = k >> 2;
    const double t = ((wsum[0][k] + wsum[1][k]) + wsum[2][k]) + wsum[3][k];
    if (i0 + q <= j) {
      double* o = (double*)(part + (((size_t)r * ldh + i0 + q) * nchunk + chunk) * 2);
      o[k & 3] = t;
    }
  }
}

// extra y-blocks of k_arnoldi_dots for the provisional column of step j - 1
static inline int hs_blocks(int j, int nchunk) { return j >= 1 ? (j + nchunk - 1) / nchunk : 0; }

// Update pass of delayed step j (formulas in the file header).  Every block
// reduces the chunk partials itself (fixed order); block 0 writes the final
// column j-1 into HuT (row-major, unrotated, for H s) and H (rotated later)
// and leaves s, z, d and 1/gamma in coef for the provisional column, which
// the next reduction pass forms; each block updates GV_ROWS rows of q_j and
// u_{j+1}.  finalize != 0: only the column j-1 (one block per rhs, w unused).
// Dynamic LDS: 3 (j + 1) double2.
constexpr int GV_ROWS = 32, GV_GRP = 8;
__global__ __launch_bounds__(256) void k_arnoldi_update(int N, int j, int nchunk, int ldh,
                                                        const double2* __restrict__ part, double2* __restrict__ V,
                                                        int64_t ldv, const double2* __restrict__ w, int64_t ld_w,
                                                        const int* __restrict__ active, double2* __restrict__ HuT,
                                                        double2* __restrict__ H, const double2* __restrict__ hp,
                                                        double2* __restrict__ coef, int finalize) {
  extern __shared__ double2 sh[];
  __shared__ double red[16];
  __shared__ double px[256], py[256], qx[256], qy[256];
  const int r = blockIdx.y;
  if (!active[r]) return;
  const int tid = threadIdx.x;
  const int j1 = j + 1;
  double2* S = sh;         // s_i (i < j), alpha at j
  double2* Z = sh + j1;    // z_i (i < j), zeta at j
  // the first basis loads of the update do not depend on the coefficients:
  // issue them before the reduction of the partials
  constexpr int UN = 8;    // basis loads in flight per thread
  const int lr = tid % GV_ROWS, g = tid / GV_ROWS;
  const int n = blockIdx.x * GV_ROWS + lr;
  const double2* vr = V + (size_t)r * ldv;
  double2 pre[UN];
  if (!finalize) {
#pragma unroll
    for (int q = 0; q < UN; ++q) {
      const int i = g + q * GV_GRP;
      pre[q] = (n < N && i < j) ? vr[(size_t)i * N + n] : make_double2(0.0, 0.0);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  const double2* pr = part + (size_t)r * ldh * nchunk * 2;
  for (int i = tid; i < j1; i += 256) {
    double ax = 0, ay = 0, bx = 0, by = 0;
    const double2* pi = pr + (size_t)i * nchunk * 2;
    int c = 0;
    for (; c + 7 < nchunk; c += 8) {   // 16 loads in flight, summed in chunk order
      double2 t[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) t[q] = pi[2 * c + q];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        ax += t[2 * q].x;
        ay += t[2 * q].y;
        bx += t[2 * q + 1].x;
        by += t[2 * q + 1].y;
      }
    }
    for (; c + 3 < nchunk; c += 4) {   // 8 loads in flight, summed in chunk order
      double2 t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = pi[2 * c + q];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ax += t[2 * q].x;
        ay += t[2 * q].y;
        bx += t[2 * q + 1].x;
        by += t[2 * q + 1].y;
      }
    }
    for (; c < nchunk; ++c) {
      const double2 a = pi[2 * c], b = pi[2 * c + 1];
      ax += a.x;
      ay += a.y;
      bx += b.x;
      by += b.y;
    }
    S[i] = make_double2(ax, ay);
    Z[i] = make_double2(bx, by);
  }
  __syncthreads();
  // |s|^2 and s^H z
  double v[3] = {0.0, 0.0, 0.0};
  for (int i = tid; i < j; i += 256) {
    const double2 a = S[i], b = Z[i];
    v[0] += a.x * a.x + a.y * a.y;
    v[1] += a.x * b.x + a.y * b.y;
    v[2] += a.x * b.y - a.y * b.x;
  }
  block_sum<3>(v, red);
  const double g2 = S[j].x - v[0];
  const double gam = g2 > 0.0 ? sqrt(g2) : 0.0;
  const double ig = gam > 0.0 ? 1.0 / gam : 0.0;
  const double2 d = make_double2((Z[j].x - v[1]) * ig, (Z[j].y - v[2]) * ig);
  const double2 e = make_double2(d.x * ig, d.y * ig);
  const size_t hcol = (size_t)r * ldh * (ldh - 1);
  const double2* hprev = hp + ((size_t)r * 2 + ((j - 1) & 1)) * ldh;   // provisional column j-1
  auto col_prev = [&](int i) -> double2 {                                // final column j-1, row i <= j
    if (i < j) return make_double2(hprev[i].x + S[i].x, hprev[i].y + S[i].y);
    return make_double2(gam, 0.0);
  };
  if (blockIdx.x == 0) {
    if (j >= 1)
      for (int i = tid; i <= j; i += 256) {
        const double2 c = col_prev(i);
        HuT[(size_t)r * ldh * ldh + (size_t)i * ldh + (j - 1)] = c;
        H[hcol + (size_t)(j - 1) * ldh + i] = c;
      }
    if (!finalize) {
      double2* cf = coef + (size_t)r * (2 * ldh + 2);
      for (int i = tid; i < j; i += 256) {
        cf[i] = S[i];
        cf[ldh + i] = Z[i];
      }
      if (tid == 0) {
        cf[2 * ldh] = d;
        cf[2 * ldh + 1] = make_double2(ig, 0.0);
      }
    }
  }
  if (finalize) return;
  // q_j and u_{j+1} for rows n
  // coefficients of Q_j in u_{j+1}: z - e s
  double2* T = sh + 2 * j1;
  for (int i = tid; i < j; i += 256) {
    const double2 c = S[i], zz = Z[i];
    T[i] = make_double2(zz.x - (e.x * c.x - e.y * c.y), zz.y - (e.x * c.y + e.y * c.x));
  }
  __syncthreads();
  double sx = 0, sy = 0, tx = 0, ty = 0;
  auto acc = [&](double2 a, int i) {
    const double2 c = S[i], t = T[i];
    sx += a.x * c.x - a.y * c.y;
    sy += a.x * c.y + a.y * c.x;
    tx += a.x * t.x - a.y * t.y;
    ty += a.x * t.y + a.y * t.x;
  };
  if (n < N) {
#pragma unroll
    for (int q = 0; q < UN; ++q)
      if (g + q * GV_GRP < j) acc(pre[q], g + q * GV_GRP);
    int i = g + UN * GV_GRP;
    for (; i + (UN - 1) * GV_GRP < j; i += UN * GV_GRP) {
      double2 a[UN];
#pragma unroll
      for (int q = 0; q < UN; ++q) a[q] = vr[(size_t)(i + q * GV_GRP) * N + n];
      __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of their uses
#pragma unroll
      for (int q = 0; q < UN; ++q) acc(a[q], i + q * GV_GRP);
    }
    for (; i < j; i += GV_GRP) acc(vr[(size_t)i * N + n], i);
  }
  px[tid] = sx;
  py[tid] = sy;
  qx[tid] = tx;
  qy[tid] = ty;
  __syncthreads();
  if (g == 0 && n < N) {
    for (int q = 1; q < GV_GRP; ++q) {
      sx += px[q * GV_ROWS + lr];
      sy += py[q * GV_ROWS + lr];
      tx += qx[q * GV_ROWS + lr];
      ty += qy[q * GV_ROWS + lr];
    }
    double2* uj = V + (size_t)r * ldv + (size_t)j * N;
    const double2 u = uj[n], wn = w[(size_t)r * ld_w + n];
    uj[n] = make_double2((u.x - sx) * ig, (u.y - sy) * ig);
    const double ox = wn.x - tx - (e.x * u.x - e.y * u.y);
    const double oy = wn.y - ty - (e.x * u.y + e.y * u.x);
    uj[N + n] = make_double2(ox * ig, oy * ig);
  }
}

// w[r] += sgn * sum_i V[r][i] c[r][i]; block = 32 rows x 8 groups of i
__global__ __launch_bounds__(256) void k_gemv(int N, int j1, const double2* __restrict__ V, int64_t ld_rhs_v,
                                              const double2* __restrict__ c, int64_t ld_c, double sgn,
                                              const int* __restrict__ active, double2* __restrict__ w,
                                              int64_t ld_w) {
  const int r = blockIdx.y;
  if (!active[r]) return;
  const int lr = threadIdx.x % GV_ROWS, g = threadIdx.x / GV_ROWS;
  const int n = blockIdx.x * GV_ROWS + lr;
  const double2* vr = V + (size_t)r * ld_rhs_v;
  const double2* cr = c + (size_t)r * ld_c;
  double sx = 0, sy = 0;
  if (n < N) {
    for (int i = g; i < j1; i += GV_GRP) {
      const double2 a = vr[(size_t)i * N + n], b = cr[i];
      sx += a.x * b.x - a.y * b.y;
      sy += a.x * b.y + a.y * b.x;
    }
  }
  __shared__ double px[256], py[256];
  px[threadIdx.x] = sx;
  py[threadIdx.x] = sy;
  __syncthreads();
  if (g == 0 && n < N) {
    for (int q = 1; q < GV_GRP; ++q) {
      sx += px[q * GV_ROWS + lr];
      sy += py[q * GV_ROWS + lr];
    }
    double2 o = w[(size_t)r * ld_w + n];
    w[(size_t)r * ld_w + n] = make_double2(o.x + sgn * sx, o.y + sgn * sy);
  }
}

// v = w / ||w||   (||w||^2 from the reduction, in nrm2[r].x)
__global__ void k_normalize(int N, const double2* nrm2, const double2* __restrict__ w, int64_t ld_w,
                            double2* __restrict__ v, int64_t ld_rhs_v, const int* __restrict__ active) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (!active[r] || n >= N) return;
  const double nr = sqrt(nrm2[r].x);
  const double s = nr > 0 ? 1.0 / nr : 0.0;
  const double2 a = w[(size_t)r * ld_w + n];
  v[(size_t)r * ld_rhs_v + n] = make_double2(a.x * s, a.y * s);
}

// residual r = b - r (in place on r)
__global__ void k_bminus(int N, const double2* b, double2* r) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (n >= N) return;
  const double2 bb = b[(size_t)c * N + n], rr = r[(size_t)c * N + n];
  r[(size_t)c * N + n] = make_double2(bb.x - rr.x, bb.y - rr.y);
}

__global__ void k_axpy(int N, const double2* d, double2* x) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (n >= N) return;
  const double2 a = d[(size_t)c * N + n], o = x[(size_t)c * N + n];
  x[(size_t)c * N + n] = make_double2(o.x + a.x, o.y + a.y);
}

__device__ __forceinline__ void rot_apply(double ci, double2 si, double2& a, double2 b, double2& out_top) {
  // [c s; -conj(s) c] (a, b) -> (out_top, a)
  out_top = make_double2(ci * a.x + si.x * b.x - si.y * b.y, ci * a.y + si.x * b.y + si.y * b.x);
  a = make_double2(-(si.x * a.x + si.y * a.y) + ci * b.x, -(si.x * a.y - si.y * a.x) + ci * b.y);
}

// Givens rotations for the Hessenberg columns j0..j1-1 of each rhs: the
// rotations 0..j0-1 are applied to the new columns in parallel (one thread
// per column, chains read from LDS), then the new rotations are formed in
// order.  Writes the residual estimates |g_{j+1}| of those steps.  One block
// per rhs; dynamic LDS: (j1 - j0) * ldh + 2 * j1 double2.
__global__ __launch_bounds__(256) void k_givens_batch(int ldh, int j0, int j1, const int* __restrict__ active,
                                                      double2* H, double2* cs, double2* sn, double2* g,
                                                      double* resid_hist, double* est_out, int est_j0,
                                                      int est_pitch) {
  extern __shared__ double2 sh[];
  const int r = blockIdx.x;
  if (!active[r]) return;
  const int R = ldh - 1;
  const int nc = j1 - j0;
  double2* Hs = sh;                        // nc columns of ldh
  double2* Cs = sh + (size_t)nc * ldh;     // j1
  double2* Ss = Cs + j1;                   // j1
  double2* Hr = H + (size_t)r * ldh * R;
  double2* c = cs + (size_t)r * R;
  double2* s = sn + (size_t)r * R;
  // the columns j0..j1-1 are contiguous in H (rows 0..j+1 of each are used):
  // one flat copy with four loads in flight per thread
  const int tot = nc * ldh;
  const double2* src = Hr + (size_t)j0 * ldh;
  for (int b = threadIdx.x; b < tot; b += 4 * 256) {
    const double2 v0 = src[b], v1 = src[min(b + 256, tot - 1)], v2 = src[min(b + 512, tot - 1)],
                  v3 = src[min(b + 768, tot - 1)];
    Hs[b] = v0;
    if (b + 256 < tot) Hs[b + 256] = v1;
    if (b + 512 < tot) Hs[b + 512] = v2;
    if (b + 768 < tot) Hs[b + 768] = v3;
  }
  for (int i = threadIdx.x; i < j0; i += 256) {
    Cs[i] = c[i];
    Ss[i] = s[i];
  }
  __syncthreads();
  if ((int)threadIdx.x < nc) {
    double2* col = Hs + (size_t)threadIdx.x * ldh;
    double2 a = col[0];
    int i = 0;
    for (; i + 4 <= j0; i += 4) {   // LDS reads of four rotations ahead of the chain
      double2 b[4], sq[4];
      double cq[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        b[q] = col[i + q + 1];
        cq[q] = Cs[i + q].x;
        sq[q] = Ss[i + q];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double2 top;
        rot_apply(cq[q], sq[q], a, b[q], top);
        col[i + q] = top;
      }
    }
    for (; i < j0; ++i) {
      double2 top;
      rot_apply(Cs[i].x, Ss[i], a, col[i + 1], top);
      col[i] = top;
    }
    col[j0] = a;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double2* gg = g + (size_t)r * ldh;
    for (int t = 0; t < nc; ++t) {
      const int jj = j0 + t;
      double2* col = Hs + (size_t)t * ldh;
      double2 a = col[j0];
      for (int i = j0; i < jj; ++i) {
        double2 top;
        rot_apply(Cs[i].x, Ss[i], a, col[i + 1], top);
        col[i] = top;
      }
      const double2 b = col[jj + 1];
      const double na = hypot(a.x, a.y), nb = hypot(b.x, b.y);
      const double den = hypot(na, nb);
      double ci;
      double2 si;
      if (na == 0.0) {
        ci = 0.0;
        si = make_double2(1.0, 0.0);
      } else {
        ci = na / den;
        const double2 ph = make_double2(a.x / na, a.y / na);
        si = make_double2((ph.x * b.x + ph.y * b.y) / den, (ph.y * b.x - ph.x * b.y) / den);
      }
      Cs[jj] = make_double2(ci, 0.0);
      Ss[jj] = si;
      col[jj] = make_double2(ci * a.x + si.x * b.x - si.y * b.y, ci * a.y + si.x * b.y + si.y * b.x);
      col[jj + 1] = make_double2(0.0, 0.0);
      const double2 gj = gg[jj];
      gg[jj + 1] = make_double2(-(si.x * gj.x + si.y * gj.y), -(si.x * gj.y - si.y * gj.x));
      gg[jj] = make_double2(ci * gj.x, ci * gj.y);
      resid_hist[(size_t)r * R + jj] = hypot(gg[jj + 1].x, gg[jj + 1].y);
      // the estimate also goes straight to the host's pinned buffer
      est_out[(size_t)r * est_pitch + (jj - est_j0)] = resid_hist[(size_t)r * R + jj];
    }
    __threadfence_system();
  }
  __syncthreads();
  double2* dst = Hr + (size_t)j0 * ldh;
  for (int b = threadIdx.x; b < tot; b += 256) {
    const int t = b / ldh, i = b - t * ldh;
    if (i <= j0 + t + 1) dst[b] = Hs[b];
  }
  for (int i = j0 + threadIdx.x; i < j1; i += 256) {
    c[i] = Cs[i];
    s[i] = Ss[i];
  }
}

// y = H^-1 g (upper triangular, jm x jm), column-oriented back substitution,
// one block per right-hand side; dynamic LDS: ldh double2.
__global__ __launch_bounds__(256) void k_trisolve(int nrhs, int ldh, const int* jm, const double2* H,
                                                  const double2* g, double2* y) {
  extern __shared__ double2 gl[];
  const int r = blockIdx.x;
  const int R = ldh - 1;
  const int m = jm[r];
  const double2* Hr = H + (size_t)r * ldh * R;
  const double2* gr = g + (size_t)r * ldh;
  double2* yr = y + (size_t)r * R;
  for (int i = threadIdx.x; i < m; i += 256) gl[i] = gr[i];
  __syncthreads();
  for (int i = m - 1; i >= 0; --i) {
    const double2* col = Hr + (size_t)i * ldh;
    const double2 d = col[i];
    const double dd = d.x * d.x + d.y * d.y;
    const double2 gi = gl[i];
    const double2 yi = make_double2((gi.x * d.x + gi.y * d.y) / dd, (gi.y * d.x - gi.x * d.y) / dd);
    if (threadIdx.x == 0) yr[i] = yi;
    for (int k = threadIdx.x; k < i; k += 256) {
      const double2 h = col[k];
      gl[k] = make_double2(gl[k].x - (h.x * yi.x - h.y * yi.y), gl[k].y - (h.x * yi.y + h.y * yi.x));
    }
    __syncthreads();
  }
  for (int i = m + threadIdx.x; i < R; i += 256) yr[i] = make_double2(0, 0);
}

__global__ void k_set_g0(int nrhs, int ldh, const double2* nrm2, const int* active, double2* g) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs || !active[r]) return;
  g[(size_t)r * ldh] = make_double2(sqrt(nrm2[r].x), 0.0);
  for (int i = 1; i < ldh; ++i) g[(size_t)r * ldh + i] = make_double2(0, 0);
}

// ---------------------------------------------------------------------------
// workspace: carved from one caller- or context-owned device region, so no
// solve path allocates device memory
// ---------------------------------------------------------------------------
__global__ void k_zero_words(size_t n, uint64_t* __restrict__ p) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}
__global__ void k_fill_int(int n, int v, int* __restrict__ p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
// up to 32 values carried in the kernel arguments (no staging memory)
struct IntChunk {
  int v[32];
};
__global__ void k_put_ints(int n, IntChunk c, int* __restrict__ dst) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = c.v[i];
}

static constexpr size_t kWorkAlign = 256;

// Carves the buffers of a (restart, nrhs) workspace out of base (nullptr:
// only counts); returns the bytes used.
static size_t carve_work(GmresWork& w, char* base, size_t N, size_t restart, size_t nrhs) {
  const size_t ldh = restart + 1, nchunk = (N + RED_CHUNK - 1) / RED_CHUNK;
  size_t off = 0;
  auto take = [&](auto** ptr, size_t bytes) {
    using P = std::remove_reference_t<decltype(**ptr)>;
    *ptr = base ? reinterpret_cast<P*>(base + off) : nullptr;
    off += (bytes + kWorkAlign - 1) / kWorkAlign * kWorkAlign;
  };
  take(&w.V, nrhs * ldh * N * 16);
  take(&w.W, nrhs * N * 16);
  take(&w.H, nrhs * ldh * restart * 16);
  take(&w.Hu, nrhs * ldh * ldh * 16);
  take(&w.hp, nrhs * 2 * ldh * 16);
  take(&w.coef, nrhs * (2 * ldh + 2) * 16);
  take(&w.g, nrhs * ldh * 16);
  take(&w.cs, nrhs * restart * 16);
  take(&w.sn, nrhs * restart * 16);
  take(&w.y, nrhs * restart * 16);
  take(&w.part, nrhs * ldh * nchunk * 2 * 16);
  take(&w.r, nrhs * N * 16);
  take(&w.d, nrhs * N * 16);
  take(&w.b2, nrhs * N * 16);
  take(&w.nrm, nrhs * 2 * 16);
  take(&w.resid, nrhs * restart * 8);
  take(&w.npart, nrhs * nchunk * 8);
  take(&w.active, nrhs * 4 * 2);
  return off;
}

size_t gmres_work_bytes(size_t N, size_t restart, size_t nrhs) {
  GmresWork w;
  return carve_work(w, nullptr, N, restart, nrhs);
}

// Binds a (restart, nrhs) workspace to `bytes` of device memory at base
// (256-byte aligned): carves its buffers, clears them with a fill kernel,
// sets the all-ones mask and sizes the host copies of the residual
// estimates.  Allocates no device memory.
aim_status bind_gmres_work(Ctx* c, GmresWork& w, void* base, size_t bytes, int restart, int nrhs) {
  if (!base || ((uintptr_t)base % kWorkAlign) != 0 || restart < 1 || nrhs < 1) return AIM_E_ARG;
  const size_t need = gmres_work_bytes(c->t.N, restart, nrhs);
  if (bytes < need) return AIM_E_ARG;
  w = GmresWork();
  w.restart = restart;
  w.nrhs = nrhs;
  w.nchunk = (c->t.N + RED_CHUNK - 1) / RED_CHUNK;
  carve_work(w, (char*)base, c->t.N, restart, nrhs);
  w.bytes = need;
  hipLaunchKernelGGL(k_zero_words, dim3(1024), dim3(256), 0, c->stream, need / 8, (uint64_t*)base);
  // all-ones mask used by the residual checks
  hipLaunchKernelGGL(k_fill_int, dim3((nrhs + 255) / 256), dim3(256), 0, c->stream, nrhs, 1, w.active + nrhs);
  AIM_HIP_CHECK(hipGetLastError());
  if (!c->h_resid || !c->d_resid_map || !c->ev_resid || nrhs > c->max_rhs) return AIM_E_STATE;
  // a check may rotate up to kCheckEvery + 1 columns (the last one of a
  // cycle is finalised with the batch); batches that do not fit one block's
  // LDS are split by close_issue
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess || lds <= 0)
    return AIM_E_HIP;
  w.lds_max = (size_t)lds;
  const size_t gb = std::min(((size_t)(kCheckEvery + 1) * (restart + 1) + 2 * (size_t)restart) * 16, w.lds_max);
  if (gb > 65536 &&
      hipFuncSetAttribute((const void*)k_givens_batch, hipFuncAttributeMaxDynamicSharedMemorySize, (int)gb) !=
          hipSuccess)
    return AIM_E_HIP;
  return AIM_OK;
}

#define TRY(x)                   \
  do {                           \
    aim_status s_ = (x);         \
    if (s_ != AIM_OK) return s_; \
  } while (0)

// squared norms of the columns of w into out (double2 .x), active columns only
static aim_status norms(Ctx* c, GmresWork& g, int nrhs, const double2* w, int64_t ldw, const int* active,
                        double2* out) {
  const int N = c->t.N;
  hipLaunchKernelGGL(k_sqnorm, dim3(g.nchunk, nrhs), dim3(256), 0, c->stream, N, w, ldw, active, g.npart, g.nchunk);
  hipLaunchKernelGGL(k_sqnorm_reduce, dim3((nrhs + 63) / 64), dim3(64), 0, c->stream, nrhs, g.nchunk, g.npart,
                     active, out);
  AIM_HIP_CHECK(hipGetLastError());
  return AIM_OK;
}

struct GmresResult {
  std::vector<int> iters, conv;
  std::vector<double> est;
  int matvecs = 0, restarts = 0;
};

// Restarted GMRES for op(x) = b (b, x: N x nrhs contiguous) to rel. tol, as
// a state machine that advances by Arnoldi steps: a cycle starts with the
// true residual of x (top), takes steps in batches of up to kCheckEvery,
// closes each batch with its rotations and residual estimates (the one host
// synchronisation), and ends with x += V y.  SolveRun drives it: to the end
// for aim_solve, a step at a time for the step-wise solver.  Both compute the
// same values in the same order; aim_solve may in addition enqueue one batch
// of steps ahead of the host's check (look), whose work is dropped when the
// check ends the cycle.
struct GmresRun {
  enum Phase { TOP, ARNOLDI, DONE };
  Ctx* c;
  GmresWork& w;
  int op, nrhs;
  const double2* b;
  double2* x;
  std::vector<double> tol;   // per right-hand side
  int maxit, restart;
  GmresResult& res;
  hipStream_t s;
  int N, ldh, gblk;
  int64_t ldv;
  dim3 gN;
  int* d_all;
  std::vector<int> act, jdone, cyc;
  std::vector<double> bn;
  int total = 0, j = 0, jfin = 0, jend = 0;
  bool batch = false;
  Phase phase = TOP;
  // Look-ahead (aim_solve only): the steps of the next batch are enqueued
  // before the host waits for the estimates of the batch just closed, so
  // the GPU does not idle through the round trip.  Steps enqueued after
  // every column has converged are discarded (their results are never
  // read) and not counted.
  bool look = false;
  int pend_c1 = 0, nspec = 0;
  bool pend_last = false;
  std::vector<double> est_prev;

  GmresRun(Ctx* c_, GmresWork& w_, int op_, int nrhs_, const double2* b_, double2* x_, std::vector<double> tol_,
           int maxit_, int restart_, GmresResult& res_)
      : c(c_), w(w_), op(op_), nrhs(nrhs_), b(b_), x(x_), tol(std::move(tol_)), maxit(maxit_), restart(restart_),
        res(res_) {
    s = c->stream;
    N = c->t.N;
    ldh = restart + 1;
    ldv = (int64_t)ldh * N;
    gN = dim3((N + 255) / 256, nrhs);
    gblk = (N + GV_ROWS - 1) / GV_ROWS;
    d_all = w.active + w.nrhs;   // all-ones mask (set when the workspace is bound)
    act.assign(nrhs, 1);
    jdone.assign(nrhs, 0);
    est_prev.assign(nrhs, 0.0);
  }

  // host values to the device through kernel arguments, 32 per launch: no
  // staging memory, and a captured launch keeps its values
  hipError_t put_mask(int* dst, const std::vector<int>& v) {
    for (int i0 = 0; i0 < nrhs; i0 += 32) {
      IntChunk ch;
      const int n = std::min(32, nrhs - i0);
      for (int i = 0; i < 32; ++i) ch.v[i] = i < n ? v[i0 + i] : 0;
      hipLaunchKernelGGL(k_put_ints, dim3(1), dim3(32), 0, s, n, ch, dst + i0);
    }
    return hipGetLastError();
  }

  // ||b||; zero right-hand sides give x = 0
  aim_status start() {
    TRY(norms(c, w, nrhs, b, N, d_all, w.nrm));
    std::vector<double2> hb(nrhs);
    AIM_HIP_CHECK(hipMemcpyAsync(hb.data(), w.nrm, nrhs * 16, hipMemcpyDeviceToHost, s));
    AIM_HIP_CHECK(hipStreamSynchronize(s));
    bn.resize(nrhs);
    for (int r = 0; r < nrhs; ++r) bn[r] = std::sqrt(hb[r].x);
    res.iters.assign(nrhs, 0);
    res.conv.assign(nrhs, 0);
    res.est.assign(nrhs, 0.0);
    for (int r = 0; r < nrhs; ++r)
      if (bn[r] == 0.0) {
        res.conv[r] = 1;
        act[r] = 0;
        hipLaunchKernelGGL(k_zero_words, dim3((N + 255) / 256), dim3(256), 0, s, (size_t)N * 2,
                           (uint64_t*)(x + (size_t)r * N));
      }
    phase = TOP;
    return AIM_OK;
  }

  // cycle start: r0 = b - A x for the unconverged columns (all columns
  // computed), convergence check, first basis vector
  aim_status top() {
    TRY(matvec(c, op, nrhs, x, N, w.W, N));
    res.matvecs++;
    hipLaunchKernelGGL(k_bminus, gN, dim3(256), 0, s, N, b, w.W);
    AIM_HIP_CHECK(put_mask(w.active, act));
    TRY(norms(c, w, nrhs, w.W, N, w.active, w.nrm));
    std::vector<double2> h0(nrhs);
    AIM_HIP_CHECK(hipMemcpyAsync(h0.data(), w.nrm, nrhs * 16, hipMemcpyDeviceToHost, s));
    AIM_HIP_CHECK(hipStreamSynchronize(s));
    bool any = false;
    for (int r = 0; r < nrhs; ++r) {
      if (!act[r]) continue;
      const double rel = std::sqrt(h0[r].x) / bn[r];
      if (!std::isfinite(rel)) return AIM_E_NUMERIC;
      res.est[r] = rel;
      if (rel <= tol[r]) { act[r] = 0; res.conv[r] = 1; }
      else any = true;
    }
    if (!any || total >= maxit) {
      phase = DONE;
      return AIM_OK;
    }
    AIM_HIP_CHECK(put_mask(w.active, act));
    hipLaunchKernelGGL(k_normalize, gN, dim3(256), 0, s, N, w.nrm, w.W, (int64_t)N, w.V, ldv, w.active);
    hipLaunchKernelGGL(k_set_g0, dim3((nrhs + 63) / 64), dim3(64), 0, s, nrhs, ldh, w.nrm, w.active, w.g);
    std::fill(jdone.begin(), jdone.end(), 0);
    cyc = act;
    // Arnoldi step j finalises Hessenberg column j - 1; jfin columns are
    // final and rotated
    j = 0;
    jfin = 0;
    batch = false;
    phase = ARNOLDI;
    return AIM_OK;
  }

  // one Arnoldi step: w = A u_j, reduction pass, update pass
  aim_status arnoldi_step() {
    TRY(matvec(c, op, nrhs, w.V + (size_t)j * N, ldv, w.W, N));
    return orthogonalise();
  }

  // the passes of step j after its operator application w = A u_j
  aim_status orthogonalise() {
    res.matvecs++;
    hipLaunchKernelGGL(k_arnoldi_dots, dim3(w.nchunk, dot_groups(j) + hs_blocks(j, w.nchunk), nrhs), dim3(256), 0, s,
                       N, j, w.V, ldv, w.W, (int64_t)N, w.active, w.part, w.nchunk, ldh, w.Hu, w.coef, w.hp);
    hipLaunchKernelGGL(k_arnoldi_update, dim3(gblk, nrhs), dim3(256), (size_t)(j + 1) * 48, s, N, j, w.nchunk,
                       ldh, w.part, w.V, ldv, w.W, (int64_t)N, w.active, w.Hu, w.H, w.hp, w.coef, 0);
    AIM_HIP_CHECK(hipGetLastError());
    total++;
    ++j;
    return AIM_OK;
  }

  // The grouped step (solver_step): an Arnoldi step whose operator
  // application is split at its column pass, which runs in one launch with
  // other solvers' (same kernels, same order of this solver's work as
  // arnoldi_step).  at_step: the next action is an Arnoldi step.
  bool at_step() const { return phase == ARNOLDI && batch && j < jend; }
  aim_status step_pre(ColsJob* job) { return matvec_pre(c, op, nrhs, w.V + (size_t)j * N, ldv, job); }
  aim_status step_post() {
    TRY(matvec_post(c, op, nrhs, w.V + (size_t)j * N, ldv, w.W, N));
    TRY(orthogonalise());
    return after_step();
  }

  // after a step: the check that closes a completed batch
  aim_status after_step() {
    if (j < jend) return AIM_OK;
    batch = false;
    bool over = false;
    TRY(close_issue());
    if (look && !pend_last && worth_speculating()) {
      jend = std::min(std::min(restart, j + kCheckEvery), j + (maxit - total));
      batch = true;
      while (j < jend) {
        TRY(arnoldi_step());
        ++nspec;
      }
    }
    TRY(close_resolve(over));
    if (over) {
      // the look-ahead steps did not happen as far as the solve is concerned
      total -= nspec;
      res.matvecs -= nspec;
      j -= nspec;
      batch = false;
    }
    nspec = 0;
    if (over) TRY(end_cycle());
    return AIM_OK;
  }

  // A look-ahead batch is wasted only if every column converges in the
  // batch being closed: skip it when each active column's estimate, reduced
  // by the factor its previous batch achieved, would reach its tolerance.
  bool worth_speculating() const {
    for (int r = 0; r < nrhs; ++r) {
      if (!act[r]) continue;
      const double e = res.est[r], ep = est_prev[r];
      const double pred = (ep > 0.0 && e > 0.0 && e < ep) ? e * (e / ep) : e;
      if (!(pred <= tol[r])) return true;
    }
    return false;
  }

  // end of a batch, GPU side: rotations of the newly final columns and the
  // copy of their residual estimates to the host buffer
  aim_status close_issue() {
    // at the end of a cycle the last column is finalised by a reduction of
    // u_j alone (no operator application)
    pend_last = j >= restart || total >= maxit;
    if (pend_last) {
      hipLaunchKernelGGL(k_arnoldi_dots, dim3(w.nchunk, dot_groups(j) + hs_blocks(j, w.nchunk), nrhs), dim3(256), 0,
                         s, N, j, w.V, ldv, (const double2*)nullptr, (int64_t)0, w.active, w.part, w.nchunk, ldh,
                         w.Hu, w.coef, w.hp);
      hipLaunchKernelGGL(k_arnoldi_update, dim3(1, nrhs), dim3(256), (size_t)(j + 1) * 48, s, N, j, w.nchunk, ldh,
                         w.part, w.V, ldv, (const double2*)nullptr, (int64_t)0, w.active, w.Hu, w.H, w.hp, w.coef,
                         1);
      AIM_HIP_CHECK(hipGetLastError());
    }
    pend_c1 = pend_last ? j : j - 1;
    if (pend_c1 <= jfin) return AIM_OK;
    // in column groups whose LDS footprint fits one block (long restarts)
    for (int a = jfin; a < pend_c1;) {
      int e = pend_c1;
      while (e > a + 1 && ((size_t)(e - a) * ldh + 2 * (size_t)e) * 16 > w.lds_max) --e;
      // the residual estimates jfin .. c1-1 of every active rhs go to the
      // context's pinned buffer (kResidPitch per rhs), written by the kernel
      // itself: no copy sits in the stream between this batch and the next.
      // close_resolve reads them before the next batch is closed, so
      // solvers sharing the context take turns.
      hipLaunchKernelGGL(k_givens_batch, dim3(nrhs), dim3(256), ((size_t)(e - a) * ldh + 2 * (size_t)e) * 16, s,
                         ldh, a, e, w.active, w.H, w.cs, w.sn, w.g, w.resid, c->d_resid_map, jfin, kResidPitch);
      AIM_HIP_CHECK(hipGetLastError());
      a = e;
    }
    AIM_HIP_CHECK(hipEventRecord(c->ev_resid, s));
    return AIM_OK;
  }

  // end of a batch, host side: wait for the copy, count the steps of each
  // column up to its convergence; over = true when no column is left in
  // this cycle
  aim_status close_resolve(bool& over) {
    over = false;
    const int c1 = pend_c1;
    if (c1 <= jfin) return AIM_OK;
    AIM_HIP_CHECK(hipEventSynchronize(c->ev_resid));
    bool left = false, changed = false;
    for (int r = 0; r < nrhs; ++r) {
      if (!act[r]) continue;
      est_prev[r] = res.est[r];
      for (int jj = jfin; jj < c1; ++jj) {
        res.iters[r]++;
        jdone[r] = jj + 1;
        const double rel = c->h_resid[(size_t)r * kResidPitch + (jj - jfin)] / bn[r];
        if (!std::isfinite(rel)) return AIM_E_NUMERIC;
        res.est[r] = rel;
        if (rel <= tol[r]) { act[r] = 0; changed = true; break; }
      }
      if (act[r]) left = true;
    }
    jfin = c1;
    if (!left) {
      over = true;
      return AIM_OK;
    }
    if (changed) AIM_HIP_CHECK(put_mask(w.active, act));
    return AIM_OK;
  }

  // cycle end: x += V y for every column that took steps in this cycle
  aim_status end_cycle() {
    std::vector<int> upd(nrhs, 0);
    for (int r = 0; r < nrhs; ++r) upd[r] = (cyc[r] && jdone[r] > 0) ? 1 : 0;
    int* d_jm = (int*)w.part;   // scratch: jm then mask
    AIM_HIP_CHECK(put_mask(d_jm, jdone));
    AIM_HIP_CHECK(put_mask(w.active, upd));
    hipLaunchKernelGGL(k_trisolve, dim3(nrhs), dim3(256), (size_t)ldh * 16, s, nrhs, ldh, d_jm, w.H, w.g, w.y);
    int jmax = 0;
    for (int r = 0; r < nrhs; ++r) jmax = std::max(jmax, jdone[r]);
    if (jmax > 0)
      hipLaunchKernelGGL(k_gemv, dim3((N + GV_ROWS - 1) / GV_ROWS, nrhs), dim3(256), 0, s, N, jmax, w.V, ldv, w.y,
                         (int64_t)restart, 1.0, w.active, x, (int64_t)N);
    AIM_HIP_CHECK(hipGetLastError());
    res.restarts++;
    // columns flagged converged by the estimate are re-checked with the true
    // residual at the top of the next cycle
    for (int r = 0; r < nrhs; ++r)
      if (cyc[r]) act[r] = 1;
    for (int r = 0; r < nrhs; ++r)
      if (res.conv[r]) act[r] = 0;
    if (total >= maxit) {
      // final true residual
      TRY(matvec(c, op, nrhs, x, N, w.W, N));
      res.matvecs++;
      hipLaunchKernelGGL(k_bminus, gN, dim3(256), 0, s, N, b, w.W);
      TRY(norms(c, w, nrhs, w.W, N, d_all, w.nrm));
      std::vector<double2> h0(nrhs);
      AIM_HIP_CHECK(hipMemcpyAsync(h0.data(), w.nrm, nrhs * 16, hipMemcpyDeviceToHost, s));
      AIM_HIP_CHECK(hipStreamSynchronize(s));
      for (int r = 0; r < nrhs; ++r)
        if (bn[r] > 0) {
          res.est[r] = std::sqrt(h0[r].x) / bn[r];
          res.conv[r] = res.est[r] <= tol[r];
        }
      phase = DONE;
    } else {
      phase = TOP;
    }
    return AIM_OK;
  }

  // Runs until `steps` more Arnoldi steps have been taken or the solve is
  // done.  The check that closes a batch runs right after the step that
  // completes it.
  aim_status advance(long steps) {
    while (phase != DONE) {
      if (phase == TOP) {
        TRY(top());
        continue;
      }
      if (batch && j >= jend) {
        // a look-ahead batch is complete: close it first (it may end the cycle)
        TRY(after_step());
        continue;
      }
      if (!(j < restart && total < maxit)) {
        TRY(end_cycle());
        continue;
      }
      if (!batch) {
        jend = std::min(std::min(restart, j + kCheckEvery), j + (maxit - total));
        batch = true;
      }
      if (j < jend) {
        if (steps <= 0) return AIM_OK;
        TRY(arnoldi_step());
        --steps;
      }
      TRY(after_step());
    }
    return AIM_OK;
  }
};

static int form_op(int form) {
  switch (form) {
    case AIM_TM_EFIE: return AIM_OP_TM;
    case AIM_TE_CALDERON: return AIM_OP_TE_CP;
    case AIM_TE_CALDERON_UNFILTERED: return AIM_OP_TE_CP_UNF;
    case AIM_TM_CALDERON: return AIM_OP_TM_CP;
    case AIM_TM_CALDERON_UNFILTERED: return AIM_OP_TM_CP_UNF;
  }
  return -1;
}

// relative true residuals ||b - op x|| / ||b|| (FP64 operator)
static aim_status true_resid(Ctx* c, GmresWork& w, int op, int nrhs, const double2* b, const double2* x,
                             std::vector<double>& out) {
  const int N = c->t.N;
  int* d_all = w.active + w.nrhs;
  TRY(matvec(c, op, nrhs, x, N, w.W, N));
  hipLaunchKernelGGL(k_bminus, dim3((N + 255) / 256, nrhs), dim3(256), 0, c->stream, N, b, w.W);
  TRY(norms(c, w, nrhs, w.W, N, d_all, w.nrm));
  TRY(norms(c, w, nrhs, b, N, d_all, w.nrm + nrhs));
  std::vector<double2> h(2 * nrhs);
  AIM_HIP_CHECK(hipMemcpyAsync(h.data(), w.nrm, 2 * nrhs * 16, hipMemcpyDeviceToHost, c->stream));
  AIM_HIP_CHECK(hipStreamSynchronize(c->stream));
  out.resize(nrhs);
  for (int r = 0; r < nrhs; ++r) out[r] = h[nrhs + r].x > 0 ? std::sqrt(h[r].x / h[nrhs + r].x) : 0.0;
  return AIM_OK;
}

// Argument checks shared by aim_solve and the step-wise solver.
static aim_status check_solve(Ctx* c, int form, int precision, int nrhs, double tol, int maxit, int restart) {
  const int op = form_op(form);
  if (op < 0 || nrhs < 1 || nrhs > c->max_rhs || !(tol > 0) || maxit < 1 || restart < 1 || restart > 1000)
    return AIM_E_ARG;
  if (precision != AIM_FP64 && precision != AIM_MIXED) return AIM_E_ARG;
  if (precision == AIM_MIXED && c->precision != AIM_MIXED) return AIM_E_ARG;
  const bool tm = form == AIM_TM_EFIE || form == AIM_TM_CALDERON || form == AIM_TM_CALDERON_UNFILTERED;
  if (c->t.basis != (tm ? AIM_PULSE : AIM_HAT)) return AIM_E_ARG;
  if ((form == AIM_TM_CALDERON || form == AIM_TM_CALDERON_UNFILTERED) && !c->dual) return AIM_E_STATE;
  return AIM_OK;
}

// The right-hand side of the iterated system: b itself for the TM EFIE, the
// preconditioned one (into w.b2) for the Calderon forms.
static aim_status system_rhs(Ctx* c, GmresWork& w, int form, int nrhs, const double2* b, const double2** rhs) {
  const int N = c->t.N;
  *rhs = b;
  if (form == AIM_TM_CALDERON || form == AIM_TM_CALDERON_UNFILTERED) {
    // preconditioned right-hand side G_pd^-T N'(alpha) G_pd^-1 b
    TRY(matvec(c, form == AIM_TM_CALDERON ? AIM_OP_TM_PC : AIM_OP_TM_PC_UNF, nrhs, b, N, w.b2, N));
    *rhs = w.b2;
  } else if (form != AIM_TM_EFIE) {
    // preconditioned right-hand side G^-1 S G^-1 b
    TRY(matvec(c, AIM_OP_GRAM_INV, nrhs, b, N, c->d_tmp1, N));
    TRY(matvec(c, form == AIM_TE_CALDERON ? AIM_OP_S_ALPHA : AIM_OP_S, nrhs, c->d_tmp1, N, c->d_tmp2, N));
    TRY(matvec(c, AIM_OP_GRAM_INV, nrhs, c->d_tmp2, N, w.b2, N));
    *rhs = w.b2;
  }
  return AIM_OK;
}

// The whole solve of aim_solve as a state machine that advances by Arnoldi
// steps: FP64 GMRES on the system of `form`, or (AIM_MIXED) iterative
// refinement whose outer checks take the FP64 true residual and whose inner
// solves are FP32-grid GMRES runs; then the final true residual.  aim_solve
// runs it to the end on the context's workspace, a step-wise solver on its
// own one.
struct SolveRun {
  enum Phase { FP64_RUN, MIX_CHECK, MIX_INNER, FINAL, DONE };
  Ctx* c;
  GmresWork& w;
  int form, precision, op, nrhs;
  const double2* b;
  double2* x;
  double tol;
  int maxit, restart;
  const double2* rhs = nullptr;
  std::vector<int> iters, conv;
  std::vector<double> est, tr;
  int matvecs = 0, restarts = 0, outer = 0;
  double tin_min = 0;
  bool look = false;   // run to the end (aim_solve): GMRES batches look ahead
  GmresResult gr;
  std::unique_ptr<GmresRun> run;
  Phase phase = FINAL;
  aim_status status = AIM_OK;   // result once DONE

  SolveRun(Ctx* c_, GmresWork& w_, int form_, int precision_, int nrhs_, const double2* b_, double2* x_,
           double tol_, int maxit_, int restart_)
      : c(c_), w(w_), form(form_), precision(precision_), op(form_op(form_)), nrhs(nrhs_), b(b_), x(x_),
        tol(tol_), maxit(maxit_), restart(restart_) {
    iters.assign(nrhs, 0);
    conv.assign(nrhs, 0);
    est.assign(nrhs, 0.0);
    // Inner solves stop no lower than 1e-5 relative (and no lower than
    // 10 tol): the FP32 grid product is accurate to ~1e-6 relative, the
    // inner Krylov convergence slows as the inner residual approaches that
    // level, and one more refinement step is cheaper than those steps.
    tin_min = std::min(1e-2, std::max(1e-5, 10.0 * tol));
  }

  aim_status begin() {
    TRY(system_rhs(c, w, form, nrhs, b, &rhs));
    if (precision == AIM_FP64) {
      run.reset(new (std::nothrow) GmresRun(c, w, op, nrhs, rhs, x, std::vector<double>(nrhs, tol), maxit, restart,
                                            gr));
      if (!run) return AIM_E_OOM;
      run->look = look;
      TRY(run->start());
      phase = FP64_RUN;
    } else {
      phase = MIX_CHECK;
    }
    return AIM_OK;
  }

  // refinement: FP64 residual, FP32-grid inner GMRES on it.  Columns are
  // refined independently: a converged column gets a zero inner right-hand
  // side (its correction is zero and it takes no steps), and each column's
  // inner tolerance follows its own residual, so a column's result does not
  // depend on the other columns of the batch.
  aim_status mix_check() {
    if (outer >= 30) {
      phase = FINAL;
      return AIM_OK;
    }
    const int N = c->t.N;
    hipStream_t s = c->stream;
    std::vector<double> rel;
    TRY(true_resid(c, w, op, nrhs, rhs, x, rel));
    matvecs++;
    bool done = true;
    for (int r = 0; r < nrhs; ++r) {
      if (!std::isfinite(rel[r])) return AIM_E_NUMERIC;
      if (rel[r] > tol) done = false;
      est[r] = rel[r];
      conv[r] = rel[r] <= tol;
    }
    int tot_it = 0;
    for (int r = 0; r < nrhs; ++r) tot_it = std::max(tot_it, iters[r]);
    if (done || tot_it >= maxit) {
      phase = FINAL;
      return AIM_OK;
    }
    // r = b - A x (left in w.W by true_resid), zero for converged columns;
    // d = 0.  The inner solve reads w.r and writes w.d.
    AIM_HIP_CHECK(hipMemcpyAsync(w.r, w.W, (size_t)N * nrhs * 16, hipMemcpyDeviceToDevice, s));
    std::vector<double> tin(nrhs, 0.5);
    for (int r = 0; r < nrhs; ++r) {
      if (conv[r])
        hipLaunchKernelGGL(k_zero_words, dim3((N + 255) / 256), dim3(256), 0, s, (size_t)N * 2,
                           (uint64_t*)(w.r + (size_t)r * N));
      else
        tin[r] = std::min(std::max(tin_min, 0.5 * tol / rel[r]), 0.5);
    }
    hipLaunchKernelGGL(k_zero_words, dim3(1024), dim3(256), 0, s, (size_t)N * nrhs * 2, (uint64_t*)w.d);
    AIM_HIP_CHECK(hipGetLastError());
    gr = GmresResult();
    run.reset(new (std::nothrow) GmresRun(c, w, op | AIM_OP_GRID_FP32, nrhs, w.r, w.d, tin, maxit - tot_it, restart,
                                          gr));
    if (!run) return AIM_E_OOM;
    run->look = look;
    TRY(run->start());
    phase = MIX_INNER;
    return AIM_OK;
  }

  aim_status mix_inner_done() {
    const int N = c->t.N;
    for (int r = 0; r < nrhs; ++r) iters[r] += gr.iters[r];
    matvecs += gr.matvecs;
    restarts += gr.restarts;
    hipLaunchKernelGGL(k_axpy, dim3((N + 255) / 256, nrhs), dim3(256), 0, c->stream, N, w.d, x);
    AIM_HIP_CHECK(hipGetLastError());
    ++outer;
    phase = MIX_CHECK;
    return AIM_OK;
  }

  aim_status finish() {
    TRY(true_resid(c, w, op, nrhs, rhs, x, tr));
    bool all = true;
    for (int r = 0; r < nrhs; ++r) {
      if (!std::isfinite(tr[r])) return AIM_E_NUMERIC;
      all = all && converged(r);
    }
    status = all ? AIM_OK : AIM_E_NOCONV;
    phase = DONE;
    return AIM_OK;
  }

  bool converged(int r) const {
    if (tr.size() != (size_t)nrhs) return false;
    return precision == AIM_FP64 ? (conv[r] && tr[r] <= tol * 1.5) : (tr[r] <= tol);
  }

  // Runs until `steps` more Arnoldi steps have been taken or the solve is
  // done; an error ends the solve with that status.
  aim_status advance(long steps) {
    while (phase != DONE) {
      aim_status st = AIM_OK;
      if (phase == FP64_RUN || phase == MIX_INNER) {
        const int before = run->total;
        st = run->advance(steps);
        steps -= run->total - before;
        if (st == AIM_OK && run->phase == GmresRun::DONE) {
          if (phase == FP64_RUN) {
            iters = gr.iters;
            conv = gr.conv;
            est = gr.est;
            matvecs = gr.matvecs;
            restarts = gr.restarts;
            phase = FINAL;
          } else {
            st = mix_inner_done();
          }
        } else if (st == AIM_OK) {
          return AIM_OK;   // the step budget is spent
        }
      } else if (phase == MIX_CHECK) {
        st = mix_check();
      } else {
        st = finish();
      }
      if (st != AIM_OK) {
        status = st;
        phase = DONE;
        return st;
      }
    }
    return AIM_OK;
  }

  // Grouped step (solver_step): the running GMRES is right before an
  // Arnoldi step; step_pre runs its operator up to the column pass,
  // step_post the rest of the step and whatever follows it up to the next
  // step (as advance(1) does).  An error ends the solve with that status.
  bool at_step() const { return (phase == FP64_RUN || phase == MIX_INNER) && run && run->at_step(); }
  int step_op() const { return run->op; }
  aim_status end_with(aim_status st) {
    if (st != AIM_OK) {
      status = st;
      phase = DONE;
    }
    return st;
  }
  aim_status step_pre(ColsJob* job) { return end_with(run->step_pre(job)); }
  aim_status step_post() {
    TRY(end_with(run->step_post()));
    return advance(0);
  }

  void fill(aim_solve_info* info, double secs) const {
    const bool fin = phase == DONE && tr.size() == (size_t)nrhs;
    for (int r = 0; r < nrhs; ++r) {
      // a running FP64 solve reports the live counts of its GMRES
      const bool live = phase == FP64_RUN && gr.iters.size() == (size_t)nrhs;
      info[r].iterations = live ? gr.iters[r] : iters[r] + (phase == MIX_INNER && gr.iters.size() ==
                                                             (size_t)nrhs ? gr.iters[r] : 0);
      info[r].matvecs = (phase == FP64_RUN || phase == MIX_INNER) ? matvecs + gr.matvecs : matvecs;
      info[r].restarts = (phase == FP64_RUN || phase == MIX_INNER) ? restarts + gr.restarts : restarts;
      info[r].outer = outer;
      info[r].converged = fin && converged(r) ? 1 : 0;
      info[r].resid_est = live ? gr.est[r] : est[r];
      info[r].resid_true = fin ? tr[r] : -1.0;
      info[r].seconds = secs;
    }
  }
};

aim_status solve(Ctx* c, int form, int precision, int nrhs, const double2* b, double2* x, double tol, int maxit,
                 int restart, aim_solve_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  TRY(check_solve(c, form, precision, nrhs, tol, maxit, restart));
  // the context's workspace, bound at set-up for max_rhs and max_restart
  if (!c->gw.V) return AIM_E_STATE;
  if (restart > c->gw.restart || nrhs > c->gw.nrhs) return AIM_E_ARG;
  SolveRun sr(c, c->gw, form, precision, nrhs, b, x, tol, maxit, restart);
  sr.look = true;
  TRY(sr.begin());
  TRY(sr.advance(std::numeric_limits<long>::max()));
  if (info) sr.fill(info, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  return sr.status;
}

// ---------------------------------------------------------------------------
// Step-wise solver: one solve of aim_solve (a SolveRun) on its own workspace,
// advanced by Arnoldi steps (serving schedulers interleave the steps of many
// requests).  Several solvers may share a context; their steps then run in
// call order on the context's stream.
// ---------------------------------------------------------------------------
}  // namespace aim

struct aim_solver_s {
  aim::Ctx* c = nullptr;
  aim::GmresWork w;
  std::unique_ptr<aim::SolveRun> run;
  std::chrono::steady_clock::time_point t0;
  double seconds = 0;
  hipEvent_t ev = nullptr;   // orders a grouped column pass across streams
};

namespace aim {

static void solver_free(aim_solver_s* sv) {
  sv->run.reset();
  if (sv->ev) (void)hipEventDestroy(sv->ev);
  delete sv;
}

aim_status solver_begin(Ctx* c, int form, int precision, int nrhs, const double2* b, double2* x, double tol,
                        int maxit, int restart, void* workspace, size_t workspace_bytes, aim_solver_s** out) {
  TRY(check_solve(c, form, precision, nrhs, tol, maxit, restart));
  aim_solver_s* sv = new (std::nothrow) aim_solver_s();
  if (!sv) return AIM_E_OOM;
  sv->c = c;
  sv->t0 = std::chrono::steady_clock::now();
  // the caller's workspace (device memory it owns until aim_solver_end)
  aim_status st = bind_gmres_work(c, sv->w, workspace, workspace_bytes, restart, nrhs);
  if (st == AIM_OK && hipEventCreateWithFlags(&sv->ev, hipEventDisableTiming) != hipSuccess) st = AIM_E_HIP;
  if (st != AIM_OK) {
    solver_free(sv);
    return st;
  }
  sv->run.reset(new (std::nothrow) SolveRun(c, sv->w, form, precision, nrhs, b, x, tol, maxit, restart));
  st = sv->run ? sv->run->begin() : AIM_E_OOM;
  if (st != AIM_OK) {
    (void)hipStreamSynchronize(c->stream);
    solver_free(sv);
    return st;
  }
  *out = sv;
  return AIM_OK;
}

// One Arnoldi step for each unfinished solver.  Solvers whose next step
// applies an operator with a single grid product (TM, S, S^alpha, N,
// N^alpha; FP64 or FP32 grid), on contexts that no other solver of this
// call uses, are grouped by spectrum: their column passes run as one
// launch over all members' tiles, which reads the shared spectrum once.
// The launch waits for the members' forward row passes (events across
// their streams) and their inverse row passes wait for it.  Every other
// solver takes its step alone.  Each tile is computed as in a step alone,
// so results do not depend on the grouping.
aim_status solver_step(aim_solver_s** group, int count) {
  if (count < 0 || (count > 0 && !group)) return AIM_E_ARG;
  aim_status first = AIM_OK;
  auto note = [&](aim_solver_s* sv, aim_status st) {
    if (sv->run->phase == SolveRun::DONE && sv->seconds == 0.0)
      sv->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - sv->t0).count();
    if (st != AIM_OK && first == AIM_OK) first = st;
  };
  std::vector<aim_solver_s*> live;
  for (int i = 0; i < count; ++i)
    if (group[i] && group[i]->run->phase != SolveRun::DONE) live.push_back(group[i]);
  // contexts stepped by more than one solver here share work buffers: those
  // solvers step alone, in call order
  std::vector<aim_solver_s*> solo, cand;
  for (aim_solver_s* sv : live) {
    int uses = 0;
    for (aim_solver_s* o : live) uses += o->c == sv->c;
    (uses > 1 ? solo : cand).push_back(sv);
  }
  for (aim_solver_s* sv : solo) note(sv, sv->run->advance(1));
  // position the others right before their next Arnoldi step
  std::vector<aim_solver_s*> split;
  for (aim_solver_s* sv : cand) {
    aim_status st = sv->run->advance(0);
    if (st != AIM_OK || sv->run->phase == SolveRun::DONE) {
      note(sv, st);
      continue;
    }
    if (sv->run->at_step() && matvec_splits(sv->c, sv->run->step_op())) split.push_back(sv);
    else note(sv, sv->run->advance(1));
  }
  // forward halves of the split steps
  std::vector<ColsJob> jobs(split.size());
  std::vector<aim_solver_s*> ok;
  std::vector<ColsJob> okjobs;
  for (size_t i = 0; i < split.size(); ++i) {
    aim_status st = split[i]->run->step_pre(&jobs[i]);
    if (st != AIM_OK) note(split[i], st);
    else {
      ok.push_back(split[i]);
      okjobs.push_back(jobs[i]);
    }
  }
  // column passes, one launch per spectrum
  std::vector<char> taken(ok.size(), 0);
  for (size_t i = 0; i < ok.size(); ++i) {
    if (taken[i]) continue;
    std::vector<size_t> mem;
    for (size_t k = i; k < ok.size(); ++k)
      if (!taken[k] && okjobs[k].Cq == okjobs[i].Cq && okjobs[k].n == okjobs[i].n && okjobs[k].f32 == okjobs[i].f32) {
        mem.push_back(k);
        taken[k] = 1;
      }
    hipStream_t lead = ok[mem[0]]->c->stream;
    aim_status st = AIM_OK;
    for (size_t q = 1; q < mem.size() && st == AIM_OK; ++q) {
      aim_solver_s* sv = ok[mem[q]];
      if (sv->c->stream == lead) continue;
      if (hipEventRecord(sv->ev, sv->c->stream) != hipSuccess || hipStreamWaitEvent(lead, sv->ev, 0) != hipSuccess)
        st = AIM_E_HIP;
    }
    std::vector<ColsJob> gj;
    for (size_t k : mem) gj.push_back(okjobs[k]);
    if (st == AIM_OK) st = launch_cols_jobs(gj.data(), (int)gj.size(), lead);
    aim_solver_s* l = ok[mem[0]];
    if (st == AIM_OK && mem.size() > 1 && hipEventRecord(l->ev, lead) != hipSuccess) st = AIM_E_HIP;
    for (size_t q = 1; q < mem.size() && st == AIM_OK; ++q) {
      aim_solver_s* sv = ok[mem[q]];
      if (sv->c->stream != lead && hipStreamWaitEvent(sv->c->stream, l->ev, 0) != hipSuccess) st = AIM_E_HIP;
    }
    for (size_t k : mem) {
      aim_solver_s* sv = ok[k];
      note(sv, st != AIM_OK ? sv->run->end_with(st) : sv->run->step_post());
    }
  }
  return first;
}

aim_status solver_poll(aim_solver_s* sv, aim_solve_info* info) {
  if (!sv) return AIM_E_ARG;
  const bool done = sv->run->phase == SolveRun::DONE;
  if (info)
    sv->run->fill(info, done ? sv->seconds
                             : std::chrono::duration<double>(std::chrono::steady_clock::now() - sv->t0).count());
  return done ? sv->run->status : AIM_PENDING;
}

aim_status solver_end(aim_solver_s* sv) {
  if (!sv) return AIM_E_ARG;
  const hipError_t e = hipStreamSynchronize(sv->c->stream);
  solver_free(sv);
  return e == hipSuccess ? AIM_OK : AIM_E_HIP;
}

}  // namespace aim
