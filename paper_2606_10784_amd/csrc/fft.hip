// Zero-padded 2D FFT convolution of eq. (8) / eq. (10) for gfx950.
//
// The grid product G_grid u is evaluated as
//     [F^-1( F(c) . F(b) )]_restr,   b = u zero-padded from m x m to n x n,
// with n the smallest power of two >= 2m and the spectrum F(c) of the
// circulant kernel resident in HBM as an even-symmetric quarter (Sec.
// III-A/B).  Three passes:
//   rows_fwd : scatter the active grid values of one grid row into LDS,
//              length-n FFT along x, write the row (only rows [y0, y0+nr)
//              that hold active points, compacted);
//   cols_conv: for a block of CW columns: length-n FFT along y (rows >= nr are
//              zero), multiply by the spectrum, inverse FFT, keep nr rows;
//   rows_inv : inverse FFT along x, gather the active points of the row.
// The circulant product commutes with cyclic shifts, so compacting the rows to
// [0, nr) changes nothing.  The 1/n^2 of the inverse DFT is folded into the
// stored spectrum.
//
// Each FFT is an in-LDS Stockham autosort with radix-16 passes (radix 8, 4
// or 2 for the remainder); each thread holds its butterflies in registers
// across a barrier, so a single LDS buffer suffices.  In the column pass the
// first forward pass reads the tile from HBM straight into registers (its
// upper half is the zero padding), the last forward pass, the spectrum
// multiply and the first inverse pass share one register round (the inverse
// runs its radices in reverse order so the butterflies line up), and the last
// inverse pass stores only the kept rows straight to HBM.
#include <hip/hip_ext.h>

#include "aim_internal.h"

namespace aim {

// ---------------------------------------------------------------------------
// small DFTs in registers (forward: e^{-2 pi i/R}, INV: conjugate)
// ---------------------------------------------------------------------------
template <typename V, bool INV>
__device__ __forceinline__ V rot_mi(V a) {      // multiply by -i (forward) or +i (inverse)
  V r;
  if (INV) { r.x = -a.y; r.y = a.x; }
  else { r.x = a.y; r.y = -a.x; }
  return r;
}

template <typename V, bool INV>
__device__ __forceinline__ void dft2(V& a, V& b) {
  V t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <typename V, bool INV>
__device__ __forceinline__ void dft4(V& a, V& b, V& c, V& d) {
  V t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), t3 = rot_mi<V, INV>(csub(b, d));
  a = cadd(t0, t2);
  c = csub(t0, t2);
  b = cadd(t1, t3);
  d = csub(t1, t3);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cplx<T>* v) {
  using V = cplx<T>;
  const T c = (T)0.70710678118654752440084436210484903928;
  // even / odd halves
  V e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  V o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<V, INV>(e0, e1, e2, e3);
  dft4<V, INV>(o0, o1, o2, o3);
  // twiddles w8^k on the odd half
  V w1, w3;
  if (!INV) {
    w1.x = c * (o1.x + o1.y); w1.y = c * (o1.y - o1.x);
    w3.x = c * (o3.y - o3.x); w3.y = -c * (o3.x + o3.y);
  } else {
    w1.x = c * (o1.x - o1.y); w1.y = c * (o1.x + o1.y);
    w3.x = -c * (o3.x + o3.y); w3.y = c * (o3.x - o3.y);
  }
  V w2 = rot_mi<V, INV>(o2);
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, w1); v[5] = csub(e1, w1);
  v[2] = cadd(e2, w2); v[6] = csub(e2, w2);
  v[3] = cadd(e3, w3); v[7] = csub(e3, w3);
}

// 16-point DFT as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
template <typename T, bool INV>
__device__ __forceinline__ void dft16(cplx<T>* v) {
  using V = cplx<T>;
  // W16^e, e = 0..9 (forward sign)
  const T c1 = (T)0.92387953251128675612818318939678829, s1 = (T)0.38268343236508977172845998403039887;
  const T c2 = (T)0.70710678118654752440084436210484903;
  dft4<V, INV>(v[0], v[4], v[8], v[12]);
  dft4<V, INV>(v[1], v[5], v[9], v[13]);
  dft4<V, INV>(v[2], v[6], v[10], v[14]);
  dft4<V, INV>(v[3], v[7], v[11], v[15]);
  // after the first stage v[4 k1 + n2] holds A[n2][k1]; twiddle by W16^{n2 k1}
  auto tw = [&](V a, T c, T sn) -> V {   // a * (c - i sn) forward, a * (c + i sn) inverse
    V r;
    if (!INV) { r.x = a.x * c + a.y * sn; r.y = a.y * c - a.x * sn; }
    else { r.x = a.x * c - a.y * sn; r.y = a.y * c + a.x * sn; }
    return r;
  };
  // n2 = 1: k1 = 1,2,3 -> e = 1,2,3
  v[5] = tw(v[5], c1, s1);
  v[9] = tw(v[9], c2, c2);
  v[13] = tw(v[13], s1, c1);
  // n2 = 2: e = 2,4,6
  v[6] = tw(v[6], c2, c2);
  v[10] = rot_mi<V, INV>(v[10]);
  v[14] = tw(v[14], -c2, c2);
  // n2 = 3: e = 3,6,9
  v[7] = tw(v[7], s1, c1);
  v[11] = tw(v[11], -c2, c2);
  v[15] = tw(v[15], -c1, -s1);
  // second stage over n2 for each k1; output X[k1 + 4 k2]
  dft4<V, INV>(v[0], v[1], v[2], v[3]);
  dft4<V, INV>(v[4], v[5], v[6], v[7]);
  dft4<V, INV>(v[8], v[9], v[10], v[11]);
  dft4<V, INV>(v[12], v[13], v[14], v[15]);
  // v[4 k1 + k2] holds X[k1 + 4 k2]: transpose the 4 x 4 block
  V t;
  t = v[1]; v[1] = v[4]; v[4] = t;
  t = v[2]; v[2] = v[8]; v[8] = t;
  t = v[3]; v[3] = v[12]; v[12] = t;
  t = v[6]; v[6] = v[9]; v[9] = t;
  t = v[7]; v[7] = v[13]; v[13] = t;
  t = v[11]; v[11] = v[14]; v[14] = t;
}

// 16-point DFT whose inputs 8..15 are zero: even and odd outputs are two
// 8-point DFTs of v and of v[r] W16^r.
template <typename T, bool INV>
__device__ __forceinline__ void dft16_halfin(cplx<T>* v) {
  using V = cplx<T>;
  const T c1 = (T)0.92387953251128675612818318939678829, s1 = (T)0.38268343236508977172845998403039887;
  const T c2 = (T)0.70710678118654752440084436210484903;
  auto tw = [&](V a, T c, T sn) -> V {   // a * (c - i sn) forward, a * (c + i sn) inverse
    V r;
    if (!INV) { r.x = a.x * c + a.y * sn; r.y = a.y * c - a.x * sn; }
    else { r.x = a.x * c - a.y * sn; r.y = a.y * c + a.x * sn; }
    return r;
  };
  V a[8], o[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) a[r] = v[r];
  o[0] = v[0];
  o[1] = tw(v[1], c1, s1);
  o[2] = tw(v[2], c2, c2);
  o[3] = tw(v[3], s1, c1);
  o[4] = rot_mi<V, INV>(v[4]);
  o[5] = tw(v[5], -s1, c1);
  o[6] = tw(v[6], -c2, c2);
  o[7] = tw(v[7], -c1, s1);
  dft8<T, INV>(a);
  dft8<T, INV>(o);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v[2 * k] = a[k];
    v[2 * k + 1] = o[k];
  }
}

// outputs 0..7 of a 16-point DFT: X[k] = E[k] + W16^k O[k] with E, O the
// 8-point DFTs of the even and odd inputs; result in v[0..7].
template <typename T, bool INV>
__device__ __forceinline__ void dft16_halfout(cplx<T>* v) {
  using V = cplx<T>;
  const T c1 = (T)0.92387953251128675612818318939678829, s1 = (T)0.38268343236508977172845998403039887;
  const T c2 = (T)0.70710678118654752440084436210484903;
  auto tw = [&](V a, T c, T sn) -> V {
    V r;
    if (!INV) { r.x = a.x * c + a.y * sn; r.y = a.y * c - a.x * sn; }
    else { r.x = a.x * c - a.y * sn; r.y = a.y * c + a.x * sn; }
    return r;
  };
  V e[8], o[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    e[r] = v[2 * r];
    o[r] = v[2 * r + 1];
  }
  dft8<T, INV>(e);
  dft8<T, INV>(o);
  v[0] = cadd(e[0], o[0]);
  v[1] = cadd(e[1], tw(o[1], c1, s1));
  v[2] = cadd(e[2], tw(o[2], c2, c2));
  v[3] = cadd(e[3], tw(o[3], s1, c1));
  v[4] = cadd(e[4], rot_mi<V, INV>(o[4]));
  v[5] = cadd(e[5], tw(o[5], -s1, c1));
  v[6] = cadd(e[6], tw(o[6], -c2, c2));
  v[7] = cadd(e[7], tw(o[7], -c1, s1));
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_r(cplx<T>* v) {
  if constexpr (R == 16) dft16<T, INV>(v);
  else if constexpr (R == 8) dft8<T, INV>(v);
  else if constexpr (R == 4) dft4<cplx<T>, INV>(v[0], v[1], v[2], v[3]);
  else dft2<cplx<T>, INV>(v[0], v[1]);
}

// LDS index with one pad slot per 16 elements: the radix-16 first pass
// stores with a stride of 16 elements, which the pad turns into 17 so the
// lanes of a wave spread over all banks.
__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int padded(int n) { return n + (n >> 4); }
// The column pass pads one slot per 256 bytes in both precisions: per 16
// FP64 or per 32 FP32 complex values.  In its fused pass consecutive lanes
// step 8 CW values apart (256 B), so the pad shifts each lane by one value
// (4 banks in FP64, 2 in FP32) and a cycle's lanes (16 of 16 B, 32 of 8 B)
// cover distinct banks.  The buffer is sized with padded(), which covers both.
template <typename T>
__device__ __forceinline__ int cidx(int i) { return i + (i >> (sizeof(T) == 4 ? 5 : 4)); }

// w^r for r = 1..R-1 from w = w^1 by a product tree of depth <= 4
template <typename V, int R>
__device__ __forceinline__ void tw_powers(V w1, V* wp) {
  wp[1] = w1;
  if constexpr (R > 2) {
    wp[2] = cmul(w1, w1);
    wp[3] = cmul(wp[2], w1);
  }
  if constexpr (R > 4) {
    wp[4] = cmul(wp[2], wp[2]);
    wp[5] = cmul(wp[4], w1);
    wp[6] = cmul(wp[4], wp[2]);
    wp[7] = cmul(wp[4], wp[3]);
  }
  if constexpr (R > 8) {
    wp[8] = cmul(wp[4], wp[4]);
#pragma unroll
    for (int r = 9; r < 16; ++r) wp[r] = cmul(wp[8], wp[r - 8]);
  }
}

// Twiddles of butterfly j of a Stockham pass (sub-transform length NS):
// input r is multiplied by w^(k r), w = e^{-2 pi i/(NS R)}, k = j mod NS.
template <typename T, int N, bool INV, int NS, int R>
__device__ __forceinline__ void pass_twiddle(cplx<T>* v, int j, const cplx<T>* __restrict__ tw) {
  using V = cplx<T>;
  if constexpr (NS > 1) {
    const int k = j & (NS - 1);
    V w1 = tw[k * (N / (NS * R))];
    if (INV) w1.y = -w1.y;
    V wp[R];
    tw_powers<V, R>(w1, wp);
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], wp[r]);
  }
}

// Base twiddle w^1 of butterfly j of a pass with sub-length NS (forward
// sign), loaded once so a later pass can reuse it without a dependent load.
template <typename T, int N, int NS, int R>
__device__ __forceinline__ cplx<T> tw_base(int j, const cplx<T>* __restrict__ tw) {
  if constexpr (NS > 1) return tw[(j & (NS - 1)) * (N / (NS * R))];
  else return mk<T>(1, 0);
}

// pass_twiddle with the base twiddle already in a register
template <typename T, bool INV, int NS, int R>
__device__ __forceinline__ void apply_twiddle(cplx<T>* v, cplx<T> w1) {
  using V = cplx<T>;
  if constexpr (NS > 1) {
    if (INV) w1.y = -w1.y;
    V wp[R];
    tw_powers<V, R>(w1, wp);
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], wp[r]);
  }
}

// One Stockham pass: sub-transform length NS -> NS*R.  Element i of column c
// lives at buf[pidx(i * NCOL + c)]; butterfly b = j * NCOL + c reads elements
// j + r N/R and writes (j - k) R + k + r NS, k = j mod NS.
template <typename T, int N, int NCOL, int NT, bool INV, int NS, int R>
__device__ __forceinline__ void stockham_pass(cplx<T>* buf, const cplx<T>* __restrict__ tw) {
  using V = cplx<T>;
  constexpr int NB = (N / R) * NCOL;
  constexpr int PER = (NB + NT - 1) / NT;
  V v[PER][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + q * NT;
    if ((NB % NT) == 0 || b < NB) {
      const int c = b % NCOL, j = b / NCOL;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[pidx((j + r * (N / R)) * NCOL + c)];
      pass_twiddle<T, N, INV, NS, R>(v[q], j, tw);
      dft_r<T, R, INV>(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + q * NT;
    if ((NB % NT) == 0 || b < NB) {
      const int c = b % NCOL, j = b / NCOL;
      const int k = j & (NS - 1);
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pidx((base + r * NS) * NCOL + c)] = v[q][r];
    }
  }
  __syncthreads();
}

// Stockham pass with the base twiddle of each butterfly given (w[q] for
// butterfly tid + q NT, forward sign); single column
template <typename T, int N, int NT, bool INV, int NS, int R>
__device__ __forceinline__ void stockham_pass_w(cplx<T>* buf, const cplx<T>* w) {
  using V = cplx<T>;
  constexpr int NB = N / R;
  constexpr int PER = (NB + NT - 1) / NT;
  V v[PER][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = tid + q * NT;
    if ((NB % NT) == 0 || j < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[pidx(j + r * (N / R))];
      apply_twiddle<T, INV, NS, R>(v[q], w[q]);
      dft_r<T, R, INV>(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = tid + q * NT;
    if ((NB % NT) == 0 || j < NB) {
      const int k = j & (NS - 1);
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pidx(base + r * NS)] = v[q][r];
    }
  }
  __syncthreads();
}

// A chain of single-column Stockham passes from sub-length NS up to NSEND,
// radix 16 (R16) or radix min(16, N/NS); the base twiddles of every pass are
// loaded up front (chain_tw) so no pass waits on a dependent load.
template <int N, int NS, bool R16> constexpr int chain_radix() { return R16 ? 16 : (N / NS >= 16 ? 16 : N / NS); }
template <int N, int NT, int NS, int NSEND, bool R16> constexpr int chain_len() {
  if constexpr (NS >= NSEND) return 0;
  else {
    constexpr int R = chain_radix<N, NS, R16>();
    return (N / R + NT - 1) / NT + chain_len<N, NT, NS * R, NSEND, R16>();
  }
}
template <typename T, int N, int NT, int NS, int NSEND, bool R16>
__device__ __forceinline__ void chain_tw(const cplx<T>* __restrict__ tw, cplx<T>* w) {
  if constexpr (NS < NSEND) {
    constexpr int R = chain_radix<N, NS, R16>();
    constexpr int NB = N / R, PER = (NB + NT - 1) / NT;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = threadIdx.x + q * NT;
      w[q] = ((NB % NT) == 0 || j < NB) ? tw_base<T, N, NS, R>(j, tw) : mk<T>(1, 0);
    }
    chain_tw<T, N, NT, NS * R, NSEND, R16>(tw, w + PER);
  }
}
template <typename T, int N, int NT, bool INV, int NS, int NSEND, bool R16>
__device__ __forceinline__ void chain_passes(cplx<T>* buf, const cplx<T>* w) {
  if constexpr (NS < NSEND) {
    constexpr int R = chain_radix<N, NS, R16>();
    stockham_pass_w<T, N, NT, INV, NS, R>(buf, w);
    chain_passes<T, N, NT, INV, NS * R, NSEND, R16>(buf, w + (N / R + NT - 1) / NT);
  }
}

// radix-16 passes, then 8, 4 or 2 for the remainder
template <typename T, int N, int NCOL, int NT, bool INV, int NS>
__device__ __forceinline__ void fft_passes(cplx<T>* buf, const cplx<T>* __restrict__ tw) {
  if constexpr (NS < N) {
    constexpr int R = (N / NS >= 16) ? 16 : (N / NS);
    stockham_pass<T, N, NCOL, NT, INV, NS, R>(buf, tw);
    fft_passes<T, N, NCOL, NT, INV, NS * R>(buf, tw);
  }
}

// radix-16 passes with sub-transform lengths NS, 16 NS, ... below NSEND
template <typename T, int N, int NCOL, int NT, bool INV, int NS, int NSEND>
__device__ __forceinline__ void passes16(cplx<T>* buf, const cplx<T>* __restrict__ tw) {
  if constexpr (NS < NSEND) {
    stockham_pass<T, N, NCOL, NT, INV, NS, 16>(buf, tw);
    passes16<T, N, NCOL, NT, INV, NS * 16, NSEND>(buf, tw);
  }
}

// One in-place Cooley-Tukey pass with stride S and radix R: butterfly
// (block, m) owns positions blk S R + m + S r.  Forward (decimation in
// frequency): R-point DFT, then output k times W_{SR}^{m k}.  Inverse
// (decimation in time, the exact reverse): input k times W_{SR}^{-m k}, then
// the inverse R-point DFT.  Each thread writes back the positions it read, so
// one barrier per pass suffices.
template <typename T, int N, int NCOL, int NT, bool INV, int S, int R>
__device__ __forceinline__ void ct_pass(cplx<T>* buf, const cplx<T>* __restrict__ tw) {
  using V = cplx<T>;
  constexpr int NB = (N / R) * NCOL;
  constexpr int PER = (NB + NT - 1) / NT;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = threadIdx.x + q * NT;
    if ((NB % NT) == 0 || b < NB) {
      const int c = b % NCOL, t = b / NCOL;
      const int m = t % S, base = (t / S) * S * R + m;
      V v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = buf[pidx((base + S * r) * NCOL + c)];
      if (!INV) {
        dft_r<T, R, false>(v);
        pass_twiddle<T, N, false, S, R>(v, m, tw);
      } else {
        pass_twiddle<T, N, true, S, R>(v, m, tw);
        dft_r<T, R, true>(v);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pidx((base + S * r) * NCOL + c)] = v[r];
    }
  }
  __syncthreads();
}

// ct_pass with the base twiddle of each of the thread's butterflies given
// (w[q] for butterfly tid + q NT, forward sign)
template <typename T, int N, int NCOL, int NT, bool INV, int S, int R>
__device__ __forceinline__ void ct_pass_w(cplx<T>* buf, const cplx<T>* w) {
  using V = cplx<T>;
  constexpr int NB = (N / R) * NCOL;
  constexpr int PER = (NB + NT - 1) / NT;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = threadIdx.x + q * NT;
    if ((NB % NT) == 0 || b < NB) {
      const int c = b % NCOL, t = b / NCOL;
      const int m = t % S, base = (t / S) * S * R + m;
      V v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = buf[cidx<T>((base + S * r) * NCOL + c)];
      if (!INV) {
        dft_r<T, R, false>(v);
        apply_twiddle<T, false, S, R>(v, w[q]);
      } else {
        apply_twiddle<T, true, S, R>(v, w[q]);
        dft_r<T, R, true>(v);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) buf[cidx<T>((base + S * r) * NCOL + c)] = v[r];
    }
  }
  __syncthreads();
}

// radix-16 forward passes with strides S, S/16, ... down to SEND (inclusive)
template <typename T, int N, int NCOL, int NT, int S, int SEND>
__device__ __forceinline__ void dif16_down(cplx<T>* buf, const cplx<T>* __restrict__ tw) {
  if constexpr (S >= SEND && S >= 1) {
    ct_pass<T, N, NCOL, NT, false, S, 16>(buf, tw);
    dif16_down<T, N, NCOL, NT, S / 16, SEND>(buf, tw);
  }
}

// radix-16 inverse passes with strides S, 16 S, ... up to SEND (inclusive)
template <typename T, int N, int NCOL, int NT, int S, int SEND>
__device__ __forceinline__ void dit16_up(cplx<T>* buf, const cplx<T>* __restrict__ tw) {
  if constexpr (S <= SEND && S >= 1) {
    ct_pass<T, N, NCOL, NT, true, S, 16>(buf, tw);
    dit16_up<T, N, NCOL, NT, S * 16, SEND>(buf, tw);
  }
}

// radix of the remainder pass: N = 16^p * last_radix(N), last_radix in 2..16
template <int N> constexpr int last_radix() {
  if constexpr (N <= 16) return N;
  else return last_radix<N / 16>();
}

// ---------------------------------------------------------------------------
// tiles: CB columns per tile; columns kx and N - kx share a tile (and,
// with two or more columns per column-pass block, a block; with one, the two
// blocks run on one XCD) so the even-symmetric quarter spectrum is fetched
// once.  Tile b, slot c holds pair q = b*(CB/2) + c/2 + 1 (c odd: the mirror
// N - q); the last slot pair of the last tile holds the self-mirrored
// columns 0 and N/2.
// ---------------------------------------------------------------------------
// CB is the tile width (columns per tile, the row passes' piece); CW the
// columns one column-pass block transforms: as many as fit the LDS budget
// of two blocks per CU.  Tiles are at least 64 bytes wide, so the row
// passes read and write whole 64-byte pieces; where CW is narrower (N >=
// 2048 in either precision) the CB / CW blocks of a tile take CW columns
// each.
template <typename T, int N> struct ColCfg {
  static constexpr int BYTES = 80000;   // padded LDS per column block: two blocks per CU
  static constexpr int CB0 = BYTES / (padded(N) * (int)sizeof(cplx<T>));
  static constexpr int CW1 = CB0 < 2 ? 1 : (CB0 > 16 ? 16 : CB0);
  static constexpr int CW = (CW1 >= 16) ? 16 : (CW1 >= 8 ? 8 : (CW1 >= 4 ? 4 : (CW1 >= 2 ? 2 : 1)));
  // tiles at least 64 bytes wide, so the row passes move whole 64-byte pieces
  static constexpr int CB64 = 64 / (int)sizeof(cplx<T>);
  static constexpr int CB = CW > CB64 ? CW : CB64;
  static constexpr int NT = (N * CW / 16 >= 512) ? 512 : 256;
};

// Column-pass block b -> tile tb and first column c0 within the tile.  The
// K = CB / CW blocks of a tile are 8 apart, which the launch deals to the
// same XCD, so the parts of each tile line meet in one L2.
template <typename T, int N>
__device__ __forceinline__ void col_block_of(int b, int& tb, int& c0) {
  constexpr int CB = ColCfg<T, N>::CB, CW = ColCfg<T, N>::CW, K = CB / CW;   // blocks per tile
  if constexpr (K == 1) {
    tb = b;
    c0 = 0;
  } else {
    static_assert(K * CW == CB && (K & (K - 1)) == 0 && (N / CB) % 8 == 0, "tile split into 2^k blocks");
    tb = (b / (8 * K)) * 8 + (b & 7);
    c0 = ((b >> 3) & (K - 1)) * CW;
  }
}

__device__ __forceinline__ void col_of(int b, int c, int N, int CB, int& kx, int& kxq) {
  const int q = b * (CB / 2) + (c >> 1) + 1;
  const int half = c & 1;
  if (q >= N / 2) {            // last pair slot of the last tile
    kx = half ? N / 2 : 0;
    kxq = kx;
  } else {
    kx = half ? N - q : q;
    kxq = q;
  }
}

// XCD-aware row order: consecutive rows go to the same XCD (blocks are
// dealt round-robin over 8 XCDs), so the pieces of a tile line written by
// neighbouring rows meet in one L2.
__device__ __forceinline__ int xcd_row(int bid, int nrows) {
  const int per = (nrows + 7) / 8;
  return (bid & 7) * per + (bid >> 3);
}

// ---------------------------------------------------------------------------
// kernels.  T layout (tiled): [pair][tile][row][CB] with ldt >= nr rows
// per tile (tile_rows); rows nr .. ldt-1 are never read or written
// ---------------------------------------------------------------------------
template <int N> constexpr int row_threads() { return N / 16 < 64 ? 64 : (N / 16 > 256 ? 256 : N / 16); }

// Pass 1: gather active values of a row into a zeroed LDS row, FFT along x.
// Active points have x < N/2, so only that half is cleared and the first pass
// reads inputs 0..7 of its radix-16 butterflies.
template <typename T, int N>
__global__ __launch_bounds__(row_threads<N>()) void k_rows_fwd(
    const cplx<T>* __restrict__ U, int n_act, const int32_t* __restrict__ row_ptr,
    const int32_t* __restrict__ act_ix, int nr, int ldt, cplx<T>* __restrict__ Tb,
    const cplx<T>* __restrict__ tw) {
  using V = cplx<T>;
  static_assert(N >= 32, "row pass assumes at least two forward passes");
  constexpr int NT = row_threads<N>();
  constexpr int CB = ColCfg<T, N>::CB;
  constexpr int NBLK = N / CB;
  __shared__ V buf[padded(N)];
  const int row = xcd_row(blockIdx.x, nr), pair = blockIdx.y;
  const int tid = threadIdx.x;
  if (row >= nr) return;
  constexpr int NW = chain_len<N, NT, 16, N, false>();
  V wt[NW > 0 ? NW : 1];
  chain_tw<T, N, NT, 16, N, false>(tw, wt);
  for (int i = tid; i < N / 2; i += NT) buf[pidx(i)] = mk<T>(0, 0);
  __syncthreads();
  const int a0 = row_ptr[row], a1 = row_ptr[row + 1];
  const V* Up = U + (size_t)pair * n_act;
  for (int a = a0 + tid; a < a1; a += NT) buf[pidx(act_ix[a])] = Up[a];
  __syncthreads();
  {
    constexpr int NB = N / 16, PER = (NB + NT - 1) / NT;
    V v[PER][16];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + q * NT;
      if ((NB % NT) == 0 || j < NB) {
#pragma unroll
        for (int r = 0; r < 8; ++r) v[q][r] = buf[pidx(j + r * (N / 16))];
        dft16_halfin<T, false>(v[q]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + q * NT;
      if ((NB % NT) == 0 || j < NB) {
#pragma unroll
        for (int r = 0; r < 16; ++r) buf[pidx(j * 16 + r)] = v[q][r];
      }
    }
    __syncthreads();
  }
  chain_passes<T, N, NT, false, 16, N, false>(buf, wt);
  // groups of CB lanes fill the CB-wide segments of the tiled layout; the LDS
  // reads of a thread are all issued before its stores
  V* out = Tb + (size_t)pair * NBLK * ldt * CB + (size_t)row * CB;
  constexpr int PER = (N + NT - 1) / NT;
  V v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + q * NT;
    if ((N % NT) == 0 || idx < N) {
      int kx, kxq;
      col_of(idx / CB, idx % CB, N, CB, kx, kxq);
      v[q] = buf[pidx(kx)];
    }
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + q * NT;
    if ((N % NT) == 0 || idx < N) out[(size_t)(idx / CB) * ldt * CB + idx % CB] = v[q];
  }
}

// Pass 3: inverse FFT along x, gather the active points of the row.  The
// inverse runs its radices in reverse order so that the last pass is radix 16
// and computes only the outputs x < N/2, where the active points lie.
template <typename T, int N>
__global__ __launch_bounds__(row_threads<N>()) void k_rows_inv(
    const cplx<T>* __restrict__ Tb, int nr, int ldt, const int32_t* __restrict__ row_ptr,
    const int32_t* __restrict__ act_ix, cplx<T>* __restrict__ Vout, int n_act,
    const cplx<T>* __restrict__ tw) {
  using V = cplx<T>;
  static_assert(N >= 32, "row pass assumes at least two inverse passes");
  constexpr int NT = row_threads<N>();
  constexpr int CB = ColCfg<T, N>::CB;
  constexpr int NBLK = N / CB;
  constexpr int RL = last_radix<N>();
  __shared__ V buf[padded(N)];
  const int row = xcd_row(blockIdx.x, nr), pair = blockIdx.y;
  const int tid = threadIdx.x;
  if (row >= nr) return;
  const V* in = Tb + (size_t)pair * NBLK * ldt * CB + (size_t)row * CB;
  // base twiddles of the radix-16 passes and of the last pass, loaded with
  // the row
  constexpr int NW = chain_len<N, NT, RL, N / 16, true>();
  constexpr int NS_L = N / 16, PER_L = (NS_L + NT - 1) / NT;
  V wt[NW > 0 ? NW : 1], wl[PER_L];
  chain_tw<T, N, NT, RL, N / 16, true>(tw, wt);
#pragma unroll
  for (int q = 0; q < PER_L; ++q) {
    const int j = tid + q * NT;
    wl[q] = ((NS_L % NT) == 0 || j < NS_L) ? tw_base<T, N, NS_L, 16>(j, tw) : mk<T>(1, 0);
  }
  {
    // all HBM loads of a thread in flight before its LDS stores
    constexpr int PER = (N + NT - 1) / NT;
    V v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * NT;
      if ((N % NT) == 0 || idx < N) v[q] = in[(size_t)(idx / CB) * ldt * CB + idx % CB];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * NT;
      if ((N % NT) == 0 || idx < N) {
        int kx, kxq;
        col_of(idx / CB, idx % CB, N, CB, kx, kxq);
        buf[pidx(kx)] = v[q];
      }
    }
  }
  __syncthreads();
  stockham_pass<T, N, 1, NT, true, 1, RL>(buf, tw);
  chain_passes<T, N, NT, true, RL, N / 16, true>(buf, wt);
  {
    constexpr int NS = NS_L, NB = NS, PER = PER_L;
    V v[PER][16];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + q * NT;
      if ((NB % NT) == 0 || j < NB) {
#pragma unroll
        for (int r = 0; r < 16; ++r) v[q][r] = buf[pidx(j + r * NS)];
        apply_twiddle<T, true, NS, 16>(v[q], wl[q]);
        dft16_halfout<T, true>(v[q]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + q * NT;
      if ((NB % NT) == 0 || j < NB) {
#pragma unroll
        for (int r = 0; r < 8; ++r) buf[pidx(j + r * NS)] = v[q][r];
      }
    }
    __syncthreads();
  }
  const int a0 = row_ptr[row], a1 = row_ptr[row + 1];
  V* Vp = Vout + (size_t)pair * n_act;
  for (int a = a0 + tid; a < a1; a += NT) Vp[a] = buf[pidx(act_ix[a])];
}

// Set-up: in-place forward FFT of full rows of length N (row-major array).
template <typename T, int N>
__global__ __launch_bounds__(row_threads<N>()) void k_rows_fft_inplace(cplx<T>* __restrict__ A,
                                                                       const cplx<T>* __restrict__ tw) {
  constexpr int NT = row_threads<N>();
  __shared__ cplx<T> buf[padded(N)];
  cplx<T>* rowp = A + (size_t)blockIdx.x * N;
  for (int i = threadIdx.x; i < N; i += NT) buf[pidx(i)] = rowp[i];
  __syncthreads();
  fft_passes<T, N, 1, NT, false, 1>(buf, tw);
  for (int i = threadIdx.x; i < N; i += NT) rowp[i] = buf[pidx(i)];
}

// Pass 2 (MODE 0): column FFT, spectrum multiply, inverse column FFT, in
// place on CW columns of one tile [row][CB] of T (nr <= N/2 rows kept, the rest is the
// zero padding).  The column FFT is an in-place decimation in frequency, so
// position p holds frequency ky_of_pos(N, p); the spectrum Cq is stored in
// that order, folded over ky -> N - ky ([kxq][spec_row_len(N)]), and the
// inverse is the matching decimation in time.
// MODE 1 (set-up): plain forward FFT of CW consecutive columns of a
// row-major N x N array.
// The column pass of CW columns of one tile [row][CB] (nr kept rows, the rest of the
// column is the zero padding), in place: column FFT, spectrum multiply,
// inverse column FFT (the MODE 0 body of k_cols and of k_cols_group).
template <typename T, int N>
__device__ __forceinline__ void cols_conv_tile(cplx<T>* buf, cplx<T>* __restrict__ tile, int nr, int b, int c0_,
                                               const cplx<T>* __restrict__ Cq, const cplx<T>* __restrict__ tw) {
  using V = cplx<T>;
  constexpr int CB = ColCfg<T, N>::CB;   // tile width (global layout)
  constexpr int CW = ColCfg<T, N>::CW;   // columns of this block, c0 .. c0 + CW - 1 (LDS layout)
  const int c0 = CW == CB ? 0 : c0_;
  constexpr int NT = ColCfg<T, N>::NT;
  const int tid = threadIdx.x;
  static_assert(N >= 32, "column pass assumes at least two forward passes");
  constexpr int RL = last_radix<N>();
  constexpr int S1 = N / 16;
  constexpr int SM = N / 256;                   // middle radix-16 pass stride
  constexpr bool MID = SM >= RL && SM >= 1;
  static_assert(!MID || SM / 16 < RL, "at most one middle pass per direction");
  constexpr int NB1 = S1 * CW, PER1 = (NB1 + NT - 1) / NT;
  constexpr int NBM = (N / 16) * CW, PERM = (NBM + NT - 1) / NT;
  constexpr int NG = N / RL, NBF = NG * CW, PERF = (NBF + NT - 1) / NT;
  // forward pass 1 (stride N/16, radix 16) from HBM: inputs m + S1 r with
  // r >= 8 lie in the zero half
  V v[PER1][16];
#pragma unroll
  for (int q = 0; q < PER1; ++q) {
    const int bb = tid + q * NT;
    if ((NB1 % NT) == 0 || bb < NB1) {
      const int c = bb % CW, m = bb / CW;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int i = m + r * S1;
        v[q][r] = i < nr ? tile[(size_t)i * CB + c0 + c] : mk<T>(0, 0);
      }
    }
  }
  // everything else this block reads from HBM does not depend on the data:
  // the spectrum values of the fused pass and the twiddles of the other
  // passes are issued now and consumed passes later, so their latency
  // overlaps the first passes instead of stalling each one (the spectrum
  // only in FP64 up to N = 2048: elsewhere the extra registers would cost
  // a wave per SIMD or spill).
  // The spectrum row is folded (ky and N - ky share a slot): group g holds
  // ky = low + W r with low the base-16 digit reversal of g; a group with
  // low > W/2 reads its mirror group W - low and reverses r (in registers,
  // at the multiply, so a prefetch never waits).
  constexpr int W = N / RL, HS = (W / 2 + 1) * RL;
  auto mirrored = [&](int g, int& lowc) {
    int low = 0;
#pragma unroll
    for (int t = 1, gg = g; t < W; t *= 16, gg >>= 4) low = low * 16 + (gg & 15);
    lowc = low > W / 2 ? W - low : low;
    return low > W / 2;
  };
  auto load_spec_part = [&](int bb, V* cv, int r0, int r1) {
    const int g = bb % NG, c = bb / NG;
    int kx, kxq, lowc;
    col_of(b, c0 + c, N, CB, kx, kxq);
    mirrored(g, lowc);
    const V* Cp = Cq + (size_t)kxq * HS + lowc * RL;
#pragma unroll
    for (int r = 0; r < RL; ++r)
      if (r >= r0 && r < r1) cv[r] = Cp[r];
  };
  auto load_spec = [&](int bb, V* cv) { load_spec_part(bb, cv, 0, RL); };
  constexpr bool PRE = sizeof(T) == 8 && N <= 2048 && PERF * RL <= 16;
  // FP64 above N = 2048 (one block per CU): half of the spectrum loads go
  // out once the first pass has left its values in LDS, so their latency
  // overlaps the middle pass in registers the first pass has freed, and the
  // other half right after the middle pass (all of them at once would spill)
  constexpr bool LATE = sizeof(T) == 8 && !PRE && MID && PERF * RL <= 16;
  V cv[PERF][RL];
  if constexpr (PRE) {
#pragma unroll
    for (int q = 0; q < PERF; ++q) {
      const int bb = tid + q * NT;
      if ((NBF % NT) == 0 || bb < NBF) load_spec(bb, cv[q]);
    }
  }
  V w1[PER1], wm[PERM];
#pragma unroll
  for (int q = 0; q < PER1; ++q) {
    const int bb = tid + q * NT;
    w1[q] = ((NB1 % NT) == 0 || bb < NB1) ? tw_base<T, N, S1, 16>(bb / CW, tw) : mk<T>(1, 0);
  }
  if constexpr (MID) {
#pragma unroll
    for (int q = 0; q < PERM; ++q) {
      const int bb = tid + q * NT;
      wm[q] = ((NBM % NT) == 0 || bb < NBM) ? tw_base<T, N, SM, 16>((bb / CW) % SM, tw) : mk<T>(1, 0);
    }
  }
#pragma unroll
  for (int q = 0; q < PER1; ++q) {
    const int bb = tid + q * NT;
    if ((NB1 % NT) == 0 || bb < NB1) {
      const int c = bb % CW, m = bb / CW;
      dft16_halfin<T, false>(v[q]);
      apply_twiddle<T, false, S1, 16>(v[q], w1[q]);
#pragma unroll
      for (int r = 0; r < 16; ++r) buf[cidx<T>((m + r * S1) * CW + c)] = v[q][r];
    }
  }
  if constexpr (LATE) {
#pragma unroll
    for (int q = 0; q < PERF; ++q) {
      const int bb = tid + q * NT;
      if ((NBF % NT) == 0 || bb < NBF) load_spec_part(bb, cv[q], 0, RL / 2);
    }
  }
  __syncthreads();
  if constexpr (MID) ct_pass_w<T, N, CW, NT, false, SM, 16>(buf, wm);
  if constexpr (LATE) {
#pragma unroll
    for (int q = 0; q < PERF; ++q) {
      const int bb = tid + q * NT;
      if ((NBF % NT) == 0 || bb < NBF) load_spec_part(bb, cv[q], RL / 2, RL);
    }
  }
  // last forward pass (contiguous groups of RL), spectrum multiply in the
  // stored frequency order, first inverse pass; lanes run along the groups
#pragma unroll
  for (int q = 0; q < PERF; ++q) {
    const int bb = tid + q * NT;
    if ((NBF % NT) == 0 || bb < NBF) {
      const int g = bb % NG, c = bb / NG;
      if constexpr (!PRE && !LATE) load_spec(bb, cv[q]);
      V u[RL];
#pragma unroll
      for (int r = 0; r < RL; ++r) u[r] = buf[cidx<T>((g * RL + r) * CW + c)];
      int lowc;
      const bool mir = mirrored(g, lowc);
      dft_r<T, RL, false>(u);
#pragma unroll
      for (int r = 0; r < RL; ++r) u[r] = cmul(u[r], mir ? cv[q][RL - 1 - r] : cv[q][r]);
      dft_r<T, RL, true>(u);
#pragma unroll
      for (int r = 0; r < RL; ++r) buf[cidx<T>((g * RL + r) * CW + c)] = u[r];
    }
  }
  __syncthreads();
  if constexpr (MID) ct_pass_w<T, N, CW, NT, true, SM, 16>(buf, wm);
  // last inverse pass (stride N/16, radix 16) straight to HBM: outputs
  // m + S1 r, only r < 8 can be a kept row
#pragma unroll
  for (int q = 0; q < PER1; ++q) {
    const int bb = tid + q * NT;
    if ((NB1 % NT) == 0 || bb < NB1) {
      const int c = bb % CW, m = bb / CW;
      V u[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) u[r] = buf[cidx<T>((m + r * S1) * CW + c)];
      apply_twiddle<T, true, S1, 16>(u, w1[q]);
      dft16_halfout<T, true>(u);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int i = m + r * S1;
        if (i < nr) tile[(size_t)i * CB + c0 + c] = u[r];
      }
    }
  }
}

template <typename T, int N, int MODE>
__global__ __launch_bounds__((ColCfg<T, N>::NT)) void k_cols(
    cplx<T>* __restrict__ Tb, int nr, int ldt, const cplx<T>* __restrict__ Cq,
    const cplx<T>* __restrict__ tw) {
  using V = cplx<T>;
  constexpr int CB = ColCfg<T, N>::CB;
  constexpr int CW = ColCfg<T, N>::CW;
  constexpr int NT = ColCfg<T, N>::NT;
  constexpr int NBLK = N / CB;
  __shared__ V buf[padded(N * CW)];
  const int b = blockIdx.x;
  const int pair = blockIdx.y;
  const int tid = threadIdx.x;
  if constexpr (MODE == 0) {
    int tb, c0;
    col_block_of<T, N>(b, tb, c0);
    cols_conv_tile<T, N>(buf, Tb + ((size_t)pair * NBLK + tb) * ldt * CB, nr, tb, c0, Cq, tw);
  } else {
    const int kx0 = b * CW;
    for (int idx = tid; idx < N * CW; idx += NT) {
      const int i = idx / CW, c = idx % CW;
      buf[pidx(idx)] = Tb[(size_t)i * N + kx0 + c];
    }
    __syncthreads();
    fft_passes<T, N, CW, NT, false, 1>(buf, tw);
    for (int idx = tid; idx < N * CW; idx += NT) {
      const int i = idx / CW, c = idx % CW;
      Tb[(size_t)i * N + kx0 + c] = buf[pidx(idx)];
    }
  }
}

// Column passes of several contexts that share one spectrum (same n, k eps
// and precision), one launch: entry e of the batch is a pair's tile set
// (tile base of column block 0, kept rows, tile stride); blockIdx.y picks
// the entry.  Each tile is computed exactly as by k_cols.
struct ColBatch {
  static constexpr int kMax = kColBatchMax;
  void* tile[kMax];
  int nr[kMax];
  int ldt[kMax];
};

template <typename T, int N>
__global__ __launch_bounds__((ColCfg<T, N>::NT)) void k_cols_group(ColBatch batch, const cplx<T>* __restrict__ Cq,
                                                                 const cplx<T>* __restrict__ tw) {
  using V = cplx<T>;
  constexpr int CB = ColCfg<T, N>::CB;
  __shared__ V buf[padded(N * ColCfg<T, N>::CW)];
  const int e = blockIdx.y;
  int tb, c0;
  col_block_of<T, N>(blockIdx.x, tb, c0);
  V* tile = (V*)batch.tile[e] + (size_t)tb * batch.ldt[e] * CB;
  cols_conv_tile<T, N>(buf, tile, batch.nr[e], tb, c0, Cq, tw);
}

// ---------------------------------------------------------------------------
// launchers with run-time size dispatch
// ---------------------------------------------------------------------------
#define AIM_FOR_SIZES(X) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

template <typename T>
aim_status launch_rows_fwd(int n, const cplx<T>* U, int n_act, const int32_t* row_ptr,
                           const int32_t* act_ix, int nr, int ldt, int pairs, cplx<T>* Tb,
                           const cplx<T>* tw, hipStream_t s) {
  if (ldt < nr) return AIM_E_ARG;
  dim3 g(8 * ((nr + 7) / 8), pairs);
  switch (n) {
#define CASE(NN)                                                                               \
  case NN:                                                                                     \
    hipLaunchKernelGGL((k_rows_fwd<T, NN>), g, dim3(row_threads<NN>()), 0, s, U, n_act, row_ptr, \
                       act_ix, nr, ldt, Tb, tw);                                               \
    break;
    AIM_FOR_SIZES(CASE)
#undef CASE
    default: return AIM_E_ARG;
  }
  return hipGetLastError() == hipSuccess ? AIM_OK : AIM_E_HIP;
}

template <typename T>
aim_status launch_rows_inv(int n, const cplx<T>* Tb, int nr, int ldt, const int32_t* row_ptr,
                           const int32_t* act_ix, int pairs, cplx<T>* V, int n_act,
                           const cplx<T>* tw, hipStream_t s) {
  if (ldt < nr) return AIM_E_ARG;
  dim3 g(8 * ((nr + 7) / 8), pairs);
  switch (n) {
#define CASE(NN)                                                                               \
  case NN:                                                                                     \
    hipLaunchKernelGGL((k_rows_inv<T, NN>), g, dim3(row_threads<NN>()), 0, s, Tb, nr, ldt,      \
                       row_ptr, act_ix, V, n_act, tw);                                         \
    break;
    AIM_FOR_SIZES(CASE)
#undef CASE
    default: return AIM_E_ARG;
  }
  return hipGetLastError() == hipSuccess ? AIM_OK : AIM_E_HIP;
}

template <typename T>
aim_status launch_cols(int n, int mode, cplx<T>* Tb, int nr, int ldt, int pairs, const cplx<T>* Cq,
                       const cplx<T>* tw, hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop) {
  // kept rows lie in the unpadded half
  if (mode == 0 && (nr < 1 || nr > n / 2 || ldt < nr)) return AIM_E_ARG;
  switch (n) {
#define CASE(NN)                                                                          \
  case NN: {                                                                              \
    dim3 g(NN / ColCfg<T, NN>::CW, pairs);                                                \
    if (mode == 0)                                                                        \
      hipExtLaunchKernelGGL((k_cols<T, NN, 0>), g, dim3(ColCfg<T, NN>::NT), 0, s, ev_start, ev_stop, 0, \
                            Tb, nr, ldt, Cq, tw);                                         \
    else                                                                                  \
      hipLaunchKernelGGL((k_cols<T, NN, 1>), g, dim3(ColCfg<T, NN>::NT), 0, s, Tb, nr, ldt, Cq, tw); \
    break;                                                                                \
  }
    AIM_FOR_SIZES(CASE)
#undef CASE
    default: return AIM_E_ARG;
  }
  return hipGetLastError() == hipSuccess ? AIM_OK : AIM_E_HIP;
}

// columns per tile of the column pass (tile layout of the intermediate)
int col_block(int n, bool f32) {
  switch (n) {
#define CASE(NN) \
  case NN: return f32 ? ColCfg<float, NN>::CB : ColCfg<double, NN>::CB;
    AIM_FOR_SIZES(CASE)
#undef CASE
  }
  return 0;
}

// grouped column pass over `count` tile sets (count <= ColBatch::kMax)
template <typename T>
aim_status launch_cols_group(int n, int count, void* const* tiles, const int* nr, const int* ldt,
                             const cplx<T>* Cq, const cplx<T>* tw, hipStream_t s) {
  if (count < 1 || count > ColBatch::kMax) return AIM_E_ARG;
  ColBatch bt;
  for (int e = 0; e < ColBatch::kMax; ++e) {
    const int q = e < count ? e : 0;
    if (nr[q] < 1 || nr[q] > n / 2 || ldt[q] < nr[q]) return AIM_E_ARG;
    bt.tile[e] = tiles[q];
    bt.nr[e] = nr[q];
    bt.ldt[e] = ldt[q];
  }
  switch (n) {
#define CASE(NN)                                                                                              \
  case NN:                                                                                                    \
    hipLaunchKernelGGL((k_cols_group<T, NN>), dim3(NN / ColCfg<T, NN>::CW, count), dim3(ColCfg<T, NN>::NT), 0, \
                       s, bt, Cq, tw);                                                                        \
    break;
    AIM_FOR_SIZES(CASE)
#undef CASE
    default: return AIM_E_ARG;
  }
  return hipGetLastError() == hipSuccess ? AIM_OK : AIM_E_HIP;
}

aim_status launch_rows_fft_inplace(int n, double2* A, const double2* tw, hipStream_t s) {
  switch (n) {
#define CASE(NN)                                                                                   \
  case NN:                                                                                         \
    hipLaunchKernelGGL((k_rows_fft_inplace<double, NN>), dim3(NN), dim3(row_threads<NN>()), 0, s, A, tw); \
    break;
    AIM_FOR_SIZES(CASE)
#undef CASE
    default: return AIM_E_ARG;
  }
  return hipGetLastError() == hipSuccess ? AIM_OK : AIM_E_HIP;
}

template aim_status launch_rows_fwd<double>(int, const double2*, int, const int32_t*, const int32_t*, int, int, int,
                                            double2*, const double2*, hipStream_t);
template aim_status launch_rows_fwd<float>(int, const float2*, int, const int32_t*, const int32_t*, int, int, int,
                                           float2*, const float2*, hipStream_t);
template aim_status launch_rows_inv<double>(int, const double2*, int, int, const int32_t*, const int32_t*, int,
                                            double2*, int, const double2*, hipStream_t);
template aim_status launch_rows_inv<float>(int, const float2*, int, int, const int32_t*, const int32_t*, int,
                                           float2*, int, const float2*, hipStream_t);
template aim_status launch_cols<double>(int, int, double2*, int, int, int, const double2*, const double2*,
                                        hipStream_t, hipEvent_t, hipEvent_t);
template aim_status launch_cols<float>(int, int, float2*, int, int, int, const float2*, const float2*, hipStream_t,
                                       hipEvent_t, hipEvent_t);
template aim_status launch_cols_group<double>(int, int, void* const*, const int*, const int*, const double2*,
                                              const double2*, hipStream_t);
template aim_status launch_cols_group<float>(int, int, void* const*, const int*, const int*, const float2*,
                                             const float2*, hipStream_t);

}  // namespace aim
