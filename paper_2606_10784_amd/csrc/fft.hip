// Zero-padded 2D FFT convolution of eq. (8) / eq. (10) for gfx950.
//
// The grid product G_grid u is evaluated as
//     [F^-1( F(c) . F(b) )]_restr,   b = u zero-padded from m x m to n x n,
// with n = 2m and the spectrum F(c) of the circulant kernel resident in HBM as
// an even-symmetric quarter (Sec. III-A/B).  Three passes:
//   rows_fwd : scatter the active grid values of one grid row into LDS,
//              length-n FFT along x, write the row (only rows [y0, y0+nr)
//              that hold active points, compacted);
//   cols_conv: for a block of CB columns: length-n FFT along y (rows >= nr are
//              zero), multiply by the spectrum, inverse FFT, keep nr rows;
//   rows_inv : inverse FFT along x, gather the active points of the row.
// The circulant product commutes with cyclic shifts, so compacting the rows to
// [0, nr) changes nothing.  The 1/n^2 of the inverse DFT is folded into the
// stored spectrum.
//
// Each FFT is an in-LDS Stockham autosort with radix-8 passes (radix 4 or 2
// for the last one); each thread holds its butterflies in registers across a
// barrier, so a single LDS buffer suffices.
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

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_r(cplx<T>* v) {
  if constexpr (R == 8) dft8<T, INV>(v);
  else if constexpr (R == 4) dft4<cplx<T>, INV>(v[0], v[1], v[2], v[3]);
  else dft2<cplx<T>, INV>(v[0], v[1]);
}

// One Stockham pass: sub-transform length NS -> NS*R.  Element i of column c
// lives at buf[i * NCOL + c].
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
      for (int r = 0; r < R; ++r) v[q][r] = buf[(j + r * (N / R)) * NCOL + c];
      if constexpr (NS > 1) {
        const int k = j & (NS - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          V w = tw[k * r * (N / (NS * R))];
          if (INV) w.y = -w.y;
          v[q][r] = cmul(v[q][r], w);
        }
      }
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
      for (int r = 0; r < R; ++r) buf[(base + r * NS) * NCOL + c] = v[q][r];
    }
  }
  __syncthreads();
}

template <typename T, int N, int NCOL, int NT, bool INV, int NS>
__device__ __forceinline__ void fft_passes(cplx<T>* buf, const cplx<T>* __restrict__ tw) {
  if constexpr (NS < N) {
    constexpr int R = (N / NS >= 8) ? 8 : (N / NS);
    stockham_pass<T, N, NCOL, NT, INV, NS, R>(buf, tw);
    fft_passes<T, N, NCOL, NT, INV, NS * R>(buf, tw);
  }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
template <int N> constexpr int row_threads() { return N / 8 < 64 ? 64 : (N / 8 > 256 ? 256 : N / 8); }

// Pass 1: gather active values of a row into a zeroed LDS row, FFT along x.
// grid = (nr, pairs); U: [pair][n_act]; T: [pair][nr][N]
template <typename T, int N>
__global__ __launch_bounds__(row_threads<N>()) void k_rows_fwd(
    const cplx<T>* __restrict__ U, int n_act, const int32_t* __restrict__ row_ptr,
    const int32_t* __restrict__ act_ix, int nr, cplx<T>* __restrict__ Tb,
    const cplx<T>* __restrict__ tw) {
  constexpr int NT = row_threads<N>();
  __shared__ cplx<T> buf[N];
  const int row = blockIdx.x, pair = blockIdx.y;
  for (int i = threadIdx.x; i < N; i += NT) buf[i] = mk<T>(0, 0);
  __syncthreads();
  const int a0 = row_ptr[row], a1 = row_ptr[row + 1];
  const cplx<T>* Up = U + (size_t)pair * n_act;
  for (int a = a0 + threadIdx.x; a < a1; a += NT) buf[act_ix[a]] = Up[a];
  __syncthreads();
  fft_passes<T, N, 1, NT, false, 1>(buf, tw);
  cplx<T>* out = Tb + ((size_t)pair * nr + row) * N;
  for (int i = threadIdx.x; i < N; i += NT) out[i] = buf[i];
}

// Pass 3: inverse FFT along x, gather the active points of the row.
template <typename T, int N>
__global__ __launch_bounds__(row_threads<N>()) void k_rows_inv(
    const cplx<T>* __restrict__ Tb, int nr, const int32_t* __restrict__ row_ptr,
    const int32_t* __restrict__ act_ix, cplx<T>* __restrict__ Vout, int n_act,
    const cplx<T>* __restrict__ tw) {
  constexpr int NT = row_threads<N>();
  __shared__ cplx<T> buf[N];
  const int row = blockIdx.x, pair = blockIdx.y;
  const cplx<T>* in = Tb + ((size_t)pair * nr + row) * N;
  for (int i = threadIdx.x; i < N; i += NT) buf[i] = in[i];
  __syncthreads();
  fft_passes<T, N, 1, NT, true, 1>(buf, tw);
  const int a0 = row_ptr[row], a1 = row_ptr[row + 1];
  cplx<T>* Vp = Vout + (size_t)pair * n_act;
  for (int a = a0 + threadIdx.x; a < a1; a += NT) Vp[a] = buf[act_ix[a]];
}

// Set-up: in-place forward FFT of nrows full rows of length N.
template <typename T, int N>
__global__ __launch_bounds__(row_threads<N>()) void k_rows_fft_inplace(cplx<T>* __restrict__ A,
                                                                       const cplx<T>* __restrict__ tw) {
  constexpr int NT = row_threads<N>();
  __shared__ cplx<T> buf[N];
  cplx<T>* rowp = A + (size_t)blockIdx.x * N;
  for (int i = threadIdx.x; i < N; i += NT) buf[i] = rowp[i];
  __syncthreads();
  fft_passes<T, N, 1, NT, false, 1>(buf, tw);
  for (int i = threadIdx.x; i < N; i += NT) rowp[i] = buf[i];
}

template <typename T, int N> struct ColCfg {
  static constexpr int BYTES = 65536;
  static constexpr int CB0 = BYTES / (N * (int)sizeof(cplx<T>));
  static constexpr int CB = CB0 < 1 ? 1 : (CB0 > 16 ? 16 : CB0);
  static constexpr int NT = 256;
};

// Pass 2: column FFT, spectrum multiply, inverse column FFT (in place on T).
// grid = (N / CB, pairs). Cq: quarter spectrum [kxq][kyq], (N/2+1)^2.
// MODE 0: convolution over rows [0, nr); MODE 1: plain forward FFT of all N rows
template <typename T, int N, int MODE>
__global__ __launch_bounds__((ColCfg<T, N>::NT)) void k_cols(
    cplx<T>* __restrict__ Tb, int nr, const cplx<T>* __restrict__ Cq,
    const cplx<T>* __restrict__ tw) {
  constexpr int CB = ColCfg<T, N>::CB;
  constexpr int NT = ColCfg<T, N>::NT;
  constexpr int H = N / 2 + 1;
  __shared__ cplx<T> buf[N * CB];
  const int kx0 = blockIdx.x * CB;
  const int pair = blockIdx.y;
  cplx<T>* base = Tb + (size_t)pair * nr * N;
  const int rows_in = (MODE == 0) ? nr : N;
  for (int idx = threadIdx.x; idx < N * CB; idx += NT) {
    const int i = idx / CB, c = idx % CB;
    buf[idx] = (i < rows_in) ? base[(size_t)i * N + kx0 + c] : mk<T>(0, 0);
  }
  __syncthreads();
  fft_passes<T, N, CB, NT, false, 1>(buf, tw);
  if constexpr (MODE == 0) {
    for (int idx = threadIdx.x; idx < N * CB; idx += NT) {
      const int ky = idx / CB, c = idx % CB;
      const int kx = kx0 + c;
      const int kxq = kx <= N / 2 ? kx : N - kx;
      const int kyq = ky <= N / 2 ? ky : N - ky;
      buf[idx] = cmul(buf[idx], Cq[(size_t)kxq * H + kyq]);
    }
    __syncthreads();
    fft_passes<T, N, CB, NT, true, 1>(buf, tw);
  }
  const int rows_out = (MODE == 0) ? nr : N;
  for (int idx = threadIdx.x; idx < rows_out * CB; idx += NT) {
    const int i = idx / CB, c = idx % CB;
    base[(size_t)i * N + kx0 + c] = buf[idx];
  }
}

// ---------------------------------------------------------------------------
// launchers with run-time size dispatch
// ---------------------------------------------------------------------------
#define AIM_FOR_SIZES(X) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192)

template <typename T>
aim_status launch_rows_fwd(int n, const cplx<T>* U, int n_act, const int32_t* row_ptr,
                           const int32_t* act_ix, int nr, int pairs, cplx<T>* Tb,
                           const cplx<T>* tw, hipStream_t s) {
  dim3 g(nr, pairs);
  switch (n) {
#define CASE(NN)                                                                               \
  case NN:                                                                                     \
    hipLaunchKernelGGL((k_rows_fwd<T, NN>), g, dim3(row_threads<NN>()), 0, s, U, n_act, row_ptr, \
                       act_ix, nr, Tb, tw);                                                    \
    break;
    AIM_FOR_SIZES(CASE)
#undef CASE
    default: return AIM_E_ARG;
  }
  return hipGetLastError() == hipSuccess ? AIM_OK : AIM_E_HIP;
}

template <typename T>
aim_status launch_rows_inv(int n, const cplx<T>* Tb, int nr, const int32_t* row_ptr,
                           const int32_t* act_ix, int pairs, cplx<T>* V, int n_act,
                           const cplx<T>* tw, hipStream_t s) {
  dim3 g(nr, pairs);
  switch (n) {
#define CASE(NN)                                                                               \
  case NN:                                                                                     \
    hipLaunchKernelGGL((k_rows_inv<T, NN>), g, dim3(row_threads<NN>()), 0, s, Tb, nr, row_ptr,  \
                       act_ix, V, n_act, tw);                                                  \
    break;
    AIM_FOR_SIZES(CASE)
#undef CASE
    default: return AIM_E_ARG;
  }
  return hipGetLastError() == hipSuccess ? AIM_OK : AIM_E_HIP;
}

template <typename T>
aim_status launch_cols(int n, int mode, cplx<T>* Tb, int nr, int pairs, const cplx<T>* Cq,
                       const cplx<T>* tw, hipStream_t s) {
  switch (n) {
#define CASE(NN)                                                                          \
  case NN: {                                                                              \
    dim3 g(NN / ColCfg<T, NN>::CB, pairs);                                                \
    if (mode == 0)                                                                        \
      hipLaunchKernelGGL((k_cols<T, NN, 0>), g, dim3(ColCfg<T, NN>::NT), 0, s, Tb, nr, Cq, tw); \
    else                                                                                  \
      hipLaunchKernelGGL((k_cols<T, NN, 1>), g, dim3(ColCfg<T, NN>::NT), 0, s, Tb, nr, Cq, tw); \
    break;                                                                                \
  }
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

template aim_status launch_rows_fwd<double>(int, const double2*, int, const int32_t*, const int32_t*, int, int,
                                            double2*, const double2*, hipStream_t);
template aim_status launch_rows_fwd<float>(int, const float2*, int, const int32_t*, const int32_t*, int, int,
                                           float2*, const float2*, hipStream_t);
template aim_status launch_rows_inv<double>(int, const double2*, int, const int32_t*, const int32_t*, int,
                                            double2*, int, const double2*, hipStream_t);
template aim_status launch_rows_inv<float>(int, const float2*, int, const int32_t*, const int32_t*, int,
                                           float2*, int, const float2*, hipStream_t);
template aim_status launch_cols<double>(int, int, double2*, int, int, const double2*, const double2*, hipStream_t);
template aim_status launch_cols<float>(int, int, float2*, int, int, const float2*, const float2*, hipStream_t);

}  // namespace aim
