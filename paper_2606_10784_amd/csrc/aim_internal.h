// Internal declarations of libaim (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/aim.h"

namespace aim {

// ---------------------------------------------------------------------------
// complex helpers (interleaved re/im, HIP vector types)
// ---------------------------------------------------------------------------
template <typename T> struct CT;
template <> struct CT<double> { using type = double2; };
template <> struct CT<float> { using type = float2; };
template <typename T> using cplx = typename CT<T>::type;

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T x, T y) { cplx<T> r; r.x = x; r.y = y; return r; }
template <typename V>
__host__ __device__ __forceinline__ V cadd(V a, V b) { V r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename V>
__host__ __device__ __forceinline__ V csub(V a, V b) { V r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename V>
__host__ __device__ __forceinline__ V cmul(V a, V b) {
  V r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// a * conj(b)
template <typename V>
__host__ __device__ __forceinline__ V cmulc(V a, V b) {
  V r; r.x = a.x * b.x + a.y * b.y; r.y = a.y * b.x - a.x * b.y; return r;
}
template <typename V, typename S>
__host__ __device__ __forceinline__ V cscale(V a, S s) { V r; r.x = a.x * s; r.y = a.y * s; return r; }

// ---------------------------------------------------------------------------
// Frequency order of the column FFT.  The column pass runs a decimation-in-
// frequency FFT of length n = 16^P * RL (radix 16 P times, then RL in 2..16)
// in place, so position p holds frequency ky_of_pos(n, p): with
// p = RL * (16^{P-1} k_1 + ... + k_P) + k_{P+1}, ky = k_1 + 16 k_2 + ... +
// 16^{P-1} k_P + 16^P k_{P+1}.  The spectrum is stored in this order, folded.
// ---------------------------------------------------------------------------
__host__ __device__ inline int ky_of_pos(int n, int p) {
  int rl = n, P = 0;
  while (rl > 16) {
    rl >>= 4;
    ++P;
  }
  const int klast = p % rl;
  int rest = p / rl, ky = 0;
  for (int i = 0; i < P; ++i) {   // rest = k_1 ... k_P, most significant first
    ky = (ky << 4) | (rest & 15);
    rest >>= 4;
  }
  // the loop reversed the digit order: ky now holds k_P ... k_1 with k_1 lowest
  return ky + (klast << (4 * P));
}

// The kernel is even in dy, so the spectrum is even in ky: only half of each
// row is stored.  Position p = RL g + r holds ky = low + W r with W = n / RL
// and low = ky_of_pos(n, RL g); its mirror n - ky = (W - low) + W (RL-1-r)
// sits at the same r reversed in the group with low' = W - low.  A row keeps
// the groups with low <= W/2: slot j = lowc RL + r holds ky = lowc + W r,
// (W/2 + 1) RL slots per kxq.
__host__ __device__ inline int spec_last_radix(int n) {
  int rl = n;
  while (rl > 16) rl >>= 4;
  return rl;
}
// Rows per tile of the row/column intermediate (the tile stride is ldt rows
// of CB values).  The row passes touch every tile of a pair at this stride,
// so a row count with a large power-of-two factor concentrates them on few
// HBM channels (960 rows of 32-byte FP64 pieces, a 30 720 B = 15 * 2^11 B
// stride: the inverse row pass 22 % slower than at 958 rows).  A multiple of 4 gets
// one padding row, which leaves at most a factor 2 in the row count.
inline int tile_rows(int nr) { return nr % 4 == 0 ? nr + 1 : nr; }

// FFT length of an m-point grid side: the smallest power of two >= 2m.  Any
// length >= 2m - 1 embeds the Toeplitz grid kernel (offsets |d| <= m - 1) in
// a circulant without wrap-around (Sec. III-A, eq. (8)); the offsets
// m <= |d| <= n - m of the embedding are zero.
inline int fft_length(int m) {
  int n = 32;
  while (n < 2 * m) n *= 2;
  return n;
}

__host__ __device__ inline int spec_row_len(int n) {
  const int rl = spec_last_radix(n);
  return (n / rl / 2 + 1) * rl;
}
__host__ __device__ inline int ky_of_slot(int n, int j) {
  const int rl = spec_last_radix(n);
  return j / rl + (n / rl) * (j % rl);
}

// ---------------------------------------------------------------------------
// host-side geometry and tables produced by aim_setup (host_setup.cpp)
// ---------------------------------------------------------------------------
struct HostTables {
  int N = 0, basis = 0, m = 0, n = 0, p = 0, R = 0, nch = 1;
  double k = 0, eta = 0, eps = 0, L = 0;
  std::vector<double> vx, vy;                 // vertices
  std::vector<double> h, tx, ty;              // per segment
  std::vector<int32_t> anc_x, anc_y;          // anchor cells per basis
  // grid map rows: S points per basis.  node_order = 0: the 4 x 4 stencil of
  // the basis (S = 16); node_order = P: the union of the P x P stencils of
  // the basis's quadrature nodes, padded to the widest basis (weight 0)
  int node_order = 0, S = 16;
  // channels: 0 = phi, 1 = dphi, 2 = t_x phi, 3 = t_y phi (hats use all four)
  std::vector<double> W[4];                   // N x S per channel
  std::vector<int32_t> aidx;                  // N x S active index of each map point
  std::vector<int32_t> act_ix, act_iy;        // active points, sorted row-major
  int n_act = 0, y0 = 0, nr = 0;              // active rows [y0, y0 + nr)
  std::vector<int32_t> row_ptr;               // nr + 1 offsets into the active list
  // transposed stencils: for active point a, entries [at_ptr[a], at_ptr[a+1])
  std::vector<int32_t> at_ptr, at_basis;
  std::vector<double> at_w[4];
  // near zone (CSR over basis rows, sorted columns)
  std::vector<int32_t> nr_ptr, nr_col;
  int band_w = -1;                            // banded symmetric near field: half-width, -1 = CSR
  std::vector<double> gl_x, gl_w;             // stencil quadrature rule on [0,1]
};

// Fills everything above; returns AIM_E_ARG / AIM_E_GEOM on bad input.
aim_status build_host_tables(const aim_params* p, HostTables& t, std::string& err);
void gauss_legendre01(int p, std::vector<double>& x, std::vector<double>& w);
// Twiddle table tw[j] = exp(-2 pi i j / n), j < n, correctly rounded.
void twiddles(int n, std::vector<double>& re_im);

// ---------------------------------------------------------------------------
// device context
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Ctx;
// residual estimates one check reads back per rhs (a batch of Arnoldi steps
// plus the column that closes a cycle), rounded up
static constexpr int kResidPitch = 16;
struct GmresWork {
  int restart = 0, nrhs = 0;
  // V: restart + 1 basis slots per rhs; H: Hessenberg (rotated in place by the
  // Givens kernel); Hu: the same columns unrotated, row-major ldh x ldh;
  // hp: two provisional columns per rhs; coef: s, z, d, 1/gamma of the last
  // step (delayed orthogonalisation)
  double2 *V = nullptr, *W = nullptr, *H = nullptr, *Hu = nullptr, *hp = nullptr, *coef = nullptr, *g = nullptr,
          *cs = nullptr,
          *sn = nullptr, *y = nullptr, *part = nullptr, *r = nullptr, *d = nullptr, *b2 = nullptr, *nrm = nullptr;
  double *resid = nullptr, *npart = nullptr;
  int* active = nullptr;
  int nchunk = 0;
  size_t lds_max = 65536;         // LDS bytes one block may use on this device
  size_t bytes = 0;
};
// Binds a (restart, nrhs) GMRES workspace to caller- or context-owned device
// memory (256-byte aligned, at least gmres_work_bytes); allocates nothing.
aim_status bind_gmres_work(Ctx* c, GmresWork& w, void* base, size_t bytes, int restart, int nrhs);

struct Ctx {
  HostTables t;
  // dual hat space of the TM Calderon operators: a hat context on the
  // refined polygon (owned), and the coefficients tau_d of T^-1, T the
  // circulant (1/8, 3/4, 1/8) with G_pd = diag(h) T
  Ctx* dual = nullptr;
  double* d_tau = nullptr;
  double* d_ih = nullptr;   // 1 / h per segment
  int tau_D = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  int precision = AIM_FP64;
  int max_rhs = 1;
  int nch_max = 1;          // grid channels of the widest operator
  double alpha = 0;         // current filter cutoff (inf: none)
  bool filtered = false;
  // geometry
  double *d_vx = nullptr, *d_vy = nullptr, *d_h = nullptr, *d_tx = nullptr, *d_ty = nullptr;
  double *d_glx = nullptr, *d_glw = nullptr;
  // stencils / maps
  double* d_W[4] = {nullptr, nullptr, nullptr, nullptr};
  float* d_Wf[4] = {nullptr, nullptr, nullptr, nullptr};
  int32_t* d_aidx = nullptr;
  int32_t *d_act_ix = nullptr, *d_row_ptr = nullptr;
  int32_t *d_at_ptr = nullptr, *d_at_basis = nullptr;
  double* d_at_w[4] = {nullptr, nullptr, nullptr, nullptr};
  float* d_at_wf[4] = {nullptr, nullptr, nullptr, nullptr};
  // spectra: [kxq][j] for kxq <= n/2 and j < spec_row_len(n), frequency
  // ky_of_slot(n, j), pre-scaled by 1/n^2
  double2 *d_C = nullptr, *d_Ca = nullptr, *own_Ca = nullptr;
  float2 *d_Cf = nullptr, *d_Caf = nullptr, *own_Caf = nullptr;
  void* spec = nullptr;          // shared spectrum cache entry
  double2* d_tw = nullptr;
  float2* d_twf = nullptr;
  double2* d_ksmall = nullptr;   // kernel at offsets |d| <= R+3 (rows dy, cols dx)
  int ks = 0;
  // near field
  int32_t *d_nr_ptr = nullptr, *d_nr_col = nullptr;
  double2 *d_CS = nullptr, *d_CN = nullptr;
  // banded symmetric copies [d][i] = C(i, (i + d) mod N), d <= band_w
  double2 *d_CSd = nullptr, *d_CNd = nullptr;
  int64_t nnz = 0;
  // matvec work (sized for max_rhs x nch_max)
  void *d_U = nullptr, *d_T = nullptr, *d_V = nullptr;
  double2 *d_tmp1 = nullptr, *d_tmp2 = nullptr;   // N x max_rhs each
  double2* d_rhs = nullptr;
  double* d_phi = nullptr;     // AIM_MAX_RHS incidence angles (aim_rhs_planewave)
  double2* d_dot = nullptr;    // max_rhs column sums, then max_rhs values (aim_rcs_monostatic)
  double* h_resid = nullptr;   // pinned (coherent) GMRES residual estimates, kResidPitch per rhs
  double* d_resid_map = nullptr;   // the device's address of h_resid
  hipEvent_t ev_resid = nullptr;   // recorded after the kernels that write h_resid
  double2* d_spec = nullptr;   // Fourier-spectrum work (modes, products, quotients), on first use
  double* d_red = nullptr;
  size_t dev_bytes = 0;
  GmresWork gw;
  std::vector<void*> allocs;
  // event timing of one pipeline kernel (aim_profile_start / stop)
  int prof_kernel = -1, prof_every = 1, prof_max = 0;
  int64_t prof_launches = 0;
  std::vector<hipEvent_t> ev0, ev1;
  int ev_used = 0;
};

// brackets one launch of pipeline kernel `kid` with events when profiling:
// recorded on the stream around the launch, or (attach) handed to the launch
// through start() / stop() so the dispatch itself timestamps them
struct ProfScope {
  Ctx* c;
  bool on = false, attach = false;
  int slot = -1;
  ProfScope(Ctx* cc, int kid, bool attach_events = false) : c(cc), attach(attach_events) {
    if (c->prof_kernel != kid) return;
    const int64_t n = c->prof_launches++;
    if (n % c->prof_every != 0 || c->ev_used >= c->prof_max) return;
    slot = c->ev_used++;
    on = attach || hipEventRecord(c->ev0[slot], c->stream) == hipSuccess;
  }
  hipEvent_t start() const { return on && attach ? c->ev0[slot] : nullptr; }
  hipEvent_t stop() const { return on && attach ? c->ev1[slot] : nullptr; }
  ~ProfScope() {
    if (on && !attach) (void)hipEventRecord(c->ev1[slot], c->stream);
  }
};

// kernels / launchers (aim_kernels.hip)
aim_status dev_alloc(Ctx* c, void** p, size_t bytes);
aim_status setup_device(Ctx* c);                        // tables, spectrum, near field
aim_status apply_filter(Ctx* c, double alpha);
aim_status apply_filter_analytic(Ctx* c, double alpha);
aim_status setup_dual(Ctx* c);                          // T^-1 coefficients of the dual pairing
aim_status acquire_spectrum(Ctx* c, double keps);
void release_spectrum(Ctx* c);
size_t cache_clear();
size_t cache_idle_bytes();
// y(:, r) = op x(:, r), column strides ldx / ldy (elements), FP64 vectors
aim_status matvec(Ctx* c, int op, int nrhs, const double2* x, int64_t ldx, double2* y, int64_t ldy);
// The column pass of a split matvec: tile sets of `pairs` pairs at `tiles`
// (pair stride n / CB tiles of ldt x CB values), spectrum Cq, twiddles tw.
struct ColsJob {
  const void* Cq = nullptr;
  const void* tw = nullptr;
  void* tiles = nullptr;
  int n = 0, nr = 0, ldt = 0, pairs = 0;
  bool f32 = false;
};
static constexpr int kColBatchMax = 32;   // tile sets per grouped column-pass launch
bool matvec_splits(Ctx* c, int op);
aim_status matvec_pre(Ctx* c, int op, int nrhs, const double2* x, int64_t ldx, ColsJob* job);
aim_status matvec_post(Ctx* c, int op, int nrhs, const double2* x, int64_t ldx, double2* y, int64_t ldy);
aim_status launch_cols_jobs(const ColsJob* jobs, int count, hipStream_t s);
aim_status rhs_planewave(Ctx* c, int nrhs, const double* phi_host, double amp, double2* b);
aim_status eval_green(Ctx* c, int n, const double* R, double2* out);
aim_status rcs(Ctx* c, int nrhs, const double2* J, const double* phi_host, double* sigma);
// aim_rcs_monostatic_noalloc: the same values with every buffer of the call
// in a fixed per-device array of kNoAllocScratch complex values
static constexpr size_t kNoAllocScratch = AIM_NOALLOC_SCRATCH;
aim_status rcs_noalloc(Ctx* c, int nrhs, const double2* J, const double* phi_host, double* sigma);
aim_status rcs_into(Ctx* c, int nrhs, const double2* J, const double* phi_host, double* sigma_host, double* phi_dev,
                    double2* b_dev, double2* dot_dev, double* sig_dev);
aim_status fourier_spectrum(Ctx* c, int op, int n_modes, const int32_t* nu_host, double2* lambda_host);
aim_status solve(Ctx* c, int form, int precision, int nrhs, const double2* b, double2* x, double tol,
                 int maxit, int restart, aim_solve_info* info);
size_t gmres_work_bytes(size_t N, size_t restart, size_t nrhs);
aim_status solver_begin(Ctx* c, int form, int precision, int nrhs, const double2* b, double2* x, double tol,
                        int maxit, int restart, void* workspace, size_t workspace_bytes, aim_solver_s** out);
aim_status solver_step(aim_solver_s** group, int count);
aim_status solver_poll(aim_solver_s* sv, aim_solve_info* info);
aim_status solver_end(aim_solver_s* sv);
void free_ctx(Ctx* c);
size_t footprint(const aim_params* p, int restart, const HostTables* t);

#define AIM_HIP_CHECK(call)                                  \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return AIM_E_HIP;                  \
  } while (0)

}  // namespace aim
