// C ABI of libaim (declared in include/aim.h).
#include <cmath>
#include <cstdio>
#include <new>
#include <vector>

#include "aim_internal.h"

using namespace aim;

struct aim_ctx_s {
  Ctx c;
};

namespace aim {

void free_ctx(Ctx* c) {
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->dual) {
    free_ctx(c->dual);
    delete c->dual;
    c->dual = nullptr;
  }
  release_spectrum(c);
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  if (c->h_resid) (void)hipHostFree(c->h_resid);
  c->h_resid = nullptr;
  c->d_resid_map = nullptr;
  if (c->ev_resid) (void)hipEventDestroy(c->ev_resid);
  c->ev_resid = nullptr;
  c->gw = GmresWork();
}

// the refined polygon of the dual hat space: v_j at 2j, midpoints at 2j+1
static std::vector<double> refined_xy(const aim_params* p) {
  const int N = p->n_vertices;
  std::vector<double> r(4 * (size_t)N);
  for (int j = 0; j < N; ++j) {
    const int j1 = (j + 1) % N;
    r[4 * j] = p->xy[2 * j];
    r[4 * j + 1] = p->xy[2 * j + 1];
    r[4 * j + 2] = 0.5 * (p->xy[2 * j] + p->xy[2 * j1]);
    r[4 * j + 3] = 0.5 * (p->xy[2 * j + 1] + p->xy[2 * j1 + 1]);
  }
  return r;
}

static aim_params dual_params(const aim_params* p, const std::vector<double>& rxy) {
  aim_params q = *p;
  q.n_vertices = 2 * p->n_vertices;
  q.xy = rxy.data();
  q.basis = AIM_HAT;
  q.node_order = 0;
  q.dual = 0;
  q.max_restart = 0;      // solves run on the pulse context
  q.workspace = nullptr;
  q.workspace_bytes = 0;
  return q;
}

size_t footprint(const aim_params* p, int restart, const HostTables* t) {
  // grid work + spectra + near field + stencils + Krylov space
  const size_t N = p->n_vertices, m = p->m, n = fft_length(p->m), R = p->max_rhs;
  const size_t nch = p->basis == AIM_HAT ? 3 : 1;
  const size_t H = n / 2 + 1;
  const size_t nr = t ? t->nr : m;
  // map points per basis: 16, or for the per-node map the cells of the
  // stencils of a basis's nodes, bounded by their box
  size_t S = 16;
  if (t) {
    S = t->S;
  } else if (p->node_order > 0 && p->xy && p->eps > 0) {
    double hmax = 0;
    for (size_t i = 0; i < N; ++i) {
      const size_t i1 = (i + 1) % N;
      hmax = std::max(hmax, std::hypot(p->xy[2 * i1] - p->xy[2 * i], p->xy[2 * i1 + 1] - p->xy[2 * i + 1]));
    }
    const size_t side = (size_t)p->node_order + (size_t)std::ceil(hmax / p->eps) + 1;
    S = side * side * (p->basis == AIM_HAT ? 2 : 1);
  }
  const size_t nact = t ? t->n_act : S * N;
  // near pairs: a basis pairs with the bases whose anchors lie in the
  // (2R+1)^2-cell box around its own; the contour inside that box is at most
  // its diagonal, (2R+1) sqrt(2) eps, long for a curve smooth on the box's
  // scale, holding that length over the mean segment length of bases (+4)
  size_t near = 0;
  if (t) {
    near = t->nr_col.size();
  } else if (p->node_order == 0 && p->xy && N > 0) {
    double len = 0;
    for (size_t i = 0; i < N; ++i) {
      const size_t i1 = (i + 1) % N;
      len += std::hypot(p->xy[2 * i1] - p->xy[2 * i], p->xy[2 * i1 + 1] - p->xy[2 * i + 1]);
    }
    const double per = (2 * p->near_radius + 1) * std::sqrt(2.0) * p->eps / (len / N) + 4;
    near = N * (size_t)std::ceil(std::min(per, (double)N));
  }
  const size_t nvals = p->basis == AIM_HAT ? 2 : 1;             // S (and N for hats) per near pair
  size_t b = 0;
  b += nch * R * ((size_t)tile_rows((int)nr) * n + 2 * nact) * 16;   // U, T, V
  b += 2 * H * spec_row_len((int)n) * 16 * (p->precision == AIM_MIXED ? 1.5 : 1.0);
  b += near * (4 + 4 + 16 * nvals) + (N + 1) * 4;               // CSR (+ row of each entry)
  if (t && t->band_w >= 0) b += (size_t)(t->band_w + 1) * N * 16 * nvals;
  else if (!t) b += near * 16 * nvals;                           // the band form, kept only when smaller
  b += N * S * (8 + 4) * (p->basis == AIM_HAT ? 4 : 1) * 2;
  b += 3 * N * R * 16 + std::max<size_t>(5 * N, 64) * R * 8;    // tmp1, tmp2, rhs, reductions
  b += (size_t)AIM_MAX_RHS * 8 + R * 24;                        // angles, column sums and values of rhs / rcs
  // the Krylov space: the context's own (max_restart) or a step-wise
  // solver's (restart), whichever is longer
  const int rs = std::max(restart, p->max_restart);
  if (rs > 0) b += gmres_work_bytes(N, rs, R);
  // the largest transient of set-up: the full n x n transform the spectrum
  // is extracted from (when it is not cached), or the near-field build's
  // work arrays (row of each pair, anchors, quadrature table)
  b += std::max(n * n * 16, near * 4 + N * 8 + 256);
  if (p->dual && p->basis == AIM_PULSE && p->xy) {   // the dual hat context (no Krylov space)
    const std::vector<double> rxy = refined_xy(p);
    aim_params q = dual_params(p, rxy);
    q.max_restart = 0;
    b += footprint(&q, 0, nullptr);
  }
  return b;
}

}  // namespace aim

extern "C" {

const char* aim_strerror(aim_status s) {
  switch (s) {
    case AIM_OK: return "ok";
    case AIM_E_ARG: return "invalid argument";
    case AIM_E_GEOM: return "stencil leaves the grid";
    case AIM_E_OOM: return "device allocation failed";
    case AIM_E_HIP: return "HIP runtime error";
    case AIM_E_STATE: return "invalid context state";
    case AIM_E_NOCONV: return "GMRES did not converge";
    case AIM_E_NUMERIC: return "non-finite residual";
    case AIM_PENDING: return "solve not finished";
  }
  return "unknown status";
}

size_t aim_footprint_bytes(const aim_params* p, int32_t restart) {
  if (!p || p->n_vertices < 1 || p->m < 1 || p->max_rhs < 1 || restart < 0 || p->max_restart < 0) return 0;
  return footprint(p, restart, nullptr);
}

size_t aim_workspace_bytes(int32_t n_unknowns, int32_t nrhs, int32_t restart) {
  if (n_unknowns < 1 || nrhs < 1 || nrhs > AIM_MAX_RHS || restart < 1 || restart > 1000) return 0;
  return gmres_work_bytes((size_t)n_unknowns, (size_t)restart, (size_t)nrhs);
}

aim_status aim_setup(const aim_params* p, aim_ctx* out) {
  if (!p || !out) return AIM_E_ARG;
  *out = nullptr;
  if (p->precision != AIM_FP64 && p->precision != AIM_MIXED) return AIM_E_ARG;
  if (p->dual != 0 && (p->dual != 1 || p->basis != AIM_PULSE || p->node_order != 0)) return AIM_E_ARG;
  if (p->max_restart < 0 || p->max_restart > 1000) return AIM_E_ARG;
  if (p->workspace && (p->max_restart < 1 || ((uintptr_t)p->workspace & 255) != 0 || p->n_vertices < 1 ||
                       p->max_rhs < 1 || p->max_rhs > AIM_MAX_RHS ||
                       p->workspace_bytes < gmres_work_bytes(p->n_vertices, p->max_restart, p->max_rhs)))
    return AIM_E_ARG;
  aim_ctx_s* h = new (std::nothrow) aim_ctx_s();
  if (!h) return AIM_E_OOM;
  Ctx* c = &h->c;
  std::string err;
  aim_status st = build_host_tables(p, c->t, err);
  std::vector<double> rxy;
  aim_params q;
  if (st == AIM_OK && p->dual) {
    // host tables of the dual hat space before any device work
    rxy = refined_xy(p);
    q = dual_params(p, rxy);
    c->dual = new (std::nothrow) Ctx();
    st = c->dual ? build_host_tables(&q, c->dual->t, err) : AIM_E_OOM;
  }
  if (st != AIM_OK) {
    delete c->dual;
    c->dual = nullptr;
    delete h;
    return st;
  }
  for (Ctx* x : {c, c->dual}) {
    if (!x) continue;
    x->stream = (hipStream_t)p->stream;
    x->precision = p->precision;
    x->max_rhs = p->max_rhs;
  }
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c->dual;
    c->dual = nullptr;
    delete h;
    return AIM_E_HIP;
  }
  st = setup_device(c);
  if (st == AIM_OK && c->dual) {
    c->dual->device = c->device;
    st = setup_device(c->dual);
    if (st == AIM_OK) st = setup_dual(c);
  }
  if (st == AIM_OK && p->max_restart > 0 && c->t.node_order == 0) {
    // the Krylov workspace of aim_solve: the caller's, or allocated here once
    void* ws = p->workspace;
    const size_t need = gmres_work_bytes(c->t.N, p->max_restart, p->max_rhs);
    if (!ws) st = dev_alloc(c, &ws, need);
    if (st == AIM_OK) st = bind_gmres_work(c, c->gw, ws, p->workspace ? p->workspace_bytes : need, p->max_restart,
                                           p->max_rhs);
    if (st == AIM_OK && hipStreamSynchronize(c->stream) != hipSuccess) st = AIM_E_HIP;
  }
  if (st != AIM_OK) {
    free_ctx(c);
    delete h;
    return st;
  }
  *out = h;
  return AIM_OK;
}

aim_status aim_filter(aim_ctx ctx, double alpha) {
  if (!ctx || std::isnan(alpha) || !(alpha > 0)) return AIM_E_ARG;
  aim_status st = apply_filter(&ctx->c, alpha);
  if (st == AIM_OK && ctx->c.dual) st = apply_filter(ctx->c.dual, alpha);
  return st;
}

aim_status aim_filter_analytic(aim_ctx ctx, double alpha) {
  if (!ctx || std::isnan(alpha)) return AIM_E_ARG;
  aim_status st = apply_filter_analytic(&ctx->c, alpha);
  if (st == AIM_OK && ctx->c.dual) st = apply_filter_analytic(ctx->c.dual, alpha);
  return st;
}

aim_status aim_matvec(aim_ctx ctx, int32_t op, int32_t nrhs, const void* x_dev, void* y_dev) {
  if (!ctx || !x_dev || !y_dev || x_dev == y_dev) return AIM_E_ARG;
  const int64_t N = ctx->c.t.N;
  return matvec(&ctx->c, op, nrhs, (const double2*)x_dev, N, (double2*)y_dev, N);
}

aim_status aim_rhs_planewave(aim_ctx ctx, int32_t nrhs, const double* phi_inc_host, double amp, void* b_dev) {
  if (!ctx || !phi_inc_host || !b_dev || nrhs < 1) return AIM_E_ARG;
  return rhs_planewave(&ctx->c, nrhs, phi_inc_host, amp, (double2*)b_dev);
}

aim_status aim_solve(aim_ctx ctx, int32_t form, int32_t precision, int32_t nrhs, const void* b_dev, void* x_dev,
                     double tol, int32_t maxit, int32_t restart, aim_solve_info* info_host) {
  if (!ctx || !b_dev || !x_dev || b_dev == x_dev) return AIM_E_ARG;
  if (ctx->c.t.node_order != 0) return AIM_E_STATE;   // every system operator needs the near field
  return solve(&ctx->c, form, precision, nrhs, (const double2*)b_dev, (double2*)x_dev, tol, maxit, restart,
               info_host);
}

aim_status aim_solver_begin(aim_ctx ctx, int32_t form, int32_t precision, int32_t nrhs, const void* b_dev,
                            void* x_dev, double tol, int32_t maxit, int32_t restart, void* workspace_dev,
                            size_t workspace_bytes, aim_solver* out) {
  if (!ctx || !b_dev || !x_dev || b_dev == x_dev || !out || !workspace_dev) return AIM_E_ARG;
  if (ctx->c.t.node_order != 0) return AIM_E_STATE;   // every system operator needs the near field
  return solver_begin(&ctx->c, form, precision, nrhs, (const double2*)b_dev, (double2*)x_dev, tol, maxit, restart,
                      workspace_dev, workspace_bytes, out);
}

aim_status aim_solver_step(aim_solver* group, int32_t count) { return solver_step(group, count); }

aim_status aim_solver_poll(aim_solver solver, aim_solve_info* info_host) { return solver_poll(solver, info_host); }

aim_status aim_solver_end(aim_solver solver) { return solver_end(solver); }

aim_status aim_rcs_monostatic(aim_ctx ctx, int32_t nrhs, const void* j_dev, const double* phi_host,
                              double* sigma_host) {
  if (!ctx || !j_dev || !phi_host || !sigma_host) return AIM_E_ARG;
  return rcs(&ctx->c, nrhs, (const double2*)j_dev, phi_host, sigma_host);
}

aim_status aim_rcs_monostatic_noalloc(aim_ctx ctx, int32_t nrhs, const void* j_dev, const double* phi_host,
                                      double* sigma_host) {
  if (!ctx || !j_dev || !phi_host || !sigma_host) return AIM_E_ARG;
  return rcs_noalloc(&ctx->c, nrhs, (const double2*)j_dev, phi_host, sigma_host);
}

aim_status aim_fourier_spectrum(aim_ctx ctx, int32_t op, int32_t n_modes, const int32_t* nu_host,
                                double* lambda_host) {
  if (!ctx) return AIM_E_ARG;
  return fourier_spectrum(&ctx->c, op, n_modes, nu_host, (double2*)lambda_host);
}

aim_status aim_get_info(aim_ctx ctx, aim_ctx_info* info) {
  if (!ctx || !info) return AIM_E_ARG;
  const Ctx& c = ctx->c;
  info->n_unknowns = c.t.N;
  info->m = c.t.m;
  info->n_pad = c.t.n;
  info->n_active = c.t.n_act;
  info->active_rows = c.t.nr;
  info->basis = c.t.basis;
  info->near_nnz_s = c.nnz;
  info->near_nnz_n = c.t.basis == AIM_HAT ? c.nnz : 0;
  info->k = c.t.k;
  info->eps = c.t.eps;
  info->alpha = c.filtered ? c.alpha : INFINITY;
  info->device_bytes = c.dev_bytes + (c.dual ? c.dual->dev_bytes : 0);
  info->near_band = c.t.band_w;
  info->node_order = c.t.node_order;
  info->map_points = c.t.S;
  info->dual_unknowns = c.dual ? c.dual->t.N : 0;
  return AIM_OK;
}

aim_status aim_eval_green(aim_ctx ctx, int32_t n, const void* R_dev, void* out_dev) {
  if (!ctx || (n > 0 && (!R_dev || !out_dev))) return AIM_E_ARG;
  return eval_green(&ctx->c, n, (const double*)R_dev, (double2*)out_dev);
}

aim_status aim_near_row(aim_ctx ctx, int32_t op, int32_t row, int32_t cap, int32_t* cols_host, double* vals_host,
                        int32_t* len) {
  if (!ctx || !len) return AIM_E_ARG;
  Ctx& c = ctx->c;
  if (row < 0 || row >= c.t.N) return AIM_E_ARG;
  const double2* C = op == AIM_OP_S ? c.d_CS : (op == AIM_OP_N ? c.d_CN : nullptr);
  if (!C) return AIM_E_ARG;
  const int q0 = c.t.nr_ptr[row], q1 = c.t.nr_ptr[row + 1];
  *len = q1 - q0;
  const int cnt = std::min(cap, q1 - q0);
  if (cnt > 0 && cols_host)
    for (int q = 0; q < cnt; ++q) cols_host[q] = c.t.nr_col[q0 + q];
  if (cnt > 0 && vals_host) {
    if (hipMemcpyAsync(vals_host, C + q0, (size_t)cnt * 16, hipMemcpyDeviceToHost, c.stream) != hipSuccess)
      return AIM_E_HIP;
    if (hipStreamSynchronize(c.stream) != hipSuccess) return AIM_E_HIP;
  }
  return AIM_OK;
}

aim_status aim_profile_start(aim_ctx ctx, int32_t kernel, int32_t every, int32_t max_samples) {
  if (!ctx || kernel < AIM_K_ANTERP || kernel > AIM_K_INTERP || every < 1 || max_samples < 1) return AIM_E_ARG;
  Ctx& c = ctx->c;
  while ((int)c.ev0.size() < max_samples) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return AIM_E_HIP;
    if (hipEventCreate(&b) != hipSuccess) return AIM_E_HIP;
    c.ev0.push_back(a);
    c.ev1.push_back(b);
  }
  c.prof_kernel = kernel;
  c.prof_every = every;
  c.prof_max = max_samples;
  c.prof_launches = 0;
  c.ev_used = 0;
  return AIM_OK;
}

aim_status aim_profile_stop(aim_ctx ctx, double* avg_ms, int64_t* samples, int64_t* launches) {
  if (!ctx) return AIM_E_ARG;
  Ctx& c = ctx->c;
  if (c.prof_kernel < 0) return AIM_E_STATE;
  if (hipStreamSynchronize(c.stream) != hipSuccess) return AIM_E_HIP;
  double tot = 0.0;
  for (int i = 0; i < c.ev_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c.ev0[i], c.ev1[i]) != hipSuccess) return AIM_E_HIP;
    tot += ms;
  }
  if (avg_ms) *avg_ms = c.ev_used ? tot / c.ev_used : 0.0;
  if (samples) *samples = c.ev_used;
  if (launches) *launches = c.prof_launches;
  c.prof_kernel = -1;
  c.ev_used = 0;
  return AIM_OK;
}

size_t aim_cache_clear(void) { return cache_clear(); }

size_t aim_cache_idle_bytes(void) { return cache_idle_bytes(); }

void aim_destroy(aim_ctx ctx) {
  if (!ctx) return;
  for (hipEvent_t e : ctx->c.ev0) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->c.ev1) (void)hipEventDestroy(e);
  free_ctx(&ctx->c);
  delete ctx;
}

}  // extern "C"
