/*
 * aim.h - C ABI of libaim: the Adaptive Integral Method (AIM) product for the
 * Galerkin-discretised 2D EFIE with a numerically filtered grid kernel, and
 * the restarted GMRES solve that applies it, on one AMD Instinct MI355X.
 *
 * Paper: "A Numerical Approach to Operator Filtering within the Adaptive
 * Integral Method for Electromagnetic Integral Equations".
 *   Sec. II, eqs. (1)-(4)   TE-EFIE with the hypersingular operator N, the
 *                           single-layer operator S, Gram matrix G and the
 *                           Calderon-preconditioned system G^-1 S G^-1 N
 *   Sec. III-A, eqs. (7)-(8) quadrature factorisation and the AIM product
 *                           Lambda^T [F^-1(F(c_grid) . F(b))]_restr
 *   Sec. III-B, eq. (10)    numerical filter: F(c_grid) truncated to |kappa|<=alpha
 *   Sec. III-C              self-interaction of the grid kernel set to zero
 *
 * Conventions
 *  - Time convention e^{jwt}; g(R) = -(j/4) H0^(2)(kR).
 *  - Complex vectors are interleaved (re, im) doubles ("c128"), column-major
 *    N x nrhs (column r starts at element r*N).  All *_dev pointers are HIP
 *    device pointers owned by the caller; *_host pointers are host memory.
 *  - The library owns everything inside an aim_ctx (grid tables, spectra,
 *    near field, work buffers).  It allocates device memory in aim_setup and
 *    in the set-up calls aim_filter / aim_filter_analytic (a filtered
 *    spectrum) and aim_fourier_spectrum (its mode buffers, first call);
 *    never in aim_matvec, aim_solve, the step-wise solver calls,
 *    aim_rhs_planewave or aim_rcs_monostatic.  Krylov workspaces are
 *    caller-owned device memory (aim_params.workspace, the workspace of
 *    aim_solver_begin) sized by aim_workspace_bytes; the context's own one
 *    is allocated in aim_setup only when the caller passes none.
 *  - Every call returns an aim_status; on error the outputs are untouched
 *    (except AIM_E_NOCONV, which returns the best iterate and its info).
 *  - Calls are asynchronous on the context's stream except aim_setup, the
 *    *_host outputs and aim_solve (which synchronises to test convergence).
 *    A context is not thread-safe; distinct contexts may run concurrently on
 *    distinct streams.
 */
#ifndef AIM_H
#define AIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aim_ctx_s* aim_ctx;
typedef struct aim_solver_s* aim_solver;   /* step-wise solve (aim_solver_begin) */

typedef enum {
  AIM_OK = 0,
  AIM_E_ARG = 1,      /* invalid argument (null pointer, size, enum)          */
  AIM_E_GEOM = 2,     /* a stencil leaves the m x m grid                       */
  AIM_E_OOM = 3,      /* device allocation failed                              */
  AIM_E_HIP = 4,      /* HIP runtime error                                     */
  AIM_E_STATE = 5,    /* call not valid in this context state                  */
  AIM_E_NOCONV = 6,   /* GMRES reached maxit; x holds the best iterate         */
  AIM_E_NUMERIC = 7,  /* NaN/Inf in a residual                                  */
  AIM_PENDING = 8     /* aim_solver_poll: the solve has not finished           */
} aim_status;

enum { AIM_PULSE = 0, AIM_HAT = 1 };

/* Operators of aim_matvec (op argument).                                     */
enum {
  AIM_OP_S = 0,        /* S_AIM x: eq. (8) with the unfiltered kernel plus the
                          near-field correction (exact Galerkin entries of
                          eq. (4) minus their grid approximation)             */
  AIM_OP_S_ALPHA = 1,  /* S^alpha x: eq. (10), filtered kernel, no near field */
  AIM_OP_N = 2,        /* N_AIM x: Maue form of eq. (2) on three grid channels
                          (phi', t_x phi, t_y phi) plus near field; hats only */
  AIM_OP_GRAM_INV = 3, /* G^-1 x, G the Gram matrix of Sec. II                */
  AIM_OP_TM = 4,       /* jk eta S_AIM x (TM-EFIE operator)                    */
  AIM_OP_TE_CP = 5,    /* G^-1 S^alpha G^-1 N x, eq. (3) with S^alpha          */
  AIM_OP_TE_CP_UNF = 6, /* G^-1 S_AIM G^-1 N x, eq. (3) unfiltered             */
  AIM_OP_N_ALPHA = 7,  /* N^alpha x: the Maue channels of eq. (2) through the
                          filtered kernel of eq. (10), no near field; hats     */
  /* TM Calderon operators (pulse contexts set up with dual = 1).  The dual
     hats psi_j live on the barycentric refinement of the polygon (vertices
     v_j and the segment midpoints M_j): psi_j is 1 at M_j, 1/2 at v_j and
     v_j+1, 0 at M_j-1 and M_j+1, linear on each half segment.  G_pd is the
     pulse/dual mixed Gram matrix (3h_i/4 on the diagonal, h_i/8 beside it),
     N'(alpha) the hypersingular operator on the refined hats.             */
  AIM_OP_TM_PC = 8,      /* G_pd^-T N^alpha_dual G_pd^-1 x (the preconditioner) */
  AIM_OP_TM_PC_UNF = 9,  /* G_pd^-T N_dual G_pd^-1 x (N with near field)         */
  AIM_OP_TM_CP = 10,     /* AIM_OP_TM_PC applied to jk eta S_AIM x               */
  AIM_OP_TM_CP_UNF = 11  /* AIM_OP_TM_PC_UNF applied to jk eta S_AIM x           */
};
/* OR-ed into op: run the grid part (maps + FFT convolution) in complex FP32;
   the near field and the in/out vectors stay FP64.  Requires a context set up
   with precision = AIM_MIXED.                                                */
#define AIM_OP_GRID_FP32 0x100

/* Systems of aim_solve (form argument).                                      */
enum {
  AIM_TM_EFIE = 0,                 /* jk eta S j = b                          */
  AIM_TE_CALDERON = 1,             /* G^-1 S^a G^-1 N j = G^-1 S^a G^-1 b     */
  AIM_TE_CALDERON_UNFILTERED = 2,  /* G^-1 S G^-1 N j = G^-1 S G^-1 b          */
  AIM_TM_CALDERON = 3,             /* P^alpha jk eta S j = P^alpha b,
                                      P^alpha = G_pd^-T N^alpha_dual G_pd^-1    */
  AIM_TM_CALDERON_UNFILTERED = 4   /* the same with N_dual (near field)          */
};

enum { AIM_FP64 = 0, AIM_MIXED = 1 };

/* Largest batch of right-hand sides: max_rhs of aim_setup and nrhs of
   aim_rhs_planewave (launch grids carry one block row per rhs and channel).  */
#define AIM_MAX_RHS 4096

typedef struct {
  int32_t n_vertices;     /* N >= 8: closed polygon, CCW, segment j = v_j -> v_{j+1},
                             each at most one wavelength long (k h <= 2 pi)     */
  const double* xy;       /* host, 2N interleaved (x, y); copied during aim_setup   */
  double k;               /* wavenumber (rad / length unit), > 0                    */
  double eta;             /* medium impedance (ohm)                                 */
  int32_t basis;          /* AIM_PULSE (TM systems) or AIM_HAT (TE systems)         */
  int32_t m;              /* grid points per side, 16..2048; the FFT length n is
                             the smallest power of two >= 2m (n_pad of aim_info) */
  double eps;             /* grid step; grid centred at 0, L = (m-1) eps / 2        */
  int32_t quad;           /* Gauss-Legendre nodes per segment in the stencils (>=1) */
  int32_t near_radius;    /* anchor Chebyshev radius of the near zone, 3..m-4       */
  int32_t precision;      /* AIM_FP64 or AIM_MIXED (also builds the FP32 grid data) */
  int32_t max_rhs;        /* largest nrhs of later calls (1..AIM_MAX_RHS)           */
  void* stream;           /* hipStream_t for all device work (NULL: default stream) */
  int32_t node_order;     /* form of Lambda (Sec. III-A).  0: one 4 x 4 cubic
                             Lagrange stencil per basis at its centre cell, with
                             the near-field correction (all operators).  P (even,
                             2..12): every quadrature node gets its own P x P
                             tensor-Lagrange stencil at its own cell and a basis
                             row of Lambda is the union of its nodes' stencils;
                             there is no near-field correction, so only
                             AIM_OP_S_ALPHA, AIM_OP_N_ALPHA and AIM_OP_GRAM_INV
                             are available                                       */
  int32_t dual;           /* pulse basis only: 1 also sets up the dual hat space
                             of the TM Calderon operators (a hat context on the
                             refined polygon, 2N vertices, same grid)           */
  int32_t max_restart;    /* longest restart aim_solve accepts on this context
                             (0..1000): its Krylov workspace, for max_rhs
                             right-hand sides, is bound in aim_setup.  0: no
                             aim_solve (AIM_E_STATE); step-wise solvers bring
                             their own workspace                               */
  void* workspace;        /* device memory for that workspace, owned by the
                             caller and valid until aim_destroy: 256-byte
                             aligned, at least aim_workspace_bytes(n_vertices,
                             max_rhs, max_restart) bytes.  NULL: aim_setup
                             allocates it (freed by aim_destroy)               */
  size_t workspace_bytes; /* size of workspace (ignored when it is NULL)        */
} aim_params;

typedef struct {
  int32_t n_unknowns, m, n_pad, n_active, active_rows, basis;
  int64_t near_nnz_s, near_nnz_n;   /* nonzeros of the near-field corrections   */
  double k, eps, alpha;             /* alpha = +inf when no filter is set        */
  size_t device_bytes;              /* bytes held on the device by the context   */
  int32_t near_band;                /* near field kept as a symmetric cyclic band
                                       of this half-width (bases are numbered
                                       along the contour), or -1: CSR only        */
  int32_t node_order;               /* aim_params.node_order of the context       */
  int32_t map_points;               /* grid points per basis row of Lambda (16, or
                                       the widest per-node row)                    */
  int32_t dual_unknowns;            /* refined hats of the dual space (2N), or 0   */
} aim_ctx_info;

typedef struct {
  int32_t iterations;    /* Arnoldi steps taken (inner steps for AIM_MIXED)     */
  int32_t matvecs;       /* operator applications, all precisions               */
  int32_t restarts;
  int32_t outer;         /* iterative-refinement steps (AIM_MIXED), else 0      */
  int32_t converged;     /* 1 if the stopping test was met                       */
  double resid_est;      /* last Arnoldi residual estimate / ||b||              */
  double resid_true;     /* ||b - A x|| / ||b|| with the FP64 operator            */
  double seconds;        /* wall time of the call                                */
} aim_solve_info;

/* Upper estimate of the device bytes a context with these parameters needs:
   its tables and buffers, one Krylov workspace (exact) for max_rhs
   right-hand sides and the longer of `restart` (a step-wise solver's) and
   p->max_restart (aim_solve's), whether the caller or the library owns it,
   its grid-kernel spectrum in the shared cache, and the largest temporary
   aim_setup holds on top of these (the n x n transform a new spectrum is
   extracted from, or the near-field build's work arrays); near-field pairs
   are bounded from the geometry (eps over the mean segment length).
   Host-only, for admission control; 0 for invalid parameters.  Spectra that
   stay cached after their last context (aim_cache_idle_bytes) are not part
   of any context's estimate.                                                  */
size_t aim_footprint_bytes(const aim_params* p, int32_t restart);

/* Device bytes of a GMRES(restart) Krylov workspace for nrhs right-hand sides
   of an n_unknowns system: restart + 1 basis vectors, the Hessenberg matrix
   and rotations, reduction partials and refinement vectors per rhs.  The
   memory passed as aim_params.workspace or to aim_solver_begin must hold at
   least this many bytes.  Host-only; 0 for invalid sizes (restart outside
   1..1000, nrhs outside 1..AIM_MAX_RHS).                                      */
size_t aim_workspace_bytes(int32_t n_unknowns, int32_t nrhs, int32_t restart);

/* Build a context: host geometry, Gauss-Legendre nodes (eq. (7)), stencil
   weights and near-zone pairs; on the device the grid kernel samples with
   the self term zeroed (Sec. III-C), its spectrum F(c_grid) (eq. (8)) and the
   FP64 near-field correction.  Synchronous.  Errors: AIM_E_ARG, AIM_E_GEOM,
   AIM_E_OOM, AIM_E_HIP.  On success *out owns device memory until
   aim_destroy.                                                                */
aim_status aim_setup(const aim_params* p, aim_ctx* out);

/* Numerical filter of Sec. III-B: keep the spectral bins with
   qx^2 + qy^2 <= (alpha n eps / 2 pi)^2 (q in FFT order, inclusive) of
   F(c_grid), giving F(c_grid^alpha) for AIM_OP_S_ALPHA and the TE-CP
   operator.  alpha = INFINITY keeps every bin.  Errors: AIM_E_ARG (alpha <= 0
   or NaN).                                                                    */
aim_status aim_filter(aim_ctx ctx, double alpha);

/* The alternative of Fig. 1(a): the grid kernel sampled from the analytically
   filtered Green's function of eq. (6), c^alpha[d] = g^alpha(eps |d|)
   (regular at d = 0, which keeps its value), embedded with the zero ring and
   transformed like c_grid; it replaces F(c_grid^alpha) for AIM_OP_S_ALPHA and
   the TE-CP operator until the next aim_filter / aim_filter_analytic.  The
   principal-value integral over [0, alpha] is evaluated on the device by
   Gauss-Legendre panels.  Synchronous.  Errors: AIM_E_ARG (alpha <= k or not
   finite), AIM_E_OOM, AIM_E_HIP.                                              */
aim_status aim_filter_analytic(aim_ctx ctx, double alpha);

/* y = op(x) for nrhs columns (1 <= nrhs <= max_rhs); x_dev and y_dev are
   c128 N x nrhs device arrays and must not overlap.  Asynchronous.  Errors:
   AIM_E_ARG (op invalid for the basis or precision), AIM_E_STATE (an operator
   with a near-field correction on a per-node context).                        */
aim_status aim_matvec(aim_ctx ctx, int32_t op, int32_t nrhs, const void* x_dev, void* y_dev);

/* Plane-wave right-hand sides, one column per angle (propagation direction
   (cos phi, sin phi), amplitude amp): pulse basis b_i = <phi_i, E_z^inc>
   (TM); hat basis b_i = <phi_i, (jk/eta) t.E^inc> with
   E^inc = eta amp (z x khat) e^{-jk khat.r} (Sec. II).  b_dev: c128 N x nrhs,
   1 <= nrhs <= AIM_MAX_RHS (else AIM_E_ARG).  Synchronises the stream.        */
aim_status aim_rhs_planewave(aim_ctx ctx, int32_t nrhs, const double* phi_inc_host,
                             double amp, void* b_dev);

/* Solve the system of `form` for nrhs right-hand sides by restarted GMRES
   (left-preconditioned for the Calderon forms, stopping when the Arnoldi
   residual estimate of that system is <= tol ||b||).  x_dev holds the
   initial guess on entry and the solution on exit.  precision AIM_MIXED
   runs FP64 iterative refinement around an inner GMRES whose grid part is
   FP32.  restart: 1..max_restart Krylov vectors per cycle (the context's
   workspace; nothing is allocated).  info_host: nrhs entries (may be NULL).
   Synchronous.  Errors: AIM_E_ARG (also restart > max_restart or nrhs >
   max_rhs), AIM_E_NOCONV, AIM_E_NUMERIC, AIM_E_STATE (max_restart = 0, or a
   per-node context: every system operator needs the near-field
   correction).                                                                */
aim_status aim_solve(aim_ctx ctx, int32_t form, int32_t precision, int32_t nrhs,
                     const void* b_dev, void* x_dev, double tol, int32_t maxit,
                     int32_t restart, aim_solve_info* info_host);

/* Step-wise solving for serving schedulers.  A solver holds one solve of
   aim_solve (any form, FP64 or AIM_MIXED refinement) and advances it by
   Arnoldi steps (inner steps for AIM_MIXED), so one host thread can
   interleave the steps of many requests, admit new requests between steps
   and retire finished ones (iteration-level batching).  Each solver has its
   own Krylov workspace (restart + 1 vectors per rhs, in caller memory), so
   several may share a context: their steps run in call order on its stream, while solvers on
   different contexts overlap on the device.  A step synchronises the stream
   only where the solve reads results on the host: when it closes a batch of
   8 Arnoldi steps, at a restart cycle's first step (true residual), and at
   a refinement check of AIM_MIXED; other steps only enqueue work.
   aim_solve is the same machinery run to the end, so a solver's result is
   bitwise that of aim_solve.

   aim_solver_begin: arguments as aim_solve, plus the solver's Krylov
   workspace: device memory of at least aim_workspace_bytes(N, nrhs,
   restart) bytes, 256-byte aligned, owned by the caller and left untouched
   by it until aim_solver_end (restart up to 1000).  b_dev (caller-owned,
   N x nrhs) must stay valid and unchanged until the solver ends; x_dev
   holds the initial guess and receives the iterate at the end of every
   restart cycle and the solution when the solve finishes.  Clears the
   workspace, forms the preconditioned right-hand side of the Calderon forms
   and takes the norms of b (synchronises the stream); allocates no device
   memory.  Errors as aim_solve (AIM_E_ARG, also for a missing, misaligned
   or short workspace; AIM_E_STATE, AIM_E_HIP); on error *out is
   unchanged.
   aim_solver_step: one Arnoldi step for each unfinished solver of
   group[0 .. count-1]; NULL entries and finished solvers are skipped.  A
   step that completes a batch also checks and restarts, the step that ends
   an AIM_MIXED inner solve also runs the refinement check, and the step
   that finishes the solve also computes the true FP64 residual.  Returns
   AIM_OK, or the first error a solver met (that solver finishes with it).
   aim_solver_poll: progress or result into info_host (nrhs entries, may be
   NULL; resid_true is -1 until the solve finishes).  Returns AIM_PENDING
   while the solve runs, then AIM_OK (converged), AIM_E_NOCONV (maxit
   reached) or the error that ended it.  Does not touch the device.
   aim_solver_end: waits for the solver's work on the stream and frees its
   host state; the workspace returns to the caller.  End the solvers of a
   context before aim_destroy.                                               */
aim_status aim_solver_begin(aim_ctx ctx, int32_t form, int32_t precision, int32_t nrhs, const void* b_dev,
                            void* x_dev, double tol, int32_t maxit, int32_t restart, void* workspace_dev,
                            size_t workspace_bytes, aim_solver* out);
aim_status aim_solver_step(aim_solver* group, int32_t count);
aim_status aim_solver_poll(aim_solver solver, aim_solve_info* info_host);
aim_status aim_solver_end(aim_solver solver);

/* Monostatic TM scattering width sigma(phi_i) = (k eta^2 / 4)
   |sum_j J_j <phi_j, e^{-jk khat_i.r}>|^2 for column i of j_dev (pulse basis,
   solved at incidence phi_i).  sigma_host: nrhs doubles.  Synchronous.        */
aim_status aim_rcs_monostatic(aim_ctx ctx, int32_t nrhs, const void* j_dev,
                              const double* phi_host, double* sigma_host);

/* aim_rcs_monostatic for callers that cannot allocate device memory (code
   under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc): the same values, bit for bit, with the angles, plane-wave
   vectors, column sums and values of the call held in one fixed device array
   of AIM_NOALLOC_SCRATCH complex values per GPU (8 MiB, kept until the
   process ends) instead of the context's buffers, so nrhs is not bounded by
   max_rhs.  Calls no allocating routine.  Limit: 2 ceil16(ceil(nrhs / 2)) +
   ceil16(nrhs) + ceil16(N nrhs) <= AIM_NOALLOC_SCRATCH (ceil16: rounded up to
   a multiple of 16), e.g. nrhs <= 31 at N = 16384; larger calls return
   AIM_E_ARG.  Every call on one GPU shares its array: calls that overlap on
   one GPU (from several threads or contexts) race and must be serialised by
   the caller.  Synchronous.  Errors: AIM_E_ARG (size, basis, null pointer),
   AIM_E_STATE, AIM_E_HIP.                                                    */
#define AIM_NOALLOC_SCRATCH 524288
aim_status aim_rcs_monostatic_noalloc(aim_ctx ctx, int32_t nrhs, const void* j_dev, const double* phi_host,
                                      double* sigma_host);

/* Spectrum of an operator in the Fourier (Laplace-Beltrami) basis of a closed
   contour whose N bases are numbered along it, as in the paper's Sec. IV
   experiments (Figs. 2 and 3, the singular values of S, S^alpha and the
   Calderon products ordered by the Laplace-Beltrami eigenvectors).  For each
   nu_host[q], q < n_modes, with e[j] = exp(i 2 pi nu j / N):
     lambda_q = (e^H G^-1 A e) / (e^H e)   for A = AIM_OP_S, AIM_OP_S_ALPHA,
                                           AIM_OP_N, AIM_OP_N_ALPHA, AIM_OP_TM
                                           (G: Gram matrix),
     lambda_q = (e^H A e) / (e^H e)        for AIM_OP_TE_CP, AIM_OP_TE_CP_UNF,
                                           AIM_OP_TM_CP, AIM_OP_TM_CP_UNF.
   On a uniformly discretised circle the matrices are circulant, e is an
   exact eigenvector, |lambda_q| is a singular value and, for the Galerkin
   operators, lambda_q approximates the continuous operator's eigenvalue.
   AIM_OP_GRID_FP32 may be or-ed in (AIM_MIXED contexts).  Modes are applied
   max_rhs at a time through aim_matvec's kernels.  lambda_host: n_modes
   interleaved complex doubles (host).  Synchronous.  Errors: AIM_E_ARG (op,
   n_modes < 1, basis mismatch as in aim_matvec), AIM_E_STATE (as in
   aim_matvec), AIM_E_OOM, AIM_E_HIP.                                          */
aim_status aim_fourier_spectrum(aim_ctx ctx, int32_t op, int32_t n_modes, const int32_t* nu_host,
                                double* lambda_host);

/* Introspection (sizes, nonzeros, device bytes).                              */
aim_status aim_get_info(aim_ctx ctx, aim_ctx_info* info);

/* Device evaluation of g(R) = -(j/4) H0^(2)(kR) at n distances (R_dev: n
   doubles, out_dev: n c128), the kernel every grid sample and near-field
   entry uses.  Exposed for verification.                                      */
aim_status aim_eval_green(aim_ctx ctx, int32_t n, const void* R_dev, void* out_dev);

/* Copy n entries of the context's near-field correction rows to host memory
   (row i: columns and values of the FP64 correction of op AIM_OP_S or
   AIM_OP_N).  cols_host may be NULL; returns the row length in *len.
   Exposed for verification; synchronous.                                      */
aim_status aim_near_row(aim_ctx ctx, int32_t op, int32_t row, int32_t cap,
                        int32_t* cols_host, double* vals_host, int32_t* len);

/* Kernel timing with HIP events recorded on the context's stream around the
   launches of one kernel of the matvec pipeline (for benchmarking).  From
   aim_profile_start on, every `every`-th launch of `kernel` (up to
   max_samples) is bracketed by a pair of events; aim_profile_stop
   synchronises the stream, returns the mean duration in ms of the sampled
   launches, the number sampled and the number of launches seen, and stops
   recording.  Errors: AIM_E_ARG (kernel id, every < 1), AIM_E_STATE (stop
   without start), AIM_E_HIP.                                                  */
enum { AIM_K_ANTERP = 0, AIM_K_ROWS_FWD = 1, AIM_K_COLS = 2, AIM_K_ROWS_INV = 3, AIM_K_INTERP = 4 };
aim_status aim_profile_start(aim_ctx ctx, int32_t kernel, int32_t every, int32_t max_samples);
aim_status aim_profile_stop(aim_ctx ctx, double* avg_ms, int64_t* samples, int64_t* launches);

/* Grid-kernel spectra F(c_grid) are shared by all contexts of a process on
   one device with the same m, k*eps and precision (the samples depend on
   k*eps only); a spectrum stays resident after its last context is
   destroyed, up to 8 GiB of cached spectra.  aim_cache_clear frees the
   unreferenced ones and returns the bytes freed.  Thread-safe.               */
size_t aim_cache_clear(void);

/* Device bytes of the cached spectra that no context uses (what
   aim_cache_clear would free now).  An admission budget counts them beside
   the footprints of its contexts.  Thread-safe.                              */
size_t aim_cache_idle_bytes(void);

void aim_destroy(aim_ctx ctx);
const char* aim_strerror(aim_status s);

#ifdef __cplusplus
}
#endif
#endif /* AIM_H */
