/*
 * ddelm.h -- C ABI of the MI355X (gfx950) DDELM-NN library.
 *
 * DDELM-NN: domain decomposition of extreme learning machines with a coarse
 * space and a theta-mixed Neumann-Neumann acceleration (Lee & Ryoo).  The
 * calls follow the paper's statement of the problem:
 *
 *   ddelm_setup   partition of the domain (sec. 2.1), local networks with
 *                 preset hidden parameters (sec. 2.2) and the collocation
 *                 sets x_I, x_B, x_Gamma of every subdomain (sec. 2.2.1);
 *   ddelm_factor  local feature matrices K_c^i, A_m^i, Kbar^i, Abar^i
 *                 (sec. 2.2.1, 3.1, 3.2), their Householder QR, and the
 *                 coarse Schur complement S_Pi, formed densely and
 *                 Cholesky-factored (sec. 3);
 *   ddelm_solve   right-hand side f = [f(x_I); g(x_B); 0] (eq. ddelm),
 *                 CG on mu_Delta for eq. nn-mixed, then
 *                 [c; mu_Pi] = K~^+ (f~ - B~ mu_Delta) (eq. coarse_sol_2);
 *   ddelm_evaluate  u(x) = NN^i(x) = sum_j c_j tanh(w_j . xi + b_j) on the
 *                 owning subdomain.
 *
 * Conventions
 *   - Two space dimensions.  Subdomain i = iy*nx + ix of a uniform nx x ny
 *     partition of the box [lo, hi].
 *   - Hidden weights act on local coordinates xi = (x - centre_i)/(h/2),
 *     so xi ranges over [-1, 1]^2 on every subdomain.
 *   - Every edge of every subdomain carries p points at parameters edge_s
 *     (both ends included).  Edge points on the domain boundary, and the
 *     extra parameters extra_s on boundary sides, are boundary points.
 *     Subdomain corners inside the domain form Pi (coarse >= 1); the other
 *     interface points form Delta.
 *   - Global orders: Pi point at lattice vertex (jx, jy) has index
 *     (jy-1)*(nx-1) + (jx-1).  Interior edges are numbered vertical first
 *     (iy*(nx-1) + jx-1), then horizontal ((nx-1)*ny + (jy-1)*nx + ix);
 *     Delta point k (1..p-2) of edge e has index e*(p-2) + k-1.  With
 *     coarse == 0 the interior vertices are Delta points numbered after all
 *     edge points, in the Pi order.
 *   - Local row order of K_c^i: interior points (as given), boundary points
 *     (sides bottom, right, top, left that lie on the domain boundary, each
 *     by increasing coordinate, a shared corner listed once; then the extra
 *     boundary points side by side), then Gamma: Pi^i then Delta^i, each by
 *     global index.
 *   - All array arguments are DEVICE pointers unless marked "host".  Arrays
 *     are dense, row-major in the index order written, float64.
 *   - Inputs are borrowed for the duration of the call; ddelm_setup copies
 *     what it keeps.  Outputs are written into caller-owned buffers.  The
 *     context owns its factors and workspaces until ddelm_destroy.
 *   - Device memory of contexts comes from a pool private to the library
 *     (one per device, stream-ordered on the context's stream); memory freed
 *     by ddelm_destroy stays in the pool for the next context, and so do the
 *     context's events, second stream and pinned staging buffer.
 *     ddelm_release_cached_memory hands the idle part back.  Destroy a
 *     context before the stream it was set up on.
 *   - Work is ordered on the stream given to ddelm_setup (a hipStream_t
 *     passed as void*; NULL = the default stream).  Calls that return
 *     statistics synchronise that stream.  A context is not thread-safe.
 *   - Errors: a negative status is an error; outputs are then unspecified
 *     and ddelm_last_error(ctx) describes it.  DDELM_WARN_NOCONV means the
 *     solve did not meet its tolerance (see ddelm_solve); the best iterate
 *     is still written.
 */
#ifndef DDELM_H
#define DDELM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ddelm_ctx_s* ddelm_ctx;

typedef enum {
  DDELM_OK = 0,
  DDELM_WARN_NOCONV = 1,
  DDELM_E_ARG = -1,        /* invalid argument value */
  DDELM_E_SHAPE = -2,      /* sizes inconsistent or beyond limits */
  DDELM_E_STATE = -3,      /* call out of order (e.g. solve before factor) */
  DDELM_E_HIP = -4,        /* HIP runtime error, or a device-side bounded wait expired */
  DDELM_E_NOMEM = -5,      /* device allocation failed */
  DDELM_E_CHOLESKY = -6,   /* S_Pi not positive definite */
  DDELM_E_NONFINITE = -7   /* NaN/Inf met in CG */
} ddelm_status;

/* Problem description (sec. 2.1 partition, sec. 2.2 networks and points). */
typedef struct {
  int nx, ny;               /* subdomains per axis, >= 1 */
  double lo[2], hi[2];      /* domain box, lo < hi */
  int p;                    /* points per edge incl. both ends, 3 <= p <= 4096 */
  const double* edge_s;     /* host [p]: 0 = s_0 < s_1 < ... < s_{p-1} = 1 */
  int n_extra;              /* extra boundary points per boundary side, >= 0 */
  const double* extra_s;    /* host [n_extra], each in (0,1); may be NULL if n_extra == 0 */
  int n_int;                /* interior collocation points per subdomain, >= 1 */
  const double* x_int;      /* device [N][n_int][2], global coordinates, inside the subdomain */
  int M;                    /* neurons per subdomain, 1 <= M <= 1024, M <= rows of K_c^i */
  const double* W;          /* device [N][M][2] hidden weights (local coordinates) */
  const double* b;          /* device [N][M] hidden biases */
} ddelm_problem;

typedef struct {
  double theta;             /* NN mixing weight of eq. nn-mixed, 0 <= theta <= 1 */
  int coarse;               /* 0: no coarse space, K and A (vanilla DDELM);
                               1: corners as Pi, K and A;
                               2: corners as Pi, K_c and A_m (sec. 3.2; default);
                               3: corners as Pi, K_c and A;  4: corners as Pi, K and A_m
                               (the other cells of the ablation of sec. 4.2) */
  int precision;            /* 0: float64 throughout;
                               1: mixed -- Householder QR in float32 on the matrix cores, its
                                  factors widened to float64 for the triangular solves, local
                                  operators, right-hand sides and recovery; float32 local
                                  operators in the CG; float64 coarse problem, dots and
                                  refinement of the coupled system (result within the
                                  float32-factor floor of the float64 one, not to tol);
                               2: float64 factors and operators, float32 copies of the local
                                  operators in the CG, refined on the float64 interface
                                  residual until it is <= tol (the float64 result) */
  double tol;               /* CG stop: ||r_k|| <= tol ||b||, 0 < tol < 1 */
  int maxit;                /* CG iteration cap (per refinement step), >= 1 */
  int max_nrhs;             /* largest nrhs a solve may pass, 1..64 */
  int cg_mode;              /* 0: auto; 1: one launch per CG phase; 2: one persistent
                               cooperative launch per CG solve */
  int refine_maxit;         /* mixed precision: outer refinement steps cap (>= 0; 0 = the
                               float32-QR solve alone) */
  double refine_tol;        /* mixed precision: stop when the correction of mu is
                               <= refine_tol relative to mu (converged), or when a step
                               shrinks the correction by less than a factor 2 (stall) */
  double inner_tol;         /* precision 1: CG tolerance of each inner solve */
} ddelm_options;

typedef struct {
  int iters;                /* CG iterations (sum over refinement steps, max over RHS) */
  int refine_steps;         /* refinement steps taken (mixed precision), else 0 */
  double rel_res;           /* final recurrence residual ||r||/||b||, max over RHS */
  double ms_rhs;            /* wall time of the right-hand-side assembly */
  double ms_cg;             /* wall time of the CG loop(s) */
  double ms_recover;        /* wall time of recovery (and refinement residuals) */
  int cg_blocks;            /* persistent CG: workgroups of the last launch (0 with cg_mode 1) */
  int cg_slices;            /* persistent CG: row slices per subdomain (tuned, see ddelm_solve) */
  int cg_coarse_dist;       /* persistent CG: 1 = coarse phases distributed over workgroups */
  int cg_restarts;          /* CG restarts on the float64 residual (see true_rel_res) */
  double true_rel_res;      /* float64: ||b - S_theta mu_Delta|| / ||b|| with S_theta applied in
                               float64 to the returned mu_Delta (eq. nn-mixed), max over RHS;
                               NaN in mixed precision, whose convergence test is refine_corr */
  double refine_corr;       /* mixed precision: relative size of the last refinement correction
                               of (mu_Pi, mu_Delta), max over RHS; 0 in float64 */
  double kappa_est_max;     /* max over the factored local matrices (K_c^i and Kbar^i) of
                               max_j |R_jj| / min_j |R_jj| of their triangular factor */
  double start_rel_res;     /* with mu0: ||b - S_theta mu0|| / ||b|| in float64 (max over RHS),
                               the residual of the starting value; 0 without mu0 */
} ddelm_stats;

typedef struct {
  int N, M, n_pi, n_dl;     /* subdomains, neurons, #Pi, #Delta */
  int n_int;                /* interior points per subdomain */
  int max_m;                /* largest local row count */
  long long sum_nB;         /* boundary points over all subdomains */
  long long sum_nG;         /* local interface points over all subdomains */
} ddelm_sizes;

/* Default options: theta 0.999 (sec. 4.2), coarse 2, fp64, tol 1e-8,
 * maxit 20000, max_nrhs 1, cg_mode auto, refine_maxit 10, refine_tol 1e-9,
 * inner_tol 1e-3. */
void ddelm_default_options(ddelm_options* opt);

/* Validate, build the interface indexing on the host and allocate the
 * context.  Errors: DDELM_E_ARG, DDELM_E_SHAPE (also for an interior point
 * outside the closed box of its subdomain, or with a NaN coordinate; checked
 * on the device, the message names the lowest such subdomain),
 * DDELM_E_NOMEM, DDELM_E_HIP.  Returns after the context's stream has
 * drained. */
ddelm_status ddelm_setup(ddelm_ctx* out, const ddelm_problem* prob,
                         const ddelm_options* opt, void* stream);

/* Variable coefficient: the operator becomes -div(rho grad u) = f with u = g
 * on the boundary (sec. 4.3, variable-coefficient Poisson equation, where
 * rho = tanh(grf) + 1.1).  Interior rows of K_c^i and Kbar^i become
 * rho (-Laplace phi) - grad rho . grad phi; every flux row (A / A_m and the
 * Delta rows of Kbar^i) becomes the conormal derivative rho dphi/dn at each of
 * its points; value and continuity rows are unchanged.
 *   rho_I  device [N][n_int][3]: rho, d rho/dx, d rho/dy at the interior points
 *          (the x_int order of ddelm_problem)
 *   rho_pi device [n_pi]: rho at the Pi points (ddelm_get_interface_points
 *          order); may be NULL when n_pi == 0
 *   rho_dl device [n_dl]: rho at the Delta points
 * All three NULL: back to rho = 1.  The arrays are copied (borrowed for the
 * call).  Call after ddelm_setup; the context then needs ddelm_factor again.
 * Synchronises the context's stream.  Errors: DDELM_E_STATE (setup did not
 * complete), DDELM_E_ARG (a required array NULL, rho <= 0 anywhere),
 * DDELM_E_NONFINITE, DDELM_E_HIP, DDELM_E_NOMEM. */
ddelm_status ddelm_set_coefficient(ddelm_ctx ctx, const double* rho_I, const double* rho_pi,
                                   const double* rho_dl);

/* Assemble local matrices, factor them (Householder QR), build the local
 * interface operators and the coarse problem.  Errors: DDELM_E_HIP,
 * DDELM_E_CHOLESKY. */
ddelm_status ddelm_factor(ddelm_ctx ctx);

/* Solve for nrhs right-hand sides (1 <= nrhs <= max_nrhs).
 *   f_I   [nrhs][N][n_int]   f at the interior points
 *   g_B   [nrhs][sum_nB]     g at the boundary points (ddelm_get_boundary_points order)
 *   mu0   [nrhs][n_dl]       may be NULL (zero): starting value of mu_Delta for the CG
 *                            (a warm start; the result does not depend on it beyond tol)
 *   coef  [nrhs][N][M]       output: last-layer coefficients c^i
 *   mu_pi [nrhs][n_pi]       output, may be NULL: mu_Pi
 *   mu_dl [nrhs][n_dl]       output, may be NULL: mu_Delta (may alias mu0)
 *   stats host, may be NULL; when given the call synchronises the stream.
 * In float64 the CG stops on its recurrence residual ||r_k|| <= tol ||b||;
 * then b - S_theta mu_Delta is formed in float64 and, while it exceeds
 * tol ||b||, the CG is restarted on it (at most 3 times).  In mixed precision
 * the float32-operator CG runs to inner_tol and the result is refined until
 * the relative correction is <= refine_tol (see ddelm_options).
 * Errors: DDELM_E_STATE (before factor), DDELM_E_ARG, DDELM_E_HIP,
 * DDELM_E_NONFINITE.  DDELM_WARN_NOCONV (result still written): float64 --
 * maxit reached or the float64 residual stayed above tol; mixed -- the
 * refinement stopped (stall or refine_maxit) with the correction above
 * refine_tol. */
ddelm_status ddelm_solve(ddelm_ctx ctx, int nrhs, const double* f_I, const double* g_B, const double* mu0,
                         double* coef, double* mu_pi, double* mu_dl, ddelm_stats* stats);

/* Allocation-free variant of ddelm_solve (without mu0), for callers that
 * cannot allocate device memory during the call: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Same
 * arguments, results and errors as ddelm_solve; the context must be factored
 * and the output arrays exist before the call.  The call's workspace (local
 * right-hand sides, interface vectors, CG state) is 8 bytes times
 * nrhs * (sum m + 12 sum_nD + 7 sum_nP + 12 n_dl + 10 n_pi + 12298), and in
 * mixed precision nrhs * (sum m + N M + sum_nD + sum_nP + 3 n_dl + 4 n_pi +
 * 512) more (sum_nD, sum_nP: local Delta and Pi points over all subdomains),
 * each buffer rounded up to 256 bytes.  It is taken from a fixed device array
 * of 64 MiB that the library holds on each GPU it runs on until the process
 * ends; a larger workspace is refused with DDELM_E_SHAPE before any work,
 * naming the bytes needed.  The call creates
 * no events (the phase times of ddelm_get_phase_times are not updated) and
 * runs no launch tuning: the persistent CG takes the launch shape an earlier
 * ddelm_solve of the same shape chose in this process, else the size
 * heuristic.  Every call on one GPU shares that GPU's array, which keeps the
 * last call's contents (the parts that must start at zero are cleared by a
 * kernel at every call): calls that overlap on one GPU race. */
ddelm_status ddelm_solve_noalloc(ddelm_ctx ctx, int nrhs, const double* f_I, const double* g_B, double* coef,
                                 double* mu_pi, double* mu_dl, ddelm_stats* stats);

/* Solve the coupled system of eq. ddelm with a general right-hand side
 * [f; h]: f given on every local row (interior, boundary and interface rows,
 * the interface rows in the K_c^i row space) and h on the flux rows of the
 * interface points (Pi block then Delta block).  The result is the DDELM-NN
 * solution for that right-hand side (d_Pi = h_Pi - A_Pi K^+ f and
 * d~ = h_Delta - A~ K~^+ f~ in sec. 3).  Used by iterative refinement and by
 * the adjoint.
 *   f_loc [nrhs][sum m]            local right-hand sides, subdomain after subdomain
 *   h     [nrhs][n_pi + n_dl]      may be NULL (zero)
 *   coef, mu_pi, mu_dl, stats      as in ddelm_solve
 * In mixed precision this call runs the float32 solve with the same
 * refinement as ddelm_solve. */
ddelm_status ddelm_solve_general(ddelm_ctx ctx, int nrhs, const double* f_loc, const double* h, double* coef,
                                 double* mu_pi, double* mu_dl, ddelm_stats* stats);

/* u(x) (and grad u if grad != NULL) on the lowest-index subdomain whose
 * closed box holds x.  coef [nrhs][N][M], x [npts][2], u [nrhs][npts],
 * grad [nrhs][npts][2].  Points outside the box are clamped to the nearest
 * subdomain. */
ddelm_status ddelm_evaluate(ddelm_ctx ctx, int nrhs, const double* coef, long long npts,
                            const double* x, double* u, double* grad);

/* Adjoint (transpose) of ddelm_solve, for gradients of a loss of the
 * coefficients with respect to the data.  The solve is a linear map
 * (f_I, g_B) -> c; this call applies its transpose to coef_bar, reusing the
 * stored factors: the transposed recovery, one CG with the same symmetric
 * operator S_theta of eq. nn-mixed, and the transposed right-hand-side map
 * (which contains theta P^T P + (1 - theta) I of sec. 3.2 and the
 * (K~^+)^T recipe of sec. 3).  Not in the paper; derived from its equations.
 *   coef_bar [nrhs][N][M]      cotangent of coef
 *   f_I_bar  [nrhs][N][n_int]  output: cotangent of f_I
 *   g_B_bar  [nrhs][sum_nB]    output, may be NULL: cotangent of g_B
 *   stats    as in ddelm_solve (iters = CG iterations of the transposed solve)
 * The CG stops at the relative residual tol, so in float64 the result is
 * exact up to that tolerance.  In mixed precision the float32 transposed
 * solve is refined on the float64 transposed residual of the coupled system
 * (refine_maxit, refine_tol, inner_tol as for the forward solve).  That
 * removes only the part of the float32 error the transposed residual sees;
 * the rest, along the difference between the float32 range of Q_i and the
 * range of K_c^i (of order eps32 * cond(K_c^i)), stays, so the result
 * carries a float32-level error.  Use precision 0 for gradients to float64
 * accuracy.
 * Errors as in ddelm_solve. */
ddelm_status ddelm_solve_adjoint(ddelm_ctx ctx, int nrhs, const double* coef_bar, double* f_I_bar,
                                 double* g_B_bar, ddelm_stats* stats);

/* Adjoint of ddelm_solve_general: cotangents of (coef, mu_Pi, mu_Delta) to
 * those of (f_loc, h).
 *   coef_bar  [nrhs][N][M]
 *   mu_pi_bar [nrhs][n_pi]          may be NULL (zero)
 *   mu_dl_bar [nrhs][n_dl]          may be NULL (zero)
 *   f_loc_bar [nrhs][sum m]         output, every local row
 *   h_bar     [nrhs][n_pi + n_dl]   output, may be NULL
 * Errors as in ddelm_solve. */
ddelm_status ddelm_solve_adjoint_general(ddelm_ctx ctx, int nrhs, const double* coef_bar,
                                         const double* mu_pi_bar, const double* mu_dl_bar,
                                         double* f_loc_bar, double* h_bar, ddelm_stats* stats);

/* Adjoint of ddelm_evaluate: coef_bar[r][i][j] = sum over the points p owned
 * by subdomain i (the owner rule of ddelm_evaluate) of
 * u_bar[r][p] phi_j(x_p) + grad_bar[r][p] . grad phi_j(x_p).
 *   x [npts][2], u_bar [nrhs][npts], grad_bar [nrhs][npts][2] (may be NULL),
 *   coef_bar [nrhs][N][M] output (overwritten).
 * The summation order over points is fixed (ascending point index), so the
 * result is reproducible bit for bit.  Errors: DDELM_E_ARG, DDELM_E_STATE,
 * DDELM_E_HIP. */
ddelm_status ddelm_evaluate_adjoint(ddelm_ctx ctx, int nrhs, long long npts, const double* x,
                                    const double* u_bar, const double* grad_bar, double* coef_bar);

/* Sizes of the problem. */
ddelm_status ddelm_get_sizes(ddelm_ctx ctx, ddelm_sizes* out);

/* Host arrays [N]: boundary, Pi, Delta and row counts per subdomain
 * (m = rows of K_c^i; the local rows of f_loc in ddelm_solve_general). */
ddelm_status ddelm_get_counts(ddelm_ctx ctx, int* n_B, int* n_P, int* n_D, int* m);

/* Host arrays: global Pi indices of the local Pi points, subdomain by
 * subdomain ([sum n_P]), and global Delta indices of the local Delta
 * points ([sum n_D]).  Bit-exact description of the interface split. */
ddelm_status ddelm_get_indexing(ddelm_ctx ctx, int* pi_glob, int* dl_glob);

/* Device [sum_nB][2]: boundary point coordinates in the g_B order. */
ddelm_status ddelm_get_boundary_points(ddelm_ctx ctx, double* x_B);

/* Device [n_pi][2] and [n_dl][2]: interface point coordinates. */
ddelm_status ddelm_get_interface_points(ddelm_ctx ctx, double* x_pi, double* x_dl);

/* Device copy of one local matrix of subdomain `sub`, row-major rows x cols
 * (host outputs rows, cols; pass out == NULL to query the shape):
 *   0 K_c^i (m x M)        1 A_m^i (n_G x M)   2 Kbar^i (m x M)   3 Abar^i (n_D x M)
 *   4 R of K_c^i (M x M)   5 I - Q_G Q_G^T (n_G x n_G)   6 A_m^i K_c^{i+} E_G (n_G x n_G)
 *   7 Abar^i Kbar^{i+} E_D (n_D x n_D)   8 S_Pi (n_pi x n_pi, sub ignored)
 * 0-3 are re-assembled on demand; 4-8 need ddelm_factor. */
ddelm_status ddelm_get_local_matrix(ddelm_ctx ctx, int which, int sub, double* out,
                                    int* rows, int* cols);

/* Host [8]: device-timeline milliseconds (HIP events on the context's
 * stream) of the phases of the last ddelm_factor and ddelm_solve:
 *   0 feature assembly   1 Householder QR   2 local interface operators
 *   3 coarse problem     4 right-hand side  5 CG   6 recovery   7 unused (0) */
ddelm_status ddelm_get_phase_times(ddelm_ctx ctx, double* ms);

const char* ddelm_last_error(ddelm_ctx ctx);
/* Synchronises the context's stream, then frees the context; its memory
 * returns to the library's pool (see the conventions above).  NULL is a
 * no-op. */
void ddelm_destroy(ddelm_ctx ctx);

/* Returns the library's idle device memory, events, streams and pinned
 * staging buffers (those of destroyed contexts) to the runtime.  Memory of
 * live contexts is not touched; allocations queued but not yet executed
 * stay with the pool until their stream reaches them.  Thread-safe. */
ddelm_status ddelm_release_cached_memory(void);

#ifdef __cplusplus
}
#endif
#endif /* DDELM_H */
