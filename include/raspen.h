/*
 * raspen.h -- C ABI of the MI355X (gfx950) RASPEN library.
 *
 * Solves the smoothed first-order optimality system of the L2/L1-regularised
 * semilinear elliptic optimal control problem
 *
 *     min 1/2 |y - y_d|^2 + nu/2 |u|^2 + mu |u|_1   s.t.  A y + phi(y) = f + u
 *
 * (paper: eq. (P); reduced smoothed system eq. (reg_OS_red), Section 3.2) with u
 * eliminated through the smoothed soft-threshold u = -(1/nu)(p + mu P_eps(-p/mu))
 * (eq. (smoothProj)), by one-level RASPEN (Section 4.2, Algorithms 2-4) whose
 * local problems are solved by damped Newton with eps-continuation (Algorithm 1).
 *
 * Discretisation: unit square, A = 5-point finite-difference -Laplacian with
 * homogeneous Dirichlet data, nx x ny interior nodes, hx = 1/(nx+1),
 * hy = 1/(ny+1).  Every grid array is float64, row-major [ny][nx] (x fastest).
 * A state vector x = (y, p) is stored as [2][ny][nx] (y first).
 *
 * Memory: unless stated otherwise, array arguments are DEVICE pointers on the
 * context's device, owned by the caller, and must stay valid until the work
 * enqueued on `stream` has completed.  Calls that return results to the host
 * (norms, histories) synchronise `stream` before they return.
 *
 * Errors: every call returns an int status.  0 = success / converged; > 0 =
 * completed with the last iterate written (RSP_NOT_CONVERGED, RSP_LINESEARCH_FAIL,
 * RSP_GMRES_STAGNATION, RSP_REFINE_FALLBACK); < 0 = hard error with outputs
 * undefined (RSP_EINVAL, RSP_ENOMEM, RSP_EHIP, RSP_ENUMERIC).  rsp_last_error()
 * returns a thread-local message for the last failing call.  No C++ exception
 * crosses this interface.  A context is not thread-safe: use one per host thread.
 */
#ifndef RASPEN_H
#define RASPEN_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RSP_VERSION 100

/* status codes */
#define RSP_OK 0
#define RSP_NOT_CONVERGED 1     /* iteration limit reached (Algorithms 1 and 2 k_max) */
#define RSP_LINESEARCH_FAIL 2   /* backtracking went below alpha_min (Algorithm 1) */
#define RSP_GMRES_STAGNATION 3  /* not converged, and a GMRES solve hit max_gmres above its tolerance */
#define RSP_REFINE_FALLBACK 4   /* converged, but only after the instance left the FP32 line
                                   factors for FP64 ones (rsp_options.fallback_rho) */
#define RSP_EINVAL (-1)
#define RSP_ENOMEM (-2)
#define RSP_EHIP (-3)
#define RSP_ENUMERIC (-4)       /* a residual or a Newton direction is not finite: NaN or Inf
                                   in the data, or a singular local Jacobian (zero pivot) */
#define RSP_EAGAIN (-5)         /* rsp_server_wait: not done within the timeout */

/* phi(y), Assumption 1 (phi in C^2, monotone increasing) */
#define RSP_PHI_ZERO 0          /* phi = 0 (linear state equation)            */
#define RSP_PHI_CUBIC 1         /* phi = y^3                                   */
#define RSP_PHI_EXP 2           /* phi = exp(y) - 1                            */
#define RSP_PHI_PAPER 3         /* phi = kappa (y^3 + exp(kappa y)), Section 4 */

/* where eps-continuation is applied (Algorithm 2 with the solver settings of
   Section 5: continuation in the local solves of the first evaluation only) */
#define RSP_CONT_FIRST 0        /* local solves of the first evaluation only */
#define RSP_CONT_NONE 1         /* never: every local solve at eps_min        */
#define RSP_CONT_EVERY 2        /* every evaluation                           */

#define RSP_FP64 0              /* local factors in FP64                        */
#define RSP_FP32_REFINED 1      /* local factors in FP32 + FP64 refinement       */

/* Problem data (eq. (P), eq. (reg_OS_red), Algorithm 1 eps schedule, Section 4.2
   partition).  The domain is the unit square.  sx x sy non-overlapping boxes of
   width ceil(n/s) per direction; each is extended by `overlap` nodes per side and
   clipped to the grid (the overlapping subdomain Omega_i). */
typedef struct rsp_problem {
  int32_t nx, ny;         /* interior nodes per direction, >= 1                     */
  int32_t phi_kind;       /* RSP_PHI_*                                             */
  double kappa;           /* parameter of RSP_PHI_PAPER                            */
  double nu;              /* > 0, L2 weight                                        */
  double mu;              /* >= 0, L1 weight (mu = 0: u = -p/nu exactly)           */
  double eps0, eps_min;   /* 0 < eps_min <= eps0: continuation start and target    */
  double gamma;           /* eps_{k+1} = max(gamma eps_k, eps_min), 0 < gamma < 1   */
  int32_t sx, sy;         /* boxes per direction, 1 <= s <= n, no box may be empty */
  int32_t overlap;        /* >= 0, nodes added on each side                        */
  const double* coef;     /* NULL: A = -Laplacian (5-point).  Else device memory, caller-
                             owned, valid until the call that reads it returns: the
                             coefficients of A y = -d/dx(a1 dy/dx) - d/dy(a2 dy/dy) + a0 y,
                             Assumption 1 (3) with a diagonal tensor, discretised in flux
                             form, (A y)_ij = sum over the four faces f of node ij of
                             a_f (y_ij - y_nb) / h_f^2 + a0_ij y_ij (y = 0 on the boundary).
                             Three float64 arrays back to back: a1 at the x-faces,
                             [ny][nx+1] (face i of row j between nodes i-1 and i), a2 at the
                             y-faces, [ny+1][nx] (face j of column i between rows j-1 and
                             j), a0 at the nodes, [ny][nx]; a1, a2 > 0 and a0 >= 0 are the
                             caller's to ensure.  rsp_solve, rsp_setup, the batch and the
                             server copy them into their workspace. */
} rsp_problem;

/* Solver options (paper Section 5 gives tol 1e-10, inner tol 1e-8, sigma 1.1).
   Norms are Euclidean norms of the discrete vectors.  The outer test of Algorithm 2
   measures the RASPEN residual, a sum of corrections in the units of x.  The inner
   test of Algorithm 1, max(tol, tol |K_i(0)|), measures the local residual K_i of the
   unscaled 5-point equations, whose stencil entries are O(h^-2).  Its two branches
   have their own tolerances: the absolute one (tol_inner) has the units of K_i, the
   relative one (tol_inner_rel) none.  A tolerance stated for equations scaled by the
   cell area hx hy (the inner 1e-8 of Section 5 read that way) therefore becomes
   tol_inner = tol / (hx hy) with tol_inner_rel = tol; taken unscaled, 1e-8 can lie
   below the FP64 rounding floor of a local residual, and the local solves then stop
   at max_inner. */
typedef struct rsp_options {
  double tol_outer;       /* Algorithm 2: stop when |F(x^k)| <= max(tol, tol |F(x^0)|)  */
  double tol_inner;       /* Algorithm 1, absolute branch of the local stopping test    */
  double gmres_rtol;      /* GMRES: stop when |r| <= rtol |b|                          */
  double sigma;           /* >= 1, relaxed backtracking, eq. (line_search)             */
  double alpha_min;       /* > 0, backtracking floor (then RSP_LINESEARCH_FAIL)        */
  int32_t gmres_restart;  /* 1 .. 64                                                    */
  int32_t max_outer;      /* Algorithm 2 k_max                                          */
  int32_t max_inner;      /* Algorithm 1 k_max                                          */
  int32_t max_gmres;      /* matrix-vector products per outer iteration                 */
  int32_t precision;      /* RSP_FP64 or RSP_FP32_REFINED                               */
  int32_t max_refine;     /* refinement steps per FP32 local solve                      */
  int32_t continuation;   /* RSP_CONT_*                                                 */
  int32_t record_eps_snapshots;  /* rsp_solve only (0 elsewhere): record at most this many
                          (<= RSP_HIST_MAX + 1) states x^0 + sum_i P~_i c_i^(k) of the
                          first evaluation into eps_snapshots, k = 0, 1, ... counting the
                          local Newton (eps) steps of Algorithm 1; c_i^(k) is subdomain i's
                          correction after its k-th step, or its last one once it stopped */
  double tol_inner_rel;   /* Algorithm 1, relative branch; < 0: equal to tol_inner       */
  double fallback_rho;    /* FP32 factors only: an instance leaves them for FP64 factors
                          when a local solve of its evaluation at x^k fails (status 1 or 2),
                          or, x^k not meeting the outer test, when the GMRES solve of step k
                          ended above fallback_rho (relative residual) or, from k = 2 on,
                          |F(x^k)| > fallback_rho |F(x^(k-1))|: the FP32 Jacobian action no
                          longer gives a contraction by fallback_rho per outer step.  It
                          continues from x^k with FP64 factors (a new budget of max_outer
                          steps) and, if it then converges, ends with RSP_REFINE_FALLBACK.
                          < 0: never; 0 forces the switch at the first open x^k, k >= 1.  */
  double* eps_snapshots;  /* device, [record_eps_snapshots][2][ny][nx], caller-owned      */
  int32_t coarse;         /* RASPEN only: 0 one level (the paper's method); 1 a second level
                          for the outer Newton systems, which the paper leaves to future
                          work (Sections 5.3, 6): the hybrid two-level Schwarz preconditioner
                          with one coarse unknown per subdomain core and field and the
                          coarse operator Z^T F'(x) Z.  Same outer iteration and fixed point,
                          fewer GMRES products as subdomains are added; at most 32
                          subdomains per row. */
} rsp_options;

#define RSP_HIST_MAX 64

/* Convergence history of one solve (host memory, filled by rsp_solve). */
typedef struct rsp_history {
  int32_t status;                       /* final status code                           */
  int32_t outer;                        /* outer iterations done                       */
  double norm[RSP_HIST_MAX + 1];        /* |F(x^k)|_2 for k = 0..outer (RASPEN residual) */
  int32_t gmres_its[RSP_HIST_MAX + 1];  /* GMRES products in outer step k (k >= 1)     */
  double gmres_rel[RSP_HIST_MAX + 1];   /* GMRES final relative residual estimate      */
  int32_t inner_min[RSP_HIST_MAX + 1];  /* local Newton iterations of evaluation k     */
  int32_t inner_max[RSP_HIST_MAX + 1];
  double inner_avg[RSP_HIST_MAX + 1];
  int32_t backtracks[RSP_HIST_MAX + 1]; /* step halvings, summed over subdomains       */
  int32_t subdomains;                   /* S                                            */
  int64_t factorizations;               /* local Jacobian factorisations (x subdomains)  */
  int64_t local_solves;                 /* local block solves                           */
  int64_t gmres_total;                  /* matrix-vector products                       */
  int64_t newton_iterations;            /* local Newton iterations, summed over subdomains */
  int64_t jac_applies;                  /* Algorithm 4 applications (GMRES + restarts)   */
  double residual_final;                /* |F_{eps_min}(y, p)|_2 on the global grid      */
  double flops;                         /* algorithmic flops of the solve               */
  double ms_eval, ms_gmres, ms_total;   /* wall time of Algorithm 3 calls, GMRES, total  */
  int32_t fallback_outer;               /* outer step after which the instance switched to
                                           FP64 factors (-1: it did not)                 */
  int32_t snapshots;                    /* states recorded into eps_snapshots           */
  double snapshot_eps[RSP_HIST_MAX + 1];/* eps_k of the local solves at snapshot k      */
} rsp_history;

typedef struct rsp_context rsp_context;

/* Library version (RSP_VERSION). */
int rsp_version(void);

/* Thread-local message describing the last error ("" if none). */
const char* rsp_last_error(void);

/* Partition of Section 4.2 (host only, no GPU needed).  Writes S (sx*sy), the
   largest overlapping-tile width txm and height tym; if `boxes` is not NULL it
   must hold 8*S int32 and receives per subdomain (row-major over boxes, x fastest):
   x0, x1, y0, y1 of the overlapping box Omega_i and x0, x1, y0, y1 of the
   non-overlapping box Omega~_i, all half-open node ranges.  RSP_EINVAL on a
   problem that leaves a box empty or a tile wider than the library supports. */
int rsp_partition(const rsp_problem* prob, int32_t* S, int32_t* txm, int32_t* tym,
                  int32_t* boxes);

/* Exact device-memory footprint (bytes) of rsp_setup for this problem/options:
   factors, tiles, Krylov basis and state.  The admission key for serving. */
size_t rsp_workspace_bytes(const rsp_problem* prob, const rsp_options* opts);

/* Create / destroy a context on HIP device `device`.  `hbm_budget` (bytes, 0 =
   unlimited) bounds what rsp_setup may allocate (RSP_ENOMEM beyond it). */
int rsp_context_create(rsp_context** ctx, int device, size_t hbm_budget);
int rsp_context_destroy(rsp_context* ctx);

/* Bind a problem to the context: partition, allocate the workspace, copy y_d and
   f (device, [ny][nx]; f may be NULL for f = 0).  Enqueued on `stream`. */
int rsp_setup(rsp_context* ctx, const rsp_problem* prob, const rsp_options* opts,
              const double* yd, const double* f, hipStream_t stream);

/* ---- steps of the hot path (after rsp_setup); tile arrays are [S][2][tym][txm],
   float64, local node (a, b) of subdomain s at [s][field][b][a], entries outside
   the subdomain's own tile zero on output and ignored on input ---- */

/* F_eps(x) on the whole grid (Section 4: the map F(x, eps)): x, out are [2][ny][nx]. */
int rsp_residual(rsp_context* ctx, const double* x, double eps, double* out,
                 hipStream_t stream);

/* u = -(1/nu)(p + mu P_eps(-p/mu)) (stationarity line of eq. (reg_OS)); p, u [ny][nx]. */
int rsp_control(rsp_context* ctx, const double* p, double eps, double* u,
                hipStream_t stream);

/* R_i x for every subdomain (Section 4.2, R_i): x [2][ny][nx] -> tiles. */
int rsp_restrict(rsp_context* ctx, const double* x, double* tiles, hipStream_t stream);

/* out = sum_i P~_i c_i (Section 4.2, P~_i; eq. (RASPEN def)): tiles -> [2][ny][nx]. */
int rsp_prolong(rsp_context* ctx, const double* tiles, double* out, hipStream_t stream);

/* Local residuals K_i(c_i) = R_i F_eps(x + P_i c_i) (eq. (c_i)) -> tiles `out`,
   and |K_i(c_i)|_2 per subdomain -> `norms` (device, S doubles). */
int rsp_local_residual(rsp_context* ctx, const double* x, const double* c, double eps,
                       double* out, double* norms, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
   tight serving loops, harnesses that forbid hipMalloc): rsp_local_residual without a
   context and without any allocation.  The problem `prob` is partitioned as in
   rsp_partition; yd (required), f (NULL: 0) are [ny][nx], x is [2][ny][nx], c, out
   are tiles [S][2][tym][txm] (tym, txm from rsp_partition) and norms gets S doubles;
   all device pointers on the current device, caller-owned.  The results are those of
   rsp_local_residual on a context set up with the same problem and data.  The staging
   (the instance's constants, the boxes and the halo tiles of R_i x) lives in a
   library-owned device array of 32 MiB on each device, held until the process ends:
   RSP_EINVAL when a problem needs more (S (txm + 2)(tym + 2) * 16 bytes plus the
   tables), or for a tile wider than the supported one.  Stream-ordered; calls that
   overlap on one device (another stream, another host thread) share the array and
   race.  Calls no hipMalloc or hipFree. */
int rsp_local_residual_noalloc(const rsp_problem* prob, const double* yd, const double* f, const double* x,
                               const double* c, double eps, double* out, double* norms, hipStream_t stream);

/* Local linear solves z_i = J_i^{-1} r_i with J_i = R_i F'_eps(x + P_i c_i) P_i
   (eq. (DerC) and the local Newton systems of Algorithm 1), by block-tridiagonal
   LU over grid lines.  c, rhs, z: tiles. */
int rsp_local_solve(rsp_context* ctx, const double* x, const double* c, double eps,
                    const double* rhs, double* z, hipStream_t stream);

/* Algorithm 3: F_eps(x) = sum_i P~_i C_i(x) -> out ([2][ny][nx]); stores the
   corrections C_i(x) and the factors of R_i F'_eps(x^(i)) P_i for rsp_jac_apply.
   continuation != 0 runs the local solves from eps0, else from eps_min.
   Returns the worst local status; `norm` (host, nullable) gets |out|_2. */
int rsp_eval(rsp_context* ctx, const double* x, int continuation, double* out,
             double* norm, hipStream_t stream);

/* Algorithm 4: out = F'_eps(x) d for the x of the last rsp_eval ([2][ny][nx]). */
int rsp_jac_apply(rsp_context* ctx, const double* d, double* out, hipStream_t stream);

/* The operator of the two-level outer Newton systems (rsp_options.coarse = 1, which the
   context must have been set up with): out = F'_RAS(x)(d - Q F'(x) d) - Q F'(x) d,
   Q = Z (Z^T F'_eps_min(x) Z)^{-1} Z^T, with x the point of the last rsp_eval (passed
   again here, [2][ny][nx]) and F'_RAS(x) its Jacobian action (Algorithm 4). */
int rsp_coarse_jac_apply(rsp_context* ctx, const double* x, const double* d, double* out, hipStream_t stream);

/* Algorithm 2 (RASPEN with eps-continuation in the local solves): from x^0 =
   (y0, p0) (both NULL for x^0 = 0) to y, p and u = D_eps_min(p), all [ny][nx].
   yd, f as in rsp_setup; `hist` (host, nullable) receives the history.  With
   opts->record_eps_snapshots > 0 the states of the first evaluation's local Newton
   steps are written to opts->eps_snapshots (their eps_k to hist->snapshot_eps). */
int rsp_solve(rsp_context* ctx, const rsp_problem* prob, const rsp_options* opts,
              const double* yd, const double* f, const double* y0, const double* p0,
              double* y, double* p, double* u, rsp_history* hist, hipStream_t stream);

/* The linearly preconditioned comparison method of Section 4.1 (Newton_RAS,eps; with
   opts->continuation == RSP_CONT_NONE, Newton_RAS at eps_min): Algorithm 1 on the
   whole system F_eps(x) = 0 from eps_0 to eps_min.  Each Newton system
   F'_eps(x^k) d = -F_eps(x^k) is solved by GMRES preconditioned from the left with
   one-level restricted additive Schwarz on the partition of Section 4.2,
   M^{-1} = sum_i P~_i (R_i F'_eps(x^k) P_i)^{-1} R_i (local line factors at x^k, FP32
   with RSP_FP32_REFINED); GMRES stops at rtol relative to |M^{-1} F|.  Backtracking
   as in Algorithm 1 (sigma, alpha_min); at most max_outer + 1 Newton steps.
   Arguments, ownership, stream ordering and status codes as rsp_solve; tol_inner,
   max_inner and max_refine are not used.  History: outer = Newton steps,
   norm[k] = |F_eps_k(x^k)|_2, gmres_its[k], gmres_rel[k], backtracks[k]; the inner
   iteration fields and newton_iterations (local solves) are 0. */
int rsp_solve_newton_ras(rsp_context* ctx, const rsp_problem* prob, const rsp_options* opts,
                         const double* yd, const double* f, const double* y0, const double* p0,
                         double* y, double* p, double* u, rsp_history* hist, hipStream_t stream);

/* The unpreconditioned monolithic method of Section 4.1 (Newton_eps; with
   opts->continuation == RSP_CONT_NONE, Newton at eps_min): Algorithm 1 on the whole
   system F_eps(x) = 0 as in rsp_solve_newton_ras, each Newton system solved by GMRES on
   F'_eps(x^k) itself (products with the whole-system Jacobian: the 5-point stencil
   and the pointwise terms).  Arguments, options, history and status codes as
   rsp_solve_newton_ras; precision does not apply (all FP64). */
int rsp_solve_newton(rsp_context* ctx, const rsp_problem* prob, const rsp_options* opts,
                     const double* yd, const double* f, const double* y0, const double* p0,
                     double* y, double* p, double* u, rsp_history* hist, hipStream_t stream);

/* Algorithm 2 for `count` independent instances at once (a batch).  Every launch of
   the hot path covers the subdomains of all instances still iterating, and each
   instance runs its own outer iteration: stopping test, GMRES (in lockstep, a
   converged instance drops out through its own stop flag) and update.  Instance q
   reads probs[q], yd[q], f[q] (f, y0, p0 may be NULL arrays, or hold NULL entries:
   f = 0, x^0 = 0) and writes y[q], p[q], u[q] (device pointers) and hist[q] (host,
   nullable array).  `opts` applies to every instance.  Per-instance reductions
   have a fixed order that depends only on the instance, so an instance's result
   does not depend on the other members of the batch when the batch's padded
   line-block size (16-multiple above twice the widest tile) equals its own.
   Instances that stall with FP32 factors (fallback_rho) finish together, after the
   others, in a layout with FP64 factors.  Returns the largest per-instance status
   (hist[q].status holds each); RSP_ENUMERIC when an instance ended with it (only that
   instance's outputs are undefined); another hard error (< 0) for the whole call.
   The single-problem calls above need rsp_setup again afterwards. */
int rsp_solve_batch(rsp_context* ctx, int count, const rsp_problem* probs, const rsp_options* opts,
                    const double* const* yd, const double* const* f, const double* const* y0,
                    const double* const* p0, double* const* y, double* const* p, double* const* u,
                    rsp_history* hist, hipStream_t stream);

/* Device bytes rsp_solve_batch needs for these problems (0 if one is invalid). */
size_t rsp_batch_workspace_bytes(int count, const rsp_problem* probs, const rsp_options* opts);

/* ---- execution tuning ----
   How a context issues its launches; none of it changes a result (the same kernels
   run in the same order either way, so results are bitwise equal). */
typedef struct rsp_tuning {
  int32_t graphs;      /* 1: the Arnoldi chunks of GMRES and the continuation runs of the
                          local Newton solves are captured once into hipGraphs (per
                          layout, options and launch shape) and replayed; 0: direct
                          stream launches.  Timed sequences (rsp_set_profiling,
                          rsp_set_profiling_sample) are launched directly. */
  int32_t gm_chunk;    /* Arnoldi steps (Jacobian action + orthogonalisation) enqueued
                          between two host reads of the GMRES stop flags, 1..64 (default 32):
                          longer chunks read back less often and waste at most
                          gm_chunk - 1 skipped steps once every instance has stopped */
  int32_t sx, sy;      /* rsp_autotune: suggested subdomain counts for the sample's grid */
  int32_t max_batch;   /* rsp_autotune: instances per batch beyond which throughput no
                          longer grows (copies of the sample) */
  double solves_per_s; /* rsp_autotune: measured throughput of the chosen settings */
  int32_t jac_form;    /* Jacobian action without refinement (Algorithm 4): 0 automatic
                          (one launch of one workgroup per subdomain when the launch's
                          subdomains fill the device's compute units, else two launches
                          of two workgroups per subdomain), 1 always the two launches,
                          2 one launch wherever the factor type allows it (FP64 factors
                          above 80 line unknowns always take two).  Same results. */
} rsp_tuning;

/* Current settings of the context (sx, sy, max_batch, solves_per_s are 0). */
int rsp_get_tuning(rsp_context* ctx, rsp_tuning* out);

/* Apply graphs, gm_chunk and jac_form (the other fields are ignored).  RSP_EINVAL if out
   of range. */
int rsp_set_tuning(rsp_context* ctx, const rsp_tuning* t);

#define RSP_TUNE_PARTITION 1   /* also try other subdomain counts (same overlap)          */
#define RSP_TUNE_BATCH 2       /* also measure batches of copies of the sample             */

/* Autotuner.  Times whole solves of the sample (device inputs yd, f as for rsp_solve)
   on this context: graphs {0, 1} x gm_chunk {4, 8, 16, restart}; with
   RSP_TUNE_PARTITION the subdomain counts whose tiles (with the sample's overlap) fill
   line blocks of 48, 64 or 80 unknowns, which changes the iteration counts but not the
   solution the method converges to (its fixed point solves the global system for any
   partition); with RSP_TUNE_BATCH batches of 1, 2, 4, ... copies up to the first that
   gains less than 5 % (max_batch: the smallest within 5 % of the best).  Applies the
   chosen graphs and gm_chunk to the context and writes everything to `out`.  Results
   are cached per grid, partition, overlap, precision, restart length and flags for
   the life of the process (a cached call measures nothing).  Allocates device memory
   for the trial outputs and replaces the problem bound by rsp_setup.  Errors:
   RSP_EINVAL (bad arguments, or the sample does not converge), RSP_ENOMEM, RSP_EHIP. */
int rsp_autotune(rsp_context* ctx, const rsp_problem* sample, const rsp_options* opts,
                 const double* yd, const double* f, int flags, rsp_tuning* out, hipStream_t stream);

/* ---- serving: continuous batching of solves on one device ----
   A server owns a context, a stream and a worker thread.  Requests are admitted
   first come first served between two outer iterations of the running batch
   (Algorithm 2 steps), while the grown batch fits `hbm_budget` (by
   rsp_batch_workspace_bytes) and `max_batch`; an instance leaves the batch at the
   end of the iteration in which it meets its stopping test.  A request's result
   does not depend on the other requests sharing its batch (see rsp_solve_batch).
   All server calls are thread-safe. */

typedef struct rsp_server rsp_server;

typedef struct rsp_server_options {
  int32_t device;       /* HIP device of the server's context and stream              */
  int32_t max_batch;    /* most instances solved together (0: no limit)               */
  size_t hbm_budget;    /* device bytes for the batch layout (0: no limit)            */
  rsp_options opts;     /* solver options of every request                            */
  rsp_tuning tune;      /* execution settings of the server's context (gm_chunk 0:
                           the defaults); e.g. from rsp_autotune on a typical request */
  int32_t profile_every;  /* 0: no kernel timing; N >= 1: HIP events around the Jacobian
                           action (class "block_solve") in one of every N launch
                           sequences of the main batch, read by rsp_server_kernel_stats */
} rsp_server_options;

#define RSP_TICKET_QUEUED 0
#define RSP_TICKET_RUNNING 1
#define RSP_TICKET_DONE 2

typedef struct rsp_server_report {
  int64_t submitted, completed, failed;   /* requests so far (failed: hard errors)       */
  int64_t queued, running;                /* requests waiting / in the running batch      */
  int64_t steps;                          /* outer iterations run by the worker           */
  double mean_batch;                      /* average instances per outer iteration        */
  double p50_ms, p99_ms, mean_ms;         /* submit-to-done latency of completed requests  */
  double solves_per_s;                    /* completed / (last completion - first submit)  */
} rsp_server_report;

/* Start a server (worker thread, stream, context on opts->device). */
int rsp_server_create(rsp_server** srv, const rsp_server_options* opts);

/* Queue one solve (Algorithm 2 from x^0 = 0).  yd, f (nullable: 0) are device
   arrays [ny][nx] whose data must be ready when this is called; y, p, u receive
   the solution.  All five must stay valid and untouched until the ticket is done.
   Returns at once with `ticket` (host); RSP_EINVAL for a problem that cannot be
   partitioned or laid out. */
int rsp_server_submit(rsp_server* srv, const rsp_problem* prob, const double* yd, const double* f,
                      double* y, double* p, double* u, uint64_t* ticket);

/* Current state of a ticket (RSP_TICKET_*). */
int rsp_server_poll(rsp_server* srv, uint64_t ticket, int32_t* state);

/* Block until the ticket is done (timeout_ms < 0: no limit; RSP_EAGAIN when it
   expires), copy its history into `hist` (host, nullable) and release the ticket.
   Returns the solve status, or the hard error that ended the request (RSP_ENOMEM
   when the problem alone exceeds the budget). */
int rsp_server_wait(rsp_server* srv, uint64_t ticket, double timeout_ms, rsp_history* hist);

/* Counters and latency percentiles (nearest rank) since the server started. */
int rsp_server_stats(rsp_server* srv, rsp_server_report* out);

/* Kernel timing of the main batch since the server started (profile_every > 0; as
   rsp_kernel_stats: up to `max` entries into `out`, their number into `count`),
   settled after each outer iteration of the worker. */
struct rsp_kernel_stat;
int rsp_server_kernel_stats(rsp_server* srv, struct rsp_kernel_stat* out, int max, int32_t* count);

/* Finish every submitted request, then stop the worker and free the server. */
int rsp_server_destroy(rsp_server* srv);

/* ---- kernel timing (HIP events around every launch of the hot-path kernels) ---- */

typedef struct rsp_kernel_stat {
  char name[32];      /* kernel (or GMRES phase) name                               */
  int64_t launches;   /* timed launches since the last reset                        */
  double ms;          /* summed device time between the launch's start/end events    */
  double flops;       /* summed algorithmic flops of those launches                 */
  double bytes;       /* summed algorithmic HBM bytes of those launches             */
} rsp_kernel_stat;

/* Turn event timing on (1) or off (0) for the calls that follow on this context. */
int rsp_set_profiling(rsp_context* ctx, int on);

/* Restrict event timing to one kernel class, named as rsp_kernel_stats names it
   ("block_solve", "factor", "gmres_ortho", ...); NULL or "" times every class.  Each
   timed launch adds two event records to the stream, so timing a single class keeps
   the overhead on the rest of the solve away.  Unknown name: RSP_EINVAL. */
int rsp_set_profiling_filter(rsp_context* ctx, const char* name);

/* Sample the event timing: with timing on, only one in `every` launch sequences
   (a chunk of Arnoldi steps, a run of continuation steps) has its launches timed,
   the first of every `every` from this call on; the other sequences run untimed, and
   are replayed as captured hipGraphs when graphs are on (rsp_tuning).  Launches
   outside such sequences are always timed.  every = 1 (the default) times every
   sequence.  RSP_EINVAL if every < 1. */
int rsp_set_profiling_sample(rsp_context* ctx, int every);

/* Zero the accumulated kernel statistics. */
int rsp_reset_kernel_stats(rsp_context* ctx);

/* Copy up to `max` kernel statistics into `out` (host) and their number into `count`.
   Synchronises with the recorded events. */
int rsp_kernel_stats(rsp_context* ctx, rsp_kernel_stat* out, int max, int32_t* count);

#ifdef __cplusplus
}
#endif
#endif /* RASPEN_H */
