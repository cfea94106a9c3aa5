// Host-side launchers of the RASPEN HIP kernels (one declaration per kernel).
// Per-subdomain launchers take a work list (Items) and run one workgroup per
// listed item; M is the batch's padded line-block size.
#pragma once
#include <hip/hip_runtime.h>
#include "rsp_device.h"

namespace rsp {

// a2: halo tiles of R_i x ([S][2][tym+2][txm+2]; nodes outside the grid are 0).
void launch_restrict_halo(const Items& I, const double* x, double* tilex, hipStream_t st);
// R_i x without halo ([S][2][tym][txm]).
void launch_restrict(const Items& I, const double* x, double* tiles, hipStream_t st);
// a7: out[core of s] = tiles[s] (every node written once: the cores tile the grid).
// If base != nullptr: out = base + (that) on the same nodes.
void launch_prolong(const Items& I, const double* tiles, const double* base, double* out, hipStream_t st);
// a3: K_i(c) at `eps`, tiles -> out, norms[s].
void launch_local_residual(const Items& I, const double* tilex, const double* yd, const double* f,
                           const double* c, double eps, double* out, double* norms, hipStream_t st);
// Algorithm 1 start at each instance's eps_start: c = 0, residual, threshold
// max(tol, tol_rel |K(0)|), active flags.
void launch_newton_init(const Items& I, const double* tilex, const double* yd, const double* f,
                        double* c, double* res, SubState* state, double tol, double tol_rel, int kmax,
                        hipStream_t st);
// a6: backtracking on |K|, update c and eps, new residual, stopping test.
void launch_linesearch(const Items& I, const double* tilex, const double* yd, const double* f,
                       double* c, const double* dir, double* res, SubState* state, double sigma,
                       double alpha_min, int kmax, hipStream_t st);
// a9: ring right-hand side h^-2 (outside neighbours of d) per tile.
void launch_ring_rhs(const Items& I, const double* d, double* rhs, hipStream_t st);
// a4 (+ fused forward sweep when rhs != nullptr): block-tridiagonal factors S_j^{-1},
// stored as double, or as float when fp32 != 0 (facT points to that type).  The
// smoothing is state[s].eps (state != nullptr; inactive items are skipped), else
// eps_fixed when > 0, the instance's eps_start when < 0 (each instance its own
// smoothing), else the instance's eps_min.  Two-ended (twisted) block LU with
// the twist at line ty / 2 (a second launch).  fallback: [items] flags, 0 between
// launches (subdomains redone with partial pivoting).
void launch_factor(const Items& I, int M, const double* tilex, const double* c, const SubState* state,
                   double eps_fixed, const double* rhs, double rhs_scale, void* facT, int fp32, double* g,
                   int* fallback, bool var, hipStream_t st);
// a5: outward sweeps after the fused inward sweeps and twist of launch_factor.
void launch_solve_bwd(const Items& I, int M, const SubState* state, const void* facT, int fp32,
                      const double* g, double* out, hipStream_t st);
// Refinement of the Newton direction: nref steps dir += F^{-1}(-res - J dir) (FP64 J).
void launch_newton_refine(const Items& I, int M, const double* tilex, const double* c,
                          const SubState* state, const void* facT, int fp32, const double* res,
                          double* dir, int nref, hipStream_t st);
// a5: forward + backward sweeps with stored factors (tile rhs -> tile out).
void launch_block_solve(const Items& I, int M, const void* facT, int fp32, const double* rhs, double* out,
                        hipStream_t st);
// a9 (Algorithm 4): ring rhs of d, the local solves (+ nref FP64 refinement steps with
// the local Jacobian at R_i x + c), out = -d + sum_i P~_i z_i.  Without refinement one
// launch of one workgroup per subdomain (one_launch, where apply_one_launch allows it),
// else two launches of two workgroups per subdomain (inward halves; twist + outward
// halves); gbuf: [items][tym][M] scratch for the latter.  ce != nullptr: the ring values
// are those of d - Z ce (the coarse correction, kernels_coarse.hip).
// ainv != nullptr (one-launch form only, with ce == nullptr): each workgroup forms the
// coarse values e = A0^{-1} cv of the cores its ring touches itself, in the order of
// launch_coarse_solve (scale 1), from A0^{-1} and the projection cv; the cores of a
// ring span at most kApplyCoarseMax / 2 cores (apply_coarse_rect).
void launch_jac_apply(const Items& I, int M, const void* facT, int fp32, const double* tilex,
                      const double* c, const double* d, const double* ce, double* out, int nref, double* gbuf,
                      bool one_launch, const double* ainv, const double* cv, hipStream_t st);
// Whether the Jacobian action without refinement may run as one launch (else two): at
// 8M threads a workgroup has at most 168 VGPRs; the FP64 sweeps spill 12 bytes per lane
// at M = 80 (still faster than two launches) and 124 at M = 96.
inline bool apply_one_launch(int M, int fp32) { return fp32 || M <= 80; }
// Coarse values held by one workgroup of the one-launch action.
constexpr int kApplyCoarseMax = 32;
// Coarse unknowns (2 per core) of the cores that the one-node ring of box bx touches, on
// an nx x ny grid with cores of cbx x cby nodes: the rectangle of cores from
// (ex0, ey0), ew cores wide.
__host__ __device__ inline int apply_coarse_rect(int4 bx, int nx, int ny, int cbx, int cby, int* ex0, int* ey0,
                                                 int* ew) {
  const int x0 = (bx.x > 0 ? bx.x - 1 : 0) / cbx, x1 = (bx.y < nx ? bx.y : nx - 1) / cbx;
  const int y0 = (bx.z > 0 ? bx.z - 1 : 0) / cby, y1 = (bx.w < ny ? bx.w : ny - 1) / cby;
  *ex0 = x0;
  *ey0 = y0;
  *ew = x1 - x0 + 1;
  return 2 * (x1 - x0 + 1) * (y1 - y0 + 1);
}
// Second level (kernels_coarse.hip).  Coarse vectors have 2 entries (fields) per item.
// Sums over each core of phi'(y), g'(p) / nu, phi''(y) p - 1 at x (eps_min) and, with
// variable coefficients of A, its face couplings and sum of a0: sums[8 items].
// The pointwise blocks of F'(x) of every core node go to pt ([3][ntot]).
void launch_coarse_sums(const Items& I, const double* x, double* sums, double* pt, long long ntot, hipStream_t st);
// cv[2 s + f] = sum over the core of item s of v (mode 0) or F'_eps_min(x) v (mode 1, the
// pointwise blocks from pt as written by launch_coarse_sums at that x).
void launch_coarse_project(const Items& I, int mode, const double* pt, long long ntot, const double* v, double* cv,
                           hipStream_t st);
// Block elimination of A0 = Z^T F' Z per instance of the list: S_r^{-1} into sinv.
void launch_coarse_factor(const DevProblem* prob, const int* list, int count, const GmState* gst,
                          const double* sums, double* sinv, hipStream_t st);
// A0^{-1} densely into ainv (max_n: the largest 2 S of the listed instances).
void launch_coarse_inverse(const DevProblem* prob, const int* list, int count, int max_n, const GmState* gst,
                           const double* sums, const double* sinv, double* ainv, hipStream_t st);
// ev = scale A0^{-1} cv on each listed instance's coarse unknowns.
void launch_coarse_solve(const DevProblem* prob, const int* list, int count, int max_n, const GmState* gst,
                         const double* ainv, const double* cv, double scale, double* ev, hipStream_t st);
// Section 4 F(x, eps) on the whole grid of one instance and its control u(p)
// (pointers at the instance's arrays).
void launch_global_residual(const DevProblem& P, const double* yd, const double* f,
                            const double* x, double eps, double* out, hipStream_t st);
void launch_coef_load(const DevProblem& P, const double* src, double* cx, double* cy, double* c0, hipStream_t st);
void launch_control(const DevProblem& P, const double* p, double eps, double* u, hipStream_t st);
// out = F'_eps(x) d on the whole grid of instance `inst` (batch vectors; eps is the
// instance's eps_start in prob, the device table; P its host copy, for the grid size).
// Nothing is done when gst != nullptr and the instance's GMRES has stopped.
void launch_global_jac_apply(const DevProblem* prob, const DevProblem& P, int inst, const GmState* gst,
                             const double* x, const double* d, double* out, hipStream_t st);

// Device-resident GMRES over the instances of B (kernels_gmres.hip); vectors are the
// batch's concatenated global vectors, V the concatenated Krylov bases.
void launch_gm_init(const GmBatch& B, int maxit, double rtol, hipStream_t s);
void launch_gm_sumsq(const GmBatch& B, const double* v, double* partial, hipStream_t s);
// out[instance] = |v|_2 over the instance's segment (fixed-order reduction).
void launch_gm_norms(const GmBatch& B, const double* v, double* partial, double* out, hipStream_t s);
void launch_gm_residual(const GmBatch& B, const double* b, const double* w, double* r, hipStream_t s);
// y = a x, or y += a x when accumulate != 0
void launch_gm_axpy(const GmBatch& B, double a, const double* x, double* y, int accumulate, hipStream_t s);
void launch_gm_zero(const GmBatch& B, double* x, hipStream_t s);
void launch_gm_start(const GmBatch& B, double* V, const double* r, const double* partial, int first_cycle,
                     hipStream_t s);
// Arnoldi step j on z = A u_j (slot j of V holds u_j after its first Gram-Schmidt
// pass, or V_0): the second pass of u_j gives V_j, the first pass of A V_j gives u_{j+1}
// in slot j + 1 (partial sums in p1, p2).  mode 0: j = 0; 1: finish column j - 1 and
// apply its Givens rotations; 2: column j - 1 was finished by launch_gm_finish.
void launch_gm_arnoldi(const GmBatch& B, double* V, int j, const double* z, double* p1, double* p2,
                       int mode, hipStream_t s);
// End of a chunk of steps ending with j - 1: column j - 1 finished (Givens rotations,
// stopping test).
void launch_gm_finish(const GmBatch& B, const double* V, int j, double* p1, double* p2, hipStream_t s);
void launch_gm_update_x(const GmBatch& B, const double* V, double* x, hipStream_t s);

}  // namespace rsp
