// Host-side launchers of the RASPEN HIP kernels (one declaration per kernel).
#pragma once
#include <hip/hip_runtime.h>
#include "rsp_device.h"

namespace rsp {

// a2: halo tiles of R_i x ([S][2][tym+2][txm+2]; nodes outside the grid are 0).
void launch_restrict_halo(const DevProblem& P, const int4* box, const double* x,
                          double* tilex, hipStream_t st);
// R_i x without halo ([S][2][tym][txm]).
void launch_restrict(const DevProblem& P, const int4* box, const double* x, double* tiles,
                     hipStream_t st);
// a7: out[core of s] = tiles[s] (every node written once: the cores tile the grid).
// If d != nullptr: out = -d + (that), the assembly of Algorithm 4.
void launch_prolong(const DevProblem& P, const int4* box, const int4* core, const double* tiles,
                    const double* d, double* out, hipStream_t st);
// a3: K_i(c) at `eps` (per subdomain from state if eps < 0), tiles -> out, norms[s].
void launch_local_residual(const DevProblem& P, const int4* box, const double* tilex,
                           const double* yd, const double* f, const double* c, double eps,
                           double* out, double* norms, hipStream_t st);
// Algorithm 1 start: c = 0, residual at eps0, threshold, active flags.
void launch_newton_init(const DevProblem& P, const int4* box, const double* tilex,
                        const double* yd, const double* f, double* c, double* res,
                        SubState* state, double eps0, double tol, int kmax, hipStream_t st);
// a6: backtracking on |K|, update c and eps, new residual, stopping test.
void launch_linesearch(const DevProblem& P, const int4* box, const double* tilex,
                       const double* yd, const double* f, double* c, const double* dir,
                       double* res, SubState* state, double sigma, double alpha_min, int kmax,
                       hipStream_t st);
// a9: ring right-hand side h^-2 (outside neighbours of d) per tile.
void launch_ring_rhs(const DevProblem& P, const int4* box, const double* d, double* rhs,
                     hipStream_t st);
// a4 (+ fused forward sweep when rhs != nullptr): block-tridiagonal factors S_j^{-1},
// stored as double, or as float when fp32 != 0 (facT points to that type).
void launch_factor(const DevProblem& P, const int4* box, const double* tilex, const double* c,
                   const SubState* state, double eps_fixed, const double* rhs, double rhs_scale,
                   void* facT, int fp32, double* g, hipStream_t st);
// a5: backward sweep after a fused forward sweep.
void launch_solve_bwd(const DevProblem& P, const int4* box, const SubState* state, const void* facT,
                      int fp32, const double* g, double* out, hipStream_t st);
// Refinement of the Newton direction: nref steps dir += F^{-1}(-res - J dir) (FP64 J).
void launch_newton_refine(const DevProblem& P, const int4* box, const double* tilex, const double* c,
                          const SubState* state, const void* facT, int fp32, const double* res,
                          double* dir, int nref, hipStream_t st);
// a5: forward + backward sweeps with stored factors (tile rhs -> tile out).
void launch_block_solve(const DevProblem& P, const int4* box, const void* facT, int fp32,
                        const double* rhs, double* out, hipStream_t st);
// a9 (Algorithm 4), fused: ring rhs of d, both sweeps (+ nref FP64 refinement steps with
// the local Jacobian at R_i x + c), out = -d + sum_i P~_i z_i.  `skip` (nullable,
// device): the launch does nothing when *skip != 0.
void launch_jac_apply(const DevProblem& P, const int4* box, const int4* core, const void* facT, int fp32,
                      const double* tilex, const double* c, const double* d, double* out,
                      const int* skip, int nref, hipStream_t st);
// Section 4 F(x, eps) on the whole grid and the control u(p).
void launch_global_residual(const DevProblem& P, const double* yd, const double* f,
                            const double* x, double eps, double* out, hipStream_t st);
void launch_control(const DevProblem& P, const double* p, double eps, double* u, hipStream_t st);

// GMRES vector kernels (length L), deterministic two-stage reductions.
int multidot_blocks(size_t L);
void launch_multidot(const double* V, size_t ldv, int nvec, const double* w, size_t L,
                     double* partial, hipStream_t st);
void launch_reduce_partials(const double* partial, int nblk, int nvec, double* out,
                            int accumulate, hipStream_t st);
void launch_axpy_multi(const double* V, size_t ldv, int nvec, const double* h, double* w,
                       size_t L, hipStream_t st);
void launch_scale_by_inv_sqrt(const double* w, const double* sumsq, double* out, size_t L,
                              hipStream_t st);
void launch_axpy(double a, const double* x, double* y, size_t L, hipStream_t st);
void launch_scale(double a, const double* x, double* y, size_t L, hipStream_t st);
void launch_combine(const double* V, size_t ldv, int k, const double* y, double* x, size_t L,
                    hipStream_t st);

// Device-resident GMRES (kernels_gmres.hip).
void gm_init_state(GmState* st_dev, int m, int maxit, double rtol, hipStream_t s);
void launch_gm_sumsq(const double* v, size_t L, double* partial, hipStream_t s);
void launch_gm_residual(const double* b, const double* w, double* r, size_t L, hipStream_t s);
void launch_gm_start(double* V0, size_t L, const double* r, GmState* st, const double* partial,
                     int first_cycle, hipStream_t s);
void launch_gm_arnoldi(const double* V, size_t L, int j, double* w, GmState* st, double* p1,
                       double* p2, hipStream_t s);
void launch_gm_update_x(const double* V, size_t L, GmState* st, double* x, hipStream_t s);

}  // namespace rsp
