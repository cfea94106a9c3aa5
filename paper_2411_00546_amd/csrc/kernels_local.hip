// Per-subdomain kernels of the RASPEN hot path (one workgroup per subdomain):
// restriction R_i with halo, local residual K_i (5-point stencil + phi + the
// smoothed soft-threshold), Algorithm 1 line search / eps update, prolongation
// P~_i, and the ring right-hand side of the RASPEN Jacobian (Algorithm 4).
#include "rsp_kernels.h"

namespace rsp {

namespace {

constexpr int kHalo = kMaxTile + 2;   // LDS stride of a staged tile with halo

__device__ __forceinline__ int4 tile_box(const int4* box, int s, int& tx, int& ty) {
  const int4 b = box[s];
  tx = b.y - b.x;
  ty = b.w - b.z;
  return b;
}

// Stage z = R_i x (+ c + alpha dir on the tile interior) into LDS, halo included.
// Returns true in a thread that staged a correction c + alpha dir that is not finite.
__device__ bool stage(const DevProblem& P, int s, int tx, int ty, const double* __restrict__ tilex,
                      const double* __restrict__ c, const double* __restrict__ dir, double alpha,
                      double* z) {
  const int W = tx + 2, H = ty + 2;
  bool nonfinite = false;
  for (int e = threadIdx.x; e < 2 * W * H; e += kBlock) {
    const int f = e / (W * H);
    const int r = e - f * W * H;
    const int b = r / W, a = r - b * W;
    double v = tilex[halo_idx(P, s, f, b, a)];
    if (c && a >= 1 && a <= tx && b >= 1 && b <= ty) {
      double cv = c[tile_idx(P, s, f, b - 1, a - 1)];
      if (dir) cv = cv + alpha * dir[tile_idx(P, s, f, b - 1, a - 1)];
      nonfinite = nonfinite || !isfinite(cv);
      v = v + cv;
    }
    z[(f * kHalo + b) * kHalo + a] = v;
  }
  return nonfinite;
}

// K_i at local node (a, b) from the staged tile: the two rows of F_eps (Section 4).
// (gi, gj): the node on the grid.
__device__ __forceinline__ void node_residual(const DevProblem& P, const double* z, int a, int b, int gi,
                                              int gj, double ydv, double fv, double eps, double& ky,
                                              double& kp) {
  const double* zy = z;
  const double* zp = z + kHalo * kHalo;
  const int c0 = (b + 1) * kHalo + (a + 1);
  const double y = zy[c0], p = zp[c0];
  const double lap_y = apply_a(P, gi, gj, y, zy[c0 - 1], zy[c0 + 1], zy[c0 - kHalo], zy[c0 + kHalo]);
  const double lap_p = apply_a(P, gi, gj, p, zp[c0 - 1], zp[c0 + 1], zp[c0 - kHalo], zp[c0 + kHalo]);
  ky = lap_y + phi_of(P.phi, y, P.kappa) - fv + g_of(p, P.mu, eps) * P.inv_nu;
  kp = lap_p + dphi_of(P.phi, y, P.kappa) * p - y + ydv;
}

// Sum of squares of K_i over the tile; optionally writes K_i to `out`.
__device__ double tile_residual(const DevProblem& P, int s, int4 bx, int tx, int ty,
                                const double* z, const double* __restrict__ yd,
                                const double* __restrict__ f, double eps, double* out,
                                double* red) {
  double acc = 0.0;
  for (int e = threadIdx.x; e < tx * ty; e += kBlock) {
    const int b = e / tx, a = e - b * tx;
    const size_t gi = (size_t)(bx.z + b) * P.nx + (bx.x + a);
    double ky, kp;
    node_residual(P, z, a, b, bx.x + a, bx.z + b, yd[gi], f ? f[gi] : 0.0, eps, ky, kp);
    if (out) {
      out[tile_idx(P, s, 0, b, a)] = ky;
      out[tile_idx(P, s, 1, b, a)] = kp;
    }
    acc += ky * ky + kp * kp;
  }
  return block_sum(acc, red);
}

__global__ __launch_bounds__(kBlock) void k_restrict_halo(Items I, const double* __restrict__ x,
                                                          double* __restrict__ tilex) {
  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  int tx, ty;
  const int4 bx = tile_box(I.box, s, tx, ty);
  const int W = P.txm + 2, H = P.tym + 2;
  const size_t n = (size_t)P.nx * P.ny;
  x += 2 * P.noff;
  for (int e = threadIdx.x; e < 2 * W * H; e += kBlock) {
    const int f = e / (W * H);
    const int r = e - f * W * H;
    const int b = r / W, a = r - b * W;
    const int gi = bx.x - 1 + a, gj = bx.z - 1 + b;
    double v = 0.0;
    if (a <= tx + 1 && b <= ty + 1 && gi >= 0 && gi < P.nx && gj >= 0 && gj < P.ny)
      v = x[f * n + (size_t)gj * P.nx + gi];
    tilex[halo_idx(P, s, f, b, a)] = v;
  }
}

__global__ __launch_bounds__(kBlock) void k_restrict(Items I, const double* __restrict__ x,
                                                     double* __restrict__ tiles) {
  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  int tx, ty;
  const int4 bx = tile_box(I.box, s, tx, ty);
  const size_t n = (size_t)P.nx * P.ny;
  x += 2 * P.noff;
  for (int e = threadIdx.x; e < 2 * P.txm * P.tym; e += kBlock) {
    const int f = e / (P.txm * P.tym);
    const int r = e - f * P.txm * P.tym;
    const int b = r / P.txm, a = r - b * P.txm;
    double v = 0.0;
    if (a < tx && b < ty) v = x[f * n + (size_t)(bx.z + b) * P.nx + (bx.x + a)];
    tiles[tile_idx(P, s, f, b, a)] = v;
  }
}

__global__ __launch_bounds__(kBlock) void k_prolong(Items I, const double* __restrict__ tiles,
                                                    const double* __restrict__ base,
                                                    double* __restrict__ out) {
  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  const int4 bx = I.box[s], co = I.core[s];
  const int cw = co.y - co.x, ch = co.w - co.z;
  const size_t n = (size_t)P.nx * P.ny;
  out += 2 * P.noff;
  if (base) base += 2 * P.noff;
  for (int e = threadIdx.x; e < 2 * cw * ch; e += kBlock) {
    const int f = e / (cw * ch);
    const int r = e - f * cw * ch;
    const int b = r / cw, a = r - b * cw;
    const int gi = co.x + a, gj = co.z + b;
    const size_t g = f * n + (size_t)gj * P.nx + gi;
    const double v = tiles[tile_idx(P, s, f, gj - bx.z, gi - bx.x)];
    out[g] = base ? base[g] + v : v;
  }
}

__global__ __launch_bounds__(kBlock) void k_local_residual(Items I, const double* __restrict__ tilex,
                                                           const double* __restrict__ yd,
                                                           const double* __restrict__ f,
                                                           const double* __restrict__ c, double eps,
                                                           double* __restrict__ out,
                                                           double* __restrict__ norms) {
  __shared__ double z[2 * kHalo * kHalo];
  __shared__ double red[kBlock];
  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  int tx, ty;
  const int4 bx = tile_box(I.box, s, tx, ty);
  // zero the padding of the output tile
  for (int e = threadIdx.x; e < 2 * P.txm * P.tym; e += kBlock) {
    const int fl = e / (P.txm * P.tym);
    const int r = e - fl * P.txm * P.tym;
    const int b = r / P.txm, a = r - b * P.txm;
    if (a >= tx || b >= ty) out[tile_idx(P, s, fl, b, a)] = 0.0;
  }
  stage(P, s, tx, ty, tilex, c, nullptr, 0.0, z);
  __syncthreads();
  const double ss = tile_residual(P, s, bx, tx, ty, z, yd + P.noff, f ? f + P.noff : nullptr, eps,
                                  out, red);
  if (threadIdx.x == 0) norms[s] = sqrt(ss);
}

// Algorithm 1 start at eps_0 = the instance's eps_start: c = 0, residual, threshold
// max(tol, tol_rel |K(0)|).  A residual that is not finite ends the solve (kSubNumeric).
__global__ __launch_bounds__(kBlock) void k_newton_init(Items I, const double* __restrict__ tilex,
                                                        const double* __restrict__ yd,
                                                        const double* __restrict__ f,
                                                        double* __restrict__ c, double* __restrict__ res,
                                                        SubState* __restrict__ state, double tol,
                                                        double tol_rel, int kmax) {
  __shared__ double z[2 * kHalo * kHalo];
  __shared__ double red[kBlock];
  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  int tx, ty;
  const int4 bx = tile_box(I.box, s, tx, ty);
  for (int e = threadIdx.x; e < 2 * P.txm * P.tym; e += kBlock) {
    c[(size_t)s * 2 * P.txm * P.tym + e] = 0.0;
    res[(size_t)s * 2 * P.txm * P.tym + e] = 0.0;
  }
  stage(P, s, tx, ty, tilex, nullptr, nullptr, 0.0, z);
  __syncthreads();
  const double eps0 = P.eps_start;
  const double r = sqrt(tile_residual(P, s, bx, tx, ty, z, yd + P.noff, f + P.noff, eps0, res, red));
  if (threadIdx.x == 0) {
    SubState S;
    S.eps = eps0;
    S.rnorm = r;
    S.thresh = fmax(tol, tol_rel * r);
    S.alpha = 0.0;
    S.k = 0;
    S.backtracks = 0;
    const bool done = (r <= S.thresh) && !(eps0 > P.eps_min);
    S.active = (!done && kmax >= 0) ? 1 : 0;
    S.status = (!done && !S.active) ? kSubNotConverged : kSubOk;
    if (!isfinite(r)) {
      S.active = 0;
      S.status = kSubNumeric;
    }
    state[s] = S;
  }
}

// One Algorithm 1 step after the Newton direction `dir` is known: alpha = 1, 1/2, ...
// until |K_{eps_k}(c + alpha dir)| <= sigma |K_{eps_k}(c)| (a NaN trial is rejected),
// then c += alpha dir, eps_{k+1} = max(gamma eps_k, eps_min), k += 1, new residual,
// and the loop test of Algorithm 1 (with the eps_k = eps_min requirement).  A
// direction that is not finite (a singular local Jacobian: a zero pivot gives an
// infinite inverse) ends the solve with kSubNumeric instead of backtracking.
__global__ __launch_bounds__(kBlock) void k_linesearch(Items I, const double* __restrict__ tilex,
                                                       const double* __restrict__ yd,
                                                       const double* __restrict__ f,
                                                       double* __restrict__ c,
                                                       const double* __restrict__ dir,
                                                       double* __restrict__ res,
                                                       SubState* __restrict__ state, double sigma,
                                                       double alpha_min, int kmax) {
  __shared__ double z[2 * kHalo * kHalo];
  __shared__ double red[kBlock];
  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  SubState S = state[s];
  if (!S.active) return;
  int tx, ty;
  const int4 bx = tile_box(I.box, s, tx, ty);
  yd += P.noff;
  f += P.noff;
  double alpha = 1.0;
  for (;;) {
    const bool nonfinite = stage(P, s, tx, ty, tilex, c, dir, alpha, z);
    if (__syncthreads_or(nonfinite) && alpha == 1.0) {
      if (threadIdx.x == 0) {
        S.status = kSubNumeric;
        S.active = 0;
        state[s] = S;
      }
      return;
    }
    const double rt = sqrt(tile_residual(P, s, bx, tx, ty, z, yd, f, S.eps, nullptr, red));
    if (rt <= sigma * S.rnorm) break;
    alpha *= 0.5;
    S.backtracks += 1;
    if (alpha < alpha_min) {
      if (threadIdx.x == 0) {
        S.status = kSubLineSearch;
        S.active = 0;
        state[s] = S;
      }
      return;
    }
  }
  // accept: c <- c + alpha dir (the staged tile already holds R_i x + c_new)
  for (int e = threadIdx.x; e < tx * ty; e += kBlock) {
    const int b = e / tx, a = e - b * tx;
    for (int fl = 0; fl < 2; ++fl) {
      const size_t i = tile_idx(P, s, fl, b, a);
      c[i] = c[i] + alpha * dir[i];
    }
  }
  S.eps = fmax(P.gamma * S.eps, P.eps_min);
  S.k += 1;
  S.alpha = alpha;
  S.rnorm = sqrt(tile_residual(P, s, bx, tx, ty, z, yd, f, S.eps, res, red));
  const bool done = (S.rnorm <= S.thresh) && !(S.eps > P.eps_min);
  S.active = (!done && S.k <= kmax) ? 1 : 0;
  S.status = (!done && !S.active) ? kSubNotConverged : kSubOk;
  if (!isfinite(S.rnorm)) {
    S.active = 0;
    S.status = kSubNumeric;
  }
  if (threadIdx.x == 0) state[s] = S;
}

__global__ __launch_bounds__(kBlock) void k_ring_rhs(Items I, const double* __restrict__ d,
                                                     double* __restrict__ rhs) {
  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  int tx, ty;
  const int4 bx = tile_box(I.box, s, tx, ty);
  const size_t n = (size_t)P.nx * P.ny;
  d += 2 * P.noff;
  for (int e = threadIdx.x; e < 2 * P.txm * P.tym; e += kBlock) {
    const int f = e / (P.txm * P.tym);
    const int r = e - f * P.txm * P.tym;
    const int b = r / P.txm, a = r - b * P.txm;
    double v = 0.0;
    if (a < tx && b < ty) {
      const int gi = bx.x + a, gj = bx.z + b;
      const double* df = d + f * n;
      if (a == 0 && gi > 0) v += c_w(P, gi, gj) * df[(size_t)gj * P.nx + gi - 1];
      if (a == tx - 1 && gi + 1 < P.nx) v += c_e(P, gi, gj) * df[(size_t)gj * P.nx + gi + 1];
      if (b == 0 && gj > 0) v += c_s(P, gi, gj) * df[(size_t)(gj - 1) * P.nx + gi];
      if (b == ty - 1 && gj + 1 < P.ny) v += c_n(P, gi, gj) * df[(size_t)(gj + 1) * P.nx + gi];
    }
    rhs[tile_idx(P, s, f, b, a)] = v;
  }
}

}  // namespace

void launch_restrict_halo(const Items& I, const double* x, double* tilex, hipStream_t st) {
  if (I.count > 0) k_restrict_halo<<<I.count, kBlock, 0, st>>>(I, x, tilex);
}
void launch_restrict(const Items& I, const double* x, double* tiles, hipStream_t st) {
  if (I.count > 0) k_restrict<<<I.count, kBlock, 0, st>>>(I, x, tiles);
}
void launch_prolong(const Items& I, const double* tiles, const double* base, double* out, hipStream_t st) {
  if (I.count > 0) k_prolong<<<I.count, kBlock, 0, st>>>(I, tiles, base, out);
}
void launch_local_residual(const Items& I, const double* tilex, const double* yd, const double* f,
                           const double* c, double eps, double* out, double* norms, hipStream_t st) {
  if (I.count > 0) k_local_residual<<<I.count, kBlock, 0, st>>>(I, tilex, yd, f, c, eps, out, norms);
}
void launch_newton_init(const Items& I, const double* tilex, const double* yd, const double* f,
                        double* c, double* res, SubState* state, double tol, double tol_rel, int kmax,
                        hipStream_t st) {
  if (I.count > 0)
    k_newton_init<<<I.count, kBlock, 0, st>>>(I, tilex, yd, f, c, res, state, tol, tol_rel, kmax);
}
void launch_linesearch(const Items& I, const double* tilex, const double* yd, const double* f,
                       double* c, const double* dir, double* res, SubState* state, double sigma,
                       double alpha_min, int kmax, hipStream_t st) {
  if (I.count > 0)
    k_linesearch<<<I.count, kBlock, 0, st>>>(I, tilex, yd, f, c, dir, res, state, sigma, alpha_min, kmax);
}
void launch_ring_rhs(const Items& I, const double* d, double* rhs, hipStream_t st) {
  if (I.count > 0) k_ring_rhs<<<I.count, kBlock, 0, st>>>(I, d, rhs);
}

}  // namespace rsp
