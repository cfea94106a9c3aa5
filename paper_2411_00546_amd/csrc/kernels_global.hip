// Whole-grid kernels of one instance: F(x, eps) and the control u(p) (Section 4).
#include "rsp_kernels.h"

namespace rsp {

namespace {

constexpr int kVecBlock = 256;

__global__ __launch_bounds__(kVecBlock) void k_global_residual(DevProblem P, const double* __restrict__ yd,
                                                               const double* __restrict__ f,
                                                               const double* __restrict__ x, double eps,
                                                               double* __restrict__ out) {
  const size_t n = (size_t)P.nx * P.ny;
  const double* y = x;
  const double* p = x + n;
  for (size_t g = blockIdx.x * (size_t)kVecBlock + threadIdx.x; g < n;
       g += (size_t)gridDim.x * kVecBlock) {
    const int j = (int)(g / P.nx), i = (int)(g - (size_t)j * P.nx);
    const double yc = y[g], pc = p[g];
    const double yl = i > 0 ? y[g - 1] : 0.0, yr = i + 1 < P.nx ? y[g + 1] : 0.0;
    const double yb = j > 0 ? y[g - P.nx] : 0.0, yt = j + 1 < P.ny ? y[g + P.nx] : 0.0;
    const double pl = i > 0 ? p[g - 1] : 0.0, pr = i + 1 < P.nx ? p[g + 1] : 0.0;
    const double pb = j > 0 ? p[g - P.nx] : 0.0, pt = j + 1 < P.ny ? p[g + P.nx] : 0.0;
    const double lap_y = apply_a(P, i, j, yc, yl, yr, yb, yt);
    const double lap_p = apply_a(P, i, j, pc, pl, pr, pb, pt);
    out[g] = lap_y + phi_of(P.phi, yc, P.kappa) - (f ? f[g] : 0.0) + g_of(pc, P.mu, eps) * P.inv_nu;
    out[n + g] = lap_p + dphi_of(P.phi, yc, P.kappa) * pc - yc + yd[g];
  }
}

// out = F'_eps(x) d on the whole grid of instance `inst`: the Jacobian of the system of
// Section 3.2,
//   [ A + diag phi'(y)        diag g'(p) / nu   ] [d_y]
//   [ diag(phi''(y) p - 1)    A + diag phi'(y)  ] [d_p],
// A the 5-point operator with homogeneous Dirichlet values.  x, d, out are batch
// vectors (the instance's segment at 2 noff) and eps is the instance's eps_start, all
// read through memory, so a captured launch stays valid while the smoothing changes.
// Returns at once when the instance's GMRES has stopped (done flag).
__global__ __launch_bounds__(kVecBlock) void k_global_jac_apply(const DevProblem* __restrict__ prob, int inst,
                                                                const GmState* __restrict__ gst,
                                                                const double* __restrict__ x,
                                                                const double* __restrict__ d,
                                                                double* __restrict__ out) {
  if (gst && gst[inst].done) return;
  const DevProblem P = prob[inst];
  const double eps = P.eps_start;
  const size_t n = (size_t)P.nx * P.ny;
  x += 2 * P.noff;
  d += 2 * P.noff;
  out += 2 * P.noff;
  for (size_t g = blockIdx.x * (size_t)kVecBlock + threadIdx.x; g < n;
       g += (size_t)gridDim.x * kVecBlock) {
    const int j = (int)(g / P.nx), i = (int)(g - (size_t)j * P.nx);
    const double yc = x[g], pc = x[n + g];
    const double* dy = d;
    const double* dp = d + n;
    const double lap_y = apply_a(P, i, j, dy[g], i > 0 ? dy[g - 1] : 0.0, i + 1 < P.nx ? dy[g + 1] : 0.0,
                                 j > 0 ? dy[g - P.nx] : 0.0, j + 1 < P.ny ? dy[g + P.nx] : 0.0);
    const double lap_p = apply_a(P, i, j, dp[g], i > 0 ? dp[g - 1] : 0.0, i + 1 < P.nx ? dp[g + 1] : 0.0,
                                 j > 0 ? dp[g - P.nx] : 0.0, j + 1 < P.ny ? dp[g + P.nx] : 0.0);
    const double a = dphi_of(P.phi, yc, P.kappa);
    out[g] = lap_y + a * dy[g] + dg_of(pc, P.mu, eps) * P.inv_nu * dp[g];
    out[n + g] = (ddphi_of(P.phi, yc, P.kappa) * pc - 1.0) * dy[g] + lap_p + a * dp[g];
  }
}

// Coefficients of A from the caller's layout (a1 [ny][nx+1], a2 [ny+1][nx], a0 [ny][nx])
// into the instance's scaled arrays cx = a1 / hx^2, cy = a2 / hy^2, c0 = a0.
__global__ __launch_bounds__(kVecBlock) void k_coef_load(DevProblem P, const double* __restrict__ src,
                                                         double* __restrict__ cx, double* __restrict__ cy,
                                                         double* __restrict__ c0) {
  const size_t nxf = (size_t)(P.nx + 1) * P.ny, nyf = (size_t)P.nx * (P.ny + 1), n = (size_t)P.nx * P.ny;
  for (size_t g = blockIdx.x * (size_t)kVecBlock + threadIdx.x; g < nxf + nyf + n;
       g += (size_t)gridDim.x * kVecBlock) {
    const double v = src[g];
    if (g < nxf) cx[g] = v * P.hx2i;
    else if (g < nxf + nyf) cy[g - nxf] = v * P.hy2i;
    else c0[g - nxf - nyf] = v;
  }
}

__global__ __launch_bounds__(kVecBlock) void k_control(DevProblem P, const double* __restrict__ p,
                                                       double eps, double* __restrict__ u) {
  const size_t n = (size_t)P.nx * P.ny;
  for (size_t g = blockIdx.x * (size_t)kVecBlock + threadIdx.x; g < n;
       g += (size_t)gridDim.x * kVecBlock)
    u[g] = -g_of(p[g], P.mu, eps) * P.inv_nu;
}

int grid_for(size_t L) {
  size_t g = (L + kVecBlock - 1) / kVecBlock;
  return (int)(g < 2048 ? (g ? g : 1) : 2048);
}

}  // namespace

void launch_global_residual(const DevProblem& P, const double* yd, const double* f,
                            const double* x, double eps, double* out, hipStream_t st) {
  k_global_residual<<<grid_for((size_t)P.nx * P.ny), kVecBlock, 0, st>>>(P, yd, f, x, eps, out);
}
void launch_global_jac_apply(const DevProblem* prob, const DevProblem& P, int inst, const GmState* gst,
                             const double* x, const double* d, double* out, hipStream_t st) {
  k_global_jac_apply<<<grid_for((size_t)P.nx * P.ny), kVecBlock, 0, st>>>(prob, inst, gst, x, d, out);
}
void launch_coef_load(const DevProblem& P, const double* src, double* cx, double* cy, double* c0, hipStream_t st) {
  const size_t tot = (size_t)(P.nx + 1) * P.ny + (size_t)P.nx * (P.ny + 1) + (size_t)P.nx * P.ny;
  k_coef_load<<<grid_for(tot), kVecBlock, 0, st>>>(P, src, cx, cy, c0);
}
void launch_control(const DevProblem& P, const double* p, double eps, double* u, hipStream_t st) {
  k_control<<<grid_for((size_t)P.nx * P.ny), kVecBlock, 0, st>>>(P, p, eps, u);
}
}  // namespace rsp
