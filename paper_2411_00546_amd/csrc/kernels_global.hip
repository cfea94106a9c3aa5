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
    const double lap_y = P.diag0 * yc - P.hx2i * (yl + yr) - P.hy2i * (yb + yt);
    const double lap_p = P.diag0 * pc - P.hx2i * (pl + pr) - P.hy2i * (pb + pt);
    out[g] = lap_y + phi_of(P.phi, yc, P.kappa) - (f ? f[g] : 0.0) + g_of(pc, P.mu, eps) * P.inv_nu;
    out[n + g] = lap_p + dphi_of(P.phi, yc, P.kappa) * pc - yc + yd[g];
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
void launch_control(const DevProblem& P, const double* p, double eps, double* u, hipStream_t st) {
  k_control<<<grid_for((size_t)P.nx * P.ny), kVecBlock, 0, st>>>(P, p, eps, u);
}
}  // namespace rsp
