// Whole-grid kernels: F(x, eps) and the control u(p) (Section 4), and the vector
// kernels of GMRES (dot products with deterministic two-stage reductions).
#include "rsp_kernels.h"

namespace rsp {

namespace {

constexpr int kVecBlock = 256;
constexpr int kMaxVec = 72;   // largest number of simultaneous dot products

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

// partial[blk][i] = sum over this block's chunk of V_i . w  (i < nvec)
__global__ __launch_bounds__(kVecBlock) void k_multidot(const double* __restrict__ V, size_t ldv, int nvec,
                                                        const double* __restrict__ w, size_t L,
                                                        double* __restrict__ partial) {
  __shared__ double red[kVecBlock];
  const size_t chunk = (L + gridDim.x - 1) / gridDim.x;
  const size_t lo = blockIdx.x * chunk;
  const size_t hi = lo + chunk < L ? lo + chunk : L;
  for (int i = 0; i < nvec; ++i) {
    const double* v = V + (size_t)i * ldv;
    double acc = 0.0;
    for (size_t e = lo + threadIdx.x; e < hi; e += kVecBlock) acc += v[e] * w[e];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kVecBlock / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * kMaxVec + i] = red[0];
    __syncthreads();
  }
}

// out[i] (+)= sum_blk partial[blk][i], fixed order.
__global__ void k_reduce_partials(const double* __restrict__ partial, int nblk, int nvec,
                                  double* __restrict__ out, int accumulate) {
  const int i = threadIdx.x;
  if (i >= nvec) return;
  double acc = 0.0;
  for (int b = 0; b < nblk; ++b) acc += partial[(size_t)b * kMaxVec + i];
  out[i] = accumulate ? out[i] + acc : acc;
}

__global__ __launch_bounds__(kVecBlock) void k_axpy_multi(const double* __restrict__ V, size_t ldv, int nvec,
                                                          const double* __restrict__ h,
                                                          double* __restrict__ w, size_t L) {
  __shared__ double hs[kMaxVec];
  if ((int)threadIdx.x < nvec) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  for (size_t e = blockIdx.x * (size_t)kVecBlock + threadIdx.x; e < L;
       e += (size_t)gridDim.x * kVecBlock) {
    double acc = w[e];
    for (int i = 0; i < nvec; ++i) acc -= hs[i] * V[(size_t)i * ldv + e];
    w[e] = acc;
  }
}

__global__ __launch_bounds__(kVecBlock) void k_combine(const double* __restrict__ V, size_t ldv, int k,
                                                       const double* __restrict__ y,
                                                       double* __restrict__ x, size_t L) {
  __shared__ double ys[kMaxVec];
  if ((int)threadIdx.x < k) ys[threadIdx.x] = y[threadIdx.x];
  __syncthreads();
  for (size_t e = blockIdx.x * (size_t)kVecBlock + threadIdx.x; e < L;
       e += (size_t)gridDim.x * kVecBlock) {
    double acc = x[e];
    for (int i = 0; i < k; ++i) acc += ys[i] * V[(size_t)i * ldv + e];
    x[e] = acc;
  }
}

__global__ __launch_bounds__(kVecBlock) void k_scale_by_inv_sqrt(const double* __restrict__ w,
                                                                 const double* __restrict__ sumsq,
                                                                 double* __restrict__ out, size_t L) {
  const double s = 1.0 / sqrt(sumsq[0]);
  for (size_t e = blockIdx.x * (size_t)kVecBlock + threadIdx.x; e < L;
       e += (size_t)gridDim.x * kVecBlock)
    out[e] = w[e] * s;
}

__global__ __launch_bounds__(kVecBlock) void k_axpy(double a, const double* __restrict__ x,
                                                    double* __restrict__ y, size_t L) {
  for (size_t e = blockIdx.x * (size_t)kVecBlock + threadIdx.x; e < L;
       e += (size_t)gridDim.x * kVecBlock)
    y[e] = y[e] + a * x[e];
}

__global__ __launch_bounds__(kVecBlock) void k_scale(double a, const double* __restrict__ x,
                                                     double* __restrict__ y, size_t L) {
  for (size_t e = blockIdx.x * (size_t)kVecBlock + threadIdx.x; e < L;
       e += (size_t)gridDim.x * kVecBlock)
    y[e] = a * x[e];
}

int grid_for(size_t L) {
  size_t g = (L + kVecBlock - 1) / kVecBlock;
  return (int)(g < 2048 ? (g ? g : 1) : 2048);
}

}  // namespace

int multidot_blocks(size_t L) {
  size_t g = (L + 4 * kVecBlock - 1) / (4 * kVecBlock);
  return (int)(g < 512 ? (g ? g : 1) : 512);
}

void launch_global_residual(const DevProblem& P, const double* yd, const double* f,
                            const double* x, double eps, double* out, hipStream_t st) {
  k_global_residual<<<grid_for((size_t)P.nx * P.ny), kVecBlock, 0, st>>>(P, yd, f, x, eps, out);
}
void launch_control(const DevProblem& P, const double* p, double eps, double* u, hipStream_t st) {
  k_control<<<grid_for((size_t)P.nx * P.ny), kVecBlock, 0, st>>>(P, p, eps, u);
}
void launch_multidot(const double* V, size_t ldv, int nvec, const double* w, size_t L,
                     double* partial, hipStream_t st) {
  k_multidot<<<multidot_blocks(L), kVecBlock, 0, st>>>(V, ldv, nvec, w, L, partial);
}
void launch_reduce_partials(const double* partial, int nblk, int nvec, double* out,
                            int accumulate, hipStream_t st) {
  k_reduce_partials<<<1, 128, 0, st>>>(partial, nblk, nvec, out, accumulate);
}
void launch_axpy_multi(const double* V, size_t ldv, int nvec, const double* h, double* w,
                       size_t L, hipStream_t st) {
  k_axpy_multi<<<grid_for(L), kVecBlock, 0, st>>>(V, ldv, nvec, h, w, L);
}
void launch_scale_by_inv_sqrt(const double* w, const double* sumsq, double* out, size_t L,
                              hipStream_t st) {
  k_scale_by_inv_sqrt<<<grid_for(L), kVecBlock, 0, st>>>(w, sumsq, out, L);
}
void launch_axpy(double a, const double* x, double* y, size_t L, hipStream_t st) {
  k_axpy<<<grid_for(L), kVecBlock, 0, st>>>(a, x, y, L);
}
void launch_scale(double a, const double* x, double* y, size_t L, hipStream_t st) {
  k_scale<<<grid_for(L), kVecBlock, 0, st>>>(a, x, y, L);
}
void launch_combine(const double* V, size_t ldv, int k, const double* y, double* x, size_t L,
                    hipStream_t st) {
  k_combine<<<grid_for(L), kVecBlock, 0, st>>>(V, ldv, k, y, x, L);
}

}  // namespace rsp
