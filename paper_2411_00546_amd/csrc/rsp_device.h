// Device-side definitions shared by the HIP kernels of the RASPEN library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsp {

constexpr int kBlock = 256;            // threads of the per-subdomain kernels
constexpr int kMaxTile = 48;           // widest overlapping tile (2*48 line unknowns)
constexpr int kMaxM = 2 * kMaxTile;    // largest line block

// Problem constants in the form the kernels use them (passed by value).
struct DevProblem {
  int nx, ny;
  int phi;            // RSP_PHI_*
  double kappa;
  double nu, inv_nu, mu;
  double hx2i, hy2i;  // 1/hx^2, 1/hy^2
  double diag0;       // 2/hx^2 + 2/hy^2
  double eps_min, gamma;
  int S;              // subdomains
  int txm, tym;       // largest tile width / height
  int M;              // padded line-block size (multiple of 16, >= 2*txm)
};

// Per-subdomain state of the local Newton solve (Algorithm 1).
struct SubState {
  double eps;        // eps_k
  double rnorm;      // |K_{eps_k}(c^k)|_2
  double thresh;     // max(tol, tol |K_{eps_0}(0)|)
  double alpha;      // last accepted step length
  int k;             // iterations done
  int status;        // 0 ok / 1 not converged / 2 line-search failure
  int active;        // another Newton step is needed
  int backtracks;    // step halvings so far
};

// Device-resident GMRES state (restart m <= kGmMaxRestart).
constexpr int kGmMaxRestart = 64;
constexpr int kGmMaxVec = kGmMaxRestart + 1;
constexpr int kGmBlocks = 128;        // fixed reduction blocks of the GMRES vector kernels
struct GmState {
  int m, maxit, steps, used, done, pad;
  double rtol, bnorm, beta, rel;
  double H[(kGmMaxRestart + 1) * kGmMaxRestart];   // H[i * m + j]
  double cs[kGmMaxRestart], sn[kGmMaxRestart], g[kGmMaxRestart + 1];
};

// ---------------------------------------------------------------- pointwise
// P_eps in the cancellation-free form 2t / (sqrt((t+1)^2+eps) + sqrt((t-1)^2+eps))
// (Lemma 3.1, proof of point (i)).
__device__ __forceinline__ double p_eps(double t, double eps) {
  const double a = t + 1.0, b = t - 1.0;
  return 2.0 * t / (sqrt(a * a + eps) + sqrt(b * b + eps));
}

// P'_eps, eq. (smoothProjDer).
__device__ __forceinline__ double dp_eps(double t, double eps) {
  const double a = t + 1.0, b = t - 1.0;
  return 0.5 * (a / sqrt(a * a + eps) - b / sqrt(b * b + eps));
}

// g(p) = p + mu P_eps(-p/mu); mu = 0 gives g = p (the term is bounded by mu).
__device__ __forceinline__ double g_of(double p, double mu, double eps) {
  return mu == 0.0 ? p : p + mu * p_eps(-p / mu, eps);
}

// g'(p) = 1 - P'_eps(-p/mu).
__device__ __forceinline__ double dg_of(double p, double mu, double eps) {
  return mu == 0.0 ? 1.0 : 1.0 - dp_eps(-p / mu, eps);
}

__device__ __forceinline__ double phi_of(int kind, double y, double kappa) {
  switch (kind) {
    case 1: return y * y * y;
    case 2: return exp(y) - 1.0;
    case 3: return kappa * (y * y * y + exp(kappa * y));
    default: return 0.0;
  }
}

__device__ __forceinline__ double dphi_of(int kind, double y, double kappa) {
  switch (kind) {
    case 1: return 3.0 * y * y;
    case 2: return exp(y);
    case 3: return kappa * (3.0 * y * y + kappa * exp(kappa * y));
    default: return 0.0;
  }
}

__device__ __forceinline__ double ddphi_of(int kind, double y, double kappa) {
  switch (kind) {
    case 1: return 6.0 * y;
    case 2: return exp(y);
    case 3: return kappa * (6.0 * y + kappa * kappa * exp(kappa * y));
    default: return 0.0;
  }
}

// ---------------------------------------------------------------- reductions
// Deterministic block sum (fixed tree over kBlock threads); every thread gets it.
__device__ __forceinline__ double block_sum(double v, double* red /* kBlock */) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
#pragma unroll
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (t < w) red[t] = red[t] + red[t + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- layouts
// Tile arrays [S][2][tym][txm]; halo tiles [S][2][tym+2][txm+2].
__device__ __forceinline__ size_t tile_idx(const DevProblem& P, int s, int f, int b, int a) {
  return (((size_t)s * 2 + f) * P.tym + b) * P.txm + a;
}
__device__ __forceinline__ size_t halo_idx(const DevProblem& P, int s, int f, int b, int a) {
  return (((size_t)s * 2 + f) * (P.tym + 2) + b) * (P.txm + 2) + a;
}

}  // namespace rsp
