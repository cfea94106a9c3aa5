// Device-side definitions shared by the HIP kernels of the RASPEN library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsp {

constexpr int kBlock = 256;            // threads of the per-subdomain kernels
constexpr int kMaxTile = 48;           // widest overlapping tile (2*48 line unknowns)
constexpr int kMaxM = 2 * kMaxTile;    // largest line block

// Constants of one problem instance in the form the kernels use them.  A batch
// holds several instances; its global arrays are the instances' arrays one after
// the other ([ny][nx] fields at offset noff, [2][ny][nx] states at 2 noff) and
// the tile and factor arrays are laid out per subdomain with one tile geometry
// for the whole batch (txm, tym, M: the same in every instance's record).
struct DevProblem {
  int nx, ny;
  int phi;            // RSP_PHI_*
  double kappa;
  double nu, inv_nu, mu;
  double hx2i, hy2i;  // 1/hx^2, 1/hy^2
  double diag0;       // 2/hx^2 + 2/hy^2
  double dom_w;       // weight of the rows of y in the line factors' dominance test
  // coefficients of A (diagonal tensor): cx = a1 / hx^2 at the x-faces [ny][nx+1], cy =
  // a2 / hy^2 at the y-faces [ny+1][nx], c0 = a0 [ny][nx]; nullptr: A = -Laplacian
  const double* cx;
  const double* cy;
  const double* c0;
  double eps_min, gamma;
  double eps_start;   // eps_0 of the local solves of the next evaluation
  long long noff;     // offset of this instance's [ny][nx] arrays
  int S;              // subdomains of the batch
  int txm, tym;       // largest tile width / height of the batch
  int M;              // padded line-block size (multiple of 16, >= 2*txm)
  // partition and second level: csx x csy cores of width cbx / height cby (the last
  // ones may be narrower); the instance's items are sub0 .. sub0 + csx csy - 1, row-major;
  // offsets of its coarse factors S_r^{-1} and of the dense A0^{-1} in their arrays
  int csx, csy, cbx, cby, sub0;
  long long sinv_off, ainv_off;
};

constexpr int kCoarseMaxNc = 64;   // 2 csx: coarse unknowns of a row of cores (csx <= 32)

// Work list of a per-subdomain launch.  Items are the (instance, subdomain) pairs
// of the batch, numbered consecutively; workgroup b handles item list[b] (or b).
// An item is skipped when skip != nullptr and skip[instance * skip_stride] != 0
// (the GMRES stop flags of the instances, for instance).
struct Items {
  const DevProblem* prob;   // [instances]
  const int* inst;          // [items] instance of the item
  const int4* box;          // [items] overlapping box (x0, x1, y0, y1), half-open
  const int4* core;         // [items] non-overlapping box
  const int* list;          // [count] or nullptr
  const int* skip;
  int skip_stride;
  int count;                // workgroups of the launch
};

// Item of this workgroup and its instance's constants; false when it is skipped.
__device__ __forceinline__ bool item_of(const Items& I, int& s, DevProblem& P) {
  s = I.list ? I.list[blockIdx.x] : (int)blockIdx.x;
  const int i = I.inst[s];
  if (I.skip && I.skip[(size_t)i * I.skip_stride]) return false;
  P = I.prob[i];
  return true;
}

// Outcome of a local Newton solve (SubState::status).
constexpr int kSubOk = 0;
constexpr int kSubNotConverged = 1;   // k_max reached
constexpr int kSubLineSearch = 2;     // backtracking below alpha_min
constexpr int kSubNumeric = 3;        // residual or direction not finite

// Per-subdomain state of the local Newton solve (Algorithm 1).
struct SubState {
  double eps;        // eps_k
  double rnorm;      // |K_{eps_k}(c^k)|_2
  double thresh;     // max(tol, tol_rel |K_{eps_0}(0)|)
  double alpha;      // last accepted step length
  int k;             // iterations done
  int status;        // kSub*
  int active;        // another Newton step is needed
  int backtracks;    // step halvings so far
};

// Device-resident GMRES (restart m <= kGmMaxRestart), one per instance: a small
// header the host reads back for the whole batch in one copy, and the Hessenberg
// matrix with the Givens rotations and the rotated right-hand side.
constexpr int kGmMaxRestart = 64;
constexpr int kGmMaxVec = kGmMaxRestart + 1;
// Reduction blocks of the GMRES vector kernels for an instance of length L: about
// kGmBlockElems elements each, at least kGmMinBlocks and at most kGmBlocks.  A function
// of L alone, so an instance's sums are formed in the same order in any batch.
constexpr int kGmBlocks = 512;
constexpr int kGmMinBlocks = 16;
constexpr long long kGmBlockElems = 1024;
__host__ __device__ inline int gm_blocks(long long L) {
  const long long b = (L + kGmBlockElems - 1) / kGmBlockElems;
  return (int)(b < kGmMinBlocks ? kGmMinBlocks : (b > kGmBlocks ? kGmBlocks : b));
}
struct GmState {
  int m, maxit, steps, used, done, pad;
  double rtol, bnorm, beta, rel;
};
constexpr int kGmDoneStride = sizeof(GmState) / sizeof(int);   // ints between two instances' done flags
struct GmHess {
  double H[(kGmMaxRestart + 1) * kGmMaxRestart];    // H[i * m + j], Givens-rotated columns
  double Hr[(kGmMaxRestart + 1) * kGmMaxRestart];   // the same columns unrotated (Arnoldi relation)
  double hf[2][kGmMaxRestart + 1];                  // first-pass column of the last step (by parity)
  double cs[kGmMaxRestart], sn[kGmMaxRestart], g[kGmMaxRestart + 1];
};
// Segment of one instance in the batch's concatenated global vectors (length L =
// 2 nx ny at offset off).  The Krylov bases are [m+1][ldv]: basis vector k of all
// instances is one concatenated vector.
struct GmSeg {
  long long off, L;
};
// Instances of a GMRES launch: blockIdx.y -> instance list[blockIdx.y] (or blockIdx.y).
struct GmBatch {
  const GmSeg* seg;
  GmState* st;
  GmHess* hs;
  const int* list;
  long long ldv;            // length of the concatenated vectors
  int count;
  int m;
  int nbx;                  // grid width: gm_blocks of the longest instance of the context
};

// ---------------------------------------------------------------- the operator A
// Coupling of node (i, j) to its west / east / south / north neighbour across the face
// between them (a1 / hx^2 or a2 / hy^2), and the diagonal of A at the node.
__device__ __forceinline__ double c_w(const DevProblem& P, int i, int j) {
  return P.cx ? P.cx[(size_t)j * (P.nx + 1) + i] : P.hx2i;
}
__device__ __forceinline__ double c_e(const DevProblem& P, int i, int j) {
  return P.cx ? P.cx[(size_t)j * (P.nx + 1) + i + 1] : P.hx2i;
}
__device__ __forceinline__ double c_s(const DevProblem& P, int i, int j) {
  return P.cx ? P.cy[(size_t)j * P.nx + i] : P.hy2i;
}
__device__ __forceinline__ double c_n(const DevProblem& P, int i, int j) {
  return P.cx ? P.cy[(size_t)(j + 1) * P.nx + i] : P.hy2i;
}
__device__ __forceinline__ double a_diag(const DevProblem& P, int i, int j) {
  if (!P.cx) return P.diag0;
  return c_w(P, i, j) + c_e(P, i, j) + c_s(P, i, j) + c_n(P, i, j) + P.c0[(size_t)j * P.nx + i];
}
// (A v)_ij from the value at the node and its four neighbours (0 beyond the boundary);
// the Laplacian keeps its own expression.
__device__ __forceinline__ double apply_a(const DevProblem& P, int i, int j, double vc, double vw, double ve,
                                          double vs, double vn) {
  if (!P.cx) return P.diag0 * vc - P.hx2i * (vw + ve) - P.hy2i * (vs + vn);
  const double w = c_w(P, i, j), e = c_e(P, i, j), s = c_s(P, i, j), n = c_n(P, i, j);
  return (w + e + s + n + P.c0[(size_t)j * P.nx + i]) * vc - (w * vw + e * ve) - (s * vs + n * vn);
}

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
