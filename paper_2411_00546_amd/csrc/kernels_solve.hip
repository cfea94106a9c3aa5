// Block-tridiagonal solves with the stored line factors (one workgroup per subdomain).
//
// With F_j = S_j^{-1} (stored transposed: facT[s][j][b][a] = F_j[a][b]) and c = 1/hy^2:
//   forward   g_0 = F_0 r_0,  g_j = F_j (r_j + c g_{j-1})
//   backward  z_{ty-1} = g_{ty-1},  z_j = g_j + c F_j z_{j+1}
// (block LU of the local Jacobian, Section 4: x-derivative of F; eq. (DerC)).
//
// Each line is an M x M matrix-vector product that only depends on the previous
// line through the (small) vector, so the matrices are streamed from HBM with
// loads issued two lines ahead of the product that consumes them.  4M threads:
// thread (a2, bg) owns output columns 2a2, 2a2+1 and rows bg*M/8 .. of the line
// matrix (double2 loads, coalesced along a), partial sums are combined in LDS in
// a fixed order.
#include "rsp_kernels.h"

namespace rsp {

namespace {

template <int M>
struct Sweep {
  static constexpr int NT = 4 * M;   // threads
  static constexpr int P2 = M / 2;   // column pairs
  static constexpr int K = M / 8;    // rows per thread per line
};

template <int M>
__device__ __forceinline__ void load_line(const double* __restrict__ F, int a2, int bg,
                                          double2 (&buf)[Sweep<M>::K]) {
  constexpr int K = Sweep<M>::K;
  const double2* p = reinterpret_cast<const double2*>(F) + (size_t)(bg * K) * (M / 2) + a2;
#pragma unroll
  for (int i = 0; i < K; ++i) buf[i] = p[(size_t)i * (M / 2)];
}

// y = F v for one line: partial sums of this thread's rows, then a fixed-order
// reduction over the 8 row groups by threads t < M.  Returns y[t] (t < M).
template <int M>
__device__ __forceinline__ double line_product(const double2 (&buf)[Sweep<M>::K], const double* v,
                                               int a2, int bg, double* red) {
  constexpr int K = Sweep<M>::K;
  double s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const double vb = v[bg * K + i];
    s0 = fma(buf[i].x, vb, s0);
    s1 = fma(buf[i].y, vb, s1);
  }
  red[bg * M + 2 * a2] = s0;
  red[bg * M + 2 * a2 + 1] = s1;
  __syncthreads();
  double y = 0.0;
  const int t = threadIdx.x;
  if (t < M) {
#pragma unroll
    for (int g = 0; g < 8; ++g) y += red[g * M + t];
  }
  return y;
}

// Forward sweep in place on gl[ty][M] (rhs -> g).
template <int M>
__device__ void forward_sweep(const double* __restrict__ Fs, int ty, double c, double* gl,
                              double* red) {
  const int t = threadIdx.x, a2 = t % (M / 2), bg = t / (M / 2);
  const size_t MM = (size_t)M * M;
  double2 b0[Sweep<M>::K], b1[Sweep<M>::K], b2[Sweep<M>::K];
  load_line<M>(Fs, a2, bg, b0);
  load_line<M>(Fs + MM * min(1, ty - 1), a2, bg, b1);
  auto step = [&](const double2(&buf)[Sweep<M>::K], int j) {
    const double y = line_product<M>(buf, gl + (size_t)j * M, a2, bg, red);
    if (t < M) {
      gl[(size_t)j * M + t] = y;
      if (j + 1 < ty) gl[(size_t)(j + 1) * M + t] += c * y;
    }
    __syncthreads();
  };
  for (int j = 0; j < ty; j += 3) {
    load_line<M>(Fs + MM * min(j + 2, ty - 1), a2, bg, b2);
    step(b0, j);
    if (j + 1 >= ty) break;
    load_line<M>(Fs + MM * min(j + 3, ty - 1), a2, bg, b0);
    step(b1, j + 1);
    if (j + 2 >= ty) break;
    load_line<M>(Fs + MM * min(j + 4, ty - 1), a2, bg, b1);
    step(b2, j + 2);
  }
}

// Backward sweep in place on gl (g -> z) for lines ty-2 down to jstop.
template <int M>
__device__ void backward_sweep(const double* __restrict__ Fs, int ty, int jstop, double c,
                               double* gl, double* red) {
  const int t = threadIdx.x, a2 = t % (M / 2), bg = t / (M / 2);
  const size_t MM = (size_t)M * M;
  const int j0 = ty - 2;
  if (j0 < jstop) return;
  double2 b0[Sweep<M>::K], b1[Sweep<M>::K], b2[Sweep<M>::K];
  load_line<M>(Fs + MM * j0, a2, bg, b0);
  load_line<M>(Fs + MM * max(j0 - 1, jstop), a2, bg, b1);
  auto step = [&](const double2(&buf)[Sweep<M>::K], int j) {
    const double y = line_product<M>(buf, gl + (size_t)(j + 1) * M, a2, bg, red);
    if (t < M) gl[(size_t)j * M + t] += c * y;
    __syncthreads();
  };
  for (int j = j0; j >= jstop; j -= 3) {
    load_line<M>(Fs + MM * max(j - 2, jstop), a2, bg, b2);
    step(b0, j);
    if (j - 1 < jstop) break;
    load_line<M>(Fs + MM * max(j - 3, jstop), a2, bg, b0);
    step(b1, j - 1);
    if (j - 2 < jstop) break;
    load_line<M>(Fs + MM * max(j - 4, jstop), a2, bg, b1);
    step(b2, j - 2);
  }
}

template <int M>
__device__ __forceinline__ void tile_to_lines(const DevProblem& P, int s, int tx, int ty,
                                              const double* __restrict__ tile, double* gl) {
  const int m = 2 * tx;
  for (int e = threadIdx.x; e < ty * M; e += Sweep<M>::NT) {
    const int j = e / M, i = e - j * M;
    double v = 0.0;
    if (i < m) {
      const int f = i >= tx;
      v = tile[tile_idx(P, s, f, j, i - f * tx)];
    }
    gl[e] = v;
  }
}

template <int M>
__device__ __forceinline__ void lines_to_tile(const DevProblem& P, int s, int tx, int ty,
                                              const double* gl, double* __restrict__ out) {
  for (int e = threadIdx.x; e < 2 * P.txm * P.tym; e += Sweep<M>::NT) {
    const int f = e / (P.txm * P.tym);
    const int r = e - f * P.txm * P.tym;
    const int b = r / P.txm, a = r - b * P.txm;
    out[tile_idx(P, s, f, b, a)] = (a < tx && b < ty) ? gl[b * M + f * tx + a] : 0.0;
  }
}

template <int M>
__global__ __launch_bounds__(4 * M) void k_block_solve(DevProblem P, const int4* __restrict__ box,
                                                       const double* __restrict__ facT,
                                                       const double* __restrict__ rhs,
                                                       double* __restrict__ out) {
  __shared__ double gl[kMaxTile * M];
  __shared__ double red[8 * M];
  const int s = blockIdx.x;
  const int4 bx = box[s];
  const int tx = bx.y - bx.x, ty = bx.w - bx.z;
  const double* Fs = facT + (size_t)s * P.tym * M * M;
  tile_to_lines<M>(P, s, tx, ty, rhs, gl);
  __syncthreads();
  forward_sweep<M>(Fs, ty, P.hy2i, gl, red);
  backward_sweep<M>(Fs, ty, 0, P.hy2i, gl, red);
  lines_to_tile<M>(P, s, tx, ty, gl, out);
}

// Backward sweep after the factorisation kernel's fused forward sweep (g in gout).
template <int M>
__global__ __launch_bounds__(4 * M) void k_solve_bwd(DevProblem P, const int4* __restrict__ box,
                                                     const SubState* __restrict__ state,
                                                     const double* __restrict__ facT,
                                                     const double* __restrict__ g,
                                                     double* __restrict__ out) {
  __shared__ double gl[kMaxTile * M];
  __shared__ double red[8 * M];
  const int s = blockIdx.x;
  if (state && !state[s].active) return;
  const int4 bx = box[s];
  const int tx = bx.y - bx.x, ty = bx.w - bx.z;
  const double* Fs = facT + (size_t)s * P.tym * M * M;
  for (int e = threadIdx.x; e < ty * M; e += Sweep<M>::NT) gl[e] = g[(size_t)s * P.tym * M + e];
  __syncthreads();
  backward_sweep<M>(Fs, ty, 0, P.hy2i, gl, red);
  lines_to_tile<M>(P, s, tx, ty, gl, out);
}

// Algorithm 4 for one subdomain, fused: right-hand side from the values of d just
// outside the tile (hx^-2 / hy^-2 weights), both sweeps, and out = -d + z on the
// non-overlapping box (every global node is written by exactly one subdomain).
template <int M>
__global__ __launch_bounds__(4 * M) void k_jac_apply(DevProblem P, const int4* __restrict__ box,
                                                     const int4* __restrict__ core,
                                                     const double* __restrict__ facT,
                                                     const double* __restrict__ d,
                                                     double* __restrict__ out,
                                                     const int* __restrict__ skip) {
  __shared__ double gl[kMaxTile * M];
  __shared__ double red[8 * M];
  if (skip && *skip) return;
  const int s = blockIdx.x;
  const int4 bx = box[s], co = core[s];
  const int tx = bx.y - bx.x, ty = bx.w - bx.z;
  const size_t n = (size_t)P.nx * P.ny;
  for (int e = threadIdx.x; e < ty * M; e += Sweep<M>::NT) {
    const int j = e / M, i = e - j * M;
    double v = 0.0;
    if (i < 2 * tx) {
      const int f = i >= tx, a = i - f * tx;
      const int gi = bx.x + a, gj = bx.z + j;
      const double* df = d + f * n;
      if (a == 0 && gi > 0) v += P.hx2i * df[(size_t)gj * P.nx + gi - 1];
      if (a == tx - 1 && gi + 1 < P.nx) v += P.hx2i * df[(size_t)gj * P.nx + gi + 1];
      if (j == 0 && gj > 0) v += P.hy2i * df[(size_t)(gj - 1) * P.nx + gi];
      if (j == ty - 1 && gj + 1 < P.ny) v += P.hy2i * df[(size_t)(gj + 1) * P.nx + gi];
    }
    gl[e] = v;
  }
  __syncthreads();
  const double* Fs = facT + (size_t)s * P.tym * M * M;
  forward_sweep<M>(Fs, ty, P.hy2i, gl, red);
  backward_sweep<M>(Fs, ty, co.z - bx.z, P.hy2i, gl, red);
  const int cw = co.y - co.x, ch = co.w - co.z;
  for (int e = threadIdx.x; e < 2 * cw * ch; e += Sweep<M>::NT) {
    const int f = e / (cw * ch);
    const int r = e - f * cw * ch;
    const int b = r / cw, a = r - b * cw;
    const int gi = co.x + a, gj = co.z + b;
    const size_t gidx = f * n + (size_t)gj * P.nx + gi;
    out[gidx] = gl[(gj - bx.z) * M + f * tx + (gi - bx.x)] - d[gidx];
  }
}

#define RSP_DISPATCH_M(M_, CALL) \
  switch (M_) {                  \
    case 16: CALL(16); break;    \
    case 32: CALL(32); break;    \
    case 48: CALL(48); break;    \
    case 64: CALL(64); break;    \
    case 80: CALL(80); break;    \
    case 96: CALL(96); break;    \
    default: break;              \
  }

}  // namespace

void launch_solve_bwd(const DevProblem& P, const int4* box, const SubState* state,
                      const double* facT, const double* g, double* out, hipStream_t st) {
#define RSP_CALL(MM) k_solve_bwd<MM><<<P.S, 4 * MM, 0, st>>>(P, box, state, facT, g, out)
  RSP_DISPATCH_M(P.M, RSP_CALL)
#undef RSP_CALL
}

void launch_block_solve(const DevProblem& P, const int4* box, const double* facT,
                        const double* rhs, double* out, hipStream_t st) {
#define RSP_CALL(MM) k_block_solve<MM><<<P.S, 4 * MM, 0, st>>>(P, box, facT, rhs, out)
  RSP_DISPATCH_M(P.M, RSP_CALL)
#undef RSP_CALL
}

void launch_jac_apply(const DevProblem& P, const int4* box, const int4* core, const double* facT,
                      const double* d, double* out, const int* skip, hipStream_t st) {
#define RSP_CALL(MM) k_jac_apply<MM><<<P.S, 4 * MM, 0, st>>>(P, box, core, facT, d, out, skip)
  RSP_DISPATCH_M(P.M, RSP_CALL)
#undef RSP_CALL
}

}  // namespace rsp
