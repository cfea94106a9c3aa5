// Block-tridiagonal solves with the stored line factors (twisted form).
//
// Lines 0 .. ty-1 of a tile, twist line t = ty / 2, c = 1/hy^2 (with variable
// coefficients of A, c is the diagonal of a2 / hy^2 on the faces between the two lines).  The factors are the
// inverses F_j of the two-ended Schur complements (kernels_factor.hip): S_j from the
// top (j < t), T_j from the bottom (j > t) and Z_t at the twist, stored transposed
// (facT[s][j][b][a] = F_j[a][b]).  A solve J z = r is
//   inward   g_0 = F_0 r_0,  g_j = F_j (r_j + c g_{j-1})            (j < t)
//            h_{ty-1} = F_{ty-1} r_{ty-1},  h_j = F_j (r_j + c h_{j+1})   (j > t)
//   twist    z_t = F_t (r_t + c g_{t-1} + c h_{t+1})
//   outward  z_j = g_j + c F_j z_{j+1} (j < t),  z_j = h_j + c F_j z_{j-1} (j > t)
// (block LU of the local Jacobian, Section 4: x-derivative of F; eq. (DerC)).  The two
// halves are independent until the twist, so the Jacobian action runs them side by side
// in the two halves of one workgroup per subdomain (k_apply_one), which meet at the
// twist line in LDS.  With fewer subdomains than compute units, and with FP64 factors
// above M = 80 (whose registers that workgroup would spill heavily), they run in two
// workgroups per subdomain instead: one launch for the inward halves, a second one in
// which each workgroup forms the twist line from the first launch's results and sweeps
// its half outward (k_apply_in, k_apply_out).
//
// Each line is an M x M matrix-vector product that only depends on the previous
// line through the (small) vector, so the matrices are streamed from HBM with
// loads issued two lines ahead of the product that consumes them.  4M threads;
// 16-byte loads of W factor entries (double2 or float4), coalesced along the
// output index; partial sums are combined in LDS in a fixed order.  Vectors and
// accumulation are FP64 for both factor types.
//
// Mixed precision (FP32 factors): a local solve is refined in FP64,
//   z <- F^{-1} b;  repeat: r = b - J_i z (J_i applied matrix-free on the tile in
//   FP64, zero outside the tile), z <- z + F^{-1} r.
#include "rsp_kernels.h"

namespace rsp {

namespace {

template <typename TF>
struct Vec;
template <>
struct Vec<double> {
  using type = double2;
  static constexpr int W = 2;
};
template <>
struct Vec<float> {
  using type = float4;
  static constexpr int W = 4;
};

template <typename TF, int M>
struct Sweep {
  using VT = typename Vec<TF>::type;
  static constexpr int W = Vec<TF>::W;
  static constexpr int NT = 4 * M;   // threads
  static constexpr int NC = M / W;   // column groups (one 16-byte load each)
  static constexpr int G = NT / NC;  // row groups
  static constexpr int K = M / G;    // rows per thread per line
};

template <typename TF, int M>
__device__ __forceinline__ void load_line(const TF* __restrict__ F, int ac, int bg,
                                          typename Sweep<TF, M>::VT (&buf)[Sweep<TF, M>::K]) {
  using S = Sweep<TF, M>;
  const typename S::VT* p = reinterpret_cast<const typename S::VT*>(F) + (size_t)(bg * S::K) * S::NC + ac;
#pragma unroll
  for (int i = 0; i < S::K; ++i) buf[i] = p[(size_t)i * S::NC];
}

// y = F v for one line: partial sums of this thread's rows, then a fixed-order
// reduction over the row groups by threads t < M.  Returns y[t] (t < M).
template <typename TF, int M>
__device__ __forceinline__ double line_product(const typename Sweep<TF, M>::VT (&buf)[Sweep<TF, M>::K],
                                               const double* v, int ac, int bg, double* red) {
  using S = Sweep<TF, M>;
  double sum[S::W];
#pragma unroll
  for (int w = 0; w < S::W; ++w) sum[w] = 0.0;
#pragma unroll
  for (int i = 0; i < S::K; ++i) {
    const double vb = v[bg * S::K + i];
    const TF* e = reinterpret_cast<const TF*>(&buf[i]);
#pragma unroll
    for (int w = 0; w < S::W; ++w) sum[w] = fma((double)e[w], vb, sum[w]);
  }
#pragma unroll
  for (int w = 0; w < S::W; ++w) red[bg * M + S::W * ac + w] = sum[w];
  __syncthreads();
  double y = 0.0;
  const int t = threadIdx.x;
  if (t < M) {
#pragma unroll
    for (int g = 0; g < S::G; ++g) y += red[g * M + t];
  }
  return y;
}

// Coupling between consecutive lines of a tile: c times the identity for the Laplacian
// (cy == nullptr), else the diagonal of a2 / hy^2 on the faces between the lines (face k
// lies between local lines k - 1 and k; both fields of a node share its face).
struct Cpl {
  double c;
  const double* cy;
  int nx, gx0, gy0, tx;
  __device__ __forceinline__ double at(int k, int i) const {
    if (!cy) return c;
    if (i >= 2 * tx) return 0.0;   // padding
    const int a = i < tx ? i : i - tx;
    return cy[(size_t)(gy0 + k) * nx + gx0 + a];
  }
};
__device__ __forceinline__ Cpl cpl_of(const DevProblem& P, int4 bx) {
  return Cpl{P.hy2i, P.cx ? P.cy : nullptr, P.nx, bx.x, bx.z, bx.y - bx.x};
}

// Inward sweep over the n lines j0, j0 + dir, ... (dir = +1 or -1), in place on
// gl[ty][M]: gl_j <- F_j gl_j, then c gl_j is added to the next line j + dir (also
// after the last one, where that is the twist line), if it lies in [0, ty).
template <typename TF, int M>
__device__ void sweep_in(const TF* __restrict__ Fs, int ty, int j0, int n, int dir, const Cpl& cp, double* gl,
                         double* red) {
  using S = Sweep<TF, M>;
  if (n <= 0) return;
  const int t = threadIdx.x, ac = t % S::NC, bg = t / S::NC;
  const size_t MM = (size_t)M * M;
  auto line = [&](int k) { return j0 + dir * min(k, n - 1); };
  typename S::VT b0[S::K], b1[S::K], b2[S::K];
  load_line<TF, M>(Fs + MM * line(0), ac, bg, b0);
  load_line<TF, M>(Fs + MM * line(1), ac, bg, b1);
  auto step = [&](const typename S::VT(&buf)[S::K], int k) {
    const int j = j0 + dir * k;
    const double y = line_product<TF, M>(buf, gl + (size_t)j * M, ac, bg, red);
    if (t < M) {
      gl[(size_t)j * M + t] = y;
      const int jn = j + dir;
      if (jn >= 0 && jn < ty) gl[(size_t)jn * M + t] += cp.at(max(j, jn), t) * y;
    }
    __syncthreads();
  };
  for (int k = 0; k < n; k += 3) {
    load_line<TF, M>(Fs + MM * line(k + 2), ac, bg, b2);
    step(b0, k);
    if (k + 1 >= n) break;
    load_line<TF, M>(Fs + MM * line(k + 3), ac, bg, b0);
    step(b1, k + 1);
    if (k + 2 >= n) break;
    load_line<TF, M>(Fs + MM * line(k + 4), ac, bg, b1);
    step(b2, k + 2);
  }
}

// Outward sweep over the n lines j0, j0 + dir, ...: gl_j += F_j (c gl_{j - dir}); vs: M
// doubles of LDS for the scaled vector when the coupling varies along the line.
template <typename TF, int M>
__device__ void sweep_out(const TF* __restrict__ Fs, int j0, int n, int dir, const Cpl& cp, double* gl,
                          double* red, double* vs) {
  using S = Sweep<TF, M>;
  if (n <= 0) return;
  const int t = threadIdx.x, ac = t % S::NC, bg = t / S::NC;
  const size_t MM = (size_t)M * M;
  auto line = [&](int k) { return j0 + dir * min(k, n - 1); };
  typename S::VT b0[S::K], b1[S::K], b2[S::K];
  load_line<TF, M>(Fs + MM * line(0), ac, bg, b0);
  load_line<TF, M>(Fs + MM * line(1), ac, bg, b1);
  auto step = [&](const typename S::VT(&buf)[S::K], int k) {
    const int j = j0 + dir * k, jp = j - dir;
    if (cp.cy) {
      if (t < M) vs[t] = cp.at(max(j, jp), t) * gl[(size_t)jp * M + t];
      __syncthreads();
      const double y = line_product<TF, M>(buf, vs, ac, bg, red);
      if (t < M) gl[(size_t)j * M + t] += y;
    } else {
      const double y = line_product<TF, M>(buf, gl + (size_t)jp * M, ac, bg, red);
      if (t < M) gl[(size_t)j * M + t] += cp.c * y;
    }
    __syncthreads();
  };
  for (int k = 0; k < n; k += 3) {
    load_line<TF, M>(Fs + MM * line(k + 2), ac, bg, b2);
    step(b0, k);
    if (k + 1 >= n) break;
    load_line<TF, M>(Fs + MM * line(k + 3), ac, bg, b0);
    step(b1, k + 1);
    if (k + 2 >= n) break;
    load_line<TF, M>(Fs + MM * line(k + 4), ac, bg, b1);
    step(b2, k + 2);
  }
}

// gl_tw <- F_tw gl_tw (the twist line, its neighbours' terms already added).
template <typename TF, int M>
__device__ void twist_line(const TF* __restrict__ Fs, int tw, double* gl, double* red) {
  using S = Sweep<TF, M>;
  const int t = threadIdx.x, ac = t % S::NC, bg = t / S::NC;
  typename S::VT b0[S::K];
  load_line<TF, M>(Fs + (size_t)M * M * tw, ac, bg, b0);
  const double y = line_product<TF, M>(b0, gl + (size_t)tw * M, ac, bg, red);
  if (t < M) gl[(size_t)tw * M + t] = y;
  __syncthreads();
}

// Whole solve in one workgroup; the outward sweeps stop at lines jlo <= t <= jhi.
template <typename TF, int M>
__device__ void full_solve(const TF* __restrict__ Fs, int ty, int jlo, int jhi, const Cpl& cp, double* gl,
                           double* red, double* vs) {
  const int tw = ty / 2;
  sweep_in<TF, M>(Fs, ty, 0, tw, 1, cp, gl, red);
  sweep_in<TF, M>(Fs, ty, ty - 1, ty - 1 - tw, -1, cp, gl, red);
  twist_line<TF, M>(Fs, tw, gl, red);
  sweep_out<TF, M>(Fs, tw - 1, tw - jlo, -1, cp, gl, red, vs);
  sweep_out<TF, M>(Fs, tw + 1, jhi - tw, 1, cp, gl, red, vs);
}

template <int M>
__device__ __forceinline__ void tile_to_lines(const DevProblem& P, int s, int tx, int ty,
                                              const double* __restrict__ tile, double scale, double* gl) {
  const int m = 2 * tx;
  for (int e = threadIdx.x; e < ty * M; e += 4 * M) {
    const int j = e / M, i = e - j * M;
    double v = 0.0;
    if (i < m) {
      const int f = i >= tx;
      v = scale * tile[tile_idx(P, s, f, j, i - f * tx)];
    }
    gl[e] = v;
  }
}

template <int M>
__device__ __forceinline__ void lines_to_tile(const DevProblem& P, int s, int tx, int ty,
                                              const double* gl, double* __restrict__ out) {
  for (int e = threadIdx.x; e < 2 * P.txm * P.tym; e += 4 * M) {
    const int f = e / (P.txm * P.tym);
    const int r = e - f * P.txm * P.tym;
    const int b = r / P.txm, a = r - b * P.txm;
    out[tile_idx(P, s, f, b, a)] = (a < tx && b < ty) ? gl[b * M + f * tx + a] : 0.0;
  }
}

// rb -= J_i z on the tile (z in line layout, zero outside the tile), J_i the local
// Jacobian at R_i x + c with smoothing eps (FP64, matrix-free 5-point stencil).
template <int M>
__device__ void sub_local_jacobian(const DevProblem& P, int s, int4 bx, int tx, int ty,
                                   const double* __restrict__ tilex, const double* __restrict__ c,
                                   double eps, const double* gl, double* rb) {
  for (int e = threadIdx.x; e < ty * tx; e += 4 * M) {
    const int j = e / tx, a = e - j * tx;
    const double y = tilex[halo_idx(P, s, 0, j + 1, a + 1)] + (c ? c[tile_idx(P, s, 0, j, a)] : 0.0);
    const double p = tilex[halo_idx(P, s, 1, j + 1, a + 1)] + (c ? c[tile_idx(P, s, 1, j, a)] : 0.0);
    // neighbours inside the tile (indices clamped, weights zero outside)
    const double* zl = gl + (size_t)j * M;
    const int al = a > 0 ? a - 1 : a, ar = a + 1 < tx ? a + 1 : a;
    const int jd = j > 0 ? j - 1 : j, ju = j + 1 < ty ? j + 1 : j;
    const double wl = a > 0 ? 1.0 : 0.0, wr = a + 1 < tx ? 1.0 : 0.0;
    const double wd = j > 0 ? 1.0 : 0.0, wu = j + 1 < ty ? 1.0 : 0.0;
    const double* zd = gl + (size_t)jd * M;
    const double* zu = gl + (size_t)ju * M;
    const double zy = zl[a], zp = zl[tx + a];
    double lap_y, lap_p;
    if (!P.cx) {
      lap_y = P.diag0 * zy - P.hx2i * (wl * zl[al] + wr * zl[ar]) - P.hy2i * (wd * zd[a] + wu * zu[a]);
      lap_p = P.diag0 * zp - P.hx2i * (wl * zl[tx + al] + wr * zl[tx + ar]) - P.hy2i * (wd * zd[tx + a] + wu * zu[tx + a]);
    } else {
      const int gi = bx.x + a, gj = bx.z + j;
      const double cw = wl * c_w(P, gi, gj), ce = wr * c_e(P, gi, gj);
      const double cs = wd * c_s(P, gi, gj), cn = wu * c_n(P, gi, gj), dg = a_diag(P, gi, gj);
      lap_y = dg * zy - (cw * zl[al] + ce * zl[ar]) - (cs * zd[a] + cn * zu[a]);
      lap_p = dg * zp - (cw * zl[tx + al] + ce * zl[tx + ar]) - (cs * zd[tx + a] + cn * zu[tx + a]);
    }
    const double dphi = dphi_of(P.phi, y, P.kappa);
    const double jy = lap_y + dphi * zy + dg_of(p, P.mu, eps) * P.inv_nu * zp;
    const double jp = (ddphi_of(P.phi, y, P.kappa) * p - 1.0) * zy + lap_p + dphi * zp;
    rb[(size_t)j * M + a] -= jy;
    rb[(size_t)j * M + tx + a] -= jp;
  }
}

// Right-hand side of Algorithm 4 on the tile, lines [j0, j1): hx^-2 / hy^-2 times the
// values of d just outside the tile (the ring), in line layout.  With the coarse
// correction (ce != nullptr) the ring values are those of d - Z e: each has the coarse
// value e of its node's core and field subtracted (core (gi / cbx, gj / cby) of the
// instance, coarse unknown 2 (sub0 + core) + f).  etab != nullptr: the same values from
// the workgroup's table of the cores its ring touches (apply_coarse_rect: from core
// (ex0, ey0), ew cores wide).
template <int M>
__device__ __forceinline__ void ring_rhs(const DevProblem& P, int4 bx, int tx, int ty, int j0, int j1,
                                         const double* __restrict__ d, const double* __restrict__ ce,
                                         double* gl, int tid, int nthr, const double* etab = nullptr,
                                         int ex0 = 0, int ey0 = 0, int ew = 0) {
  const size_t n = (size_t)P.nx * P.ny;
  d += 2 * P.noff;
  auto val = [&](const double* df, int f, int gi, int gj) {
    double v = df[(size_t)gj * P.nx + gi];
    if (etab) v -= etab[2 * ((gj / P.cby - ey0) * ew + gi / P.cbx - ex0) + f];
    else if (ce) v -= ce[2 * (size_t)(P.sub0 + (gj / P.cby) * P.csx + gi / P.cbx) + f];
    return v;
  };
  for (int e = j0 * M + tid; e < j1 * M; e += nthr) {
    const int j = e / M, i = e - j * M;
    double v = 0.0;
    if (i < 2 * tx) {
      const int f = i >= tx, a = i - f * tx;
      const int gi = bx.x + a, gj = bx.z + j;
      const double* df = d + f * n;
      if (a == 0 && gi > 0) v += c_w(P, gi, gj) * val(df, f, gi - 1, gj);
      if (a == tx - 1 && gi + 1 < P.nx) v += c_e(P, gi, gj) * val(df, f, gi + 1, gj);
      if (j == 0 && gj > 0) v += c_s(P, gi, gj) * val(df, f, gi, gj - 1);
      if (j == ty - 1 && gj + 1 < P.ny) v += c_n(P, gi, gj) * val(df, f, gi, gj + 1);
    }
    gl[e] = v;
  }
}

// out = -d + z on the core nodes of lines [j0, j1) (every global node is written by one
// subdomain: the cores tile the grid).
template <int M>
__device__ __forceinline__ void core_out(const DevProblem& P, int4 bx, int4 co, int tx, int j0, int j1,
                                         const double* gl, const double* __restrict__ d,
                                         double* __restrict__ out, int tid, int nthr) {
  const size_t n = (size_t)P.nx * P.ny;
  const int cw = co.y - co.x;
  const int b0 = max(j0, co.z - bx.z), b1 = min(j1, co.w - bx.z);
  if (b1 <= b0) return;
  const int ch = b1 - b0;
  d += 2 * P.noff;
  out += 2 * P.noff;
  for (int e = tid; e < 2 * cw * ch; e += nthr) {
    const int f = e / (cw * ch);
    const int r = e - f * cw * ch;
    const int b = b0 + r / cw, a = co.x - bx.x + (r % cw);
    const size_t gidx = f * n + (size_t)(bx.z + b) * P.nx + (bx.x + a);
    out[gidx] = gl[b * M + f * tx + a] - d[gidx];
  }
}

template <typename TF, int M>
__global__ __launch_bounds__(4 * M) void k_block_solve(Items I, const TF* __restrict__ facT,
                                                       const double* __restrict__ rhs,
                                                       double* __restrict__ out) {
  __shared__ double gl[kMaxTile * M];
  __shared__ double red[Sweep<TF, M>::G * M];
  __shared__ double vsc[M];
  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  const int4 bx = I.box[s];
  const int tx = bx.y - bx.x, ty = bx.w - bx.z;
  const TF* Fs = facT + (size_t)s * P.tym * M * M;
  tile_to_lines<M>(P, s, tx, ty, rhs, 1.0, gl);
  __syncthreads();
  full_solve<TF, M>(Fs, ty, 0, ty - 1, cpl_of(P, bx), gl, red, vsc);
  lines_to_tile<M>(P, s, tx, ty, gl, out);
}

// Outward half-sweeps after the factorisation kernel's fused inward sweeps and twist
// (g, h and z_t in gout); blockIdx.y = 0: lines t .. 0, 1: lines t+1 .. ty-1.
template <typename TF, int M>
__global__ __launch_bounds__(4 * M) void k_solve_bwd(Items I, const SubState* __restrict__ state,
                                                     const TF* __restrict__ facT,
                                                     const double* __restrict__ g,
                                                     double* __restrict__ out) {
  __shared__ double gl[kMaxTile * M];
  __shared__ double red[Sweep<TF, M>::G * M];
  __shared__ double vsc[M];
  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  if (state && !state[s].active) return;
  const int4 bx = I.box[s];
  const int tx = bx.y - bx.x, ty = bx.w - bx.z, tw = ty / 2;
  const int half = blockIdx.y;
  const int j0 = half == 0 ? 0 : tw, j1 = half == 0 ? tw + 1 : ty;   // lines read
  const TF* Fs = facT + (size_t)s * P.tym * M * M;
  for (int e = j0 * M + threadIdx.x; e < j1 * M; e += 4 * M) gl[e] = g[(size_t)s * P.tym * M + e];
  __syncthreads();
  const Cpl cp = cpl_of(P, bx);
  if (half == 0) sweep_out<TF, M>(Fs, tw - 1, tw, -1, cp, gl, red, vsc);
  else sweep_out<TF, M>(Fs, tw + 1, ty - 1 - tw, 1, cp, gl, red, vsc);
  // tile rows of this half (half 1 also writes the padding rows)
  const int r0 = half == 0 ? 0 : tw + 1, r1 = half == 0 ? tw + 1 : P.tym;
  for (int e = threadIdx.x; e < 2 * P.txm * (r1 - r0); e += 4 * M) {
    const int f = e / (P.txm * (r1 - r0));
    const int r = e - f * P.txm * (r1 - r0);
    const int b = r0 + r / P.txm, a = r % P.txm;
    out[tile_idx(P, s, f, b, a)] = (a < tx && b < ty) ? gl[b * M + f * tx + a] : 0.0;
  }
}

// nref refinement steps of the Newton direction of Algorithm 1:
// dir <- dir + F^{-1}(-K - J dir) with J at the subdomain's current c and eps_k.
template <typename TF, int M>
__global__ __launch_bounds__(4 * M) void k_newton_refine(Items I, const double* __restrict__ tilex,
                                                         const double* __restrict__ c,
                                                         const SubState* __restrict__ state,
                                                         const TF* __restrict__ facT,
                                                         const double* __restrict__ res,
                                                         double* __restrict__ dir, int nref) {
  __shared__ double gl[kMaxTile * M];
  __shared__ double rb[kMaxTile * M];
  __shared__ double red[Sweep<TF, M>::G * M];
  __shared__ double vsc[M];
  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  if (!state[s].active) return;
  const double eps = state[s].eps;
  const int4 bx = I.box[s];
  const int tx = bx.y - bx.x, ty = bx.w - bx.z;
  const TF* Fs = facT + (size_t)s * P.tym * M * M;
  tile_to_lines<M>(P, s, tx, ty, dir, 1.0, gl);
  for (int it = 0; it < nref; ++it) {
    tile_to_lines<M>(P, s, tx, ty, res, -1.0, rb);
    __syncthreads();
    sub_local_jacobian<M>(P, s, bx, tx, ty, tilex, c, eps, gl, rb);
    __syncthreads();
    full_solve<TF, M>(Fs, ty, 0, ty - 1, cpl_of(P, bx), rb, red, vsc);
    for (int e = threadIdx.x; e < ty * M; e += 4 * M) gl[e] += rb[e];
    __syncthreads();
  }
  lines_to_tile<M>(P, s, tx, ty, gl, dir);
}

// Algorithm 4, inward part, two workgroups per subdomain (blockIdx.y: 0 top lines
// 0 .. t-1, 1 bottom lines ty-1 .. t+1): right-hand side from the values of d just
// outside the tile, inward sweep, the half's lines g_j / h_j to gbuf.
template <typename TF, int M>
__global__ __launch_bounds__(4 * M) void k_apply_in(Items I, const TF* __restrict__ facT,
                                                    const double* __restrict__ d, const double* __restrict__ ce,
                                                    double* __restrict__ gbuf) {
  __shared__ double gl[kMaxTile * M];
  __shared__ double red[Sweep<TF, M>::G * M];
  __shared__ double vsc[M];
  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  const int4 bx = I.box[s];
  const int tx = bx.y - bx.x, ty = bx.w - bx.z, tw = ty / 2;
  const int half = blockIdx.y;
  const int j0 = half == 0 ? 0 : tw + 1, j1 = half == 0 ? tw : ty;   // lines of the half
  const TF* Fs = facT + (size_t)s * P.tym * M * M;
  double* gs = gbuf + (size_t)s * P.tym * M;
  ring_rhs<M>(P, bx, tx, ty, j0, j1, d, ce, gl, threadIdx.x, 4 * M);
  __syncthreads();
  const Cpl cp = cpl_of(P, bx);
  if (half == 0) sweep_in<TF, M>(Fs, ty, 0, tw, 1, cp, gl, red);
  else sweep_in<TF, M>(Fs, ty, ty - 1, ty - 1 - tw, -1, cp, gl, red);
  for (int e = j0 * M + threadIdx.x; e < j1 * M; e += 4 * M) gs[e] = gl[e];
}

// Algorithm 4, outward part (blockIdx.y as above; half 0 also owns the twist line):
// both workgroups form z_t = F_t (r_t + c g_{t-1} + c h_{t+1}) from the inward results,
// then sweep outward to the half's last core line; out = -d + z on the core.
template <typename TF, int M>
__global__ __launch_bounds__(4 * M) void k_apply_out(Items I, const TF* __restrict__ facT,
                                                     const double* __restrict__ gbuf,
                                                     const double* __restrict__ d, const double* __restrict__ ce,
                                                     double* __restrict__ out) {
  __shared__ double gl[kMaxTile * M];
  __shared__ double red[Sweep<TF, M>::G * M];
  __shared__ double vsc[M];
  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  const int4 bx = I.box[s], co = I.core[s];
  const int tx = bx.y - bx.x, ty = bx.w - bx.z, tw = ty / 2;
  const int half = blockIdx.y;
  const int clo = co.z - bx.z, chi = co.w - bx.z - 1;   // core lines
  const TF* Fs = facT + (size_t)s * P.tym * M * M;
  const double* gs = gbuf + (size_t)s * P.tym * M;
  const int jlo = half == 0 ? min(clo, tw) : tw + 1;   // lines read back (besides the twist)
  const int jhi = half == 0 ? tw - 1 : max(chi, tw);
  for (int e = jlo * M + threadIdx.x; e < (jhi + 1) * M; e += 4 * M) gl[e] = gs[e];
  ring_rhs<M>(P, bx, tx, ty, tw, tw + 1, d, ce, gl, threadIdx.x, 4 * M);
  __syncthreads();
  const Cpl cp = cpl_of(P, bx);
  for (int i = threadIdx.x; i < M; i += 4 * M) {
    double v = gl[(size_t)tw * M + i];
    if (tw > 0) v += cp.at(tw, i) * gs[(size_t)(tw - 1) * M + i];
    if (tw + 1 < ty) v += cp.at(tw + 1, i) * gs[(size_t)(tw + 1) * M + i];
    gl[(size_t)tw * M + i] = v;
  }
  __syncthreads();
  twist_line<TF, M>(Fs, tw, gl, red);
  if (half == 0) {
    sweep_out<TF, M>(Fs, tw - 1, tw - jlo, -1, cp, gl, red, vsc);
    core_out<M>(P, bx, co, tx, jlo, tw + 1, gl, d, out, threadIdx.x, 4 * M);
  } else {
    sweep_out<TF, M>(Fs, tw + 1, jhi - tw, 1, cp, gl, red, vsc);
    core_out<M>(P, bx, co, tx, tw + 1, jhi + 1, gl, d, out, threadIdx.x, 4 * M);
  }
}

// ---------------------------------------------------------------- one-workgroup action
// Algorithm 4 in one workgroup per subdomain of 8M threads: two halves of 4M threads
// (half 0: lines 0 .. t-1 inward and t-1 .. outward, half 1: lines ty-1 .. t+1 inward and
// t+1 .. outward) run their sweeps side by side.  The halves meet at block barriers, so
// each runs as many steps as the longer one (idle steps load and compute nothing but
// pass the same barriers), and the twist line is formed between the inward and the
// outward sweeps in LDS instead of across two launches.  Every value is formed by the
// same operations in the same order as in k_apply_in / k_apply_out.

// One line product of a half (act: this half has a line at this step): the half's
// threads form their partial sums into their own red, every thread of the block passes
// the barrier, then the half's threads tl < M add the row groups in order.
template <typename TF, int M>
__device__ __forceinline__ double line_product_half(const typename Sweep<TF, M>::VT (&buf)[Sweep<TF, M>::K],
                                                    const double* v, int ac, int bg, int tl, bool act,
                                                    double* red) {
  using S = Sweep<TF, M>;
  if (act) {
    double sum[S::W];
#pragma unroll
    for (int w = 0; w < S::W; ++w) sum[w] = 0.0;
#pragma unroll
    for (int i = 0; i < S::K; ++i) {
      const double vb = v[bg * S::K + i];
      const TF* e = reinterpret_cast<const TF*>(&buf[i]);
#pragma unroll
      for (int w = 0; w < S::W; ++w) sum[w] = fma((double)e[w], vb, sum[w]);
    }
#pragma unroll
    for (int w = 0; w < S::W; ++w) red[bg * M + S::W * ac + w] = sum[w];
  }
  __syncthreads();
  double y = 0.0;
  if (act && tl < M) {
#pragma unroll
    for (int g = 0; g < S::G; ++g) y += red[g * M + tl];
  }
  return y;
}

// The inward (out == false) or outward sweep of both halves: this half's n lines from
// j0 in direction dir, nmax (>= n, the same in both halves) steps.  Inward: gl_j <- F_j
// gl_j and c gl_j added to line j + dir unless that is the twist line tw; outward:
// gl_j += F_j (c gl_{j - dir}).
template <typename TF, int M, bool OUT>
__device__ void sweep_half(const TF* __restrict__ Fs, int ty, int tw, int j0, int n, int dir, int nmax,
                           const Cpl& cp, double* gl, double* red, double* vs, int tl) {
  using S = Sweep<TF, M>;
  const int ac = tl % S::NC, bg = tl / S::NC;
  const size_t MM = (size_t)M * M;
  auto line = [&](int k) { return j0 + dir * min(k, n - 1); };
  auto load = [&](int k, typename S::VT(&buf)[S::K]) {
    if (n > 0) load_line<TF, M>(Fs + MM * line(k), ac, bg, buf);
  };
  typename S::VT b0[S::K], b1[S::K], b2[S::K];
  load(0, b0);
  load(1, b1);
  auto step = [&](const typename S::VT(&buf)[S::K], int k) {
    const bool act = k < n;
    const int j = j0 + dir * k;
    if constexpr (!OUT) {
      const double y = line_product_half<TF, M>(buf, gl + (size_t)j * M, ac, bg, tl, act, red);
      if (act && tl < M) {
        gl[(size_t)j * M + tl] = y;
        const int jn = j + dir;
        if (jn >= 0 && jn < ty && jn != tw) gl[(size_t)jn * M + tl] += cp.at(max(j, jn), tl) * y;
      }
    } else {
      const int jp = j - dir;
      if (cp.cy) {
        if (act && tl < M) vs[tl] = cp.at(max(j, jp), tl) * gl[(size_t)jp * M + tl];
        __syncthreads();
        const double y = line_product_half<TF, M>(buf, vs, ac, bg, tl, act, red);
        if (act && tl < M) gl[(size_t)j * M + tl] += y;
      } else {
        const double y = line_product_half<TF, M>(buf, gl + (size_t)jp * M, ac, bg, tl, act, red);
        if (act && tl < M) gl[(size_t)j * M + tl] += cp.c * y;
      }
    }
    __syncthreads();
  };
  for (int k = 0; k < nmax; k += 3) {
    load(k + 2, b2);
    step(b0, k);
    if (k + 1 >= nmax) break;
    load(k + 3, b0);
    step(b1, k + 1);
    if (k + 2 >= nmax) break;
    load(k + 4, b1);
    step(b2, k + 2);
  }
}

// ainv != nullptr: the coarse values of the cores the ring touches are formed here, each
// by one wave in the order of k_coarse_solve, from A0^{-1} and the projection cv.
template <typename TF, int M>
__global__ __launch_bounds__(8 * M) void k_apply_one(Items I, const TF* __restrict__ facT,
                                                     const double* __restrict__ d, const double* __restrict__ ce,
                                                     const double* __restrict__ ainv,
                                                     const double* __restrict__ cv, double* __restrict__ out) {
  using S = Sweep<TF, M>;
  __shared__ double gl[kMaxTile * M];
  __shared__ double red[2 * S::G * M];
  __shared__ double vsc[2 * M];
  __shared__ double etab[kApplyCoarseMax];
  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  const int4 bx = I.box[s], co = I.core[s];
  const int tx = bx.y - bx.x, ty = bx.w - bx.z, tw = ty / 2;
  const int half = threadIdx.x >= 4 * M, tl = threadIdx.x - half * 4 * M;
  const int clo = co.z - bx.z, chi = co.w - bx.z - 1;   // core lines
  const TF* Fs = facT + (size_t)s * P.tym * M * M;
  double* rh = red + half * S::G * M;
  double* vh = vsc + half * M;
  int ex0 = 0, ey0 = 0, ew = 0;
  if (ainv) {
    const int ne = min(apply_coarse_rect(bx, P.nx, P.ny, P.cbx, P.cby, &ex0, &ey0, &ew), kApplyCoarseMax);
    const int N = 2 * P.csx * P.csy;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double* c = cv + 2 * (size_t)P.sub0;
    for (int r = wave; r < ne; r += 8 * M / 64) {
      const int q = r >> 1, f = r & 1;
      const int row = 2 * ((ey0 + q / ew) * P.csx + ex0 + q % ew) + f;
      const double* Ar = ainv + P.ainv_off + (size_t)row * N;
      double acc = 0.0;
#pragma unroll 8
      for (int k = lane; k < N; k += 64) acc += Ar[k] * c[k];
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
      if (lane == 0) etab[r] = acc;
    }
    __syncthreads();
  }
  ring_rhs<M>(P, bx, tx, ty, 0, ty, d, ce, gl, threadIdx.x, 8 * M, ainv ? etab : nullptr, ex0, ey0, ew);
  __syncthreads();
  const Cpl cp = cpl_of(P, bx);
  // inward: half 0 lines 0 .. tw-1, half 1 lines ty-1 .. tw+1
  const int n0 = tw, n1 = ty - 1 - tw;
  sweep_half<TF, M, false>(Fs, ty, tw, half == 0 ? 0 : ty - 1, half == 0 ? n0 : n1, half == 0 ? 1 : -1,
                           max(n0, n1), cp, gl, rh, vh, tl);
  // twist line: z_t = F_t (r_t + c g_{t-1} + c h_{t+1}), by half 0
  if (half == 0 && tl < M) {
    double v = gl[(size_t)tw * M + tl];
    if (tw > 0) v += cp.at(tw, tl) * gl[(size_t)(tw - 1) * M + tl];
    if (tw + 1 < ty) v += cp.at(tw + 1, tl) * gl[(size_t)(tw + 1) * M + tl];
    gl[(size_t)tw * M + tl] = v;
  }
  __syncthreads();
  {
    typename S::VT b0[S::K];
    const int ac = tl % S::NC, bg = tl / S::NC;
    if (half == 0) load_line<TF, M>(Fs + (size_t)M * M * tw, ac, bg, b0);
    const double y = line_product_half<TF, M>(b0, gl + (size_t)tw * M, ac, bg, tl, half == 0, rh);
    if (half == 0 && tl < M) gl[(size_t)tw * M + tl] = y;
    __syncthreads();
  }
  // outward to the core lines: half 0 lines tw-1 .. jlo, half 1 lines tw+1 .. jhi
  const int jlo = min(clo, tw), jhi = max(chi, tw);
  const int m0 = tw - jlo, m1 = jhi - tw;
  sweep_half<TF, M, true>(Fs, ty, tw, half == 0 ? tw - 1 : tw + 1, half == 0 ? m0 : m1, half == 0 ? -1 : 1,
                          max(m0, m1), cp, gl, rh, vh, tl);
  if (half == 0) core_out<M>(P, bx, co, tx, jlo, tw + 1, gl, d, out, tl, 4 * M);
  else core_out<M>(P, bx, co, tx, tw + 1, jhi + 1, gl, d, out, tl, 4 * M);
}

// Algorithm 4 with nref FP64 refinement steps of each local solve (the local Jacobian at
// x^(i) = R_i x + c, eps_min), one workgroup per subdomain.
template <typename TF, int M>
__global__ __launch_bounds__(4 * M) void k_apply_refined(Items I, const TF* __restrict__ facT,
                                                         const double* __restrict__ tilex,
                                                         const double* __restrict__ c,
                                                         const double* __restrict__ d,
                                                         const double* __restrict__ ce,
                                                         double* __restrict__ out, int nref) {
  __shared__ double gl[kMaxTile * M];
  __shared__ double rb[kMaxTile * M];
  __shared__ double red[Sweep<TF, M>::G * M];
  __shared__ double vsc[M];
  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  const int4 bx = I.box[s], co = I.core[s];
  const int tx = bx.y - bx.x, ty = bx.w - bx.z;
  const TF* Fs = facT + (size_t)s * P.tym * M * M;
  ring_rhs<M>(P, bx, tx, ty, 0, ty, d, ce, gl, threadIdx.x, 4 * M);
  __syncthreads();
  const Cpl cp = cpl_of(P, bx);
  full_solve<TF, M>(Fs, ty, 0, ty - 1, cp, gl, red, vsc);
  for (int it = 0; it < nref; ++it) {
    ring_rhs<M>(P, bx, tx, ty, 0, ty, d, ce, rb, threadIdx.x, 4 * M);
    __syncthreads();
    sub_local_jacobian<M>(P, s, bx, tx, ty, tilex, c, P.eps_min, gl, rb);
    __syncthreads();
    full_solve<TF, M>(Fs, ty, 0, ty - 1, cp, rb, red, vsc);
    for (int e = threadIdx.x; e < ty * M; e += 4 * M) gl[e] += rb[e];
    __syncthreads();
  }
  core_out<M>(P, bx, co, tx, 0, ty, gl, d, out, threadIdx.x, 4 * M);
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

void launch_solve_bwd(const Items& I, int M, const SubState* state, const void* facT, int fp32,
                      const double* g, double* out, hipStream_t st) {
  if (I.count <= 0) return;
  const dim3 grid(I.count, 2);
  if (fp32) {
#define RSP_CALL(MM) k_solve_bwd<float, MM><<<grid, 4 * MM, 0, st>>>(I, state, (const float*)facT, g, out)
    RSP_DISPATCH_M(M, RSP_CALL)
#undef RSP_CALL
  } else {
#define RSP_CALL(MM) k_solve_bwd<double, MM><<<grid, 4 * MM, 0, st>>>(I, state, (const double*)facT, g, out)
    RSP_DISPATCH_M(M, RSP_CALL)
#undef RSP_CALL
  }
}

void launch_newton_refine(const Items& I, int M, const double* tilex, const double* c,
                          const SubState* state, const void* facT, int fp32, const double* res,
                          double* dir, int nref, hipStream_t st) {
  if (nref <= 0 || I.count <= 0) return;
  if (fp32) {
#define RSP_CALL(MM) \
  k_newton_refine<float, MM><<<I.count, 4 * MM, 0, st>>>(I, tilex, c, state, (const float*)facT, res, dir, nref)
    RSP_DISPATCH_M(M, RSP_CALL)
#undef RSP_CALL
  } else {
#define RSP_CALL(MM) \
  k_newton_refine<double, MM><<<I.count, 4 * MM, 0, st>>>(I, tilex, c, state, (const double*)facT, res, dir, nref)
    RSP_DISPATCH_M(M, RSP_CALL)
#undef RSP_CALL
  }
}

void launch_block_solve(const Items& I, int M, const void* facT, int fp32, const double* rhs, double* out,
                        hipStream_t st) {
  if (I.count <= 0) return;
  if (fp32) {
#define RSP_CALL(MM) k_block_solve<float, MM><<<I.count, 4 * MM, 0, st>>>(I, (const float*)facT, rhs, out)
    RSP_DISPATCH_M(M, RSP_CALL)
#undef RSP_CALL
  } else {
#define RSP_CALL(MM) k_block_solve<double, MM><<<I.count, 4 * MM, 0, st>>>(I, (const double*)facT, rhs, out)
    RSP_DISPATCH_M(M, RSP_CALL)
#undef RSP_CALL
  }
}

void launch_jac_apply(const Items& I, int M, const void* facT, int fp32, const double* tilex,
                      const double* c, const double* d, const double* ce, double* out, int nref, double* gbuf,
                      bool one_launch, const double* ainv, const double* cv, hipStream_t st) {
  if (I.count <= 0) return;
  const dim3 grid(I.count, 2);
  if (nref > 0) {
#define RSP_REF(TT, MM) \
  k_apply_refined<TT, MM><<<I.count, 4 * MM, 0, st>>>(I, (const TT*)facT, tilex, c, d, ce, out, nref)
    if (fp32) {
#define RSP_CALL(MM) RSP_REF(float, MM)
      RSP_DISPATCH_M(M, RSP_CALL)
#undef RSP_CALL
    } else {
#define RSP_CALL(MM) RSP_REF(double, MM)
      RSP_DISPATCH_M(M, RSP_CALL)
#undef RSP_CALL
    }
#undef RSP_REF
    return;
  }
// one workgroup of 8M threads per subdomain when one_launch; else, and for FP64 factors
// above M = 80 (whose registers the wider workgroup would spill heavily), two launches
// of 4M threads
#define RSP_TWO(TT, MM)                                                                        \
  if (!one_launch || !apply_one_launch(MM, sizeof(TT) == 4)) {                                 \
    k_apply_in<TT, MM><<<grid, 4 * MM, 0, st>>>(I, (const TT*)facT, d, ce, gbuf);              \
    k_apply_out<TT, MM><<<grid, 4 * MM, 0, st>>>(I, (const TT*)facT, gbuf, d, ce, out);        \
  } else {                                                                                     \
    k_apply_one<TT, MM><<<I.count, 8 * MM, 0, st>>>(I, (const TT*)facT, d, ce, ainv, cv, out); \
  }
  if (fp32) {
#define RSP_CALL(MM) RSP_TWO(float, MM)
    RSP_DISPATCH_M(M, RSP_CALL)
#undef RSP_CALL
  } else {
#define RSP_CALL(MM) RSP_TWO(double, MM)
    RSP_DISPATCH_M(M, RSP_CALL)
#undef RSP_CALL
  }
#undef RSP_TWO
}

}  // namespace rsp
