// Second level of RASPEN: a coarse correction for the outer Newton systems.
//
// The paper leaves a second level to future work (end of Section 5.3, Section 6).  The
// one taken here is the hybrid two-level Schwarz preconditioner
//   P2 = Q + M^{-1} (I - F' Q),  Q = Z A0^{-1} Z^T,  A0 = Z^T F'(x) Z,
// with M^{-1} the one-level RAS part of the RASPEN Jacobian and Z the indicators of the
// non-overlapping boxes (cores) per field: the coarse unknown (i, f) is subdomain i's
// core in field f, numbered 2 i + f over the items of the batch.  On the RASPEN Newton
// system it gives the operator
//   d -> F_RAS'(x)(d - Z e) - Z e,  e = A0^{-1} Z^T F'(x) d,
// and, because F_RAS'(x) w = -w - sum_i P~_i J_i^{-1} B_i w with B_i the one-node ring
// outside Omega_i, this is -d - sum_i P~_i J_i^{-1} B_i (d - Z e): the Jacobian action of
// Algorithm 4 whose ring values have the coarse values of their cores subtracted.
//
// A0 is block tridiagonal over the rows of cores: with the 2 sx coarse unknowns of core
// row r (core column c, field f at 2 c + f), the diagonal block T_r holds the sums over
// each core of the pointwise blocks of F' (phi'(y), g'(p) / nu, phi''(y) p - 1) plus the
// 5-point Laplacian summed over cores: 2 (ch hx^-2 + cw hy^-2) on a cw x ch core itself,
// -ch hx^-2 with its left and right neighbours; the coupling between rows r - 1 and r
// is diagonal, -cw hy^-2 for core column c in both fields.  With variable coefficients of
// A the same structure holds with sums over faces: each coupling is minus the sum of
// a_f / h^2 over the faces between the two cores, and the diagonal holds the sum over
// the faces on the core's boundary plus the sum of a0 over the core.  It is factored by block
// elimination with explicit inverses of the Schur complements S_r = T_r - C S_{r-1}^{-1} C
// (Gauss-Jordan, one workgroup per instance), and A0^{-1} is
// formed densely from them (2 S columns in blocks, many workgroups), so that each coarse
// solve in GMRES is one dense product.
#include "rsp_kernels.h"
#include "rsp_mfma.h"

namespace rsp {

namespace {

constexpr int kCoarseThreads = 256;
// per item of the core sums: phi'(y), g'(p)/nu, phi''(y) p - 1, and (variable
// coefficients) the face couplings west, east, south, north and the sum of a0
constexpr int kCSum = 8;
constexpr int kColBlock = 8;            // columns of A0^{-1} per workgroup

// Width of core column c / height of core row r of an instance.
__device__ __forceinline__ int core_w(const DevProblem& P, int c) { return min((c + 1) * P.cbx, P.nx) - c * P.cbx; }
__device__ __forceinline__ int core_h(const DevProblem& P, int r) { return min((r + 1) * P.cby, P.ny) - r * P.cby; }

// Sums over each core of phi'(y), g'(p) / nu and phi''(y) p - 1 at x (eps_min), and
// with variable coefficients the couplings over the core's four sides and its sum of a0.
// The three pointwise values of each node also go to pt ([3][ntot], batch layout), for the
// products with F'(x) of the GMRES solve at this x (the first with a0 added).
__global__ __launch_bounds__(kBlock) void k_coarse_sums(Items I, const double* __restrict__ x,
                                                        double* __restrict__ sums, double* __restrict__ pt,
                                                        long long ntot) {
  __shared__ double red[kBlock];
  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  const int4 co = I.core[s];
  const int cw = co.y - co.x, ch = co.w - co.z;
  const size_t n = (size_t)P.nx * P.ny;
  const double* y = x + 2 * P.noff;
  const double* p = y + n;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int e = threadIdx.x; e < cw * ch; e += kBlock) {
    const int r = e / cw, q = e - r * cw;
    const size_t g = (size_t)(co.z + r) * P.nx + (co.x + q);
    const double yv = y[g], pv = p[g];
    const double va = dphi_of(P.phi, yv, P.kappa);
    const double vb = dg_of(pv, P.mu, P.eps_min) * P.inv_nu;
    const double vc = ddphi_of(P.phi, yv, P.kappa) * pv - 1.0;
    a += va;
    b += vb;
    c += vc;
    const size_t o = (size_t)P.noff + g;
    // the diagonal of the pointwise blocks for the products: phi'(y), plus a0 of A
    pt[o] = P.cx ? va + P.c0[g] : va;
    pt[(size_t)ntot + o] = vb;
    pt[2 * (size_t)ntot + o] = vc;
  }
  a = block_sum(a, red);
  b = block_sum(b, red);
  c = block_sum(c, red);
  double* o = sums + kCSum * (size_t)s;
  if (threadIdx.x == 0) {
    o[0] = a;
    o[1] = b;
    o[2] = c;
  }
  if (P.cx) {
    double w = 0.0, e = 0.0, so = 0.0, no = 0.0, z = 0.0;
    for (int r = threadIdx.x; r < ch; r += kBlock) {
      w += c_w(P, co.x, co.z + r);
      e += c_e(P, co.y - 1, co.z + r);
    }
    for (int q = threadIdx.x; q < cw; q += kBlock) {
      so += c_s(P, co.x + q, co.z);
      no += c_n(P, co.x + q, co.w - 1);
    }
    for (int el = threadIdx.x; el < cw * ch; el += kBlock) {
      const int r = el / cw, q = el - r * cw;
      z += P.c0[(size_t)(co.z + r) * P.nx + co.x + q];
    }
    w = block_sum(w, red);
    e = block_sum(e, red);
    so = block_sum(so, red);
    no = block_sum(no, red);
    z = block_sum(z, red);
    if (threadIdx.x == 0) {
      o[3] = w;
      o[4] = e;
      o[5] = so;
      o[6] = no;
      o[7] = z;
    }
  }
}

// c[2 s + f] = sum over the core of item s of v (mode 0) or of (F'_eps_min(x) v) (mode 1,
// with the pointwise blocks of F'(x) from pt, written by k_coarse_sums at this x), field f.
// Summed over a core, the 5-point operator telescopes: each face between two nodes of
// the core adds c (v_a - v_b) + c (v_b - v_a) = 0, so only the faces on the core's
// boundary remain, c (v_inside - v_outside) with v = 0 beyond the grid; the a0 part of
// A is in the first pointwise value.
__global__ __launch_bounds__(kBlock) void k_coarse_project(Items I, int mode, const double* __restrict__ pt,
                                                           long long ntot, const double* __restrict__ v,
                                                           double* __restrict__ cv) {
  __shared__ double red[kBlock];
  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  const int4 co = I.core[s];
  const int cw = co.y - co.x, ch = co.w - co.z;
  const size_t n = (size_t)P.nx * P.ny;
  const double* vy = v + 2 * P.noff;
  const double* vp = vy + n;
  double ay = 0.0, ap = 0.0;
  for (int e = threadIdx.x; e < cw * ch; e += kBlock) {
    const int r = e / cw, q = e - r * cw;
    const int i = co.x + q, j = co.z + r;
    const size_t g = (size_t)j * P.nx + i;
    if (mode == 0) {
      ay += vy[g];
      ap += vp[g];
      continue;
    }
    const double dy = vy[g], dp = vp[g];
    const size_t o = (size_t)P.noff + g;
    const double d1 = pt[o], gq = pt[(size_t)ntot + o], cc = pt[2 * (size_t)ntot + o];
    ay += d1 * dy + gq * dp;
    ap += cc * dy + d1 * dp;
  }
  if (mode != 0) {
    // the faces on the core's boundary: west, east, south and north sides in turn
    const int nside = 2 * ch + 2 * cw;
    for (int e = threadIdx.x; e < nside; e += kBlock) {
      int i, j, di, dj;
      double c;
      if (e < ch) {
        i = co.x, j = co.z + e, di = -1, dj = 0;
        c = c_w(P, i, j);
      } else if (e < 2 * ch) {
        i = co.y - 1, j = co.z + e - ch, di = 1, dj = 0;
        c = c_e(P, i, j);
      } else if (e < 2 * ch + cw) {
        i = co.x + e - 2 * ch, j = co.z, di = 0, dj = -1;
        c = c_s(P, i, j);
      } else {
        i = co.x + e - 2 * ch - cw, j = co.w - 1, di = 0, dj = 1;
        c = c_n(P, i, j);
      }
      const size_t g = (size_t)j * P.nx + i;
      const int io = i + di, jo = j + dj;
      const bool in = io >= 0 && io < P.nx && jo >= 0 && jo < P.ny;
      const size_t go = in ? (size_t)jo * P.nx + io : g;
      ay += c * (vy[g] - (in ? vy[go] : 0.0));
      ap += c * (vp[g] - (in ? vp[go] : 0.0));
    }
  }
  // both sums in one pass: butterfly inside each wave, then the waves in order (fixed
  // order for thread 0, which writes them)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    ay += __shfl_xor(ay, off, 64);
    ap += __shfl_xor(ap, off, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[w] = ay;
    red[kBlock / 64 + w] = ap;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sy = 0.0, sp = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) {
      sy += red[q];
      sp += red[kBlock / 64 + q];
    }
    cv[2 * (size_t)s] = sy;
    cv[2 * (size_t)s + 1] = sp;
  }
}

// Block elimination of A0 over the core rows: S_r^{-1} for r = 0 .. sy-1, one workgroup
// per instance (blockIdx.x -> instance list[blockIdx.x]).  A column diagonally dominant
// S_r (the usual case: the Laplacian part dominates the pointwise sums) keeps its
// diagonal pivots under partial pivoting and is inverted with its pivots in order: for
// nc <= 32 by the blocked Gauss-Jordan with 16 x 16 pivot blocks on the matrix cores
// (two block steps instead of nc scalar ones), wider rows in place in LDS, one barrier
// per step (two buffers alternate).  Otherwise W = [S_r | I] is reduced to
// [I | S_r^{-1}] with partial pivoting (rows swapped).
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_factor(const DevProblem* __restrict__ prob,
                                                                  const int* __restrict__ list,
                                                                  const GmState* __restrict__ gst,
                                                                  const double* __restrict__ sums,
                                                                  double* __restrict__ sinv) {
  constexpr int LDW = 2 * kCoarseMaxNc + 1;                // W = [S_r | I], pivoting path
  constexpr int LDB = kCoarseMaxNc + 1;                    // the two buffers of the in-place path
  constexpr int kWords = 2 * kCoarseMaxNc * LDB;           // >= kCoarseMaxNc * LDW: both fit
  static_assert(kWords >= kCoarseMaxNc * LDW, "LDS buffers");
  constexpr int kPer = kCoarseMaxNc * kCoarseMaxNc / kCoarseThreads;
  __shared__ double W[kWords];
  __shared__ double colk[kCoarseMaxNc];
  __shared__ int piv;
  // staging panels of the blocked Gauss-Jordan of rows of at most 32 coarse unknowns
  __shared__ __attribute__((aligned(16))) double Stc[2 * 32 * padded<double>(16)];
  const int q = list ? list[blockIdx.x] : (int)blockIdx.x;
  if (gst && gst[q].done) return;
  const DevProblem P = prob[q];
  const int sx = P.csx, nc = 2 * sx, t = threadIdx.x;
  double* Sq = sinv + P.sinv_off;
  double* const B0 = W;
  double* const B1 = W + kCoarseMaxNc * LDB;
  for (int r = 0; r < P.csy; ++r) {
    const int ch = core_h(P, r);
    for (int e = t; e < nc * 2 * nc; e += kCoarseThreads) {
      const int a = e / (2 * nc), b = e - a * 2 * nc;
      double v;
      if (b < nc) {
        const int ca = a >> 1, fa = a & 1, cb = b >> 1, fb = b & 1;
        v = 0.0;
        const double* sa = sums + kCSum * (size_t)(P.sub0 + r * sx + ca);
        const double* sb = sums + kCSum * (size_t)(P.sub0 + r * sx + cb);
        if (ca == cb) {
          const double lap = P.cx ? sa[3] + sa[4] + sa[5] + sa[6] + sa[7]
                                  : 2.0 * ch * P.hx2i + 2.0 * core_w(P, ca) * P.hy2i;
          v = fa == fb ? lap + sa[0] : (fa == 0 ? sa[1] : sa[2]);
        } else if (fa == fb && (ca == cb + 1 || cb == ca + 1)) {
          v = P.cx ? -(cb == ca + 1 ? sa[4] : sa[3]) : -ch * P.hx2i;
        }
        if (r > 0) {
          // couplings to the row of cores below: the south sides of this row's cores
          const double wa = P.cx ? sa[5] : core_w(P, ca) * P.hy2i, wb = P.cx ? sb[5] : core_w(P, cb) * P.hy2i;
          v -= wa * wb * Sq[((size_t)(r - 1) * nc + a) * nc + b];
        }
      } else {
        v = (b - nc == a) ? 1.0 : 0.0;
      }
      W[a * LDW + b] = v;
    }
    __syncthreads();
    // column diagonal dominance of S_r (the left half of W)
    if (t < 64) {
      bool bad = false;
      for (int b = t; b < nc; b += 64) {
        double off = 0.0;
        for (int a = 0; a < nc; ++a)
          if (a != b) off += fabs(W[a * LDW + b]);
        bad = bad || !(fabs(W[b * LDW + b]) > off);
      }
      const bool any_bad = __any(bad);
      if (t == 0) piv = any_bad ? 1 : 0;
    }
    __syncthreads();
    if (piv == 0 && nc <= 32) {
      // S_r padded to 32 x 32 with the identity, inverted by the blocked Gauss-Jordan on
      // the matrix cores (pivot blocks in order, as partial pivoting would take them):
      // waves 0 and 1 own the two column blocks, waves 2 and 3 only meet the barriers
      using Vd = Mfma<double>::V;
      const int lane = t & 63, J = t >> 6;
      Vd c[2];
#pragma unroll
      for (int I = 0; I < 2; ++I)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int a = 16 * I + Mfma<double>::row(lane, q), b = 16 * J + (lane & 15);
          c[I][q] = J >= 2 ? 0.0 : (a < nc && b < nc) ? W[a * LDW + b] : (a == b ? 1.0 : 0.0);
        }
      block_gauss_jordan<double, 32>(c, Stc);
      if (J < 2) {
#pragma unroll
        for (int I = 0; I < 2; ++I)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int a = 16 * I + Mfma<double>::row(lane, q), b = 16 * J + (lane & 15);
            if (a < nc && b < nc) Sq[((size_t)r * nc + a) * nc + b] = c[I][q];
          }
      }
      __syncthreads();   // S_r^{-1} is read back by every thread for the next row
      continue;
    }
    if (piv == 0) {
      // in place, pivots in order: W -> S_r^{-1}.  Step k reads buffer `cur` and writes
      // the other: a_kk <- 1 / a_kk, row k <- row k / a_kk, column k <- -column k / a_kk,
      // a_ij <- a_ij - a_ik a_kj / a_kk.
      {
        // the buffers overlap W: every thread holds its entries before any is rewritten
        double own[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int e = t + u * kCoarseThreads, a = e / nc, b = e - a * nc;
          own[u] = e < nc * nc ? W[a * LDW + b] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int e = t + u * kCoarseThreads, a = e / nc, b = e - a * nc;
          if (e < nc * nc) B0[a * LDB + b] = own[u];
        }
        __syncthreads();
      }
      double* cur = B0;
      double* nxt = B1;
      int ra[kPer], rb[kPer];   // this thread's entries (row, column), -1: none
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = t + u * kCoarseThreads;
        ra[u] = e < nc * nc ? e / nc : -1;
        rb[u] = e < nc * nc ? e - ra[u] * nc : -1;
      }
      for (int k = 0; k < nc; ++k) {
        const double inv = 1.0 / cur[k * LDB + k];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int a = ra[u], b = rb[u];
          if (a < 0) continue;
          double v;
          if (a == k) v = b == k ? inv : cur[k * LDB + b] * inv;
          else if (b == k) v = -cur[a * LDB + k] * inv;
          else v = cur[a * LDB + b] - cur[a * LDB + k] * inv * cur[k * LDB + b];
          nxt[a * LDB + b] = v;
        }
        __syncthreads();
        double* tmp = cur;
        cur = nxt;
        nxt = tmp;
      }
      for (int e = t; e < nc * nc; e += kCoarseThreads) {
        const int a = e / nc, b = e - a * nc;
        Sq[((size_t)r * nc + a) * nc + b] = cur[a * LDB + b];
      }
      __syncthreads();   // S_r^{-1} is read back by every thread for the next row
      continue;
    }
    for (int k = 0; k < nc; ++k) {
      if (t < 64) {   // pivot: largest |W[i][k]|, i >= k (ties to the smaller row)
        double best = -1.0;
        int bi = nc;
        for (int i = k + t; i < nc; i += 64) {
          const double m = fabs(W[i * LDW + k]);
          if (m > best) {
            best = m;
            bi = i;
          }
        }
        for (int off = 32; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off, 64);
          const int oi = __shfl_xor(bi, off, 64);
          if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
          }
        }
        if (t == 0) piv = bi < nc ? bi : k;
      }
      __syncthreads();
      const int pr = piv;
      if (pr != k) {
        for (int b = t; b < 2 * nc; b += kCoarseThreads) {
          const double u = W[k * LDW + b];
          W[k * LDW + b] = W[pr * LDW + b];
          W[pr * LDW + b] = u;
        }
        __syncthreads();
      }
      const double inv = 1.0 / W[k * LDW + k];
      for (int i = t; i < nc; i += kCoarseThreads) colk[i] = W[i * LDW + k];
      __syncthreads();
      for (int b = t; b < 2 * nc; b += kCoarseThreads) W[k * LDW + b] *= inv;
      __syncthreads();
      for (int e = t; e < nc * 2 * nc; e += kCoarseThreads) {
        const int a = e / (2 * nc), b = e - a * 2 * nc;
        if (a != k) W[a * LDW + b] -= colk[a] * W[k * LDW + b];
      }
      __syncthreads();
    }
    for (int e = t; e < nc * nc; e += kCoarseThreads) {
      const int a = e / nc, b = e - a * nc;
      Sq[((size_t)r * nc + a) * nc + b] = W[a * LDW + nc + b];
    }
    __syncthreads();   // S_r^{-1} is read back by every thread for the next row
  }
}

// A0^{-1} densely, kColBlock columns per workgroup (blockIdx.y -> instance, blockIdx.x ->
// column block).  Column k (core row rk = k / nc, position lk) is the solution of
// A0 z = e_k by the block sweeps g_r = S_r^{-1}(e_k[r] - C g_{r-1}),
// z_r = g_r - S_r^{-1} C z_{r+1}; C = -diag(cw hy^-2), so -C multiplies by cw hy^-2.
// Each row's S_r^{-1} and couplings are staged in LDS once for the workgroup's columns.
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_inverse(const DevProblem* __restrict__ prob,
                                                                   const int* __restrict__ list,
                                                                   const GmState* __restrict__ gst,
                                                                   const double* __restrict__ sums,
                                                                   const double* __restrict__ sinv,
                                                                   double* __restrict__ ainv) {
  constexpr int LDS_ = kCoarseMaxNc + 1;
  __shared__ double Gl[kCoarseMaxNc * kColBlock];
  __shared__ double Sl[kCoarseMaxNc * LDS_];
  __shared__ double cb[kCoarseMaxNc];
  const int q = list ? list[blockIdx.y] : (int)blockIdx.y;
  if (gst && gst[q].done) return;
  const DevProblem P = prob[q];
  const int nc = 2 * P.csx, sy = P.csy, N = nc * sy, t = threadIdx.x;
  const int k0 = blockIdx.x * kColBlock;
  if (k0 >= N) return;
  const double* Sq = sinv + P.sinv_off;
  double* Aq = ainv + P.ainv_off;
  constexpr int PER = (kCoarseMaxNc * kColBlock + kCoarseThreads - 1) / kCoarseThreads;   // (a, column) pairs per thread
  double own[PER];
  // S_r^{-1} and the couplings of core row r to the row below (side 5: south) or above
  // (side 6: north) into LDS
  auto stage = [&](int r, int side) {
    const double* Sr = Sq + (size_t)r * nc * nc;
    for (int e = t; e < nc * nc; e += kCoarseThreads) {
      const int a = e / nc, b = e - a * nc;
      Sl[a * LDS_ + b] = Sr[e];
    }
    for (int b = t; b < nc; b += kCoarseThreads)
      cb[b] = P.cx ? sums[kCSum * (size_t)(P.sub0 + r * P.csx + (b >> 1)) + side] : core_w(P, b >> 1) * P.hy2i;
    __syncthreads();
  };
  // forward sweep
  for (int r = 0; r < sy; ++r) {
    stage(r, 5);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = t + u * kCoarseThreads;
      const int a = e / kColBlock, kk = e - a * kColBlock, k = k0 + kk;
      double v = 0.0;
      if (a < nc && k < N) {
        const int rk = k / nc, lk = k - rk * nc;
        if (r == rk) {
          v = Sl[a * LDS_ + lk];
        } else if (r > rk) {
          for (int b = 0; b < nc; ++b) v += Sl[a * LDS_ + b] * cb[b] * Gl[b * kColBlock + kk];
        }
      }
      own[u] = v;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = t + u * kCoarseThreads;
      const int a = e / kColBlock, kk = e - a * kColBlock, k = k0 + kk;
      if (a < nc) {
        Gl[a * kColBlock + kk] = own[u];
        if (k < N) Aq[(size_t)(r * nc + a) * N + k] = own[u];
      }
    }
    __syncthreads();
  }
  // backward sweep (the last block row is final); each thread reads back its own g_r
  for (int r = sy - 2; r >= 0; --r) {
    stage(r, 6);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = t + u * kCoarseThreads;
      const int a = e / kColBlock, kk = e - a * kColBlock, k = k0 + kk;
      double v = 0.0;
      if (a < nc && k < N) {
        double acc = 0.0;
        for (int b = 0; b < nc; ++b) acc += Sl[a * LDS_ + b] * cb[b] * Gl[b * kColBlock + kk];
        v = Aq[(size_t)(r * nc + a) * N + k] + acc;
      }
      own[u] = v;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = t + u * kCoarseThreads;
      const int a = e / kColBlock, kk = e - a * kColBlock, k = k0 + kk;
      if (a < nc) {
        Gl[a * kColBlock + kk] = own[u];
        if (k < N) Aq[(size_t)(r * nc + a) * N + k] = own[u];
      }
    }
    __syncthreads();
  }
}

// e[2 sub0 + r] = scale * sum_k A0^{-1}[r][k] c[2 sub0 + k] for the rows of the instance,
// one wave per row (blockIdx.y -> instance, blockIdx.x -> rows 4 bx .. 4 bx + 3).
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_solve(const DevProblem* __restrict__ prob,
                                                                 const int* __restrict__ list,
                                                                 const GmState* __restrict__ gst,
                                                                 const double* __restrict__ ainv,
                                                                 const double* __restrict__ cv, double scale,
                                                                 double* __restrict__ ev) {
  const int q = list ? list[blockIdx.y] : (int)blockIdx.y;
  if (gst && gst[q].done) return;
  const DevProblem P = prob[q];
  const int N = 2 * P.csx * P.csy;
  const int row = blockIdx.x * (kCoarseThreads / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= N) return;
  const double* Ar = ainv + P.ainv_off + (size_t)row * N;
  const double* c = cv + 2 * (size_t)P.sub0;
  double acc = 0.0;
#pragma unroll 8
  for (int k = lane; k < N; k += 64) acc += Ar[k] * c[k];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) ev[2 * (size_t)P.sub0 + row] = scale * acc;
}

}  // namespace

void launch_coarse_sums(const Items& I, const double* x, double* sums, double* pt, long long ntot, hipStream_t st) {
  if (I.count > 0) k_coarse_sums<<<I.count, kBlock, 0, st>>>(I, x, sums, pt, ntot);
}
void launch_coarse_project(const Items& I, int mode, const double* pt, long long ntot, const double* v, double* cv,
                           hipStream_t st) {
  if (I.count > 0) k_coarse_project<<<I.count, kBlock, 0, st>>>(I, mode, pt, ntot, v, cv);
}
void launch_coarse_factor(const DevProblem* prob, const int* list, int count, const GmState* gst,
                          const double* sums, double* sinv, hipStream_t st) {
  if (count > 0) k_coarse_factor<<<count, kCoarseThreads, 0, st>>>(prob, list, gst, sums, sinv);
}
void launch_coarse_inverse(const DevProblem* prob, const int* list, int count, int max_n, const GmState* gst,
                           const double* sums, const double* sinv, double* ainv, hipStream_t st) {
  if (count > 0 && max_n > 0)
    k_coarse_inverse<<<dim3((max_n + kColBlock - 1) / kColBlock, count), kCoarseThreads, 0, st>>>(prob, list, gst,
                                                                                                  sums, sinv, ainv);
}
void launch_coarse_solve(const DevProblem* prob, const int* list, int count, int max_n, const GmState* gst,
                         const double* ainv, const double* cv, double scale, double* ev, hipStream_t st) {
  constexpr int rows = kCoarseThreads / 64;
  if (count > 0 && max_n > 0)
    k_coarse_solve<<<dim3((max_n + rows - 1) / rows, count), kCoarseThreads, 0, st>>>(prob, list, gst, ainv, cv,
                                                                                     scale, ev);
}

}  // namespace rsp
