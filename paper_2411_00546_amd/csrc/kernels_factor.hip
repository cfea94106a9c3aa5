// Local Jacobian factorisation and solves (one workgroup per subdomain).
//
// J_i = R_i F'_eps(x + P_i c) P_i (Section 4: x-derivative of F; eq. (DerC)) is
// block tridiagonal over the grid lines of the tile: with the unknowns of line j
// ordered (y_0..y_{tx-1}, p_0..p_{tx-1}) the diagonal block is
//   D_j = [[T + diag(phi'(y)),        diag(g'(p)/nu)   ],
//          [diag(phi''(y) p - 1),     T + diag(phi'(y))]]
// with T = tridiag(-1/hx^2, 2/hx^2 + 2/hy^2, -1/hx^2), and both off-diagonal
// blocks are -(1/hy^2) I.  Block LU: S_0 = D_0, S_j = D_j - hy^-4 S_{j-1}^{-1};
// forward g_j = S_j^{-1}(r_j + hy^-2 g_{j-1}); backward z_j = g_j + hy^-2 S_j^{-1} z_{j+1}.
// Each S_j^{-1} comes from in-place Gauss-Jordan with partial pivoting (rows are
// not moved: step k pivots on row pr[k]; afterwards S^{-1}[a][b] = A[pr[a]][pinv[b]]).
// The line block lives in registers (256 threads, an R x R slice each); per step the
// pivot is found inside the wave that holds the column, the column goes through LDS
// (one barrier per step) and the pivot row is broadcast with in-wave shuffles.
// The inverses are stored transposed, facT[s][j][b][a] = S_j^{-1}[a][b], so that
// the solves read them coalesced.  Lines are padded to M (multiple of 16) with
// an identity block.
#include "rsp_kernels.h"

namespace rsp {

namespace {

// DPP lane exchange inside 16-lane rows (quad_perm [1,0,3,2], quad_perm [2,3,0,1],
// row_half_mirror, row_mirror): four steps give every lane of a row the row-wide
// result of a symmetric combine.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = dpp_i<CTRL>(__double2loint(v));
  const int hi = dpp_i<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_d(float v) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
// Keep the larger |value|, ties to the smaller row index (a total order, so every
// lane of the row ends with the same winner).
template <int CTRL, typename T>
__device__ __forceinline__ void pivot_step(T& best, int& bi, T& bv) {
  const T ob = dpp_d<CTRL>(best);
  const int oi = dpp_i<CTRL>(bi);
  const T ov = dpp_d<CTRL>(bv);
  const bool take = (ob > best) | ((ob == best) & (oi < bi));
  best = take ? ob : best;
  bi = take ? oi : bi;
  bv = take ? ov : bv;
}

// Sum over the 16 lanes of a DPP row (every lane gets the sum, same order in all).
template <typename T>
__device__ __forceinline__ T row_sum16(T v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return v;
}

constexpr int kFacThreads = 256;   // 16 x 16 threads; thread (ti, tj) owns rows ti + 16 rr, cols tj + 16 cc

// T: arithmetic and storage type of the line inverses (double, or float for the
// FP32 factors of the mixed-precision form); coefficients and the fused forward
// sweep stay in double.
template <typename T, int M>
__global__ __launch_bounds__(kFacThreads) void k_factor(Items I, const double* __restrict__ tilex,
                                                        const double* __restrict__ c,
                                                        const SubState* __restrict__ state,
                                                        double eps_fixed, const double* __restrict__ rhs,
                                                        double rhs_scale, T* __restrict__ facT,
                                                        double* __restrict__ gout) {
  constexpr int R = M / 16;          // rows (and columns) of the line block per thread
  constexpr int LD = M + 1;
  __shared__ T Mx[M * LD];      // finished in-place Gauss-Jordan result of the line
  __shared__ T colb[2][M];      // pivot column of the current step (double buffered)
  __shared__ int pivb[2];
  __shared__ T pivv[2][2];      // pivot value and its reciprocal
  __shared__ int pr[2][M], pinv[2][M];
  __shared__ double la[M / 2], lb[M / 2], lc[M / 2];
  __shared__ double vin[M], gprev[M];
  __shared__ int nondom;

  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  const int t = threadIdx.x, ti = t & 15, tj = t >> 4;
  const int lane = t & 63;
  double eps = eps_fixed > 0.0 ? eps_fixed : P.eps_min;
  if (state) {
    if (!state[s].active) return;
    eps = state[s].eps;
  }
  const int4 bx = I.box[s];
  const int tx = bx.y - bx.x, ty = bx.w - bx.z;
  const int m = 2 * tx;
  const double hy4i = P.hy2i * P.hy2i;
  T A[R][R];

  for (int i = t; i < M; i += kFacThreads) gprev[i] = 0.0;

  for (int j = 0; j < ty; ++j) {
    const int pj = j & 1, pp = pj ^ 1;
    if (t == 0) nondom = 0;
    // coefficients of line j at z = R_i x + c
    for (int a = t; a < tx; a += kFacThreads) {
      const double y = tilex[halo_idx(P, s, 0, j + 1, a + 1)] + (c ? c[tile_idx(P, s, 0, j, a)] : 0.0);
      const double p = tilex[halo_idx(P, s, 1, j + 1, a + 1)] + (c ? c[tile_idx(P, s, 1, j, a)] : 0.0);
      la[a] = dphi_of(P.phi, y, P.kappa);
      lb[a] = dg_of(p, P.mu, eps) * P.inv_nu;
      lc[a] = ddphi_of(P.phi, y, P.kappa) * p - 1.0;
    }
    __syncthreads();
    // S_j = D_j - hy^-4 S_{j-1}^{-1} on the active m x m block, identity padding;
    // S_{j-1}^{-1}[a][b] = Mx[pr[a]][pinv[b]] of the previous line
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int a = ti + 16 * rr;
#pragma unroll
      for (int cc = 0; cc < R; ++cc) {
        const int b = tj + 16 * cc;
        double d;
        if (a >= m || b >= m) {
          d = (a == b) ? 1.0 : 0.0;
        } else {
          const int fr = a >= tx, fc = b >= tx;
          const int ar = a - fr * tx, ac = b - fc * tx;
          d = 0.0;
          if (fr == fc) {
            if (ar == ac) d = P.diag0 + la[ar];
            else if (ar == ac + 1 || ac == ar + 1) d = -P.hx2i;
          } else if (ar == ac) {
            d = fr == 0 ? lb[ar] : lc[ar];
          }
          if (j > 0) d -= hy4i * (double)Mx[pr[pp][a] * LD + pinv[pp][b]];
        }
        A[rr][cc] = (T)d;
      }
    }
    // Column diagonal dominance |S_kk| >= sum_{i != k} |S_ik| of the active block:
    // then Gauss-Jordan with partial pivoting keeps every diagonal pivot (the
    // property is inherited by the Schur complements), so the static-pivot steps
    // below compute exactly what the pivoted ones would.
    {
      bool bad = false;
#pragma unroll
      for (int cc = 0; cc < R; ++cc) {
        const int b = tj + 16 * cc;
        T off = 0, dia = 0;
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          const T v = fabs(A[rr][cc]);
          const bool d = (ti + 16 * rr) == b;
          dia += d ? v : (T)0;
          off += d ? (T)0 : v;
        }
        off = row_sum16(off);
        dia = row_sum16(dia);
        bad |= (b < m) & !(dia >= off);
      }
      if (bad) nondom = 1;
    }
    __syncthreads();
    if (!nondom) {
      // static pivots: step k eliminates with row k
#pragma unroll
      for (int ck = 0; ck < R; ++ck) {
        for (int kk = 0; kk < 16; ++kk) {
          const int k = 16 * ck + kk;
          if (k >= m) break;
          const int pb = k & 1;
          if (tj == kk) {
#pragma unroll
            for (int rr = 0; rr < R; ++rr) colb[pb][ti + 16 * rr] = A[rr][ck];
            if (ti == kk) {
              pivv[pb][0] = A[ck][ck];
              pivv[pb][1] = (T)1 / A[ck][ck];
            }
          }
          __syncthreads();
          const T ipiv = pivv[pb][1];
          T rs[R], mult[R];
#pragma unroll
          for (int cc = 0; cc < R; ++cc) rs[cc] = __shfl(A[ck][cc], (lane & 48) | kk, 64) * ipiv;
#pragma unroll
          for (int rr = 0; rr < R; ++rr) mult[rr] = colb[pb][ti + 16 * rr];
#pragma unroll
          for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int cc = 0; cc < R; ++cc) A[rr][cc] = fma(-mult[rr], rs[cc], A[rr][cc]);
          // the pivot row becomes row / piv (assigned, not updated: the update would
          // cancel catastrophically for |piv| >> 1)
          if (ti == kk) {
#pragma unroll
            for (int cc = 0; cc < R; ++cc) A[ck][cc] = rs[cc];
          }
          if (tj == kk) {
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
              const T cv = colb[pb][ti + 16 * rr];
              A[rr][ck] = (rr == ck && ti == kk) ? ipiv : -cv * ipiv;
            }
          }
        }
      }
      for (int k = t; k < m; k += kFacThreads) {
        pr[pj][k] = k;
        pinv[pj][k] = k;
      }
    } else {
      unsigned used = 0;                 // bit rr: row ti + 16 rr already pivoted
      // in-place Gauss-Jordan with partial pivoting over the m active columns
#pragma unroll
      for (int ck = 0; ck < R; ++ck) {
        for (int kk = 0; kk < 16; ++kk) {
          const int k = 16 * ck + kk;
          if (k >= m) break;
          const int pb = k & 1;
          // pivot search by the 16 lanes that hold column k (DPP reduction inside the
          // row), only in the wave that holds them; the winner's value and reciprocal
          // are published with its row index
          if ((t >> 6) == (kk >> 2)) {
            T best = -1, bv = 0;
            int bi = 1 << 30;
            if (tj == kk) {
#pragma unroll
              for (int rr = 0; rr < R; ++rr) {
                const T v = fabs(A[rr][ck]);
                const bool take = !((used >> rr) & 1u) & (v > best);
                best = take ? v : best;
                bi = take ? ti + 16 * rr : bi;
                bv = take ? A[rr][ck] : bv;
              }
            }
            pivot_step<0xB1>(best, bi, bv);
            pivot_step<0x4E>(best, bi, bv);
            pivot_step<0x141>(best, bi, bv);
            pivot_step<0x140>(best, bi, bv);
            if (tj == kk) {
              if (ti == 0) {
                const bool ok = bi < M;                     // a NaN column has no candidate
                const T pv = ok ? bv : (T)__builtin_nan("");
                pivb[pb] = ok ? bi : k;
                pivv[pb][0] = pv;
                pivv[pb][1] = (T)1 / pv;
              }
#pragma unroll
              for (int rr = 0; rr < R; ++rr) colb[pb][ti + 16 * rr] = A[rr][ck];
            }
          }
          __syncthreads();
          const int r = __builtin_amdgcn_readfirstlane(pivb[pb]);
          const int rq = r >> 4, rl = r & 15;
          const T ipiv = pivv[pb][1];
          // pivot row: held by lane (rl) of this 16-lane group, register row rq (wave-uniform)
          T rs[R], mult[R], src[R];
          // rq is wave-uniform: one scalar branch picks the register row (the empty asm
          // keeps the compiler from turning the cases into per-element selects)
#pragma unroll
          for (int q = 0; q < R; ++q)
            if (q == rq) {
              asm volatile("" ::: "memory");
#pragma unroll
              for (int cc = 0; cc < R; ++cc) src[cc] = A[q][cc];
            }
#pragma unroll
          for (int cc = 0; cc < R; ++cc) rs[cc] = __shfl(src[cc], (lane & 48) | rl, 64) * ipiv;
          // rank-1 update, then the pivot row is assigned row / piv (see the static steps)
#pragma unroll
          for (int rr = 0; rr < R; ++rr) mult[rr] = colb[pb][ti + 16 * rr];
#pragma unroll
          for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int cc = 0; cc < R; ++cc) A[rr][cc] = fma(-mult[rr], rs[cc], A[rr][cc]);
          if (ti == rl) {
#pragma unroll
            for (int q = 0; q < R; ++q)
              if (q == rq) {
                asm volatile("" ::: "memory");
#pragma unroll
                for (int cc = 0; cc < R; ++cc) A[q][cc] = rs[cc];
              }
          }
          // column k becomes -column k / piv, and (r, k) = 1 / piv
          if (tj == kk) {
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
              const T cv = colb[pb][ti + 16 * rr];
              A[rr][ck] = (ti + 16 * rr == r) ? ipiv : -cv * ipiv;
            }
          }
          if (ti == rl) used |= 1u << rq;
          if (t == 0) {
            pr[pj][k] = r;
            pinv[pj][r] = k;
          }
        }
      }
    }
    // padded steps are identities: pivot row k for k >= m
    for (int k = m + t; k < M; k += kFacThreads) {
      pr[pj][k] = k;
      pinv[pj][k] = k;
    }
#pragma unroll
    for (int rr = 0; rr < R; ++rr)
#pragma unroll
      for (int cc = 0; cc < R; ++cc) Mx[(ti + 16 * rr) * LD + tj + 16 * cc] = A[rr][cc];
    __syncthreads();

    // fused forward sweep: g_j = S_j^{-1}(rhs_scale r_j + hy^-2 g_{j-1})
    if (rhs) {
      for (int i = t; i < M; i += kFacThreads) {
        double rv = 0.0;
        if (i < m) {
          const int f = i >= tx;
          rv = rhs_scale * rhs[tile_idx(P, s, f, j, i - f * tx)];
        }
        vin[i] = rv + P.hy2i * gprev[i];
      }
      __syncthreads();
      if (t < M) {
        const T* row = Mx + pr[pj][t] * LD;
        double acc = 0.0;
        for (int k = 0; k < M; ++k) acc += (double)row[k] * vin[pr[pj][k]];
        gprev[t] = acc;
        gout[((size_t)s * P.tym + j) * M + t] = acc;
      }
    }
    // store S_j^{-1} transposed: facT[b][a] = Mx[pr[a]][pinv[b]]
    T* F = facT + ((size_t)s * P.tym + j) * M * M;
#pragma unroll
    for (int cc = 0; cc < R; ++cc) {
      const int b = tj + 16 * cc;
      const int cb = pinv[pj][b];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int a = ti + 16 * rr;
        F[(size_t)b * M + a] = Mx[pr[pj][a] * LD + cb];
      }
    }
    __syncthreads();
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

void launch_factor(const Items& I, int M, const double* tilex, const double* c, const SubState* state,
                   double eps_fixed, const double* rhs, double rhs_scale, void* facT, int fp32, double* g,
                   hipStream_t st) {
  if (I.count <= 0) return;
  if (fp32) {
#define RSP_CALL(MM)                                                                                  \
  k_factor<float, MM><<<I.count, kFacThreads, 0, st>>>(I, tilex, c, state, eps_fixed, rhs, rhs_scale, \
                                                       (float*)facT, g)
    RSP_DISPATCH_M(M, RSP_CALL)
#undef RSP_CALL
  } else {
#define RSP_CALL(MM)                                                                                   \
  k_factor<double, MM><<<I.count, kFacThreads, 0, st>>>(I, tilex, c, state, eps_fixed, rhs, rhs_scale, \
                                                        (double*)facT, g)
    RSP_DISPATCH_M(M, RSP_CALL)
#undef RSP_CALL
  }
}

}  // namespace rsp
