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
// The inverses are stored transposed, facT[s][j][b][a] = S_j^{-1}[a][b], so that
// the solves read them coalesced.  Lines are padded to M (multiple of 16) with
// an identity block.
#include "rsp_kernels.h"

namespace rsp {

namespace {

template <int M>
__global__ __launch_bounds__(kBlock) void k_factor(DevProblem P, const int4* __restrict__ box,
                                                   const double* __restrict__ tilex,
                                                   const double* __restrict__ c,
                                                   const SubState* __restrict__ state,
                                                   double eps_fixed, const double* __restrict__ rhs,
                                                   double rhs_scale, double* __restrict__ facT,
                                                   double* __restrict__ gout) {
  constexpr int LD = M + 1;
  constexpr int NE = (M * M + kBlock - 1) / kBlock;
  __shared__ double A[M * LD];
  __shared__ double colk[M], rowr[M], vin[M], gprev[M];
  __shared__ double la[M / 2], lb[M / 2], lc[M / 2];
  __shared__ double redv[kBlock];
  __shared__ int redi[kBlock];
  __shared__ int pr[M], pinv[M], used[M];

  const int s = blockIdx.x;
  const int t = threadIdx.x;
  double eps = eps_fixed;
  if (state) {
    if (!state[s].active) return;
    eps = state[s].eps;
  }
  const int4 bx = box[s];
  const int tx = bx.y - bx.x, ty = bx.w - bx.z;
  const int m = 2 * tx;
  const double hy4i = P.hy2i * P.hy2i;

  for (int i = t; i < M; i += kBlock) gprev[i] = 0.0;

  for (int j = 0; j < ty; ++j) {
    // coefficients of line j at z = R_i x + c
    for (int a = t; a < tx; a += kBlock) {
      const double y = tilex[halo_idx(P, s, 0, j + 1, a + 1)] + (c ? c[tile_idx(P, s, 0, j, a)] : 0.0);
      const double p = tilex[halo_idx(P, s, 1, j + 1, a + 1)] + (c ? c[tile_idx(P, s, 1, j, a)] : 0.0);
      la[a] = dphi_of(P.phi, y, P.kappa);
      lb[a] = dg_of(p, P.mu, eps) * P.inv_nu;
      lc[a] = ddphi_of(P.phi, y, P.kappa) * p - 1.0;
    }
    __syncthreads();
    // S_j = D_j - hy^-4 S_{j-1}^{-1} (active m x m block), identity padding
    double nv[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = t + q * kBlock;
      double d = 0.0;
      if (e < M * M) {
        const int r = e / M, col = e - r * M;
        if (r >= m || col >= m) {
          d = (r == col) ? 1.0 : 0.0;
        } else {
          const int fr = r >= tx, fc = col >= tx;
          const int ar = r - fr * tx, ac = col - fc * tx;
          if (fr == fc) {
            if (ar == ac) d = P.diag0 + la[ar];
            else if (ar == ac + 1 || ac == ar + 1) d = -P.hx2i;
          } else if (ar == ac) {
            d = fr == 0 ? lb[ar] : lc[ar];
          }
          if (j > 0) d -= hy4i * A[pr[r] * LD + pinv[col]];
        }
      }
      nv[q] = d;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = t + q * kBlock;
      if (e < M * M) {
        const int r = e / M, col = e - r * M;
        A[r * LD + col] = nv[q];
      }
    }
    for (int i = t; i < M; i += kBlock) used[i] = 0;
    __syncthreads();

    // in-place Gauss-Jordan with partial pivoting
    for (int k = 0; k < M; ++k) {
      double v = -1.0;
      if (t < M && !used[t]) v = fabs(A[t * LD + k]);
      redv[t] = v;
      redi[t] = t;
      __syncthreads();
      for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (t < w) {
          const double o = redv[t + w];
          if (o > redv[t]) {          // ties keep the smaller row index
            redv[t] = o;
            redi[t] = redi[t + w];
          }
        }
        __syncthreads();
      }
      const int r = redi[0];
      if (t < M) {
        colk[t] = A[t * LD + k];
        rowr[t] = A[r * LD + t];
      }
      if (t == 0) {
        used[r] = 1;
        pr[k] = r;
        pinv[r] = k;
      }
      __syncthreads();
      const double ipiv = 1.0 / rowr[k];
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const int e = t + q * kBlock;
        if (e < M * M) {
          const int i = e / M, jj = e - i * M;
          double a;
          if (i == r) a = (jj == k) ? ipiv : rowr[jj] * ipiv;
          else a = (jj == k) ? -colk[i] * ipiv : A[i * LD + jj] - colk[i] * (rowr[jj] * ipiv);
          A[i * LD + jj] = a;
        }
      }
      __syncthreads();
    }

    // fused forward sweep: g_j = S_j^{-1}(rhs_scale r_j + hy^-2 g_{j-1})
    if (rhs) {
      for (int i = t; i < M; i += kBlock) {
        double r = 0.0;
        if (i < m) {
          const int f = i >= tx;
          r = rhs_scale * rhs[tile_idx(P, s, f, j, i - f * tx)];
        }
        vin[i] = r + P.hy2i * gprev[i];
      }
      __syncthreads();
      double acc = 0.0;
      if (t < M) {
        const double* row = A + pr[t] * LD;
        for (int k = 0; k < M; ++k) acc += row[k] * vin[pr[k]];
      }
      __syncthreads();
      if (t < M) {
        gprev[t] = acc;
        gout[((size_t)s * P.tym + j) * M + t] = acc;
      }
    }
    // store S_j^{-1} transposed
    double* F = facT + ((size_t)s * P.tym + j) * M * M;
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = t + q * kBlock;
      if (e < M * M) {
        const int b = e / M, a = e - b * M;
        F[e] = A[pr[a] * LD + pinv[b]];
      }
    }
    __syncthreads();
  }
}

// z_{ty-1} = g_{ty-1}; z_j = g_j + hy^-2 S_j^{-1} z_{j+1}; written to the tile `out`.
template <int M>
__global__ __launch_bounds__(kBlock) void k_solve_bwd(DevProblem P, const int4* __restrict__ box,
                                                      const SubState* __restrict__ state,
                                                      const double* __restrict__ facT,
                                                      const double* __restrict__ g,
                                                      double* __restrict__ out) {
  __shared__ double z[M];
  const int s = blockIdx.x, t = threadIdx.x;
  if (state && !state[s].active) return;
  const int4 bx = box[s];
  const int tx = bx.y - bx.x, ty = bx.w - bx.z;
  const int m = 2 * tx;
  for (int j = ty - 1; j >= 0; --j) {
    double v = 0.0;
    if (t < M) {
      v = g[((size_t)s * P.tym + j) * M + t];
      if (j < ty - 1) {
        const double* F = facT + ((size_t)s * P.tym + j) * M * M;
        double acc = 0.0;
        for (int b = 0; b < M; ++b) acc += F[(size_t)b * M + t] * z[b];
        v += P.hy2i * acc;
      }
    }
    __syncthreads();
    if (t < M) {
      z[t] = v;
      if (t < m) {
        const int f = t >= tx;
        out[tile_idx(P, s, f, j, t - f * tx)] = v;
      }
    }
    __syncthreads();
  }
}

// Forward and backward sweeps with stored factors: out = J_i^{-1} rhs.
template <int M>
__global__ __launch_bounds__(kBlock) void k_block_solve(DevProblem P, const int4* __restrict__ box,
                                                        const double* __restrict__ facT,
                                                        const double* __restrict__ rhs,
                                                        double* __restrict__ out) {
  __shared__ double gl[kMaxTile * M];
  __shared__ double v[M];
  const int s = blockIdx.x, t = threadIdx.x;
  const int4 bx = box[s];
  const int tx = bx.y - bx.x, ty = bx.w - bx.z;
  const int m = 2 * tx;
  for (int e = t; e < 2 * P.txm * P.tym; e += kBlock) {       // zero padding of the output
    const int f = e / (P.txm * P.tym);
    const int r = e - f * P.txm * P.tym;
    const int b = r / P.txm, a = r - b * P.txm;
    if (a >= tx || b >= ty) out[tile_idx(P, s, f, b, a)] = 0.0;
  }
  for (int j = 0; j < ty; ++j) {
    if (t < M) {
      double r = 0.0;
      if (t < m) {
        const int f = t >= tx;
        r = rhs[tile_idx(P, s, f, j, t - f * tx)];
      }
      v[t] = r + (j > 0 ? P.hy2i * gl[(j - 1) * M + t] : 0.0);
    }
    __syncthreads();
    if (t < M) {
      const double* F = facT + ((size_t)s * P.tym + j) * M * M;
      double acc = 0.0;
      for (int b = 0; b < M; ++b) acc += F[(size_t)b * M + t] * v[b];
      gl[j * M + t] = acc;
    }
    __syncthreads();
  }
  for (int j = ty - 2; j >= 0; --j) {
    if (t < M) {
      const double* F = facT + ((size_t)s * P.tym + j) * M * M;
      double acc = 0.0;
      for (int b = 0; b < M; ++b) acc += F[(size_t)b * M + t] * gl[(j + 1) * M + b];
      v[t] = gl[j * M + t] + P.hy2i * acc;
    }
    __syncthreads();
    if (t < M) gl[j * M + t] = v[t];
    __syncthreads();
  }
  for (int j = 0; j < ty; ++j)
    for (int i = t; i < m; i += kBlock) {
      const int f = i >= tx;
      out[tile_idx(P, s, f, j, i - f * tx)] = gl[j * M + i];
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

void launch_factor(const DevProblem& P, const int4* box, const double* tilex, const double* c,
                   const SubState* state, double eps_fixed, const double* rhs, double rhs_scale,
                   double* facT, double* g, hipStream_t st) {
#define RSP_CALL(MM) \
  k_factor<MM><<<P.S, kBlock, 0, st>>>(P, box, tilex, c, state, eps_fixed, rhs, rhs_scale, facT, g)
  RSP_DISPATCH_M(P.M, RSP_CALL)
#undef RSP_CALL
}

void launch_solve_bwd(const DevProblem& P, const int4* box, const SubState* state,
                      const double* facT, const double* g, double* out, hipStream_t st) {
#define RSP_CALL(MM) k_solve_bwd<MM><<<P.S, kBlock, 0, st>>>(P, box, state, facT, g, out)
  RSP_DISPATCH_M(P.M, RSP_CALL)
#undef RSP_CALL
}

void launch_block_solve(const DevProblem& P, const int4* box, const double* facT,
                        const double* rhs, double* out, hipStream_t st) {
#define RSP_CALL(MM) k_block_solve<MM><<<P.S, kBlock, 0, st>>>(P, box, facT, rhs, out)
  RSP_DISPATCH_M(P.M, RSP_CALL)
#undef RSP_CALL
}

}  // namespace rsp
