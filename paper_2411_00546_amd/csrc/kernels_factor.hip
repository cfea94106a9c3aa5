// Local Jacobian factorisation for the local Newton solves and Algorithm 4.
//
// J_i = R_i F'_eps(x + P_i c) P_i (Section 4: x-derivative of F; eq. (DerC)) is
// block tridiagonal over the grid lines of the tile: with the unknowns of line j
// ordered (y_0..y_{tx-1}, p_0..p_{tx-1}) the diagonal block is
//   D_j = [[T + diag(phi'(y)),        diag(g'(p)/nu)   ],
//          [diag(phi''(y) p - 1),     T + diag(phi'(y))]]
// with T = tridiag(-1/hx^2, 2/hx^2 + 2/hy^2, -1/hx^2), and both off-diagonal
// blocks are -(1/hy^2) I.  It is factored two-ended (twisted block LU) around the
// twist line t = ty / 2:
//   from the top     S_0 = D_0,       S_j = D_j - hy^-4 S_{j-1}^{-1}      (j < t)
//   from the bottom  T_{ty-1} = D_{ty-1}, T_j = D_j - hy^-4 T_{j+1}^{-1}  (j > t)
//   twist            Z_t = D_t - hy^-4 (S_{t-1}^{-1} + T_{t+1}^{-1})
// and the explicit inverses F_j of S_j, T_j and Z_t are stored (the solves are
// described in kernels_solve.hip).  The two chains are independent, so each
// subdomain takes two workgroups for them; the twist lines follow in a second launch.
//
// Each line block is assembled and tested for column diagonal dominance with the rows
// of y weighted by dom_w, a power of two near sqrt(nu) that balances the couplings
// g'(p)/nu and phi''(y) p - 1 between the fields: the dominance of W S W^{-1},
// W = diag(dom_w I, I), on which partial pivoting would keep the diagonal.  Without
// pivoting, the elimination of S performs the operations of that of W S W^{-1} scaled
// exactly by powers of two, so it is that elimination.  A dominant block (the usual
// case) is inverted by Gauss-Jordan with 16 x 16 pivot blocks whose block products run
// on the matrix cores.  The twist block adds the
// contributions of both chains and need not be dominant: when it is not, its block
// elimination checks the partial-pivoting condition of W Z W^{-1} exactly (every
// weighted multiplier at most 1 in magnitude) instead.  A subdomain where a test fails is redone by a second kernel
// with in-place Gauss-Jordan with partial pivoting in registers (rows are not moved:
// step k pivots on row pr[k]; afterwards S^{-1}[a][b] = A[pr[a]][pinv[b]]): per step
// the pivot is found inside the wave that holds the column, the column goes through
// LDS (one barrier per step) and the pivot row is broadcast with in-wave shuffles.
// The inverses are stored transposed, facT[s][j][b][a] = F_j[a][b], so that the
// solves read them coalesced.  Lines are padded to M (multiple of 16) with an
// identity block.
#include <type_traits>

#include "rsp_kernels.h"
#include "rsp_mfma.h"

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
static_assert(kMaxTile < kFacThreads, "one thread per node of a line");

// In-place inverse of the M x M matrix A (LDS, row stride LD, rows 16-byte aligned)
// by Gauss-Jordan with 16 x 16 pivot blocks taken in order (no pivot search): for
// pivot block K,
//   A_KK <- A_KK^{-1},  A_KJ <- A_KK^{-1} A_KJ,  A_IK <- -A_IK A_KK^{-1},
//   A_IJ <- A_IJ - A_IK A_KK^{-1} A_KJ                      (I, J != K),
// checking the partial-pivoting condition on the way (for the twist line, whose block
// need not be column diagonally dominant), on the block with its rows of the first
// field (rows below tx) weighted by wy, as the dominance test (see k_factor_mfma).  M / 16 waves; wave J owns column block J.
// Wave K eliminates the whole column panel A[:, K] (a copy in one of the two staging
// panels of Pn, M x padded(16) each, taken in turn: wave K copies its panel back to A
// after the step's last barrier while wave K + 1 already fills the other), which gives
// A_KK^{-1} and the new column K at once and every multiplier a_ik / a_kk of the
// elimination in natural order; if one exceeds 1 in magnitude for an unpivoted row,
// partial pivoting would have swapped rows, and the function returns true (A is then
// left partly eliminated).  The other waves form their row-panel tile A_KK^{-1} A_KJ
// and update their column.  Returns false otherwise.
template <typename T, int M>
__device__ __forceinline__ bool panel_gauss_jordan(T* A, int LD, T* Pn, int* flag, int tx, T wy) {
  constexpr int NB = M / 16;
  constexpr int PLD = padded<T>(16);
  using V = typename Mfma<T>::V;
  const int t = threadIdx.x, lane = t & 63, J = t >> 6;
  const int li = lane & 15, q4 = lane >> 4;
  if (t == 0) *flag = 0;
#pragma unroll 1
  for (int K = 0; K < NB; ++K) {
    T* const Pk = Pn + (K & 1) * M * PLD;   // this step's staging panel
    const T* Pinv = Pk + 16 * K * PLD;      // where the other waves find A_KK^{-1}
    if (J == K) {
      // lane (li, q4) owns rows li + 16 r (r < NB), columns 4 q4 .. 4 q4 + 3 of the panel
      T own[NB][4];
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        load4<T>(A + (li + 16 * r) * LD + 16 * K + 4 * q4, own[r]);
        store4<T>(Pk + (li + 16 * r) * PLD + 4 * q4, own[r]);
      }
      bool swap = false;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int kk = 16 * K + k;               // pivot row
        T prow[4];
        load4<T>(Pk + kk * PLD + 4 * q4, prow);
        T pcol[NB];
#pragma unroll
        for (int r = 0; r < NB; ++r) pcol[r] = Pk[(li + 16 * r) * PLD + k];
        const T piv = Pk[kk * PLD + k];
        const T inv = recip(piv);
        const T wpiv = (kk < tx ? wy : (T)1) * fabs(piv);
#pragma unroll
        for (int r = 0; r < NB; ++r) {
          const int i = li + 16 * r;
          swap |= i > kk && (i < tx ? wy : (T)1) * fabs(pcol[r]) > wpiv;
          const bool on_row = i == kk;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const bool on_col = 4 * q4 + q == k;
            const T tr = prow[q] * inv;
            own[r][q] = on_col ? (on_row ? inv : -pcol[r] * inv)
                               : (on_row ? tr : fma(-pcol[r], tr, own[r][q]));
          }
          store4<T>(Pk + i * PLD + 4 * q4, own[r]);
        }
      }
      if (__any(swap) && lane == 0) *flag = 1;
    }
    __syncthreads();
    if (*flag) return true;
    if (J != K) {
      // row-panel tile R = A_KK^{-1} A_KJ, then column J: A_IJ -= A_IK R, A_KJ = R
      T a[4], b[4];
      a_operand<T>(Pinv, PLD, lane, a);
      b_operand<T>(A + 16 * K * LD + 16 * J, LD, lane, b);
      V r = {0, 0, 0, 0};
      r = mma16<T>(a, b, (T)1, r);
      T rb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) rb[q] = r[q];
#pragma unroll
      for (int I = 0; I < NB; ++I) {
        T* AIJ = A + 16 * I * LD + 16 * J;
        if (I == K) {
          tile_store<T>(AIJ, LD, r, lane);
        } else {
          T ai[4];
          a_operand<T>(A + 16 * I * LD + 16 * K, LD, lane, ai);
          V c = tile_load<T>(AIJ, LD, lane);
          c = mma16<T>(ai, rb, (T)-1, c);
          tile_store<T>(AIJ, LD, c, lane);
        }
      }
    }
    __syncthreads();
    if (J == K) {
      // the eliminated panel is the new column K (A_KK^{-1} in rows K)
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        T v[4];
        load4<T>(Pk + (li + 16 * r) * PLD + 4 * q4, v);
        store4<T>(A + (li + 16 * r) * LD + 16 * K + 4 * q4, v);
      }
    }
  }
  __syncthreads();
  return false;
}

// The usual path, two-ended (twisted) block LU over the lines of the tile, t = ty / 2,
// in two launches.  phase 0, two workgroups per subdomain: blockIdx.y = 0 factors lines
// 0 .. t-1 from the top (S_j = D_j - hy^-4 S_{j-1}^{-1}), blockIdx.y = 1 lines ty-1 ..
// t+1 from the bottom (T_j = D_j - hy^-4 T_{j+1}^{-1}).  phase 1, one workgroup per
// subdomain: the twist line Z_t = D_t - hy^-4 (S_{t-1}^{-1} + T_{t+1}^{-1}) from the
// stored inverses (the launch boundary makes both chains' stores visible; a hand-over
// between the two workgroups inside one launch needs device-scope fences, which write
// back the L2 and cost more than the second launch).  Each line block is assembled in LDS with its
// column sums, checked for column diagonal dominance and inverted by the blocked
// Gauss-Jordan on the matrix cores.  The fused sweep gives g_j (top), h_j (bottom) and
// z_t = Z_t^{-1}(r_t + hy^-2 (g_{t-1} + h_{t+1})) for the Newton right-hand side.  A
// subdomain with a line that is not dominant is marked in fallback[s] and redone by
// k_factor_pivot.  M / 16 waves per workgroup.
template <typename T, int M, bool VAR>
__global__ __launch_bounds__(4 * M, (sizeof(T) == 4 && M <= 80) ? 4 : 1) void k_factor_mfma(Items I, const double* __restrict__ tilex,
                                                       const double* __restrict__ c,
                                                       const SubState* __restrict__ state,
                                                       double eps_fixed, const double* __restrict__ rhs,
                                                       double rhs_scale, T* __restrict__ facT,
                                                       double* __restrict__ gout, int* __restrict__ fallback,
                                                       int phase) {
  constexpr int NT = 4 * M;             // 64 threads per column block
  constexpr int LD = padded<T>(M);
  constexpr int KC = M / 4;             // the forward sweep adds each row in 4 parts
  __shared__ __attribute__((aligned(16))) T Mx[M * LD];   // S_j, then S_j^{-1}
  __shared__ double la[M / 2], lb[M / 2], lc[M / 2];
  // variable coefficients of A (VAR): diagonal of A, west and east couplings of each node
  // of the line, and its couplings to the previous line (lp) and, at the twist, to the
  // line below the twist (lq; lp then couples to the line above)
  __shared__ double ldg[M / 2], lw[M / 2], le[M / 2], lp[M / 2], lq[M / 2];
  __shared__ double vin[M], gprev[M];
  __shared__ double part[4 * M];
  __shared__ int flag;
  // the two staging panels of the blocked and of the panel Gauss-Jordan
  __shared__ __attribute__((aligned(16))) T St[2 * M * padded<T>(16)];
  T* const Pn = St;

  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double eps = eps_fixed > 0.0 ? eps_fixed : eps_fixed < 0.0 ? P.eps_start : P.eps_min;
  if (state) {
    if (!state[s].active) return;
    eps = state[s].eps;
  }
  const int4 bx = I.box[s];
  const int tx = bx.y - bx.x, ty = bx.w - bx.z, tw = ty / 2;
  const int m = 2 * tx;
  const double hy4i = P.hy2i * P.hy2i;
  const T nh4 = (T)(-hy4i);
  // row weight of the first field in the dominance tests (a power of two, so the
  // weighted and the plain block take the same elimination arithmetic)
  const T wy = (T)P.dom_w;
  const int half = phase == 0 ? (int)blockIdx.y : 0;   // phase 1 combines as half 0 would
  const int j0 = half == 0 ? 0 : ty - 1, dir = half == 0 ? 1 : -1;
  const int nlines = phase != 0 ? 0 : half == 0 ? tw : ty - 1 - tw;
  T* Fs = facT + (size_t)s * P.tym * M * M;
  double* gs = gout + (size_t)s * P.tym * M;
  for (int i = t; i < M; i += NT) gprev[i] = 0.0;

  auto state_at = [&](int jj, double& y, double& p) {
    y = tilex[halo_idx(P, s, 0, jj + 1, t + 1)] + (c ? c[tile_idx(P, s, 0, jj, t)] : 0.0);
    p = tilex[halo_idx(P, s, 1, jj + 1, t + 1)] + (c ? c[tile_idx(P, s, 1, jj, t)] : 0.0);
  };
  // The loads of state_at without the sums, so that the loads of the next line stay in
  // flight while the current line is factored.
  struct Raw { double xy, cy, xp, cp; };
  auto fetch = [&](int jj, Raw& r) {
    r.xy = tilex[halo_idx(P, s, 0, jj + 1, t + 1)];
    r.xp = tilex[halo_idx(P, s, 1, jj + 1, t + 1)];
    r.cy = c ? c[tile_idx(P, s, 0, jj, t)] : 0.0;
    r.cp = c ? c[tile_idx(P, s, 1, jj, t)] : 0.0;
  };
  // the pointwise coefficients of node t of line jj; with VAR also the operator's (the
  // previous line of the chain is jj - dir; at the twist lp and lq couple to tw - 1 and
  // tw + 1)
  auto coefficients = [&](double y, double p, int jj, bool twist) {
    la[t] = dphi_of(P.phi, y, P.kappa);
    lb[t] = dg_of(p, P.mu, eps) * P.inv_nu;
    lc[t] = ddphi_of(P.phi, y, P.kappa) * p - 1.0;
    if constexpr (VAR) {
      const int gi = bx.x + t, gj = bx.z + jj;
      ldg[t] = a_diag(P, gi, gj);
      lw[t] = c_w(P, gi, gj);
      le[t] = c_e(P, gi, gj);
      lp[t] = (twist || dir == 1) ? c_s(P, gi, gj) : c_n(P, gi, gj);
      lq[t] = c_n(P, gi, gj);
    }
  };
  // node of line-vector entry i < m
  auto node = [&](int i) { return i < tx ? i : i - tx; };
  // Line block of line j: D_j + (mode 0: nothing; 1: hy^-4 times -(the previous inverse
  // in Mx); 2: Mx as it stands), identity padding, column sums; returns true when some
  // active column is not dominant.  Column b = 16 wave + (lane & 15), rows (lane >> 4) + 4 r.
  auto build = [&](int mode) -> bool {
    const int b = 16 * wave + (lane & 15), rg = lane >> 4;
    T off = 0, dia = 0;
    if (b < m) {
      // column b of D_j has entries in four rows only: the diagonal, the x-neighbours in
      // the same field and the same node in the other field (the y-p coupling)
      const int fc = b >= tx, bc = b - fc * tx;
      const int r_l = bc > 0 ? b - 1 : -1, r_r = bc + 1 < tx ? b + 1 : -1;
      const int r_c = fc ? bc : tx + bc;
      const T d_d = (T)((VAR ? ldg[bc] : P.diag0) + la[bc]), d_c = (T)(fc ? lb[bc] : lc[bc]);
      const T d_xl = (T)(VAR ? -lw[bc] : -P.hx2i), d_xr = (T)(VAR ? -le[bc] : -P.hx2i);
#pragma unroll 4
      for (int r = 0; r < M / 4; ++r) {
        const int a = rg + 4 * r;
        T v = 0;
        if (a < m) {
          T d = 0;
          d = a == b ? d_d : d;
          d = a == r_l ? d_xl : d;
          d = a == r_r ? d_xr : d;
          d = a == r_c ? d_c : d;
          const T prev = Mx[a * LD + b];
          v = (mode == 0 ? (T)0 : (mode == 1 ? nh4 * prev : prev)) + d;
        }
        Mx[a * LD + b] = v;
        const T wv = (a < tx ? wy : (T)1) * fabs(v);
        if (a == b) dia = wv;
        else off += wv;
      }
    } else {
      // padding: identity
#pragma unroll 4
      for (int r = 0; r < M / 4; ++r) {
        const int a = rg + 4 * r;
        Mx[a * LD + b] = (T)(a == b ? 1 : 0);
      }
    }
    off += __shfl_xor(off, 16, 64);
    off += __shfl_xor(off, 32, 64);
    dia += __shfl_xor(dia, 16, 64);
    dia += __shfl_xor(dia, 32, 64);
    return __syncthreads_or(b < m && !(dia >= off)) != 0;
  };
  // fused sweep: y = S^{-1}(rhs_scale r_j + extra), extra in vin on entry; y -> gprev, gout
  auto solve_line = [&](int j) {
    for (int i = t; i < M; i += NT) {
      double rv = 0.0;
      if (i < m) {
        const int f = i >= tx;
        rv = rhs_scale * rhs[tile_idx(P, s, f, j, i - f * tx)];
      }
      vin[i] += rv;
    }
    __syncthreads();
    {
      const int row_i = t % M, g = t / M;
      const T* row = Mx + row_i * LD + g * KC;
      double acc = 0.0;
#pragma unroll 4
      for (int k = 0; k < KC; ++k) acc += (double)row[k] * vin[g * KC + k];
      part[g * M + row_i] = acc;
    }
    __syncthreads();
    if (t < M) {
      const double acc = part[t] + part[M + t] + part[2 * M + t] + part[3 * M + t];
      gprev[t] = acc;
      gs[(size_t)j * M + t] = acc;
    }
  };
  // S^{-1} of line j, transposed: facT[j][b][a] = S^{-1}[a][b]
  auto store = [&](int j) {
    T* F = Fs + (size_t)j * M * M;
    for (int e = t; e < M * M / 4; e += NT) {
      const int b = e / (M / 4), a0 = 4 * (e - b * (M / 4));
      T v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = Mx[(a0 + q) * LD + b];
      store4<T>(F + (size_t)b * M + a0, v);
    }
    __syncthreads();
  };

  // this workgroup's half; thread a < tx keeps (y, p) of node a of the next line in
  // registers, so that the HBM loads overlap the work of the current line
  // The line block stays in registers from one line to the next: wave J holds column
  // block J in accumulator layout (c[I]: rows 16 I .. 16 I + 15).  form_block turns the
  // previous inverse (mode 1; mode 0: nothing) into the next line block, D_j +
  // (-hy^-4) S_{j-1}^{-1}: column b of D_j has entries in the diagonal row, the
  // x-neighbours in the same field and the coupling row in the other field.  Identity
  // padding; returns true when some active column is not dominant.
  using VT = typename Mfma<T>::V;
  constexpr int NB = M / 16;
  VT blk[NB];
  auto form_block = [&](auto mode_c) -> bool {
    constexpr int mode = decltype(mode_c)::value;
    const int bl = lane & 15, b = 16 * wave + bl;
    const bool act = b < m;
    const int fc = b >= tx, bc = act ? b - fc * tx : 0;
    const int r_l = act && bc > 0 ? b - 1 : -1, r_r = act && bc + 1 < tx ? b + 1 : -1;
    const int r_c = act ? (fc ? bc : tx + bc) : -1;
    // a padding column is the identity column: its previous inverse column is the
    // identity column too (finite), which the zero scale removes
    const T d_d = act ? (T)((VAR ? ldg[bc] : P.diag0) + la[bc]) : (T)1, d_c = (T)(fc ? lb[bc] : lc[bc]);
    const T d_xl = (T)(VAR ? -lw[bc] : -P.hx2i), d_xr = (T)(VAR ? -le[bc] : -P.hx2i);
    const T sc = act ? nh4 : (T)0;
    const double cpb = VAR && act ? lp[bc] : 0.0;
    T off = 0, dia = 0;
#pragma unroll
    for (int I = 0; I < NB; ++I) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int a = 16 * I + Mfma<T>::row(lane, r);
        // the row tests are the same for every line; recomputing them here keeps the
        // compiler from holding 3 NB * 4 lane masks in scalar registers across the line loop
        asm volatile("" : "+v"(a));
        T d = a == b ? d_d : (T)0;
        d = a == r_l ? d_xl : d;
        d = a == r_r ? d_xr : d;
        d = a == r_c ? d_c : d;
        // -hy^-4 S^{-1} + D (VAR: -C S^{-1} C + D, C the couplings to the previous line),
        // rounded after the product and after the sum (padding rows of an active column: 0)
        T scv = sc;
        if constexpr (VAR) scv = (T)(-(cpb * (a < m ? lp[node(a)] : 0.0)));
        const T v = mode == 0 ? d : add_rn(mul_rn(scv, (T)blk[I][r]), d);
        blk[I][r] = v;
        const T wv = (a < tx ? wy : (T)1) * fabs(v);
        dia = a == b ? wv : dia;
        off += a == b ? (T)0 : wv;
      }
    }
    off = rows_sum(off);
    dia = rows_sum(dia);
    return __syncthreads_or(act && !(dia >= off)) != 0;
  };

  // The inverse of line j goes to HBM straight from the registers (16-byte stores,
  // padding columns included): lane (column b, group g = lane >> 4) writes rows
  // 4 g .. 4 g + 3 of row block I, which are consecutive in the transposed layout
  // facT[j][b][a].  FP32 lanes hold exactly those rows; FP64 lanes hold rows g + 4 r,
  // so the four lane groups first transpose their 4 x 4 block (two 32-lane swaps,
  // then two 16-lane swaps).
  auto store_regs = [&](int j) {
    T* F = Fs + (size_t)j * M * M + (size_t)(16 * wave + (lane & 15)) * M + 4 * (lane >> 4);
#pragma unroll
    for (int I = 0; I < NB; ++I) {
      T r0 = blk[I][0], r1 = blk[I][1], r2 = blk[I][2], r3 = blk[I][3];
      if constexpr (sizeof(T) == 8) {
        swap_lanes32(r0, r2);
        swap_lanes32(r1, r3);
        swap_lanes16(r0, r1);
        swap_lanes16(r2, r3);
      }
      const T v[4] = {r0, r1, r2, r3};
      store4<T>(F + 16 * I, v);
    }
  };

  bool bad = false;
  Raw next{0.0, 0.0, 0.0, 0.0};
  if (nlines > 0 && t < tx) fetch(j0, next);
  for (int k = 0; k < nlines; ++k) {
    const int j = j0 + dir * k;
    if (t < tx) {
      const double y = next.xy + next.cy, p = next.xp + next.cp;
      if (k + 1 < nlines) fetch(j + dir, next);
      coefficients(y, p, j, false);
    }
    __syncthreads();
    if (k == 0 ? form_block(std::integral_constant<int, 0>{}) : form_block(std::integral_constant<int, 1>{})) {
      bad = true;
      break;
    }
    block_gauss_jordan<T, M>(blk, St);
    store_regs(j);
    // the inverse also to LDS, for the fused sweep of the next line
#pragma unroll
    for (int I = 0; I < NB; ++I) tile_store<T>(Mx + 16 * I * LD + 16 * wave, LD, blk[I], lane);
    __syncthreads();
    if (rhs) {
      for (int i = t; i < M; i += NT) {
        if constexpr (VAR) vin[i] = (i < m ? lp[node(i)] : 0.0) * gprev[i];
        else vin[i] = P.hy2i * gprev[i];
      }
      solve_line(j);
    }
  }
  if (phase == 0) {
    if (bad && t == 0) atomicExch(fallback + s, 1);
    return;
  }
  // phase 1: a subdomain one of whose chains failed is redone by k_factor_pivot
  if (fallback[s]) return;
  // the inverse of line t - 1 into Mx, where the top chain leaves it (F[b][a] =
  // inverse[a][b]: 16-byte loads along a)
  if (tw > 0) {
    const T* Fm = Fs + (size_t)(tw - 1) * M * M;
    for (int e4 = t; e4 < M * M / 4; e4 += NT) {
      const int e = 4 * e4, b = e / M, a0 = e - b * M;
      T v[4];
      load4<T>(Fm + e, v);
#pragma unroll
      for (int q = 0; q < 4; ++q) Mx[(a0 + q) * LD + b] = v[q];
    }
  }
  __syncthreads();

  // the twist line: Mx = -hy^-4 (F_{t-1} + F_{t+1}) from the stored inverses, then + D_t
  if (t < tx) {
    double y, p;
    state_at(tw, y, p);
    coefficients(y, p, tw, true);
  }
  if constexpr (VAR) __syncthreads();   // the twist couplings are read below
  // The inverse of line t - 1 is in Mx; that of line t + 1 comes from global memory
  // (stored transposed, F[b][a] = inverse[a][b]), 16-byte loads along a.
  {
    const bool mine = tw > 0;
    const int jo = half == 0 ? tw + 1 : tw - 1;   // the other side's line
    const T* Fo = jo >= 0 && jo < ty ? Fs + (size_t)jo * M * M : nullptr;
    constexpr int PER = M * M / 4 / NT;           // 16-byte groups per thread (M = 16 k)
    T v[PER][4];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = 4 * (t + i * NT);
      if (Fo) load4<T>(Fo + e, v[i]);
      else v[i][0] = v[i][1] = v[i][2] = v[i][3] = 0;
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = 4 * (t + i * NT), b = e / M, a0 = e - b * M;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T* x = Mx + (a0 + q) * LD + b;
        const double own = mine ? (double)*x : 0.0;
        if (VAR && P.cx) {
          // couplings of the row's and the column's nodes to this side's line and the other's
          const double* cm = half == 0 ? lp : lq;
          const double* co = half == 0 ? lq : lp;
          const int na = a0 + q < m ? node(a0 + q) : -1, nb = b < m ? node(b) : -1;
          const double km = na >= 0 && nb >= 0 ? cm[na] * cm[nb] : 0.0;
          const double ko = na >= 0 && nb >= 0 ? co[na] * co[nb] : 0.0;
          *x = (T)(-(km * own + ko * (double)v[i][q]));
        } else {
          *x = (T)(-hy4i * (own + (double)v[i][q]));
        }
      }
    }
  }
  __syncthreads();
  // Z_t subtracts both neighbours' Schur terms and is often close to the boundary of
  // column dominance.  A dominant Z_t takes the register elimination of the chain
  // lines (partial pivoting would keep its diagonal); otherwise its elimination checks
  // the partial-pivoting choice exactly.  Each wave reads and writes only its own
  // column block of Mx here.
  const bool dominant = !build(2);
  if (dominant) {
#pragma unroll
    for (int I = 0; I < NB; ++I) blk[I] = tile_load<T>(Mx + 16 * I * LD + 16 * wave, LD, lane);
    block_gauss_jordan<T, M>(blk, St);
    store_regs(tw);
#pragma unroll
    for (int I = 0; I < NB; ++I) tile_store<T>(Mx + 16 * I * LD + 16 * wave, LD, blk[I], lane);
    __syncthreads();
  } else if (panel_gauss_jordan<T, M>(Mx, LD, Pn, &flag, tx, wy)) {
    if (t == 0) atomicExch(fallback + s, 1);
    return;
  }
  if (rhs) {
    for (int i = t; i < M; i += NT) {
      if (VAR && P.cx) {
        vin[i] = i < m ? (tw > 0 ? lp[node(i)] * gs[(size_t)(tw - 1) * M + i] : 0.0) +
                             (tw + 1 < ty ? lq[node(i)] * gs[(size_t)(tw + 1) * M + i] : 0.0)
                       : 0.0;
      } else {
        vin[i] = P.hy2i * ((tw > 0 ? gs[(size_t)(tw - 1) * M + i] : 0.0) +
                           (tw + 1 < ty ? gs[(size_t)(tw + 1) * M + i] : 0.0));
      }
    }
    solve_line(tw);
  }
  if (!dominant) store(tw);
}

// Fallback for subdomains with a line block that is not column diagonally dominant
// (only the items with only[s] != 0): in-place Gauss-Jordan with partial pivoting in
// registers.  T: arithmetic and storage type of the line inverses (double, or float
// for the FP32 factors of the mixed-precision form); coefficients and the fused
// forward sweep stay in double.
template <typename T, int M>
__global__ __launch_bounds__(kFacThreads) void k_factor_pivot(Items I, const double* __restrict__ tilex,
                                                              const double* __restrict__ c,
                                                              const SubState* __restrict__ state,
                                                              double eps_fixed, const double* __restrict__ rhs,
                                                              double rhs_scale, T* __restrict__ facT,
                                                              double* __restrict__ gout,
                                                              int* __restrict__ only) {
  constexpr int R = M / 16;          // rows (and columns) of the line block per thread
  constexpr int LD = M + 1;
  __shared__ T Mx[M * LD];      // finished in-place Gauss-Jordan result of the line
  __shared__ T colb[2][M];      // pivot column of the current step (double buffered)
  __shared__ int pivb[2];
  __shared__ T pivv[2][2];      // pivot value and its reciprocal
  __shared__ int pr[2][M], pinv[2][M];
  __shared__ double la[M / 2], lb[M / 2], lc[M / 2];
  // variable coefficients of A (as in k_factor_mfma): diagonal, west / east couplings,
  // couplings to the previous line (twist: to line tw - 1) and, at the twist, to tw + 1
  __shared__ double ldg[M / 2], lw[M / 2], le[M / 2], lp[M / 2], lq[M / 2];
  __shared__ double vin[M], gprev[M];

  int s;
  DevProblem P;
  if (!item_of(I, s, P)) return;
  if (!only[s]) return;
  const bool var = P.cx != nullptr;
  const int t = threadIdx.x, ti = t & 15, tj = t >> 4;
  const int lane = t & 63;
  double eps = eps_fixed > 0.0 ? eps_fixed : eps_fixed < 0.0 ? P.eps_start : P.eps_min;
  if (state) {
    if (!state[s].active) return;
    eps = state[s].eps;
  }
  const int4 bx = I.box[s];
  const int tx = bx.y - bx.x, ty = bx.w - bx.z;
  const int m = 2 * tx;
  const double hy4i = P.hy2i * P.hy2i;
  T A[R][R];

  const int tw = ty / 2;
  const T* Fm = tw > 0 ? facT + ((size_t)s * P.tym + tw - 1) * M * M : nullptr;
  const T* Fp = tw + 1 < ty ? facT + ((size_t)s * P.tym + tw + 1) * M * M : nullptr;
  for (int i = t; i < M; i += kFacThreads) gprev[i] = 0.0;

  // the two-ended order of k_factor_mfma: top lines 0 .. t-1, bottom lines ty-1 .. t+1,
  // then the twist line t, whose neighbours' inverses and vectors are read back from
  // facT and gout
  for (int q = 0; q < ty; ++q) {
    const bool twist = q == ty - 1;
    const int j = q < tw ? q : (twist ? tw : ty - 1 - (q - tw));
    const bool has_prev = q < tw ? q > 0 : (!twist && q > tw);
    if (twist) __threadfence();
    const int pj = q & 1, pp = pj ^ 1;
    // coefficients of line j at z = R_i x + c
    for (int a = t; a < tx; a += kFacThreads) {
      const double y = tilex[halo_idx(P, s, 0, j + 1, a + 1)] + (c ? c[tile_idx(P, s, 0, j, a)] : 0.0);
      const double p = tilex[halo_idx(P, s, 1, j + 1, a + 1)] + (c ? c[tile_idx(P, s, 1, j, a)] : 0.0);
      la[a] = dphi_of(P.phi, y, P.kappa);
      lb[a] = dg_of(p, P.mu, eps) * P.inv_nu;
      lc[a] = ddphi_of(P.phi, y, P.kappa) * p - 1.0;
      if (var) {
        const int gi = bx.x + a, gj = bx.z + j;
        ldg[a] = a_diag(P, gi, gj);
        lw[a] = c_w(P, gi, gj);
        le[a] = c_e(P, gi, gj);
        lp[a] = (q < tw || twist) ? c_s(P, gi, gj) : c_n(P, gi, gj);
        lq[a] = c_n(P, gi, gj);
      }
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
            if (ar == ac) d = (var ? ldg[ar] : P.diag0) + la[ar];
            else if (ar == ac + 1) d = var ? -lw[ar] : -P.hx2i;
            else if (ac == ar + 1) d = var ? -le[ar] : -P.hx2i;
          } else if (ar == ac) {
            d = fr == 0 ? lb[ar] : lc[ar];
          }
          if (var) {
            // -C S^{-1} C with the diagonal couplings C of the faces to the neighbour lines
            if (has_prev) d -= lp[ar] * lp[ac] * (double)Mx[pr[pp][a] * LD + pinv[pp][b]];
            if (twist)
              d -= lp[ar] * lp[ac] * (Fm ? (double)Fm[(size_t)b * M + a] : 0.0) +
                   lq[ar] * lq[ac] * (Fp ? (double)Fp[(size_t)b * M + a] : 0.0);
          } else {
            if (has_prev) d -= hy4i * (double)Mx[pr[pp][a] * LD + pinv[pp][b]];
            if (twist) d -= hy4i * ((Fm ? (double)Fm[(size_t)b * M + a] : 0.0) +
                                   (Fp ? (double)Fp[(size_t)b * M + a] : 0.0));
          }
        }
        A[rr][cc] = (T)d;
      }
    }
    {
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
        if (var) {
          const int nd = i < tx ? i : i - tx;
          double nb = 0.0;
          if (i < m) {
            if (has_prev) nb += lp[nd] * gprev[i];
            if (twist) {
              const double* gs = gout + (size_t)s * P.tym * M;
              if (tw > 0) nb += lp[nd] * gs[(size_t)(tw - 1) * M + i];
              if (tw + 1 < ty) nb += lq[nd] * gs[(size_t)(tw + 1) * M + i];
            }
          }
          vin[i] = rv + nb;
        } else {
          double nb = has_prev ? gprev[i] : 0.0;
          if (twist) {
            const double* gs = gout + (size_t)s * P.tym * M;
            if (tw > 0) nb += gs[(size_t)(tw - 1) * M + i];
            if (tw + 1 < ty) nb += gs[(size_t)(tw + 1) * M + i];
          }
          vin[i] = rv + P.hy2i * nb;
        }
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
  if (t == 0) only[s] = 0;   // consumed: the flags start at 0 for the next launch
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

// The chains (phase 0), the twist lines (phase 1), then the pivoting redo of the flagged
// subdomains.
template <typename T, int MM>
void factor_launches(const Items& I, const double* tilex, const double* c, const SubState* state,
                     double eps_fixed, const double* rhs, double rhs_scale, T* facT, double* g, int* fallback,
                     bool var, hipStream_t st) {
  const dim3 chains(I.count, 2), twist(I.count, 1);
  if (var) {
    k_factor_mfma<T, MM, true><<<chains, 4 * MM, 0, st>>>(I, tilex, c, state, eps_fixed, rhs, rhs_scale, facT, g,
                                                          fallback, 0);
    k_factor_mfma<T, MM, true><<<twist, 4 * MM, 0, st>>>(I, tilex, c, state, eps_fixed, rhs, rhs_scale, facT, g,
                                                         fallback, 1);
  } else {
    k_factor_mfma<T, MM, false><<<chains, 4 * MM, 0, st>>>(I, tilex, c, state, eps_fixed, rhs, rhs_scale, facT, g,
                                                           fallback, 0);
    k_factor_mfma<T, MM, false><<<twist, 4 * MM, 0, st>>>(I, tilex, c, state, eps_fixed, rhs, rhs_scale, facT, g,
                                                          fallback, 1);
  }
  k_factor_pivot<T, MM><<<I.count, kFacThreads, 0, st>>>(I, tilex, c, state, eps_fixed, rhs, rhs_scale, facT, g,
                                                         fallback);
}

void launch_factor(const Items& I, int M, const double* tilex, const double* c, const SubState* state,
                   double eps_fixed, const double* rhs, double rhs_scale, void* facT, int fp32, double* g,
                   int* fallback, bool var, hipStream_t st) {
  if (I.count <= 0) return;
  if (fp32) {
#define RSP_CALL(MM) \
  factor_launches<float, MM>(I, tilex, c, state, eps_fixed, rhs, rhs_scale, (float*)facT, g, fallback, var, st)
    RSP_DISPATCH_M(M, RSP_CALL)
#undef RSP_CALL
  } else {
#define RSP_CALL(MM) \
  factor_launches<double, MM>(I, tilex, c, state, eps_fixed, rhs, rhs_scale, (double*)facT, g, fallback, var, st)
    RSP_DISPATCH_M(M, RSP_CALL)
#undef RSP_CALL
  }
}

}  // namespace rsp
