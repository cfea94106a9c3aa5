// Matrix-core tiles and the blocked Gauss-Jordan inverse on them (device helpers shared
// by the line factors and the coarse factor).
#pragma once
#include <hip/hip_runtime.h>

namespace rsp {

namespace {

// ---------------------------------------------------------------- MFMA tiles
// 16 x 16 x 4 matrix-core products (one wave).  Operand A[i][k] sits in lane i + 16 k,
// operand B[k][j] in lane j + 16 k; the accumulator D[i][j] sits in lane j + 16 g,
// register r, with i = 4 g + r for float and i = 4 r + g for double.  A product over
// 16 values of k takes four instructions; instruction q of lane group k0 uses
// k = kappa(q, k0), with kappa = 4 k0 + q for float and 4 q + k0 for double, so that
// register q of an accumulator tile is exactly the B operand of instruction q: a
// result tile feeds the next product from registers.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  using V = f32x4;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
  static __device__ __forceinline__ int kap(int q, int k0) { return 4 * k0 + q; }
};
template <>
struct Mfma<double> {
  using V = f64x4;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
  static __device__ __forceinline__ int kap(int q, int k0) { return 4 * q + k0; }
};

// Row stride (in elements) that keeps the rows of an LDS matrix 16-byte aligned.
template <typename T>
constexpr int padded(int n) { return n + 16 / (int)sizeof(T); }

template <typename T>
__device__ __forceinline__ void load4(const T* p, T (&v)[4]);
template <>
__device__ __forceinline__ void load4<float>(const float* p, float (&v)[4]) {
  const f32x4 x = *reinterpret_cast<const f32x4*>(p);
  v[0] = x[0]; v[1] = x[1]; v[2] = x[2]; v[3] = x[3];
}
template <>
__device__ __forceinline__ void load4<double>(const double* p, double (&v)[4]) {
  const double2 x = reinterpret_cast<const double2*>(p)[0];
  const double2 y = reinterpret_cast<const double2*>(p)[1];
  v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
}
template <typename T>
__device__ __forceinline__ void store4(T* p, const T (&v)[4]);
template <>
__device__ __forceinline__ void store4<float>(float* p, const float (&v)[4]) {
  f32x4 x;
  x[0] = v[0]; x[1] = v[1]; x[2] = v[2]; x[3] = v[3];
  *reinterpret_cast<f32x4*>(p) = x;
}
template <>
__device__ __forceinline__ void store4<double>(double* p, const double (&v)[4]) {
  reinterpret_cast<double2*>(p)[0] = make_double2(v[0], v[1]);
  reinterpret_cast<double2*>(p)[1] = make_double2(v[2], v[3]);
}

// Pivot reciprocal: the hardware reciprocal (1 ulp) for the FP32 factors; for FP64 the
// hardware estimate refined by two Newton steps r <- r + r (1 - x r) (each squares the
// relative error).
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// Lane exchanges inside one wave, as VALU operations (no LDS).  Rows are the four
// groups of 16 lanes.
//   row_bcast<n>(v): lane n of each row, to every lane of that row (DPP row_newbcast);
//   col_bcast<R>(v): lane (i, row R), to lane (i, any row) (two permlane swaps: the
//     16-lane swap pairs rows 0-1 and 2-3, the 32-lane swap pairs the halves);
//   read_lane(v, l): lane l, to every lane.
template <int N>
__device__ __forceinline__ int row_bcast_i(int v) {
  // every lane reads a lane of its own row, so no lane keeps its old value: the move
  // needs no copy of the source
  return __builtin_amdgcn_mov_dpp(v, 0x150 + N, 0xF, 0xF, false);
}
template <int R>
__device__ __forceinline__ int col_bcast_i(int v) {
  const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);   // rows (0,0,2,2), (1,1,3,3)
  const int c = (int)((R & 1) ? p[1] : p[0]);
  const auto q = __builtin_amdgcn_permlane32_swap(c, c, false, false);   // (c0,c1,c0,c1), (c2,c3,c2,c3)
  return (int)((R & 2) ? q[1] : q[0]);
}
template <int N>
__device__ __forceinline__ float row_bcast(float v) {
  return __int_as_float(row_bcast_i<N>(__float_as_int(v)));
}
template <int N>
__device__ __forceinline__ double row_bcast(double v) {
  return __hiloint2double(row_bcast_i<N>(__double2hiint(v)), row_bcast_i<N>(__double2loint(v)));
}
template <int R>
__device__ __forceinline__ float col_bcast(float v) {
  return __int_as_float(col_bcast_i<R>(__float_as_int(v)));
}
template <int R>
__device__ __forceinline__ double col_bcast(double v) {
  return __hiloint2double(col_bcast_i<R>(__double2hiint(v)), col_bcast_i<R>(__double2loint(v)));
}
// Exchanges between lane groups of two double registers a, b (groups = 16-lane rows):
//   swap_lanes32: a <- (a rows 0,1; b rows 0,1), b <- (a rows 2,3; b rows 2,3);
//   swap_lanes16: a <- (a row 0, b row 0, a row 2, b row 2), b <- (a row 1, b row 1,
//                 a row 3, b row 3).
__device__ __forceinline__ void swap_lanes32(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
  a = __hiloint2double((int)hi[0], (int)lo[0]);
  b = __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ void swap_lanes16(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
  a = __hiloint2double((int)hi[0], (int)lo[0]);
  b = __hiloint2double((int)hi[1], (int)lo[1]);
}
// Product and sum rounded separately (never contracted into one fused operation).
__device__ __forceinline__ float mul_rn(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ float add_rn(float a, float b) { return __fadd_rn(a, b); }
__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }

// Sum over the four 16-lane rows of a wave (lanes i, i + 16, i + 32, i + 48), the
// same value in all four: the 16-lane swap adds rows 0+1 and 2+3, the 32-lane swap
// adds the halves.
__device__ __forceinline__ int2 swap_pair16(int v) {
  const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return make_int2((int)p[0], (int)p[1]);
}
__device__ __forceinline__ int2 swap_pair32(int v) {
  const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return make_int2((int)p[0], (int)p[1]);
}
__device__ __forceinline__ float rows_sum(float v) {
  int2 p = swap_pair16(__float_as_int(v));
  v = __int_as_float(p.x) + __int_as_float(p.y);
  p = swap_pair32(__float_as_int(v));
  return __int_as_float(p.x) + __int_as_float(p.y);
}
__device__ __forceinline__ double rows_sum(double v) {
  int2 lo = swap_pair16(__double2loint(v)), hi = swap_pair16(__double2hiint(v));
  v = __hiloint2double(hi.x, lo.x) + __hiloint2double(hi.y, lo.y);
  lo = swap_pair32(__double2loint(v));
  hi = swap_pair32(__double2hiint(v));
  return __hiloint2double(hi.x, lo.x) + __hiloint2double(hi.y, lo.y);
}
__device__ __forceinline__ float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double read_lane(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// In-place inverse of the 16 x 16 block X (LDS, row stride ld) by Gauss-Jordan with
// pivots in order, by one wave in registers: lane (i, r) = i + 16 r holds row i,
// columns 4 r .. 4 r + 3.  Step k takes the pivot row from lane (k, r) (row_bcast),
// the pivot-column entry of row i from lane (i, k / 4) (col_bcast) and the pivot from
// lane (k, k / 4).  Row i != k becomes a_i - m_i a_k with m_i = a_ik / a_kk, the pivot
// row a_k / a_kk, and column k holds -m_i (row i != k) and 1 / a_kk (row k): one fused
// multiply-add per entry with the row factor f_i = -m_i (f_k = 1 / a_kk, applied to a
// zeroed pivot row), which is also the new column-k entry.
template <typename T, int K>
__device__ __forceinline__ void gj16_step(T (&own)[4], int li, int q4) {
  constexpr int KQ = K >> 2, KR = K & 3;
  T prow[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) prow[q] = row_bcast<K>(own[q]);
  const T pcol = col_bcast<KQ>(own[KR]);
  const T inv = recip(read_lane(own[KR], K + 16 * KQ));
  const bool on_row = li == K;
  const T f = on_row ? inv : -(pcol * inv);
#pragma unroll
  for (int q = 0; q < 4; ++q) own[q] = fma(f, prow[q], on_row ? (T)0 : own[q]);
  own[KR] = q4 == KQ ? f : own[KR];
}
template <typename T, int K>
__device__ __forceinline__ void gj16_steps(T (&own)[4], int li, int q4) {
  if constexpr (K < 16) {
    gj16_step<T, K>(own, li, q4);
    gj16_steps<T, K + 1>(own, li, q4);
  }
}

// A operand (row-major 16 x 16 tile X, stride ldx) of instruction q.
template <typename T>
__device__ __forceinline__ void a_operand(const T* X, int ldx, int lane, T (&a)[4]) {
  const int i = lane & 15, k0 = lane >> 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) a[q] = X[i * ldx + Mfma<T>::kap(q, k0)];
}
// B operand (row-major 16 x 16 tile Y, stride ldy) of instruction q.
template <typename T>
__device__ __forceinline__ void b_operand(const T* Y, int ldy, int lane, T (&b)[4]) {
  const int j = lane & 15, k0 = lane >> 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) b[q] = Y[Mfma<T>::kap(q, k0) * ldy + j];
}
// c += sgn a b over the 16 values of k
template <typename T>
__device__ __forceinline__ typename Mfma<T>::V mma16(const T (&a)[4], const T (&b)[4], T sgn,
                                                     typename Mfma<T>::V c) {
#pragma unroll
  for (int q = 0; q < 4; ++q) c = Mfma<T>::mma(sgn * a[q], b[q], c);
  return c;
}

template <typename T>
__device__ __forceinline__ typename Mfma<T>::V tile_load(const T* X, int ldx, int lane) {
  typename Mfma<T>::V c;
#pragma unroll
  for (int r = 0; r < 4; ++r) c[r] = X[Mfma<T>::row(lane, r) * ldx + (lane & 15)];
  return c;
}

template <typename T>
__device__ __forceinline__ void tile_store(T* X, int ldx, typename Mfma<T>::V c, int lane) {
#pragma unroll
  for (int r = 0; r < 4; ++r) X[Mfma<T>::row(lane, r) * ldx + (lane & 15)] = c[r];
}

// Inverse of the M x M matrix A by Gauss-Jordan with 16 x 16 pivot blocks taken in
// order (no pivot search): for pivot block K,
//   A_KK <- A_KK^{-1},  A_KJ <- A_KK^{-1} A_KJ,  A_IK <- -A_IK A_KK^{-1},
//   A_IJ <- A_IJ - A_IK A_KK^{-1} A_KJ                      (I, J != K).
// This is the partial-pivoting Gauss-Jordan result whenever partial pivoting would
// keep the diagonal: for column diagonally dominant A always (the Schur complements
// inherit the property).  M / 16 waves; wave J owns column block J in registers, c[I]
// holding tile (I, J) in accumulator layout (a tile in that layout is exactly the B
// operand of a product), on entry the matrix and on return its inverse.  Step K: wave K publishes its old column and
// the inverse of A_KK (inverted by one wave in registers, gj16_steps) into a staging
// panel, the other waves take the inverse and their A_IK from there as A operands and
// update their tiles in registers, and wave K forms its new column.  The staging
// panels alternate between steps, so a step needs one barrier.  St: 2 panels of
// M x padded(16).
template <typename T, int M>
__device__ __forceinline__ void block_gauss_jordan(typename Mfma<T>::V (&c)[M / 16], T* St) {
  constexpr int NB = M / 16;
  constexpr int PLD = padded<T>(16);
  using V = typename Mfma<T>::V;
  const int t = threadIdx.x, lane = t & 63, J = t >> 6;
  const int li = lane & 15, q4 = lane >> 4;
#pragma unroll
  for (int K = 0; K < NB; ++K) {
    T* S = St + (K & 1) * M * PLD;
    if (J == K) {
      if constexpr (sizeof(T) == 4) {
        // FP32: lane (j, g) holds rows 4 g .. 4 g + 3 of column j, which is the row
        // layout of gj16_steps for the transpose; inverting the transpose in place
        // leaves A_KK^{-1} in accumulator layout, without a trip through LDS
#pragma unroll
        for (int I = 0; I < NB; ++I)
          if (I != K) tile_store<T>(S + 16 * I * PLD, PLD, c[I], lane);
        T own[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) own[q] = c[K][q];
        gj16_steps<T, 0>(own, li, q4);
#pragma unroll
        for (int q = 0; q < 4; ++q) c[K][q] = own[q];
        tile_store<T>(S + 16 * K * PLD, PLD, c[K], lane);
      } else {
#pragma unroll
        for (int I = 0; I < NB; ++I) tile_store<T>(S + 16 * I * PLD, PLD, c[I], lane);
        T own[4];
        load4<T>(S + (16 * K + li) * PLD + 4 * q4, own);
        gj16_steps<T, 0>(own, li, q4);
        store4<T>(S + (16 * K + li) * PLD + 4 * q4, own);
      }
    }
    __syncthreads();
    if (J != K) {
      // row-panel tile R = A_KK^{-1} A_KJ, then A_IJ -= A_IK R, A_KJ = R
      T a[4], b[4];
      a_operand<T>(S + 16 * K * PLD, PLD, lane, a);
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = c[K][q];
      V r = {0, 0, 0, 0};
      r = mma16<T>(a, b, (T)1, r);
      T rb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) rb[q] = r[q];
#pragma unroll
      for (int I = 0; I < NB; ++I) {
        if (I == K) continue;
        T ai[4];
        a_operand<T>(S + 16 * I * PLD, PLD, lane, ai);
        c[I] = mma16<T>(ai, rb, (T)-1, c[I]);
      }
      c[K] = r;
    } else {
      // new column K: A_IK <- -A_IK A_KK^{-1} (I != K), A_KK <- its inverse (FP32: c[K]
      // already holds it, in the B-operand layout)
      T b[4];
      if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int q = 0; q < 4; ++q) b[q] = c[K][q];
      } else {
        b_operand<T>(S + 16 * K * PLD, PLD, lane, b);
      }
#pragma unroll
      for (int I = 0; I < NB; ++I) {
        if (I == K) continue;
        T ai[4];
        a_operand<T>(S + 16 * I * PLD, PLD, lane, ai);
        V z = {0, 0, 0, 0};
        c[I] = mma16<T>(ai, b, (T)-1, z);
      }
      if constexpr (sizeof(T) != 4) c[K] = tile_load<T>(S + 16 * K * PLD, PLD, lane);
    }
  }
}

}  // namespace

}  // namespace rsp
