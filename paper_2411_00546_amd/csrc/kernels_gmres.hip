// Device-resident restarted GMRES (x_0 = 0) for the RASPEN Newton system of
// Algorithm 2: Arnoldi with classical Gram-Schmidt applied twice, Givens rotations
// on the Hessenberg column, the stopping test |g_{j+1}| <= rtol |b| and the
// triangular solve, all on the device.  A stop flag written by the Givens kernel
// lets the host enqueue a whole restart cycle without reading anything back:
// every kernel of a later step returns at once when the flag is set.
//
// Reductions are deterministic: kGmBlocks fixed blocks each own a contiguous
// chunk, write their partial sums, and every consumer adds the partials in block
// order.
#include "rsp_kernels.h"

namespace rsp {

namespace {

constexpr int kT = 256;

__device__ __forceinline__ void chunk_of(size_t L, size_t& lo, size_t& hi) {
  const size_t ch = (L + kGmBlocks - 1) / kGmBlocks;
  lo = blockIdx.x * ch;
  hi = lo + ch < L ? lo + ch : L;
  if (lo > L) lo = L;
}

// Block sums of acc[i] for i < nv (wave shuffles, then the 4 wave results in order);
// thread i < nv of the block returns sum i.  Fixed order: deterministic.
template <int NB>
__device__ __forceinline__ double block_sums(const double (&acc)[NB], int nv, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (i < nv) {
      double v = acc[i];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) red[wave * kGmMaxVec + i] = v;
    }
  }
  __syncthreads();
  double r = 0.0;
  if ((int)threadIdx.x < nv)
    for (int w = 0; w < kT / 64; ++w) r += red[w * kGmMaxVec + threadIdx.x];
  return r;
}

// h[i] = sum_blk partial[blk][i] for i < nv -> LDS hs (every block, same fixed order):
// thread (i, q) adds blocks q, q + Q, ... with independent loads, then thread i adds
// the Q segment sums in order.
__device__ __forceinline__ void gather_partials(const double* __restrict__ partial, int nv,
                                                double* hs) {
  __shared__ double seg[kT];
  const int Q = nv > 0 ? (kT / nv < kGmBlocks ? kT / nv : kGmBlocks) : 1;
  const int t = threadIdx.x;
  if (t < nv * Q) {
    const int i = t / Q, q = t - i * Q;
    double acc = 0.0;
#pragma unroll 8
    for (int b = q; b < kGmBlocks; b += Q) acc += partial[b * kGmMaxVec + i];
    seg[t] = acc;
  }
  __syncthreads();
  if (t < nv) {
    double acc = 0.0;
    for (int q = 0; q < Q; ++q) acc += seg[t * Q + q];
    hs[t] = acc;
  }
  __syncthreads();
}

// NB: compile-time bound on the number of basis vectors (bucket >= nv).  Loads of all
// NB vectors are issued unconditionally (index clamped to nv - 1, the extra ones hit
// the cache) and the unused products are masked, so the loads are not serialised.

// partial sums of V_i . w for i < nv over this block's chunk
template <int NB>
__global__ __launch_bounds__(kT) void k_gm_dots(const double* __restrict__ V, size_t L, int nv,
                                                const double* __restrict__ w,
                                                const GmState* __restrict__ st,
                                                double* __restrict__ partial) {
  __shared__ double red[(kT / 64) * kGmMaxVec];
  if (st->done) return;
  size_t lo, hi;
  chunk_of(L, lo, hi);
  double acc[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) acc[i] = 0.0;
  for (size_t e = lo + threadIdx.x; e < hi; e += kT) {
    const double we = w[e];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const double v = V[(size_t)min(i, nv - 1) * L + e];
      acc[i] = fma(v, i < nv ? we : 0.0, acc[i]);
    }
  }
  const double r = block_sums<NB>(acc, nv, red);
  if ((int)threadIdx.x < nv) partial[blockIdx.x * kGmMaxVec + threadIdx.x] = r;
}

// h = sum of the previous partials; w -= V h; then either the partial dots of the new
// w with V (next = 0) or its partial squared norm (next = 1).  Block 0 adds h into
// the Hessenberg column j.
template <int NB>
__global__ __launch_bounds__(kT) void k_gm_update(const double* __restrict__ V, size_t L, int nv,
                                                  double* __restrict__ w, GmState* __restrict__ st,
                                                  const double* __restrict__ pin, int first,
                                                  int next, double* __restrict__ pout, int j) {
  __shared__ double red[(kT / 64) * kGmMaxVec];
  __shared__ double hs[kGmMaxVec];
  if (st->done) return;
  gather_partials(pin, nv, hs);
  if (blockIdx.x == 0 && (int)threadIdx.x < nv) {
    const int m = st->m;
    double* Hc = st->H + threadIdx.x * m + j;
    *Hc = first ? hs[threadIdx.x] : *Hc + hs[threadIdx.x];
  }
  double h[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) h[i] = i < nv ? hs[i] : 0.0;
  size_t lo, hi;
  chunk_of(L, lo, hi);
  double acc[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) acc[i] = 0.0;
  for (size_t e = lo + threadIdx.x; e < hi; e += kT) {
    double v[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) v[i] = V[(size_t)min(i, nv - 1) * L + e];
    double we = w[e];
#pragma unroll
    for (int i = 0; i < NB; ++i) we = fma(-h[i], v[i], we);
    w[e] = we;
    if (next == 0) {
#pragma unroll
      for (int i = 0; i < NB; ++i) acc[i] = fma(v[i], i < nv ? we : 0.0, acc[i]);
    } else {
      acc[0] = fma(we, we, acc[0]);
    }
  }
  const int nout = next == 0 ? nv : 1;
  const double r = block_sums<NB>(acc, nout, red);
  if ((int)threadIdx.x < nout) pout[blockIdx.x * kGmMaxVec + threadIdx.x] = r;
}

// |w| from the partials; V_{j+1} = w / |w|; block 0 stores H[j+1][j].
__global__ __launch_bounds__(kT) void k_gm_normalize(double* __restrict__ Vn, size_t L,
                                                     const double* __restrict__ w,
                                                     GmState* __restrict__ st,
                                                     const double* __restrict__ pin, int j) {
  __shared__ double hs[1];
  if (st->done) return;
  gather_partials(pin, 1, hs);
  const double nrm = sqrt(hs[0]);
  if (blockIdx.x == 0 && threadIdx.x == 0) st->H[(j + 1) * st->m + j] = nrm;
  const double inv = 1.0 / nrm;
  size_t lo, hi;
  chunk_of(L, lo, hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += kT) Vn[e] = w[e] * inv;
}

// Givens rotations on Hessenberg column j, residual estimate and stopping test.  The
// column and the rotations are staged in LDS so the sequential part runs from LDS.
__global__ __launch_bounds__(kT) void k_gm_givens(GmState* __restrict__ st, int j) {
  __shared__ double col[kGmMaxVec], cs[kGmMaxRestart], sn[kGmMaxRestart];
  if (st->done) return;
  const int m = st->m;
  const int t = threadIdx.x;
  if (t <= j + 1) col[t] = st->H[t * m + j];
  if (t < j) {
    cs[t] = st->cs[t];
    sn[t] = st->sn[t];
  }
  __syncthreads();
  if (t != 0) return;
  for (int i = 0; i < j; ++i) {
    const double a = col[i], b = col[i + 1];
    col[i] = cs[i] * a + sn[i] * b;
    col[i + 1] = -sn[i] * a + cs[i] * b;
  }
  const double a = col[j], b = col[j + 1];
  const double den = hypot(a, b);
  const double c = a / den, s = b / den;
  st->cs[j] = c;
  st->sn[j] = s;
  col[j] = den;
  col[j + 1] = 0.0;
  for (int i = 0; i <= j + 1; ++i) st->H[i * m + j] = col[i];
  const bool breakdown = !(b > 0.0);
  const double gj = st->g[j];
  st->g[j + 1] = -s * gj;
  st->g[j] = c * gj;
  st->rel = fabs(st->g[j + 1]) / st->bnorm;
  st->steps = j + 1;
  st->used += 1;
  if (!(st->rel > st->rtol) || st->used >= st->maxit || breakdown || j + 1 >= m) st->done = 1;
}

// Cycle start: beta = |r| from partials, V_0 = r / beta, g = (beta, 0, ...).
__global__ __launch_bounds__(kT) void k_gm_start(double* __restrict__ V0, size_t L,
                                                 const double* __restrict__ r,
                                                 GmState* __restrict__ st,
                                                 const double* __restrict__ pin, int first_cycle) {
  __shared__ double hs[1];
  gather_partials(pin, 1, hs);
  const double beta = sqrt(hs[0]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (first_cycle) st->bnorm = beta;
    st->beta = beta;
    for (int i = 0; i <= st->m; ++i) st->g[i] = 0.0;
    st->g[0] = beta;
    st->steps = 0;
    st->rel = st->bnorm > 0.0 ? beta / st->bnorm : 0.0;
    st->done = (!(beta > st->rtol * st->bnorm) || st->used >= st->maxit) ? 1 : 0;
  }
  if (!(beta > 0.0)) return;
  const double inv = 1.0 / beta;
  size_t lo, hi;
  chunk_of(L, lo, hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += kT) V0[e] = r[e] * inv;
}

// y = R^{-1} g (back substitution over the steps done), x += V y.
__global__ __launch_bounds__(kT) void k_gm_update_x(const double* __restrict__ V, size_t L,
                                                    GmState* __restrict__ st,
                                                    double* __restrict__ x) {
  __shared__ double ys[kGmMaxVec];
  const int k = st->steps;
  if (threadIdx.x == 0) {
    const int m = st->m;
    for (int i = k - 1; i >= 0; --i) {
      double s = st->g[i];
      for (int l = i + 1; l < k; ++l) s -= st->H[i * m + l] * ys[l];
      ys[i] = s / st->H[i * m + i];
    }
  }
  __syncthreads();
  size_t lo, hi;
  chunk_of(L, lo, hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += kT) {
    double acc = x[e];
    for (int i = 0; i < k; ++i) acc += ys[i] * V[(size_t)i * L + e];
    x[e] = acc;
  }
}

// partial squared norms of v (for k_gm_start)
__global__ __launch_bounds__(kT) void k_gm_sumsq(const double* __restrict__ v, size_t L,
                                                 double* __restrict__ partial) {
  __shared__ double red[(kT / 64) * kGmMaxVec];
  size_t lo, hi;
  chunk_of(L, lo, hi);
  double acc[kGmMaxVec];
#pragma unroll
  for (int i = 0; i < kGmMaxVec; ++i) acc[i] = 0.0;
  for (size_t e = lo + threadIdx.x; e < hi; e += kT) acc[0] = fma(v[e], v[e], acc[0]);
  const double r = block_sums(acc, 1, red);
  if (threadIdx.x == 0) partial[blockIdx.x * kGmMaxVec] = r;
}

// r = b - w
__global__ __launch_bounds__(kT) void k_gm_residual(const double* __restrict__ b,
                                                    const double* __restrict__ w,
                                                    double* __restrict__ r, size_t L) {
  size_t lo, hi;
  chunk_of(L, lo, hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += kT) r[e] = b[e] - w[e];
}

}  // namespace

void gm_init_state(GmState* st_dev, int m, int maxit, double rtol, hipStream_t s) {
  GmState h{};
  h.m = m;
  h.maxit = maxit;
  h.rtol = rtol;
  (void)hipMemcpyAsync(st_dev, &h, sizeof(GmState), hipMemcpyHostToDevice, s);
}

void launch_gm_sumsq(const double* v, size_t L, double* partial, hipStream_t s) {
  k_gm_sumsq<<<kGmBlocks, kT, 0, s>>>(v, L, partial);
}
void launch_gm_residual(const double* b, const double* w, double* r, size_t L, hipStream_t s) {
  k_gm_residual<<<kGmBlocks, kT, 0, s>>>(b, w, r, L);
}
void launch_gm_start(double* V0, size_t L, const double* r, GmState* st, const double* partial,
                     int first_cycle, hipStream_t s) {
  k_gm_start<<<kGmBlocks, kT, 0, s>>>(V0, L, r, st, partial, first_cycle);
}
template <int NB>
void arnoldi_nb(const double* V, size_t L, int j, double* w, GmState* st, double* p1, double* p2,
                hipStream_t s) {
  const int nv = j + 1;
  k_gm_dots<NB><<<kGmBlocks, kT, 0, s>>>(V, L, nv, w, st, p1);
  k_gm_update<NB><<<kGmBlocks, kT, 0, s>>>(V, L, nv, w, st, p1, 1, 0, p2, j);
  k_gm_update<NB><<<kGmBlocks, kT, 0, s>>>(V, L, nv, w, st, p2, 0, 1, p1, j);
  k_gm_normalize<<<kGmBlocks, kT, 0, s>>>(const_cast<double*>(V) + (size_t)(j + 1) * L, L, w, st, p1, j);
  k_gm_givens<<<1, kT, 0, s>>>(st, j);
}

void launch_gm_arnoldi(const double* V, size_t L, int j, double* w, GmState* st, double* p1,
                       double* p2, hipStream_t s) {
  const int nv = j + 1;
  if (nv <= 8) arnoldi_nb<8>(V, L, j, w, st, p1, p2, s);
  else if (nv <= 16) arnoldi_nb<16>(V, L, j, w, st, p1, p2, s);
  else if (nv <= 32) arnoldi_nb<32>(V, L, j, w, st, p1, p2, s);
  else arnoldi_nb<64>(V, L, j, w, st, p1, p2, s);
}
void launch_gm_update_x(const double* V, size_t L, GmState* st, double* x, hipStream_t s) {
  k_gm_update_x<<<kGmBlocks, kT, 0, s>>>(V, L, st, x);
}

}  // namespace rsp
