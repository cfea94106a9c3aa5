// Device-resident restarted GMRES (x_0 = 0) for the RASPEN Newton systems of
// Algorithm 2, for every instance of a batch at once: Arnoldi with classical
// Gram-Schmidt applied twice, Givens rotations on the Hessenberg column, the
// stopping test |g_{j+1}| <= rtol |b| and the triangular solve, all on the device.
//
// Normalisation is deferred by one step: the second Gram-Schmidt pass of step j
// writes the orthogonalised vector unscaled into V_{j+1} together with partial sums
// of its squared norm, the Jacobian action of step j+1 takes it unscaled (the
// operator is linear), and the first kernel of step j+1 scales V_{j+1} and the
// product by 1/|V_{j+1}| while it forms the dot products, and applies the Givens
// rotations to column j.  An Arnoldi step is three launches; a chunk of steps ends
// with one small launch that finishes its last column.
// Launch grid: (kGmBlocks, instances); blockIdx.y selects the instance, whose
// vectors are its segment of the batch's concatenated vectors (basis vector k of
// every instance: V + k ldv).  A per-instance stop
// flag written by the Givens kernel lets the host enqueue a whole restart cycle
// without reading anything back: the kernels of a stopped instance return at once.
//
// Reductions are deterministic and depend only on the instance's own length:
// kGmBlocks fixed blocks each own a contiguous chunk, write their partial sums, and
// every consumer adds the partials in block order.
#include "rsp_kernels.h"

namespace rsp {

namespace {

constexpr int kT = 256;
constexpr size_t kPart = (size_t)kGmBlocks * kGmMaxVec;   // partial sums per instance

// Partial sum i of block b, laid out [i][b] so the consumers read runs of blocks.
__device__ __forceinline__ size_t part_at(int i, int b) { return (size_t)i * kGmBlocks + b; }

struct Seg {
  int i;          // instance
  size_t off, L;  // its vector segment
};

__device__ __forceinline__ Seg seg_of(const GmBatch& B) {
  Seg g;
  g.i = B.list ? B.list[blockIdx.y] : (int)blockIdx.y;
  const GmSeg sg = B.seg[g.i];
  g.off = (size_t)sg.off;
  g.L = (size_t)sg.L;
  return g;
}

__device__ __forceinline__ void chunk_of(size_t L, size_t& lo, size_t& hi) {
  const size_t ch = (L + kGmBlocks - 1) / kGmBlocks;
  lo = blockIdx.x * ch;
  hi = lo + ch < L ? lo + ch : L;
  if (lo > L) lo = L;
}

// Sum over the 64 lanes of a wave, the same value in every lane, by VALU lane
// exchanges only: four DPP steps inside each 16-lane row (quad_perm [1,0,3,2],
// quad_perm [2,3,0,1], row_half_mirror, row_mirror), then the 16-lane swap adds rows
// 0+1 and 2+3 and the 32-lane swap adds the two halves.  Fixed order: deterministic.
template <int CTRL>
__device__ __forceinline__ double dpp_swap(double v) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_swap<0xB1>(v);
  v += dpp_swap<0x4E>(v);
  v += dpp_swap<0x141>(v);
  v += dpp_swap<0x140>(v);
  {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
    v = __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
  }
  {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
    v = __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
  }
  return v;
}

// Block sums of acc[i] for i < nv (wave sums, then the 4 wave results in order);
// thread i < nv of the block returns sum i.  Fixed order: deterministic.
template <int NB>
__device__ __forceinline__ double block_sums(const double (&acc)[NB], int nv, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (i < nv) {
      const double v = wave_sum(acc[i]);
      if (lane == 0) red[wave * kGmMaxVec + i] = v;
    }
  }
  __syncthreads();
  double r = 0.0;
  if ((int)threadIdx.x < nv)
    for (int w = 0; w < kT / 64; ++w) r += red[w * kGmMaxVec + threadIdx.x];
  return r;
}

// h[i] = sum over blocks of partial[i][b] for i < nv -> LDS hs (every block, the same
// fixed order for a given nv).
//   nv <= 4 (norms, short bases): output i is summed by wave i, whose lane l adds
//     blocks l, l + 64, l + 128, l + 192 in that order before the wave sum;
//   nv > 4: thread (i, q) adds blocks q, q + Q, ... with independent loads, then
//     thread i adds the Q segment sums in order.
__device__ __forceinline__ void gather_partials(const double* __restrict__ partial, int nv, double* hs) {
  constexpr int R = kGmBlocks / 64;   // partials per lane and output
  static_assert(kGmBlocks % 64 == 0 && kT == 256, "four waves, whole waves of partials");
  const int t = threadIdx.x;
  if (nv <= kT / 64) {
    const int lane = t & 63, wave = t >> 6;
    if (wave < nv) {
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) acc += partial[part_at(wave, lane + 64 * r)];
      acc = wave_sum(acc);
      if (lane == 0) hs[wave] = acc;
    }
    __syncthreads();
    return;
  }
  __shared__ double seg[kT];
  const int Q = kT / nv < kGmBlocks ? kT / nv : kGmBlocks;
  if (t < nv * Q) {
    const int i = t / Q, q = t - i * Q;
    double acc = 0.0;
#pragma unroll 8
    for (int b = q; b < kGmBlocks; b += Q) acc += partial[part_at(i, b)];
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

// Givens rotations on Hessenberg column j, whose subdiagonal entry is nrm: residual
// estimate and stopping test.  Called by every thread of one block; the column and
// the rotations are staged in LDS so the sequential part runs from LDS.
__device__ void givens_column(const GmBatch& B, int inst, int j, double nrm) {
  __shared__ double col[kGmMaxVec], cs[kGmMaxRestart], sn[kGmMaxRestart];
  GmState* st = B.st + inst;
  GmHess* hz = B.hs + inst;
  const int m = B.m;
  const int t = threadIdx.x;
  if (t <= j) col[t] = hz->H[t * m + j];
  if (t == j + 1) col[t] = nrm;
  if (t < j) {
    cs[t] = hz->cs[t];
    sn[t] = hz->sn[t];
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
  hz->cs[j] = c;
  hz->sn[j] = s;
  col[j] = den;
  col[j + 1] = 0.0;
  for (int i = 0; i <= j + 1; ++i) hz->H[i * m + j] = col[i];
  const bool breakdown = !(b > 0.0);
  const double gj = hz->g[j];
  hz->g[j + 1] = -s * gj;
  hz->g[j] = c * gj;
  st->rel = fabs(hz->g[j + 1]) / st->bnorm;
  st->steps = j + 1;
  st->used += 1;
  if (!(st->rel > st->rtol) || st->used >= st->maxit || breakdown || j + 1 >= m) st->done = 1;
}

// First kernel of Arnoldi step j = nv - 1 (w = A V_j as the Jacobian action left it):
// partial sums of V_i . w for i < nv over this block's chunk.  mode 0 (j = 0): V_j is
// normalised already.  mode 1: V_j is unscaled; sigma = 1/|V_j| from the squared-norm
// partials `pnorm`, V_j <- sigma V_j and w <- sigma w in place, and block 0 applies
// the Givens rotations to column j - 1.  mode 2: as 1, but column j - 1 was finished
// by k_gm_column at the end of the previous chunk.
template <int NB>
__global__ __launch_bounds__(kT) void k_gm_dots(GmBatch B, double* __restrict__ V, int nv,
                                                double* __restrict__ w, const double* __restrict__ pnorm,
                                                double* __restrict__ partial, int mode) {
  __shared__ double red[(kT / 64) * kGmMaxVec];
  __shared__ double hs[1];
  const Seg g = seg_of(B);
  if (B.st[g.i].done) return;
  const int j = nv - 1;
  const size_t L = g.L;
  V += g.off;
  w += g.off;
  double* Vj = V + (size_t)j * B.ldv;
  partial += g.i * kPart;
  size_t lo, hi;
  chunk_of(L, lo, hi);
  // all NB loads of an element are issued together; the first element's go out
  // before the norm partials are gathered
  double v[NB], wf = 0.0;
  const size_t e0 = lo + threadIdx.x;
  if (e0 < hi) {
#pragma unroll
    for (int i = 0; i < NB; ++i) v[i] = V[(size_t)min(i, j) * B.ldv + e0];
    wf = w[e0];
  }
  double nrm = 1.0, sig = 1.0;
  if (mode != 0) {
    gather_partials(pnorm + g.i * kPart, 1, hs);
    nrm = sqrt(hs[0]);
    sig = 1.0 / nrm;
  }
  double acc[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) acc[i] = 0.0;
  for (size_t e = e0; e < hi; e += kT) {
    if (e != e0) {
#pragma unroll
      for (int i = 0; i < NB; ++i) v[i] = V[(size_t)min(i, j) * B.ldv + e];
      wf = w[e];
    }
    const double we = wf * sig;
    if (mode != 0) {
      Vj[e] = Vj[e] * sig;
      w[e] = we;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) acc[i] = fma(v[i], i < nv ? we : 0.0, acc[i]);
  }
  // V_j entered the sums unscaled
#pragma unroll
  for (int i = 0; i < NB; ++i)
    if (i == j) acc[i] *= sig;
  const double r = block_sums<NB>(acc, nv, red);
  if ((int)threadIdx.x < nv) partial[part_at(threadIdx.x, blockIdx.x)] = r;
  if (mode == 1 && blockIdx.x == 0) givens_column(B, g.i, j - 1, nrm);
}

// h = sum of the previous partials; w -= V h; then either the partial dots of the new
// w with V (next = 0, result back into w) or its partial squared norm (next = 1,
// result into `out`, the unscaled V_{j+1}).  Block 0 adds h into the Hessenberg
// column j.
template <int NB>
__global__ __launch_bounds__(kT) void k_gm_update(GmBatch B, const double* __restrict__ V, int nv,
                                                  double* w, const double* __restrict__ pin, int first,
                                                  int next, double* __restrict__ pout, int j, double* out) {
  __shared__ double red[(kT / 64) * kGmMaxVec];
  __shared__ double hs[kGmMaxVec];
  const Seg g = seg_of(B);
  if (B.st[g.i].done) return;
  const size_t L = g.L;
  V += g.off;
  w += g.off;
  out += g.off;
  pin += g.i * kPart;
  pout += g.i * kPart;
  size_t lo, hi;
  chunk_of(L, lo, hi);
  // the first element's loads go out before the partial sums are gathered
  double v[NB], wf = 0.0;
  const size_t e0 = lo + threadIdx.x;
  if (e0 < hi) {
#pragma unroll
    for (int i = 0; i < NB; ++i) v[i] = V[(size_t)min(i, nv - 1) * B.ldv + e0];
    wf = w[e0];
  }
  gather_partials(pin, nv, hs);
  if (blockIdx.x == 0 && (int)threadIdx.x < nv) {
    double* Hc = B.hs[g.i].H + threadIdx.x * B.m + j;
    *Hc = first ? hs[threadIdx.x] : *Hc + hs[threadIdx.x];
  }
  double h[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) h[i] = i < nv ? hs[i] : 0.0;
  double acc[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) acc[i] = 0.0;
  for (size_t e = e0; e < hi; e += kT) {
    if (e != e0) {
#pragma unroll
      for (int i = 0; i < NB; ++i) v[i] = V[(size_t)min(i, nv - 1) * B.ldv + e];
      wf = w[e];
    }
    double we = wf;
#pragma unroll
    for (int i = 0; i < NB; ++i) we = fma(-h[i], v[i], we);
    out[e] = we;
    if (next == 0) {
#pragma unroll
      for (int i = 0; i < NB; ++i) acc[i] = fma(v[i], i < nv ? we : 0.0, acc[i]);
    } else {
      acc[0] = fma(we, we, acc[0]);
    }
  }
  const int nout = next == 0 ? nv : 1;
  const double r = block_sums<NB>(acc, nout, red);
  if ((int)threadIdx.x < nout) pout[part_at(threadIdx.x, blockIdx.x)] = r;
}

// End of a chunk of Arnoldi steps whose last step is j: Givens rotations on column j
// with |V_{j+1}| from the squared-norm partials (V_{j+1} is scaled by the next step).
__global__ __launch_bounds__(kT) void k_gm_column(GmBatch B, const double* __restrict__ pnorm, int j) {
  __shared__ double hs[1];
  const Seg g = seg_of(B);
  if (B.st[g.i].done) return;
  gather_partials(pnorm + g.i * kPart, 1, hs);
  givens_column(B, g.i, j, sqrt(hs[0]));
}

// Fresh solve: header of every instance of the launch (one block per instance).
__global__ void k_gm_init(GmBatch B, int maxit, double rtol) {
  const Seg g = seg_of(B);
  if (threadIdx.x != 0) return;
  GmState s;
  s.m = B.m;
  s.maxit = maxit;
  s.steps = 0;
  s.used = 0;
  s.done = 0;
  s.pad = 0;
  s.rtol = rtol;
  s.bnorm = 0.0;
  s.beta = 0.0;
  s.rel = 0.0;
  B.st[g.i] = s;
}

// Cycle start: beta = |r| from partials, V_0 = r / beta, g = (beta, 0, ...).
__global__ __launch_bounds__(kT) void k_gm_start(GmBatch B, double* __restrict__ V,
                                                 const double* __restrict__ r,
                                                 const double* __restrict__ pin, int first_cycle) {
  __shared__ double hs[1];
  const Seg g = seg_of(B);
  const size_t L = g.L;
  double* V0 = V + g.off;
  r += g.off;
  gather_partials(pin + g.i * kPart, 1, hs);
  const double beta = sqrt(hs[0]);
  GmState* st = B.st + g.i;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    GmHess* hz = B.hs + g.i;
    if (first_cycle) st->bnorm = beta;
    st->beta = beta;
    for (int i = 0; i <= B.m; ++i) hz->g[i] = 0.0;
    hz->g[0] = beta;
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
__global__ __launch_bounds__(kT) void k_gm_update_x(GmBatch B, const double* __restrict__ V,
                                                    double* __restrict__ x) {
  __shared__ double ys[kGmMaxVec];
  const Seg g = seg_of(B);
  const size_t L = g.L;
  V += g.off;
  x += g.off;
  const GmHess* hz = B.hs + g.i;
  const int k = B.st[g.i].steps;
  if (threadIdx.x == 0) {
    const int m = B.m;
    for (int i = k - 1; i >= 0; --i) {
      double s = hz->g[i];
      for (int l = i + 1; l < k; ++l) s -= hz->H[i * m + l] * ys[l];
      ys[i] = s / hz->H[i * m + i];
    }
  }
  __syncthreads();
  size_t lo, hi;
  chunk_of(L, lo, hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += kT) {
    double acc = x[e];
    for (int i = 0; i < k; ++i) acc += ys[i] * V[(size_t)i * B.ldv + e];
    x[e] = acc;
  }
}

// partial squared norms of v (for k_gm_start and the norms)
__global__ __launch_bounds__(kT) void k_gm_sumsq(GmBatch B, const double* __restrict__ v,
                                                 double* __restrict__ partial) {
  __shared__ double red[(kT / 64) * kGmMaxVec];
  const Seg g = seg_of(B);
  v += g.off;
  size_t lo, hi;
  chunk_of(g.L, lo, hi);
  double acc[1] = {0.0};
  for (size_t e = lo + threadIdx.x; e < hi; e += kT) acc[0] = fma(v[e], v[e], acc[0]);
  const double r = block_sums<1>(acc, 1, red);
  if (threadIdx.x == 0) partial[g.i * kPart + part_at(0, blockIdx.x)] = r;
}

// out[instance] = sqrt(sum of its partials) (one block per instance)
__global__ __launch_bounds__(kT) void k_gm_norms(GmBatch B, const double* __restrict__ partial,
                                                 double* __restrict__ out) {
  __shared__ double hs[1];
  const Seg g = seg_of(B);
  gather_partials(partial + g.i * kPart, 1, hs);
  if (threadIdx.x == 0) out[g.i] = sqrt(hs[0]);
}

// r = b - w
__global__ __launch_bounds__(kT) void k_gm_residual(GmBatch B, const double* __restrict__ b,
                                                    const double* __restrict__ w,
                                                    double* __restrict__ r) {
  const Seg g = seg_of(B);
  size_t lo, hi;
  chunk_of(g.L, lo, hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += kT) r[g.off + e] = b[g.off + e] - w[g.off + e];
}

// y = a x (+ y when accumulate)
__global__ __launch_bounds__(kT) void k_gm_axpy(GmBatch B, double a, const double* __restrict__ x,
                                                double* __restrict__ y, int accumulate) {
  const Seg g = seg_of(B);
  size_t lo, hi;
  chunk_of(g.L, lo, hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += kT)
    y[g.off + e] = accumulate ? fma(a, x[g.off + e], y[g.off + e]) : a * x[g.off + e];
}

// x = 0
__global__ __launch_bounds__(kT) void k_gm_zero(GmBatch B, double* __restrict__ x) {
  const Seg g = seg_of(B);
  size_t lo, hi;
  chunk_of(g.L, lo, hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += kT) x[g.off + e] = 0.0;
}

dim3 grid_of(const GmBatch& B) { return dim3(kGmBlocks, B.count); }

}  // namespace

void launch_gm_init(const GmBatch& B, int maxit, double rtol, hipStream_t s) {
  if (B.count > 0) k_gm_init<<<dim3(1, B.count), 64, 0, s>>>(B, maxit, rtol);
}
void launch_gm_sumsq(const GmBatch& B, const double* v, double* partial, hipStream_t s) {
  if (B.count > 0) k_gm_sumsq<<<grid_of(B), kT, 0, s>>>(B, v, partial);
}
void launch_gm_norms(const GmBatch& B, const double* v, double* partial, double* out, hipStream_t s) {
  if (B.count <= 0) return;
  k_gm_sumsq<<<grid_of(B), kT, 0, s>>>(B, v, partial);
  k_gm_norms<<<dim3(1, B.count), kT, 0, s>>>(B, partial, out);
}
void launch_gm_residual(const GmBatch& B, const double* b, const double* w, double* r, hipStream_t s) {
  if (B.count > 0) k_gm_residual<<<grid_of(B), kT, 0, s>>>(B, b, w, r);
}
void launch_gm_axpy(const GmBatch& B, double a, const double* x, double* y, int accumulate, hipStream_t s) {
  if (B.count > 0) k_gm_axpy<<<grid_of(B), kT, 0, s>>>(B, a, x, y, accumulate);
}
void launch_gm_zero(const GmBatch& B, double* x, hipStream_t s) {
  if (B.count > 0) k_gm_zero<<<grid_of(B), kT, 0, s>>>(B, x);
}
void launch_gm_start(const GmBatch& B, double* V, const double* r, const double* partial, int first_cycle,
                     hipStream_t s) {
  if (B.count > 0) k_gm_start<<<grid_of(B), kT, 0, s>>>(B, V, r, partial, first_cycle);
}
template <int NB>
void arnoldi_nb(const GmBatch& B, double* V, int j, double* w, double* p1, double* p2, double* p3,
                int mode, hipStream_t s) {
  const int nv = j + 1;
  const dim3 gr = grid_of(B);
  k_gm_dots<NB><<<gr, kT, 0, s>>>(B, V, nv, w, p3, p1, mode);
  k_gm_update<NB><<<gr, kT, 0, s>>>(B, V, nv, w, p1, 1, 0, p2, j, w);
  k_gm_update<NB><<<gr, kT, 0, s>>>(B, V, nv, w, p2, 0, 1, p3, j, V + (size_t)(j + 1) * B.ldv);
}
void launch_gm_arnoldi(const GmBatch& B, double* V, int j, double* w, double* p1, double* p2, double* p3,
                       int mode, hipStream_t s) {
  if (B.count <= 0) return;
  const int nv = j + 1;
  switch ((nv + 3) / 4) {
    case 1: arnoldi_nb<4>(B, V, j, w, p1, p2, p3, mode, s); break;
    case 2: arnoldi_nb<8>(B, V, j, w, p1, p2, p3, mode, s); break;
    case 3: arnoldi_nb<12>(B, V, j, w, p1, p2, p3, mode, s); break;
    case 4: arnoldi_nb<16>(B, V, j, w, p1, p2, p3, mode, s); break;
    case 5: arnoldi_nb<20>(B, V, j, w, p1, p2, p3, mode, s); break;
    case 6: arnoldi_nb<24>(B, V, j, w, p1, p2, p3, mode, s); break;
    case 7: arnoldi_nb<28>(B, V, j, w, p1, p2, p3, mode, s); break;
    case 8: arnoldi_nb<32>(B, V, j, w, p1, p2, p3, mode, s); break;
    default:
      if (nv <= 48) arnoldi_nb<48>(B, V, j, w, p1, p2, p3, mode, s);
      else arnoldi_nb<64>(B, V, j, w, p1, p2, p3, mode, s);
  }
}
void launch_gm_column(const GmBatch& B, const double* p3, int j, hipStream_t s) {
  if (B.count > 0) k_gm_column<<<dim3(1, B.count), kT, 0, s>>>(B, p3, j);
}
void launch_gm_update_x(const GmBatch& B, const double* V, double* x, hipStream_t s) {
  if (B.count > 0) k_gm_update_x<<<grid_of(B), kT, 0, s>>>(B, V, x);
}

}  // namespace rsp
