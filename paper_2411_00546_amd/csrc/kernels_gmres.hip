// Device-resident restarted GMRES (x_0 = 0) for the RASPEN Newton systems of
// Algorithm 2, for every instance of a batch at once: Arnoldi with classical
// Gram-Schmidt applied twice, Givens rotations on the Hessenberg column, the
// stopping test |g_{j+1}| <= rtol |b| and the triangular solve, all on the device.
//
// The second Gram-Schmidt pass of a vector is delayed by one step and shares the
// global reduction of the next, so a step has one reduction.  At step j the basis
// V_0 .. V_{j-1} is orthonormal and slot j holds u_j, the new vector after its first
// pass (unscaled); the Jacobian action gives z = A u_j.  One pass over the vectors
// forms a = V_{j-1}^T u_j, b = u_j . u_j, c = V_{j-1}^T z and d = u_j . z.  Then:
//   second pass of u_j:  v_j = (u_j - V_{j-1} a) / nu,  nu^2 = b - |a|^2, and column
//                        j - 1 of the Hessenberg matrix is its first pass plus a, with
//                        subdiagonal nu (it gets its Givens rotations here);
//   A v_j from z:        A u_j = nu A v_j + A V_{j-1} a and A V_{j-1} = V_j H (the
//                        Arnoldi relation, unrotated columns), so with t = H a,
//                        A v_j = (z - V_j t) / nu;
//   first pass of A v_j: h = V_j^T A v_j = ((c - t_{<j}) / nu, (v_j . z - t_j) / nu),
//                        v_j . z = (d - a . c) / nu, and
//                        u_{j+1} = (z - V_j s) / nu with s = t + nu h.
// A second pass over the vectors writes v_j and u_{j+1}.  In exact arithmetic this is
// the classical Gram-Schmidt process applied twice.  An Arnoldi step is two launches
// after the Jacobian action; a chunk of steps ends with one reduction and one small
// launch that finish its last column.
// Launch grid: (blocks, instances); blockIdx.y selects the instance, whose
// vectors are its segment of the batch's concatenated vectors (basis vector k of
// every instance: V + k ldv), and the instance uses gm_blocks(L) blocks of the row.  A per-instance stop
// flag written by the Givens kernel lets the host enqueue a whole restart cycle
// without reading anything back: the kernels of a stopped instance return at once.
//
// Reductions are deterministic and depend only on the instance's own length:
// gm_blocks(L) blocks each own a contiguous chunk, write their partial sums, and
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
  int nb;         // its reduction blocks, gm_blocks(L)
};

__device__ __forceinline__ Seg seg_of(const GmBatch& B) {
  Seg g;
  g.i = B.list ? B.list[blockIdx.y] : (int)blockIdx.y;
  const GmSeg sg = B.seg[g.i];
  g.off = (size_t)sg.off;
  g.L = (size_t)sg.L;
  g.nb = gm_blocks(sg.L);
  return g;
}

// Chunk of block blockIdx.x < nb of a vector of length L.
__device__ __forceinline__ void chunk_of(size_t L, int nb, size_t& lo, size_t& hi) {
  const size_t ch = (L + nb - 1) / nb;
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

// h[i] = sum over the nb blocks of partial[i][b] for i < nv -> LDS hs (every block, the
// same fixed order for given nv and nb).
//   nv <= 4 (norms, short bases): output i is summed by wave i, whose lane l adds
//     blocks l, l + 64, l + 128, ... in that order before the wave sum;
//   nv > 4: thread (i, q) adds blocks q, q + Q, ... with independent loads, then
//     thread i adds the Q segment sums in order.
__device__ __forceinline__ void gather_partials(const double* __restrict__ partial, int nv, int nb, double* hs) {
  constexpr int R = kGmBlocks / 64;   // partials per lane and output, at most
  static_assert(kGmBlocks % 64 == 0 && kT == 256, "four waves, whole waves of partials");
  const int t = threadIdx.x;
  if (nv <= kT / 64) {
    const int lane = t & 63, wave = t >> 6;
    if (wave < nv) {
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (lane + 64 * r < nb) acc += partial[part_at(wave, lane + 64 * r)];
      acc = wave_sum(acc);
      if (lane == 0) hs[wave] = acc;
    }
    __syncthreads();
    return;
  }
  __shared__ double seg[kT];
  const int Q = kT / nv < nb ? kT / nv : nb;
  if (t < nv * Q) {
    const int i = t / Q, q = t - i * Q;
    double acc = 0.0;
#pragma unroll 8
    for (int b = q; b < nb; b += Q) acc += partial[part_at(i, b)];
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

// Givens rotations on Hessenberg column j, whose subdiagonal entry is nrm: residual
// estimate and stopping test (`lucky`: the basis cannot be extended, the cycle ends).  Called by every thread of one block; the column and
// the rotations are staged in LDS so the sequential part runs from LDS.
__device__ void givens_column(const GmBatch& B, int inst, int j, double nrm, bool lucky) {
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
  const bool breakdown = lucky || !(b > 0.0);
  const double gj = hz->g[j];
  hz->g[j + 1] = -s * gj;
  hz->g[j] = c * gj;
  st->rel = fabs(hz->g[j + 1]) / st->bnorm;
  st->steps = j + 1;
  st->used += 1;
  if (!(st->rel > st->rtol) || st->used >= st->maxit || breakdown || j + 1 >= m) st->done = 1;
}

// NB: compile-time bound on the number of basis vectors read besides u (bucket >= j).
// Loads of all NB vectors are issued unconditionally (index clamped to j - 1, the
// extra ones hit the cache) and the unused products are masked, so the loads of an
// element are in flight together.

// Reduction of Arnoldi step j (slot j holds u: unscaled after its first pass, or the
// normalised V_0 for j = 0): partial sums over this block's chunk of
//   p1: a_i = V_i . u (i < j), and b = u . u in slot j;
//   p2: c_i = V_i . z (i < j), and d = u . z in slot j (withz = 0: not formed).
// The basis vectors are split over the four waves (wave w takes V_w, V_{w+4}, ...), each
// wave covering the whole chunk with KE elements per lane in flight: a wave holds the
// sums of NB / 4 vectors only, so more loads stay in flight (a stand-alone copy of the
// access pattern streamed 5.6 TB/s this way against 3.8 with every thread reading all
// vectors).  Each partial is a fixed-order wave sum of the lanes' sums, and every lane
// adds its elements in order.  u and z are read by all four waves (from the caches).
template <int NB>
__global__ __launch_bounds__(kT) void k_gm_reduce(GmBatch B, const double* __restrict__ V, int j,
                                                  const double* __restrict__ z, double* __restrict__ p1,
                                                  double* __restrict__ p2, int withz) {
  static_assert(NB % 4 == 0, "basis vectors split over four waves");
  constexpr int NV = NB / 4;   // basis vectors of a wave
  constexpr int KE = 4;        // elements per lane in flight
  const Seg g = seg_of(B);
  if (blockIdx.x >= g.nb || B.st[g.i].done) return;
  V += g.off;
  z += g.off;
  const double* u = V + (size_t)j * B.ldv;
  p1 += g.i * kPart;
  p2 += g.i * kPart;
  size_t lo, hi;
  chunk_of(g.L, g.nb, lo, hi);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double aa[NV], cc[NV], bb = 0.0, dd = 0.0;
#pragma unroll
  for (int i = 0; i < NV; ++i) aa[i] = cc[i] = 0.0;
  for (size_t e0 = lo + lane; e0 < hi; e0 += 64 * KE) {
    double ue[KE], ze[KE], v[KE][NV];
#pragma unroll
    for (int k = 0; k < KE; ++k) {
      const size_t e = e0 + 64 * (size_t)k;
      const bool in = e < hi;
      const size_t ee = in ? e : e0;   // past the chunk: an element of it, counted 0
      const double ur = u[ee], zr = withz ? z[ee] : 0.0;
      ue[k] = in ? ur : 0.0;
      ze[k] = in ? zr : 0.0;
      if (j > 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) v[k][i] = V[(size_t)min(w + 4 * i, j - 1) * B.ldv + ee];
      }
    }
#pragma unroll
    for (int k = 0; k < KE; ++k) {
      if (j > 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
          const bool act = w + 4 * i < j;
          aa[i] = fma(v[k][i], act ? ue[k] : 0.0, aa[i]);
          cc[i] = fma(v[k][i], act ? ze[k] : 0.0, cc[i]);
        }
      }
      bb = fma(ue[k], ue[k], bb);
      dd = fma(ue[k], ze[k], dd);
    }
  }
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int vi = w + 4 * i;
    if (vi >= j) continue;   // wave-uniform
    const double ra = wave_sum(aa[i]);
    const double rc = withz ? wave_sum(cc[i]) : 0.0;
    if (lane == 0) {
      p1[part_at(vi, blockIdx.x)] = ra;
      if (withz) p2[part_at(vi, blockIdx.x)] = rc;
    }
  }
  // b and d (slot j): every wave formed them over the same elements; wave 0 writes
  if (w == 0) {
    const double rb = wave_sum(bb);
    const double rd = withz ? wave_sum(dd) : 0.0;
    if (lane == 0) {
      p1[part_at(j, blockIdx.x)] = rb;
      if (withz) p2[part_at(j, blockIdx.x)] = rd;
    }
  }
}

// u_j is taken to lie in span(V_0 .. V_{j-1}) (a lucky breakdown: the Krylov space is
// invariant up to rounding) when nu^2 = |u|^2 - |a|^2 is at most this fraction of
// |A v_{j-1}|^2.  Below it the difference of two nearly equal sums is not resolved in
// FP64: its sign and size are rounding residue (on the order of 1e-16 |A v|^2).
constexpr double kGmLucky = 1e-12;

// The two reductions of an Arnoldi step gathered in one pass: ha[i] = sum over the nb
// blocks of pa[i][b] and hb[i] of pb[i][b], i < nv.  Thread (v, q), v < 2 nv (v < nv:
// pa), adds blocks q, q + Q, ... (Q = kT / (2 nv)) with independent loads, then thread v
// adds its Q segment sums in order: every block, the same fixed order for given nv, nb.
// The loads of both arrays are in flight together.
__device__ __forceinline__ void gather_pair(const double* __restrict__ pa, const double* __restrict__ pb, int nv,
                                            int nb, double* ha, double* hb) {
  __shared__ double seg[kT];
  const int t = threadIdx.x;
  const int Q = kT / (2 * nv);
  if (t < 2 * nv * Q) {
    const int v = t / Q, q = t - v * Q;
    const double* src = v < nv ? pa : pb;
    const int i = v < nv ? v : v - nv;
    double acc = 0.0;
#pragma unroll 8
    for (int b = q; b < nb; b += Q) acc += src[part_at(i, b)];
    seg[t] = acc;
  }
  __syncthreads();
  if (t < 2 * nv) {
    double acc = 0.0;
    for (int q = 0; q < Q; ++q) acc += seg[t * Q + q];
    (t < nv ? ha : hb)[t < nv ? t : t - nv] = acc;
  }
  __syncthreads();
}

// Second pass of u_j against V_0 .. V_{j-1} from the partial sums a, b (p1, j + 1
// values): nu and the finished column j - 1 (its first pass plus a, subdiagonal nu),
// into colv[0 .. j], nu and the breakdown flag into out[0], out[1] (1.0: lucky
// breakdown, nu is then max(nu^2, 0)^(1/2) and v_j is not formed).  `mode` 2: the
// column is final in Hr already.  Every thread of the block calls it; the result is in
// LDS for all.
__device__ __forceinline__ void second_pass_column(const GmHess* hz, int m, int j, const double* ha,
                                                   int mode, double* colv, double* out) {
  const int t = threadIdx.x;
  if (t < j) colv[t] = mode == 2 ? hz->Hr[t * m + j - 1] : hz->hf[(j - 1) & 1][t] + ha[t];
  __syncthreads();
  if (t == 0) {
    // |A v_{j-1}|^2 = |H column|^2 + |u_j|^2 (z = V h + u after the first pass)
    double ss = 0.0, zz = ha[j];
    for (int i = 0; i < j; ++i) {
      ss = fma(ha[i], ha[i], ss);
      zz = fma(colv[i], colv[i], zz);
    }
    const double nu2 = ha[j] - ss;
    const double nu = sqrt(fmax(nu2, 0.0));
    out[0] = nu;
    out[1] = nu2 > kGmLucky * zz ? 0.0 : 1.0;
    colv[j] = nu;
  }
  __syncthreads();
}

// Arnoldi step j after the reduction (p1: a and b, p2: c and d): every block forms nu,
// t = H a, h and s (small, in LDS), then writes v_j over u_j (j > 0) and u_{j+1} into
// slot j + 1.  Block 0 stores h as the first pass of column j and, for mode 1, the
// finished column j - 1 with its Givens rotations (residual estimate, stopping test).
// mode 0: j = 0 (V_0 is normalised, no column to finish); mode 2: column j - 1 was
// finished at the end of the previous chunk.
template <int NB>
__global__ __launch_bounds__(kT) void k_gm_vupdate(GmBatch B, double* __restrict__ V, int j,
                                                   const double* __restrict__ z,
                                                   const double* __restrict__ p1,
                                                   const double* __restrict__ p2, int mode) {
  __shared__ double ha[kGmMaxVec], hc[kGmMaxVec], colv[kGmMaxVec], tv[kGmMaxVec], hv[kGmMaxVec],
      sv[kGmMaxVec];
  __shared__ double hl[kGmMaxVec * kGmMaxRestart];   // unrotated columns 0 .. j - 2, rows 0 .. j
  __shared__ double scal[3];   // nu, lucky flag, v_j . z
  const Seg g = seg_of(B);
  GmState* st = B.st + g.i;
  if (blockIdx.x >= g.nb || st->done) return;
  GmHess* hz = B.hs + g.i;
  const int m = B.m;
  const int t = threadIdx.x;
  // loads that do not depend on the partial sums go out first: the Hessenberg block
  // for t = H a, and the first two elements of this thread (the second one up to 12
  // basis vectors: the registers of both)
  for (int q = t; q < (j + 1) * j; q += kT) {
    const int r = q / j, i = q - r * j;
    hl[q] = (i < j - 1 && r <= i + 1) ? hz->Hr[r * m + i] : 0.0;
  }
  V += g.off;
  z += g.off;
  double* Vj = V + (size_t)j * B.ldv;
  double* Vn = V + (size_t)(j + 1) * B.ldv;
  size_t lo, hi;
  chunk_of(g.L, g.nb, lo, hi);
  constexpr int EP = NB <= 12 ? 2 : 1;
  const size_t e0 = lo + threadIdx.x, e1 = e0 + kT;
  double v[NB], ue = 0.0, ze = 0.0;
  double v1[EP == 2 ? NB : 1], ue1 = 0.0, ze1 = 0.0;
  if (e0 < hi) {
    if (j > 0) {
#pragma unroll
      for (int i = 0; i < NB; ++i) v[i] = V[(size_t)min(i, j - 1) * B.ldv + e0];
    }
    ue = Vj[e0];
    ze = z[e0];
  }
  if constexpr (EP == 2) {
    if (e1 < hi) {
      if (j > 0) {
#pragma unroll
        for (int i = 0; i < NB; ++i) v1[i] = V[(size_t)min(i, j - 1) * B.ldv + e1];
      }
      ue1 = Vj[e1];
      ze1 = z[e1];
    }
  }
  // a, b (p1) and c, d (p2) of this step, in one gather
  gather_pair(p1 + g.i * kPart, p2 + g.i * kPart, j + 1, g.nb, ha, hc);
  if (j == 0) {
    if (t == 0) {
      scal[0] = 1.0;
      scal[1] = 0.0;
      hv[0] = hc[0];
      sv[0] = hc[0];
    }
    __syncthreads();
  } else {
    second_pass_column(hz, m, j, ha, mode, colv, scal);
    if (t == 0) {
      double ac = 0.0;
      for (int i = 0; i < j; ++i) ac = fma(ha[i], hc[i], ac);
      scal[2] = scal[1] != 0.0 ? 0.0 : (hc[j] - ac) / scal[0];   // v_j . z
    }
    // t = H a over the unrotated columns 0 .. j - 1 (column j - 1 as just finished)
    if (t <= j) {
      double acc = 0.0;
      for (int i = 0; i < j; ++i) {
        const double hki = i == j - 1 ? colv[t] : hl[t * j + i];
        acc = fma(hki, ha[i], acc);
      }
      tv[t] = acc;
    }
    __syncthreads();
    if (t <= j) {
      // (after a lucky breakdown nothing of this step is used; it stays finite)
      const double nu = scal[1] != 0.0 ? 1.0 : scal[0];
      const double hk = (t < j ? hc[t] - tv[t] : scal[2] - tv[j]) / nu;
      hv[t] = hk;
      sv[t] = fma(nu, hk, tv[t]);
    }
    __syncthreads();
  }
  const double inv = scal[1] != 0.0 ? 0.0 : 1.0 / scal[0];
  double a[NB], sc[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    a[i] = i < j ? ha[i] : 0.0;
    sc[i] = i < j ? sv[i] : 0.0;
  }
  const double sj = sv[j];
  // v_j over u_j and u_{j+1} at element e from the basis values vv, u_j and z there
  auto update = [&](size_t e, const double (&vv)[NB], double uu, double zz) {
    double vj = uu, un = zz;
    if (j > 0) {
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        vj = fma(-a[i], vv[i], vj);
        un = fma(-sc[i], vv[i], un);
      }
      vj *= inv;
      Vj[e] = vj;
    }
    un = fma(-sj, vj, un) * inv;
    Vn[e] = un;
  };
  if constexpr (EP == 2) {
    if (e0 < hi) update(e0, v, ue, ze);
    if (e1 < hi) update(e1, v1, ue1, ze1);
    for (size_t e = e1 + kT; e < hi; e += kT) {
      if (j > 0) {
#pragma unroll
        for (int i = 0; i < NB; ++i) v[i] = V[(size_t)min(i, j - 1) * B.ldv + e];
      }
      update(e, v, Vj[e], z[e]);
    }
  } else {
    for (size_t e = e0; e < hi; e += kT) {
      if (e != e0) {
        if (j > 0) {
#pragma unroll
          for (int i = 0; i < NB; ++i) v[i] = V[(size_t)min(i, j - 1) * B.ldv + e];
        }
        ue = Vj[e];
        ze = z[e];
      }
      double vj = ue, un = ze;
      if (j > 0) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          vj = fma(-a[i], v[i], vj);
          un = fma(-sc[i], v[i], un);
        }
        vj *= inv;
        Vj[e] = vj;
      }
      un = fma(-sj, vj, un) * inv;
      Vn[e] = un;
    }
  }
  if (blockIdx.x != 0) return;
  if (t <= j) hz->hf[j & 1][t] = hv[t];
  if (mode == 1) {
    if (t <= j) hz->Hr[t * m + j - 1] = colv[t];
    if (t < j) hz->H[t * m + j - 1] = colv[t];
    __syncthreads();
    givens_column(B, g.i, j - 1, colv[j], scal[1] != 0.0);
  }
}

// End of a chunk whose last step was j - 1 (slot j holds u_j): column j - 1 finished
// from the partial sums a, b (p1) and its Givens rotations applied (one block per
// instance).
__global__ __launch_bounds__(kT) void k_gm_finish(GmBatch B, const double* __restrict__ p1, int j) {
  __shared__ double ha[kGmMaxVec], colv[kGmMaxVec];
  __shared__ double nu[2];
  const Seg g = seg_of(B);
  if (B.st[g.i].done) return;
  GmHess* hz = B.hs + g.i;
  const int m = B.m;
  const int t = threadIdx.x;
  // a, b in the order of the step kernel's gather (its second array is not used here)
  gather_pair(p1 + g.i * kPart, p1 + g.i * kPart, j + 1, g.nb, ha, colv);
  second_pass_column(hz, m, j, ha, 1, colv, nu);
  if (t <= j) hz->Hr[t * m + j - 1] = colv[t];
  if (t < j) hz->H[t * m + j - 1] = colv[t];
  __syncthreads();
  givens_column(B, g.i, j - 1, colv[j], nu[1] != 0.0);
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
  if (blockIdx.x >= g.nb) return;
  const size_t L = g.L;
  double* V0 = V + g.off;
  r += g.off;
  gather_partials(pin + g.i * kPart, 1, g.nb, hs);
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
  chunk_of(L, g.nb, lo, hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += kT) V0[e] = r[e] * inv;
}

// y = R^{-1} g (back substitution over the steps done), x += V y.
__global__ __launch_bounds__(kT) void k_gm_update_x(GmBatch B, const double* __restrict__ V,
                                                    double* __restrict__ x) {
  __shared__ double ys[kGmMaxVec];
  __shared__ double rs[kGmMaxRestart * kGmMaxRestart];   // the k x k triangle R
  const Seg g = seg_of(B);
  if (blockIdx.x >= g.nb) return;
  const size_t L = g.L;
  V += g.off;
  x += g.off;
  const GmHess* hz = B.hs + g.i;
  const int k = B.st[g.i].steps;
  // R and g to LDS by all threads (independent loads), then the substitution from LDS
  {
    const int m = B.m;
    for (int q = threadIdx.x; q < k * k; q += kT) {
      const int i = q / k, l = q - i * k;
      rs[q] = l >= i ? hz->H[i * m + l] : 0.0;
    }
    if ((int)threadIdx.x < k) ys[threadIdx.x] = hz->g[threadIdx.x];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = k - 1; i >= 0; --i) {
      double s = ys[i];
      for (int l = i + 1; l < k; ++l) s -= rs[i * k + l] * ys[l];
      ys[i] = s / rs[i * k + i];
    }
  }
  __syncthreads();
  size_t lo, hi;
  chunk_of(L, g.nb, lo, hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += kT) {
    double acc = x[e];
    // the basis loads are independent: eight in flight at a time, added in order
    int i = 0;
    for (; i + 8 <= k; i += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = V[(size_t)(i + q) * B.ldv + e];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc += ys[i + q] * v[q];
    }
    for (; i < k; ++i) acc += ys[i] * V[(size_t)i * B.ldv + e];
    x[e] = acc;
  }
}

// partial squared norms of v (for k_gm_start and the norms)
__global__ __launch_bounds__(kT) void k_gm_sumsq(GmBatch B, const double* __restrict__ v,
                                                 double* __restrict__ partial) {
  __shared__ double red[(kT / 64) * kGmMaxVec];
  const Seg g = seg_of(B);
  if (blockIdx.x >= g.nb) return;
  v += g.off;
  size_t lo, hi;
  chunk_of(g.L, g.nb, lo, hi);
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
  gather_partials(partial + g.i * kPart, 1, g.nb, hs);
  if (threadIdx.x == 0) out[g.i] = sqrt(hs[0]);
}

// r = b - w
__global__ __launch_bounds__(kT) void k_gm_residual(GmBatch B, const double* __restrict__ b,
                                                    const double* __restrict__ w,
                                                    double* __restrict__ r) {
  const Seg g = seg_of(B);
  if (blockIdx.x >= g.nb) return;
  size_t lo, hi;
  chunk_of(g.L, g.nb, lo, hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += kT) r[g.off + e] = b[g.off + e] - w[g.off + e];
}

// y = a x (+ y when accumulate)
__global__ __launch_bounds__(kT) void k_gm_axpy(GmBatch B, double a, const double* __restrict__ x,
                                                double* __restrict__ y, int accumulate) {
  const Seg g = seg_of(B);
  if (blockIdx.x >= g.nb) return;
  size_t lo, hi;
  chunk_of(g.L, g.nb, lo, hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += kT)
    y[g.off + e] = accumulate ? fma(a, x[g.off + e], y[g.off + e]) : a * x[g.off + e];
}

// x = 0
__global__ __launch_bounds__(kT) void k_gm_zero(GmBatch B, double* __restrict__ x) {
  const Seg g = seg_of(B);
  if (blockIdx.x >= g.nb) return;
  size_t lo, hi;
  chunk_of(g.L, g.nb, lo, hi);
  for (size_t e = lo + threadIdx.x; e < hi; e += kT) x[g.off + e] = 0.0;
}

dim3 grid_of(const GmBatch& B) { return dim3(B.nbx, B.count); }

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
void arnoldi_nb(const GmBatch& B, double* V, int j, const double* z, double* p1, double* p2, int mode,
                hipStream_t s) {
  const dim3 gr = grid_of(B);
  k_gm_reduce<NB><<<gr, kT, 0, s>>>(B, V, j, z, p1, p2, 1);
  k_gm_vupdate<NB><<<gr, kT, 0, s>>>(B, V, j, z, p1, p2, mode);
}
template <int NB>
void finish_nb(const GmBatch& B, const double* V, int j, double* p1, double* p2, hipStream_t s) {
  k_gm_reduce<NB><<<grid_of(B), kT, 0, s>>>(B, V, j, V, p1, p2, 0);   // z not read (withz = 0)
  k_gm_finish<<<dim3(1, B.count), kT, 0, s>>>(B, p1, j);
}
// NB bucket for j basis vectors before u: multiples of 4 up to 32, then 48, 64
#define RSP_GM_BUCKET(j_, CALL)                    \
  switch (((j_) > 0 ? (j_) + 3 : 4) / 4) {         \
    case 1: CALL(4); break;                        \
    case 2: CALL(8); break;                        \
    case 3: CALL(12); break;                       \
    case 4: CALL(16); break;                       \
    case 5: CALL(20); break;                       \
    case 6: CALL(24); break;                       \
    case 7: CALL(28); break;                       \
    case 8: CALL(32); break;                       \
    default:                                       \
      if ((j_) <= 48) CALL(48);                    \
      else CALL(64);                               \
  }
void launch_gm_arnoldi(const GmBatch& B, double* V, int j, const double* z, double* p1, double* p2, int mode,
                       hipStream_t s) {
  if (B.count <= 0) return;
#define RSP_CALL(NB) arnoldi_nb<NB>(B, V, j, z, p1, p2, mode, s)
  RSP_GM_BUCKET(j, RSP_CALL)
#undef RSP_CALL
}
void launch_gm_finish(const GmBatch& B, const double* V, int j, double* p1, double* p2, hipStream_t s) {
  if (B.count <= 0) return;
#define RSP_CALL(NB) finish_nb<NB>(B, V, j, p1, p2, s)
  RSP_GM_BUCKET(j, RSP_CALL)
#undef RSP_CALL
}
void launch_gm_update_x(const GmBatch& B, const double* V, double* x, hipStream_t s) {
  if (B.count > 0) k_gm_update_x<<<grid_of(B), kT, 0, s>>>(B, V, x);
}

}  // namespace rsp
