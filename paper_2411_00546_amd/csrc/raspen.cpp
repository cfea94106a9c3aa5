// Host side of the RASPEN library: C ABI, the batch engine and its memory layout,
// the partition of Section 4.2, and the drivers of Algorithms 1-4 (local Newton
// loop, evaluation of the RASPEN residual, Jacobian action, outer Newton-GMRES).
// All arithmetic of the method runs in the HIP kernels; the host sequences the
// launches and reads back per-subdomain and per-instance scalars.
//
// Memory of a context: a global arena with the instances' persistent arrays
// (y_d, f, x; two of them, so that a new layout can take over the state of the
// instances of the old one) and a work arena with everything an outer iteration
// rebuilds (tiles, line factors, Krylov bases, per-item and per-instance tables).
#include "engine.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

using rsp::DevProblem;
using rsp::GmBatch;
using rsp::GmHess;
using rsp::GmSeg;
using rsp::GmState;
using rsp::Inst;
using rsp::Items;
using rsp::Partition;
using rsp::SubState;
using rsp::fail;
using rsp::Clock;

namespace rsp {

namespace {
thread_local std::string g_err;
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

const char* last_error() { return g_err.c_str(); }

}  // namespace rsp

#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) return fail(RSP_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define RSPCHK(expr)        \
  do {                      \
    int r_ = (expr);        \
    if (r_ < 0) return r_;  \
  } while (0)

namespace {

constexpr int kMaxRestart = rsp::kGmMaxRestart;
constexpr long long kAlignN = 32;   // instance offsets in the batch arrays: multiples of 32 nodes

int split_1d(int n, int s, std::vector<std::pair<int, int>>* out) {
  if (s < 1 || s > n) return fail(RSP_EINVAL, "need 1 <= subdomains (%d) <= nodes (%d)", s, n);
  const int B = (n + s - 1) / s;
  out->clear();
  for (int j = 0; j < s; ++j) {
    const int lo = j * B, hi = std::min((j + 1) * B, n);
    if (lo >= hi) return fail(RSP_EINVAL, "%d boxes of width %d leave an empty box on %d nodes", s, B, n);
    out->push_back({lo, hi});
  }
  return 0;
}

}  // namespace

namespace rsp {

int validate_problem(const rsp_problem* p) {
  if (!p) return fail(RSP_EINVAL, "problem is NULL");
  if (p->nx < 1 || p->ny < 1) return fail(RSP_EINVAL, "grid must have nx, ny >= 1");
  if (p->phi_kind < RSP_PHI_ZERO || p->phi_kind > RSP_PHI_PAPER) return fail(RSP_EINVAL, "unknown phi_kind %d", p->phi_kind);
  if (!(p->nu > 0)) return fail(RSP_EINVAL, "nu must be > 0");
  if (!(p->mu >= 0)) return fail(RSP_EINVAL, "mu must be >= 0");
  if (!(p->eps_min > 0) || !(p->eps0 >= p->eps_min)) return fail(RSP_EINVAL, "need 0 < eps_min <= eps0");
  if (p->eps0 > p->eps_min && !(p->gamma > 0 && p->gamma < 1)) return fail(RSP_EINVAL, "need 0 < gamma < 1");
  if (p->overlap < 0) return fail(RSP_EINVAL, "overlap must be >= 0");
  return 0;
}

int line_block(int txm) { return ((2 * txm + 15) / 16) * 16; }

DevProblem dev_problem(const rsp_problem& p, long long noff, int S, int txm, int tym, int M) {
  DevProblem P{};
  P.nx = p.nx;
  P.ny = p.ny;
  P.phi = p.phi_kind;
  P.kappa = p.kappa;
  P.nu = p.nu;
  P.inv_nu = 1.0 / p.nu;
  P.mu = p.mu;
  const double hx = 1.0 / (p.nx + 1), hy = 1.0 / (p.ny + 1);
  P.hx2i = 1.0 / (hx * hx);
  P.hy2i = 1.0 / (hy * hy);
  P.diag0 = 2.0 * P.hx2i + 2.0 * P.hy2i;
  // Line blocks couple the fields through g'(p)/nu (rows of y, columns of p) and
  // phi''(y) p - 1 (rows of p): weighting the rows of y by about sqrt(nu), rounded to a
  // power of two, balances the two in the column dominance test of the line factors.
  P.dom_w = std::ldexp(1.0, std::max(-60, std::min(0, (int)std::lround(0.5 * std::log2(p.nu)))));
  P.eps_min = p.eps_min;
  P.gamma = p.gamma;
  P.eps_start = p.eps_min;
  P.noff = noff;
  P.S = S;
  P.txm = txm;
  P.tym = tym;
  P.M = M;
  return P;
}

}  // namespace rsp

using rsp::validate_problem;
using rsp::line_block;

namespace rsp {

int validate_options(const rsp_options* o) {
  if (!o) return fail(RSP_EINVAL, "options are NULL");
  if (!(o->sigma >= 1)) return fail(RSP_EINVAL, "sigma must be >= 1");
  if (!(o->alpha_min > 0 && o->alpha_min <= 1)) return fail(RSP_EINVAL, "need 0 < alpha_min <= 1");
  if (o->gmres_restart < 1 || o->gmres_restart > kMaxRestart) return fail(RSP_EINVAL, "gmres_restart must be in 1..%d", kMaxRestart);
  if (o->max_outer < 0 || o->max_inner < 0 || o->max_gmres < 1) return fail(RSP_EINVAL, "negative iteration limit");
  if (o->precision != RSP_FP64 && o->precision != RSP_FP32_REFINED)
    return fail(RSP_EINVAL, "unknown precision %d", o->precision);
  if (o->max_refine < 0 || o->max_refine > 8) return fail(RSP_EINVAL, "max_refine must be in 0..8");
  if (o->continuation < RSP_CONT_FIRST || o->continuation > RSP_CONT_EVERY) return fail(RSP_EINVAL, "unknown continuation mode");
  if (!(o->tol_outer >= 0) || !(o->tol_inner >= 0) || !(o->gmres_rtol >= 0)) return fail(RSP_EINVAL, "negative tolerance");
  if (std::isnan(o->tol_inner_rel)) return fail(RSP_EINVAL, "tol_inner_rel is NaN");
  if (std::isnan(o->fallback_rho)) return fail(RSP_EINVAL, "fallback_rho is NaN");
  if (o->record_eps_snapshots < 0 || o->record_eps_snapshots > RSP_HIST_MAX + 1)
    return fail(RSP_EINVAL, "record_eps_snapshots must be in 0..%d", RSP_HIST_MAX + 1);
  if (o->record_eps_snapshots > 0 && !o->eps_snapshots)
    return fail(RSP_EINVAL, "record_eps_snapshots needs the eps_snapshots array");
  if (o->coarse != 0 && o->coarse != 1) return fail(RSP_EINVAL, "coarse must be 0 or 1");
  return 0;
}

rsp_options fallback_options(const rsp_options& o) {
  rsp_options r = o;
  r.precision = RSP_FP64;
  r.max_refine = 0;
  r.fallback_rho = -1.0;
  r.record_eps_snapshots = 0;
  r.eps_snapshots = nullptr;
  return r;
}

int make_partition(const rsp_problem* p, Partition* out) {
  RSPCHK(validate_problem(p));
  std::vector<std::pair<int, int>> xs, ys;
  RSPCHK(split_1d(p->nx, p->sx, &xs));
  RSPCHK(split_1d(p->ny, p->sy, &ys));
  out->box.clear();
  out->core.clear();
  out->txm = out->tym = 0;
  for (auto& yy : ys)
    for (auto& xx : xs) {
      int4 c = make_int4(xx.first, xx.second, yy.first, yy.second);
      int4 b = make_int4(std::max(0, c.x - p->overlap), std::min(p->nx, c.y + p->overlap),
                         std::max(0, c.z - p->overlap), std::min(p->ny, c.w + p->overlap));
      out->core.push_back(c);
      out->box.push_back(b);
      out->txm = std::max(out->txm, b.y - b.x);
      out->tym = std::max(out->tym, b.w - b.z);
    }
  out->S = (int)out->box.size();
  out->sx = p->sx;
  out->sy = p->sy;
  if (out->txm > kMaxTile)
    return fail(RSP_EINVAL, "tile width %d exceeds the supported %d nodes", out->txm, kMaxTile);
  if (out->tym > kMaxTile)
    return fail(RSP_EINVAL, "tile height %d exceeds the supported %d nodes", out->tym, kMaxTile);
  return 0;
}

int inst_init(Inst* in, const rsp_problem* prob) {
  Partition part;
  RSPCHK(make_partition(prob, &part));
  *in = Inst{};
  in->prob = *prob;
  in->part = std::move(part);
  in->n = (size_t)prob->nx * prob->ny;
  in->t0 = Clock::now();
  in->hist.fallback_outer = -1;
  return 0;
}

}  // namespace rsp

namespace {

// Tile geometry and sizes of a layout.
struct Geometry {
  int ninst = 0, S = 0, txm = 0, tym = 0, M = 0;
  long long ntot = 0;   // nodes of the concatenated [ny][nx] arrays (instances 32-aligned)
  long long ncoef = 0;  // doubles of the coefficient arrays of A (instances that have them)
  // second level: entries of the coarse factors S_r^{-1} and of the dense A0^{-1} of all
  // instances, the widest row of cores
  long long sinv = 0, ainv = 0;
  int csx_max = 0;
};

// Carves 256-byte aligned buffers; with base == nullptr it only counts the bytes,
// so sizing and carving can never disagree.
struct Carve {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    const size_t o = off;
    off += (count * sizeof(T) + 255) / 256 * 256;
    return base ? reinterpret_cast<T*>(base + o) : nullptr;
  }
};

enum { kLEval, kLGo, kLCyc, kLFin, kLists };

// Buffers of the work arena.
struct Work {
  DevProblem* prob = nullptr;   // [ninst]
  GmSeg* seg = nullptr;         // [ninst]
  GmState* gst = nullptr;       // [ninst]
  GmHess* ghs = nullptr;        // [ninst]
  double* norms = nullptr;      // [ninst]
  int* ilist[kLists] = {};      // [ninst] instance lists
  int4 *box = nullptr, *core = nullptr;   // [S]
  int* inst = nullptr;                    // [S]
  SubState* state = nullptr;              // [S]
  int* fallback = nullptr;                // [S] factor fallback flags (0 between launches)
  int* list[kLists] = {};                 // [S] item lists
  double *F = nullptr, *w = nullptr, *b = nullptr, *dx = nullptr, *r = nullptr;   // [2 ntot]
  double *tilex = nullptr, *c = nullptr, *dir = nullptr, *res = nullptr, *t1 = nullptr, *t2 = nullptr;
  void* fac = nullptr;
  double *g = nullptr, *V = nullptr, *p1 = nullptr, *p2 = nullptr;
  // second level (rsp_options.coarse): core sums [3 S], coarse vectors [2 S], factors
  double *csum = nullptr, *cvec = nullptr, *evec = nullptr, *sinv = nullptr, *ainv = nullptr;
  double* cpt = nullptr;   // pointwise blocks of F'(x) at the outer iterate, [3][ntot]
};

void carve_global(Carve& cv, const Geometry& g, double** yd, double** f, double** x, double** coef) {
  *yd = cv.take<double>(g.ntot);
  *f = cv.take<double>(g.ntot);
  *x = cv.take<double>(2 * g.ntot);
  *coef = g.ncoef ? cv.take<double>(g.ncoef) : nullptr;
}

// Doubles of the scaled coefficient arrays of one instance (cx, cy, c0), 32-aligned each.
long long coef_doubles(int nx, int ny) {
  auto al = [](long long v) { return (v + kAlignN - 1) / kAlignN * kAlignN; };
  return al((long long)(nx + 1) * ny) + al((long long)nx * (ny + 1)) + al((long long)nx * ny);
}

void carve_work(Carve& cv, const Geometry& g, const rsp_options& o, Work* w) {
  const size_t S = g.S, ni = g.ninst, L = 2 * (size_t)g.ntot;
  const size_t tile = S * 2 * g.txm * g.tym, halo = S * 2 * (g.txm + 2) * (g.tym + 2);
  const size_t fe = o.precision == RSP_FP32_REFINED ? 4 : 8;
  const size_t part = ni * rsp::kGmBlocks * rsp::kGmMaxVec;
  w->prob = cv.take<DevProblem>(ni);
  w->seg = cv.take<GmSeg>(ni);
  w->gst = cv.take<GmState>(ni);
  w->ghs = cv.take<GmHess>(ni);
  w->norms = cv.take<double>(ni);
  for (auto& l : w->ilist) l = cv.take<int>(ni);
  w->box = cv.take<int4>(S);
  w->core = cv.take<int4>(S);
  w->inst = cv.take<int>(S);
  w->state = cv.take<SubState>(S);
  w->fallback = cv.take<int>(S);
  for (auto& l : w->list) l = cv.take<int>(S);
  w->F = cv.take<double>(L);
  w->w = cv.take<double>(L);
  w->b = cv.take<double>(L);
  w->dx = cv.take<double>(L);
  w->r = cv.take<double>(L);
  w->tilex = cv.take<double>(halo);
  w->c = cv.take<double>(tile);
  w->dir = cv.take<double>(tile);
  w->res = cv.take<double>(tile);
  w->t1 = cv.take<double>(tile);
  w->t2 = cv.take<double>(tile);
  w->fac = cv.take<char>(fe * S * g.tym * g.M * g.M);
  w->g = cv.take<double>(S * g.tym * g.M);
  w->V = cv.take<double>((size_t)(o.gmres_restart + 1) * L);
  w->p1 = cv.take<double>(part);
  w->p2 = cv.take<double>(part);
  if (o.coarse) {
    w->csum = cv.take<double>(8 * S);
    w->cvec = cv.take<double>(2 * S);
    w->evec = cv.take<double>(2 * S);
    w->sinv = cv.take<double>(g.sinv);
    w->ainv = cv.take<double>(g.ainv);
    w->cpt = cv.take<double>(3 * (size_t)g.ntot);
  }
}

Geometry geometry_of(const std::vector<const Partition*>& parts, const std::vector<size_t>& ns,
                     const std::vector<long long>& ncoef) {
  Geometry g;
  g.ninst = (int)parts.size();
  for (size_t q = 0; q < parts.size(); ++q) {
    g.ncoef += ncoef[q];
    g.S += parts[q]->S;
    g.txm = std::max(g.txm, parts[q]->txm);
    g.tym = std::max(g.tym, parts[q]->tym);
    g.ntot += ((long long)ns[q] + kAlignN - 1) / kAlignN * kAlignN;
    const long long nc = 2LL * parts[q]->sx, N = nc * parts[q]->sy;
    g.sinv += parts[q]->sy * nc * nc;
    g.ainv += N * N;
    g.csx_max = std::max(g.csx_max, parts[q]->sx);
  }
  g.M = line_block(g.txm);
  return g;
}

size_t layout_bytes(const Geometry& g, const rsp_options& o) {
  Carve a, b;
  double *yd, *f, *x, *coef;
  Work w;
  carve_global(a, g, &yd, &f, &x, &coef);
  carve_work(b, g, o, &w);
  return a.off + b.off;
}

// Kernel timing: HIP events around launches, resolved at synchronisation points.
enum Kid {
  KID_RESTRICT, KID_INIT, KID_FACTOR, KID_SOLVE_BWD, KID_LINESEARCH, KID_PROLONG, KID_RING,
  KID_BLOCK_SOLVE, KID_GMRES_ORTHO, KID_GLOBAL, KID_REFINE, KID_PRECOND, KID_GJAC, KID_COARSE,
  KID_COARSE_SETUP, KID_N
};
const char* const kKidName[KID_N] = {"restrict_halo", "newton_init", "factor", "solve_bwd",
                                     "linesearch", "prolong", "ring_rhs", "block_solve",
                                     "gmres_ortho", "global_residual", "newton_refine",
                                     "ras_precond", "global_jacobian", "coarse_correction",
                                     "coarse_setup"};

struct Pending {
  int kid;
  hipEvent_t a, b;
  double flops, bytes;
  int step;   // Arnoldi step of a GMRES launch whose work is settled afterwards, else -1
};

// A launch sequence that is captured once and replayed: its kind and the integers
// that shape its launches (list slot, item and instance counts, first step, length).
enum SeqKind { SEQ_ARNOLDI, SEQ_NEWTON };
struct GraphKey {
  int kind, a, b, c, d;
  bool operator<(const GraphKey& o) const {
    return std::tie(kind, a, b, c, d) < std::tie(o.kind, o.a, o.b, o.c, o.d);
  }
};
constexpr size_t kMaxGraphs = 256;

}  // namespace

struct rsp_context {
  int device = 0;
  int n_cu = 1;                 // compute units of the device
  size_t budget = 0;
  rsp_options opts{};
  Geometry geo;
  // global arenas (the current one holds the placed instances' y_d, f, x)
  void* gmem[2] = {nullptr, nullptr};
  size_t gcap[2] = {0, 0};
  int gcur = 0;
  double *yd = nullptr, *f = nullptr, *x = nullptr;
  double* coef = nullptr;   // scaled coefficient arrays of A of the instances that have them
  bool var = false;         // some instance of the layout has variable coefficients
  // work arena (capacity grows)
  void* wmem = nullptr;
  size_t wcap = 0;
  Work w;
  int fp32 = 0;       // FP32 line factors (mixed precision)
  int nref = 0;       // FP64 refinement steps per local solve with FP32 factors
  // host mirrors
  std::vector<DevProblem> hprob;
  std::vector<GmSeg> hseg;
  std::vector<SubState> hstate;
  std::vector<GmState> hgm;
  // pinned staging for the small device-to-host reads (a read from pageable memory is
  // staged through an extra copy kernel and a host copy)
  void* pin = nullptr;
  size_t pin_cap = 0;
  hipEvent_t wait_ev = nullptr;   // completion of the work before a read-back
  std::vector<double> hnorm;
  std::vector<int> hlist[kLists], hilist[kLists];
  // the instance bound by rsp_setup / rsp_solve for the single-problem calls
  Inst single;
  bool ready = false;
  // captured launch sequences (hipGraphs), valid while the launch signature holds
  int graphs = 0;               // capture and replay (else plain stream launches)
  int gm_chunk = 32;            // Arnoldi steps between two reads of the GMRES headers
  int jac_form = 0;             // rsp_tuning.jac_form
  int gm_nbx = 1;               // grid width of the GMRES vector kernels (longest instance)
  int gm_op = 0;                // operator of GMRES: 0 the Jacobian action of Algorithm 4,
                                // 1 F'_eps(x) of the whole system (monolithic Newton)
  bool coarse_in_apply = false; // the two-level action forms the coarse values of each ring
                                // in its own workgroups (no separate coarse solve launch)
  hipStream_t cap = nullptr;    // private stream, only ever in capture mode
  uint64_t gsig = 0;
  std::map<GraphKey, hipGraphExec_t> gcache;
  // kernel timing
  bool prof = false;
  int prof_only = -1;   // time only this kernel class (-1: every class)
  int prof_every = 1;   // time the launches of one in prof_every launch sequences
  uint64_t prof_seq = 0;
  bool prof_mute = false;   // inside a launch sequence that is not timed
  std::vector<hipEvent_t> ev_pool;
  std::vector<Pending> pending;
  rsp_kernel_stat kstat[KID_N]{};
};

namespace {

// Waits until the work enqueued on `st` so far has completed, polling an event: a
// read-back decides the next launches, and a polling thread resumes sooner than one
// that blocks in hipStreamSynchronize.
int wait_stream(rsp_context* ctx, hipStream_t st) {
  if (!ctx->wait_ev) HIPCHK(hipEventCreateWithFlags(&ctx->wait_ev, hipEventDisableTiming));
  HIPCHK(hipEventRecord(ctx->wait_ev, st));
  for (;;) {
    const hipError_t e = hipEventQuery(ctx->wait_ev);
    if (e == hipSuccess) return 0;
    if (e != hipErrorNotReady) return fail(RSP_EHIP, "waiting for the stream: %s", hipGetErrorString(e));
  }
}

// Enqueues the copy of n host bytes (pageable memory) to device memory `dst` on `st`.
// HIP stages a pageable source before the call returns, so `src` may be reused at once.
// (A pinned staging ring measured no faster on the solves: these copies are small.)
int upload(rsp_context* ctx, void* dst, const void* src, size_t n, hipStream_t st) {
  (void)ctx;
  if (n == 0) return 0;
  HIPCHK(hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, st));
  return 0;
}

// Copies n bytes of device memory to host memory `dst` through the pinned staging
// buffer and waits for them (every read-back of the solver goes through here).
int read_back(rsp_context* ctx, void* dst, const void* src, size_t n, hipStream_t st) {
  if (n == 0) return 0;
  if (ctx->pin_cap < n) {
    HIPCHK(hipStreamSynchronize(st));
    if (ctx->pin) HIPCHK(hipHostFree(ctx->pin));
    ctx->pin = nullptr;
    ctx->pin_cap = 0;
    const size_t cap = std::max(n, (size_t)4096);
    HIPCHK(hipHostMalloc(&ctx->pin, cap, hipHostMallocDefault));
    ctx->pin_cap = cap;
  }
  HIPCHK(hipMemcpyAsync(ctx->pin, src, n, hipMemcpyDeviceToHost, st));
  RSPCHK(wait_stream(ctx, st));
  std::memcpy(dst, ctx->pin, n);
  return 0;
}

int account(rsp_context* ctx, const Pending& p) {
  HIPCHK(hipEventSynchronize(p.b));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
  rsp_kernel_stat& k = ctx->kstat[p.kid];
  k.launches += 1;
  k.ms += ms;
  k.flops += p.flops;
  k.bytes += p.bytes;
  return 0;
}

// Accounts the pending timings (those of GMRES launches whose work is not settled
// yet stay pending).
int resolve_events(rsp_context* ctx) {
  std::vector<Pending> keep;
  for (auto& p : ctx->pending) {
    if (p.step >= 0) {
      keep.push_back(p);
      continue;
    }
    RSPCHK(account(ctx, p));
    ctx->ev_pool.push_back(p.a);
    ctx->ev_pool.push_back(p.b);
  }
  ctx->pending.swap(keep);
  return 0;
}

hipEvent_t event_get(rsp_context* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  // timing only: no system-scope fence (cache writeback) at each record, which would
  // slow the work between the events
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

// Brackets the launches issued during its lifetime with events (when timing is on),
// attributing the given algorithmic flops and bytes to kernel `kid`.
struct Timed {
  rsp_context* c;
  int kid;
  hipStream_t st;
  double fl, by;
  int step;
  hipEvent_t a = nullptr;
  Timed(rsp_context* c_, int kid_, hipStream_t st_, double fl_, double by_, int step_ = -1)
      : c(c_), kid(kid_), st(st_), fl(fl_), by(by_), step(step_) {
    if (c->prof && !c->prof_mute && (c->prof_only < 0 || c->prof_only == kid) && (a = event_get(c)) != nullptr &&
        hipEventRecord(a, st) != hipSuccess)
      a = nullptr;
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = event_get(c);
    if (!b || hipEventRecord(b, st) != hipSuccess) return;
    c->pending.push_back({kid, a, b, fl, by, step});
    if (c->pending.size() > 16384) (void)resolve_events(c);
  }
};

// Everything the captured launches take as arguments besides the graph key: the
// layout, the arena pointers and the options the kernels read.  A change drops
// every captured graph.
uint64_t launch_signature(const rsp_context* ctx) {
  uint64_t h = 1469598103934665603ull;   // FNV-1a
  auto add = [&h](const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  };
  auto val = [&add](auto v) { add(&v, sizeof v); };
  const Geometry& g = ctx->geo;
  val(g.ninst), val(g.S), val(g.txm), val(g.tym), val(g.M), val(g.ntot);
  add(&ctx->w, sizeof(Work));   // pointers only
  val(ctx->yd), val(ctx->f), val(ctx->x);
  const rsp_options& o = ctx->opts;
  val(o.tol_inner), val(o.sigma), val(o.alpha_min), val(o.gmres_restart), val(o.max_inner);
  val(o.precision), val(ctx->fp32), val(ctx->nref), val(ctx->gm_op), val(ctx->gm_nbx), val(ctx->coarse_in_apply), val(ctx->jac_form);
  return h;
}

// Drops the captured graphs (after the stream has drained: none may still run).
int drop_graphs(rsp_context* ctx, hipStream_t st) {
  if (ctx->gcache.empty()) return 0;
  HIPCHK(hipStreamSynchronize(st));
  for (auto& kv : ctx->gcache) (void)hipGraphExecDestroy(kv.second);
  ctx->gcache.clear();
  return 0;
}

// Runs the launches `enqueue(stream)` issues on `st`: directly, or (graphs on) as a
// graph captured from them once on the private stream and replayed for every later
// call with the same key and launch signature.  The sequences captured here are
// kernel launches only.  A sequence whose launches are timed is launched directly:
// event pairs recorded inside a graph do not give usable elapsed times.  With event
// timing on, one in prof_every sequences is timed; the others run untimed (muted),
// as graphs when graphs are on.
// Kernel classes each kind of sequence launches.
constexpr unsigned kSeqKids[2] = {(1u << KID_BLOCK_SOLVE) | (1u << KID_GMRES_ORTHO),
                                  (1u << KID_FACTOR) | (1u << KID_SOLVE_BWD) | (1u << KID_REFINE) |
                                      (1u << KID_LINESEARCH)};

template <class F>
int launch_seq(rsp_context* ctx, const GraphKey& key, hipStream_t st, F&& enqueue) {
  // a sequence with no launch of the timed class is never timed
  const bool timeable = ctx->prof && (ctx->prof_only < 0 || ((kSeqKids[key.kind] >> ctx->prof_only) & 1u));
  const bool timed = timeable && ctx->prof_seq++ % (uint64_t)ctx->prof_every == 0;
  struct Mute {
    rsp_context* c;
    bool old;
    ~Mute() { c->prof_mute = old; }
  } mute{ctx, ctx->prof_mute};
  ctx->prof_mute = ctx->prof && !timed;
  if (!ctx->graphs || timed) {
    enqueue(st);
    HIPCHK(hipGetLastError());
    return 0;
  }
  const uint64_t sig = launch_signature(ctx);
  if (sig != ctx->gsig) {
    RSPCHK(drop_graphs(ctx, st));
    ctx->gsig = sig;
  }
  auto it = ctx->gcache.find(key);
  if (it == ctx->gcache.end()) {
    if (ctx->gcache.size() >= kMaxGraphs) RSPCHK(drop_graphs(ctx, st));
    if (!ctx->cap) HIPCHK(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
    enqueue(ctx->cap);
    const hipError_t le = hipGetLastError();
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(ctx->cap, &g);
    hipGraphExec_t ex = nullptr;
    hipError_t ie = hipSuccess;
    if (le == hipSuccess && ce == hipSuccess && g) ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (le != hipSuccess || ce != hipSuccess || !g || ie != hipSuccess) {
      const hipError_t e = le != hipSuccess ? le : ce != hipSuccess ? ce : ie;
      return fail(RSP_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    }
    it = ctx->gcache.emplace(key, ex).first;
  }
  HIPCHK(hipGraphLaunch(it->second, st));
  return 0;
}

// Algorithmic work of the per-subdomain kernels (m = 2 tx line unknowns, ty lines).
struct SubWork {
  double factor_fl = 0, factor_by = 0, bwd_fl = 0, bwd_by = 0, solve_fl = 0, solve_by = 0;
  double tile_by = 0, halo_by = 0;
  void add(int4 b, double fe) {
    const double tx = b.y - b.x, ty = b.w - b.z, m = 2 * tx;
    factor_fl += 16.0 * ty * tx * tx * tx;           // ty Gauss-Jordan inversions of m x m
    factor_by += fe * ty * m * m;                    // the inverses written once
    bwd_fl += 2.0 * (ty - 1) * m * m;
    bwd_by += fe * (ty - 1) * m * m;
    solve_fl += 2.0 * (2 * ty - 1) * m * m;          // forward + backward sweeps
    solve_by += fe * (2 * ty - 1) * m * m + 8.0 * 2 * m * ty;
    tile_by += 8.0 * m * ty;
    halo_by += 8.0 * 2 * (tx + 2) * (ty + 2);
  }
};

// Work of the items in `items` (optionally only the active ones).
SubWork sub_work(const rsp_context* ctx, const std::vector<Inst*>& set, bool active_only) {
  SubWork w;
  const double fe = ctx->fp32 ? 4.0 : 8.0;
  for (const Inst* in : set)
    for (int q = 0; q < in->part.S; ++q) {
      if (active_only && !ctx->hstate[in->sub0 + q].active) continue;
      w.add(in->part.box[q], fe);
    }
  return w;
}

// Number of Algorithm 1 steps until eps reaches eps_min (evaluated like the device).
int continuation_steps(double eps0, double eps_min, double gamma) {
  int k = 0;
  double e = eps0;
  while (e > eps_min && k < 100000) {
    e = std::max(gamma * e, eps_min);
    ++k;
  }
  return k;
}

Items items_of(const rsp_context* ctx, const int* list, int count) {
  Items I;
  I.prob = ctx->w.prob;
  I.inst = ctx->w.inst;
  I.box = ctx->w.box;
  I.core = ctx->w.core;
  I.list = list;
  I.skip = nullptr;
  I.skip_stride = 0;
  I.count = count;
  return I;
}

Items all_items(const rsp_context* ctx) { return items_of(ctx, nullptr, ctx->geo.S); }

GmBatch gm_of(const rsp_context* ctx, const int* list, int count) {
  GmBatch B;
  B.seg = ctx->w.seg;
  B.st = ctx->w.gst;
  B.hs = ctx->w.ghs;
  B.list = list;
  B.ldv = 2 * ctx->geo.ntot;
  B.count = count;
  B.m = ctx->opts.gmres_restart;
  B.nbx = ctx->gm_nbx;
  return B;
}

// Uploads the item list and the instance list of `set` into list slot `l`.
int upload_lists(rsp_context* ctx, int l, const std::vector<Inst*>& set, hipStream_t st) {
  auto& it = ctx->hlist[l];
  auto& il = ctx->hilist[l];
  it.clear();
  il.clear();
  for (const Inst* in : set) {
    il.push_back(in->slot);
    for (int q = 0; q < in->part.S; ++q) it.push_back(in->sub0 + q);
  }
  RSPCHK(upload(ctx, ctx->w.list[l], it.data(), sizeof(int) * it.size(), st));
  RSPCHK(upload(ctx, ctx->w.ilist[l], il.data(), sizeof(int) * il.size(), st));
  return 0;
}

struct EvalStats {
  int status = 0, inner_min = 0, inner_max = 0, backtracks = 0;
  double inner_avg = 0;
};

// Algorithm 3 for the instances of `set` on the device: local Newton solves
// (Algorithm 1) for their subdomains, factorisation at x^(i), and the assembly
// F(x) = sum_i P~_i C_i(x) into `out`.  cont[q]: instance q starts its local
// solves at eps0 (continuation), else at eps_min.  x, out: batch arrays.
int run_eval(rsp_context* ctx, const std::vector<Inst*>& set, const std::vector<char>& cont,
             const double* x, double* out, std::vector<EvalStats>* es, hipStream_t st) {
  const rsp_options& o = ctx->opts;
  const int M = ctx->geo.M;
  int ncont = 0;
  for (size_t q = 0; q < set.size(); ++q) {
    const Inst* in = set[q];
    DevProblem& P = ctx->hprob[in->slot];
    P.eps_start = cont[q] ? in->prob.eps0 : in->prob.eps_min;
    ncont = std::max(ncont, continuation_steps(P.eps_start, in->prob.eps_min, in->prob.gamma));
  }
  RSPCHK(upload(ctx, ctx->w.prob, ctx->hprob.data(), sizeof(DevProblem) * ctx->hprob.size(), st));
  RSPCHK(upload_lists(ctx, kLEval, set, st));
  const int count = (int)ctx->hlist[kLEval].size();
  const Items I = items_of(ctx, ctx->w.list[kLEval], count);
  const SubWork all = sub_work(ctx, set, false);
  Work& w = ctx->w;
  {
    Timed t(ctx, KID_RESTRICT, st, 0, all.halo_by * 2);
    rsp::launch_restrict_halo(I, x, w.tilex, st);
  }
  {
    Timed t(ctx, KID_INIT, st, 40.0 * all.tile_by / 8, all.halo_by + 3 * all.tile_by);
    rsp::launch_newton_init(I, w.tilex, ctx->yd, ctx->f, w.c, w.res, w.state, o.tol_inner,
                            o.tol_inner_rel < 0 ? o.tol_inner : o.tol_inner_rel, o.max_inner, st);
  }
  HIPCHK(hipGetLastError());
  // snapshots of the first evaluation of a single instance: x + sum_i P~_i c_i^(k) after
  // local Newton step k (k = 0: c = 0), with the eps_k of the steps
  Inst* rec = (set.size() == 1 && set[0]->snap && cont[0] && !set[0]->started) ? set[0] : nullptr;
  double rec_eps = rec ? ctx->hprob[rec->slot].eps_start : 0.0;
  auto record = [&](int k, hipStream_t s) {
    if (!rec || k >= rec->snap_max) return;
    // the prolongation writes at the instance's offset in the batch arrays: its own
    // array is addressed relative to that (the single instance sits at offset 0)
    double* dst = rec->snap + (size_t)k * 2 * rec->n - 2 * rec->noff;
    rsp::launch_prolong(I, w.c, x, dst, s);
    rec->hist.snapshot_eps[k] = rec_eps;
    rec->hist.snapshots = k + 1;
    rec_eps = std::max(rec->prob.gamma * rec_eps, rec->prob.eps_min);
  };
  record(0, st);
  auto read_state = [&]() -> int {
    return read_back(ctx, ctx->hstate.data(), w.state, sizeof(SubState) * ctx->hstate.size(), st);
  };
  auto count_active = [&]() {
    int a = 0;
    for (int s : ctx->hlist[kLEval]) a += ctx->hstate[s].active;
    return a;
  };
  RSPCHK(read_state());
  int it = 0;
  int active = count_active();
  while (active && it < o.max_inner + 1) {
    // the continuation steps are needed by every subdomain that continues: run them
    // without looking, then check after every step
    const int batch = std::max(1, std::min(ncont - it, o.max_inner + 1 - it));
    const SubWork sw = sub_work(ctx, set, true);
    auto steps = [&](hipStream_t s) {
      for (int b = 0; b < batch; ++b) {
        {
          Timed t(ctx, KID_FACTOR, s, sw.factor_fl + sw.bwd_fl / 2, sw.factor_by);
          rsp::launch_factor(I, M, w.tilex, w.c, w.state, 0.0, w.res, -1.0, w.fac, ctx->fp32, w.g,
                             w.fallback, ctx->var, s);
        }
        {
          Timed t(ctx, KID_SOLVE_BWD, s, sw.bwd_fl, sw.bwd_by);
          rsp::launch_solve_bwd(I, M, w.state, w.fac, ctx->fp32, w.g, w.dir, s);
        }
        if (ctx->nref > 0) {
          Timed t(ctx, KID_REFINE, s, ctx->nref * (sw.solve_fl + 20.0 * sw.tile_by / 8),
                  ctx->nref * (sw.solve_by + 2 * sw.tile_by));
          rsp::launch_newton_refine(I, M, w.tilex, w.c, w.state, w.fac, ctx->fp32, w.res, w.dir, ctx->nref, s);
        }
        {
          Timed t(ctx, KID_LINESEARCH, s, 40.0 * sw.tile_by / 8, 6 * sw.tile_by);
          rsp::launch_linesearch(I, w.tilex, ctx->yd, ctx->f, w.c, w.dir, w.res, w.state, o.sigma,
                                 o.alpha_min, o.max_inner, s);
        }
        record(it + b + 1, s);
      }
    };
    if (rec) steps(st);   // recorded steps write to step-dependent addresses: no graph
    else RSPCHK(launch_seq(ctx, GraphKey{SEQ_NEWTON, count, batch, 0, 0}, st, steps));
    it += batch;
    RSPCHK(read_state());
    active = count_active();
  }
  es->assign(set.size(), EvalStats{});
  for (size_t q = 0; q < set.size(); ++q) {
    Inst* in = set[q];
    EvalStats& e = (*es)[q];
    int64_t ksum = 0;
    e.inner_min = 1 << 30;
    double fl = 0, ffl = 0;
    for (int j = 0; j < in->part.S; ++j) {
      const SubState& S = ctx->hstate[in->sub0 + j];
      ksum += S.k;
      e.inner_min = std::min(e.inner_min, S.k);
      e.inner_max = std::max(e.inner_max, S.k);
      e.backtracks += S.backtracks;
      e.status = std::max(e.status, S.status);
      const int4 b = in->part.box[j];
      const double tx = b.y - b.x, ty = b.w - b.z;
      fl += S.k * (16.0 * ty * tx * tx * tx + 2.0 * (2 * ty - 1) * 4 * tx * tx);
      ffl += 16.0 * ty * tx * tx * tx;
    }
    e.inner_avg = (double)ksum / in->part.S;
    in->n_factor += ksum + in->part.S;
    in->n_solve += ksum;
    in->n_newton += ksum;
    in->flops += fl + ffl;
  }
  // factor at x^(i) = x + P_i C_i(x) for Algorithm 4
  {
    Timed t(ctx, KID_FACTOR, st, all.factor_fl, all.factor_by);
    rsp::launch_factor(I, M, w.tilex, w.c, nullptr, 0.0, nullptr, 0.0, w.fac, ctx->fp32, w.g, w.fallback, ctx->var, st);
  }
  {
    Timed t(ctx, KID_PROLONG, st, 0, all.tile_by * 2);
    rsp::launch_prolong(I, w.c, nullptr, out, st);
  }
  HIPCHK(hipGetLastError());
  return 0;
}

// Algorithm 4 for the items I: out = -d + sum_i P~_i J_i^{-1}(h^-2 weighted outside
// neighbours of d) on their instances' segments.
// Algorithmic flops and bytes of one Jacobian action over the subdomains of `sw`, and
// of Arnoldi step q (classical Gram-Schmidt twice, normalisation) on vectors of total
// length L.
double apply_flops(const rsp_context* ctx, const SubWork& sw) { return (1 + ctx->nref) * sw.solve_fl; }
double apply_bytes(const rsp_context* ctx, const SubWork& sw) {
  return (1 + ctx->nref) * sw.solve_by + 2 * sw.tile_by;
}
double ortho_flops(double L, int q) { return L * (8.0 * q + 8); }
double ortho_bytes(double L, int q) { return 8.0 * L * (2.0 * q + 6); }

// step >= 0: Arnoldi step of a GMRES cycle (its timing is settled by settle_gmres_timing).
// Whether the Jacobian action over the items I runs as one launch of one workgroup per
// subdomain: with at least as many subdomains as compute units.  Below that, the two
// launches of two workgroups per subdomain keep twice as many compute units streaming
// the factors (at 64 subdomains of 255^2 the one-launch form was 1.5x slower).
bool apply_one(const rsp_context* ctx, const Items& I) {
  if (!rsp::apply_one_launch(ctx->geo.M, ctx->fp32) || ctx->jac_form == 1) return false;
  return ctx->jac_form == 2 || I.count >= ctx->n_cu;
}

// ce: the coarse values (d - Z ce on the rings); ainv, cv: the action forms them itself
// from A0^{-1} and the projection cv (coarse_in_apply, one-launch form only).
void jac_apply(rsp_context* ctx, const Items& I, const SubWork& sw, const double* d, double* out,
               hipStream_t st, int step = -1, const double* ce = nullptr, const double* ainv = nullptr,
               const double* cv = nullptr) {
  Timed t(ctx, KID_BLOCK_SOLVE, st, apply_flops(ctx, sw), apply_bytes(ctx, sw), step);
  rsp::launch_jac_apply(I, ctx->geo.M, ctx->w.fac, ctx->fp32, ctx->w.tilex, ctx->w.c, d, ce, out, ctx->nref,
                        ctx->w.g, apply_one(ctx, I), ainv, cv, st);
}

// Largest number of coarse unknowns (2 S) over the instances of `set`.
int coarse_max_n(const std::vector<Inst*>& set) {
  int m = 0;
  for (const Inst* in : set) m = std::max(m, 2 * in->part.S);
  return m;
}

// Algorithmic work of the coarse correction in one GMRES product over the instances of
// `set`: the core sums of F'(x) v (two vectors read, 28 flops per node) and, unless the
// action forms the coarse values itself, the dense coarse solve (2 S)^2.
void coarse_work(const std::vector<Inst*>& set, bool with_solve, double* fl, double* by) {
  *fl = *by = 0;
  for (const Inst* in : set) {
    const double N = with_solve ? 2.0 * in->part.S : 0.0;
    *fl += 28.0 * in->n + 2 * N * N;
    *by += 32.0 * in->n + 8 * N * N;
  }
}

// The operator of GMRES on the instances of `set` (items I): the Jacobian action of
// Algorithm 4, or (gm_op 1) F'_eps(x) of the whole system with each instance's current
// smoothing.  skip_done: instances whose GMRES has stopped are skipped.
void gm_apply(rsp_context* ctx, const Items& I, const SubWork& sw, const std::vector<Inst*>& set,
              const GmBatch& B, const double* d, double* out, hipStream_t st, bool skip_done, int step = -1) {
  if (ctx->gm_op == 0) {
    jac_apply(ctx, I, sw, d, out, st, step);
    return;
  }
  if (ctx->gm_op == 2) {
    // the two-level operator d -> -d - sum_i P~_i J_i^{-1} B_i (d - Z e), e = A0^{-1} Z^T F'(x) d
    Work& w = ctx->w;
    const bool fused = ctx->coarse_in_apply && apply_one(ctx, I);
    {
      double fl, by;
      coarse_work(set, !fused, &fl, &by);
      Timed t(ctx, KID_COARSE, st, fl, by, step);
      rsp::launch_coarse_project(I, 1, w.cpt, ctx->geo.ntot, d, w.cvec, st);
      if (!fused)
        rsp::launch_coarse_solve(w.prob, B.list, B.count, coarse_max_n(set), skip_done ? w.gst : nullptr, w.ainv,
                                 w.cvec, 1.0, w.evec, st);
    }
    if (fused) jac_apply(ctx, I, sw, d, out, st, step, nullptr, w.ainv, w.cvec);
    else jac_apply(ctx, I, sw, d, out, st, step, w.evec);
    return;
  }
  double L = 0;
  for (const Inst* in : set) L += 2.0 * in->n;
  Timed t(ctx, KID_GJAC, st, 14.0 * L, 24.0 * L, step);
  for (const Inst* in : set)
    rsp::launch_global_jac_apply(ctx->w.prob, ctx->hprob[in->slot], in->slot, skip_done ? ctx->w.gst : nullptr,
                                 ctx->x, d, out, st);
}

// After the headers of a GMRES chunk are read: Arnoldi step q did work for the
// instances whose step count now exceeds q (a stopped instance's kernels return at
// once).  The timed launches of the chunk are re-priced by those instances, and
// launches that did no work for any instance are dropped from the statistics.
void settle_gmres_timing(rsp_context* ctx, const std::vector<Inst*>& cyc) {
  std::vector<Pending> keep;
  keep.reserve(ctx->pending.size());
  for (Pending p : ctx->pending) {
    if (p.step < 0) {
      keep.push_back(p);
      continue;
    }
    std::vector<Inst*> act;
    double L = 0;
    for (Inst* in : cyc)
      if (ctx->hgm[in->slot].steps > p.step) {
        act.push_back(in);
        L += 2.0 * in->n;
      }
    if (act.empty()) {
      ctx->ev_pool.push_back(p.a);
      ctx->ev_pool.push_back(p.b);
      continue;
    }
    if (p.kid == KID_BLOCK_SOLVE) {
      const SubWork sw = sub_work(ctx, act, false);
      p.flops = apply_flops(ctx, sw);
      p.bytes = apply_bytes(ctx, sw);
    } else if (p.kid == KID_GJAC) {
      p.flops = 14.0 * L;
      p.bytes = 24.0 * L;
    } else {
      p.flops = ortho_flops(L, p.step);
      p.bytes = ortho_bytes(L, p.step);
    }
    p.step = -1;
    keep.push_back(p);
  }
  ctx->pending.swap(keep);
}

// |v|_2 of every instance of `set` (list slot l must hold set), read back into hnorm.
int read_norms(rsp_context* ctx, int l, int count, const double* v, hipStream_t st) {
  const GmBatch B = gm_of(ctx, ctx->w.ilist[l], count);
  rsp::launch_gm_norms(B, v, ctx->w.p1, ctx->w.norms, st);
  HIPCHK(hipGetLastError());
  return read_back(ctx, ctx->hnorm.data(), ctx->w.norms, sizeof(double) * ctx->hnorm.size(), st);
}

int read_gm_headers(rsp_context* ctx, hipStream_t st) {
  return read_back(ctx, ctx->hgm.data(), ctx->w.gst, sizeof(GmState) * ctx->hgm.size(), st);
}

// Second level at the outer iterate x of the instances of `go` (list slot kLGo): the
// coarse operator A0 = Z^T F'(x) Z is assembled, factored by core rows and inverted
// densely, and the right-hand side of the two-level Newton system gets its coarse part:
// b = -F_RAS(x) + (F_RAS'(x) + I) Q F(x) = -F_RAS(x) - sum_i P~_i J_i^{-1} B_i (Z e_F), with
// e_F = A0^{-1} Z^T F(x) (Jacobian action on d = 0 with ring values -(-Z e_F)).
// A0 = Z^T F'(x) Z of the instances of `set` (items I, device instance list ilist),
// factored by rows of cores and inverted densely into the work arena.
void coarse_factorize(rsp_context* ctx, const Items& I, const int* ilist, const std::vector<Inst*>& set,
                      const double* x, hipStream_t st) {
  Work& w = ctx->w;
  double fl = 0, by = 0;
  for (const Inst* in : set) {
    const double N = 2.0 * in->part.S, nc = 2.0 * in->part.sx;
    fl += 12.0 * in->n + in->part.sy * (2 * nc * nc * nc + 4 * nc * nc * N);
    by += 16.0 * in->n + 8.0 * (N * N + in->part.sy * nc * nc);
  }
  Timed t(ctx, KID_COARSE_SETUP, st, fl, by);
  rsp::launch_coarse_sums(I, x, w.csum, w.cpt, ctx->geo.ntot, st);
  rsp::launch_coarse_factor(w.prob, ilist, (int)set.size(), nullptr, w.csum, w.sinv, st);
  rsp::launch_coarse_inverse(w.prob, ilist, (int)set.size(), coarse_max_n(set), nullptr, w.csum, w.sinv, w.ainv,
                             st);
}

int coarse_setup(rsp_context* ctx, const std::vector<Inst*>& go, const GmBatch& B, hipStream_t st) {
  Work& w = ctx->w;
  const Items I = items_of(ctx, w.list[kLGo], (int)ctx->hlist[kLGo].size());
  const int max_n = coarse_max_n(go);
  coarse_factorize(ctx, I, w.ilist[kLGo], go, ctx->x, st);
  {
    double fl = 0, by = 0;
    for (const Inst* in : go) {
      const double N = 2.0 * in->part.S;
      fl += 28.0 * in->n + 2 * N * N;
      by += 40.0 * in->n + 8.0 * N * N;
    }
    Timed t(ctx, KID_COARSE, st, fl, by);
    for (const Inst* in : go)
      rsp::launch_global_residual(ctx->hprob[in->slot], ctx->yd + in->noff, ctx->f + in->noff, ctx->x + 2 * in->noff,
                                  in->prob.eps_min, w.r + 2 * in->noff, st);
    rsp::launch_coarse_project(I, 0, nullptr, 0, w.r, w.cvec, st);
    rsp::launch_coarse_solve(w.prob, w.ilist[kLGo], (int)go.size(), max_n, nullptr, w.ainv, w.cvec, -1.0, w.evec,
                             st);
    rsp::launch_gm_zero(B, w.dx, st);
  }
  jac_apply(ctx, I, sub_work(ctx, go, false), w.dx, w.w, st, -1, w.evec);
  rsp::launch_gm_axpy(B, 1.0, w.w, w.b, 1, st);
  HIPCHK(hipGetLastError());
  for (Inst* in : go) {
    const double N = 2.0 * in->part.S;
    in->flops += 40.0 * in->n + 2 * N * N;
  }
  return 0;
}

// Restarted GMRES(m), x_0 = 0, on the device for every instance of `go` (list slot
// kLGo must hold go): dx = F'(x)^{-1} b with b = -F.  All instances run their cycles
// in lockstep (a finished one is skipped through its stop flag); the host enqueues
// Arnoldi steps in chunks and reads the headers back once per chunk.
int run_gmres(rsp_context* ctx, const std::vector<Inst*>& go, hipStream_t st) {
  const rsp_options& o = ctx->opts;
  const int m = o.gmres_restart;
  Work& w = ctx->w;
  const size_t ldv = 2 * (size_t)ctx->geo.ntot;
  const GmBatch Bgo = gm_of(ctx, w.ilist[kLGo], (int)go.size());
  rsp::launch_gm_axpy(Bgo, -1.0, w.F, w.b, 0, st);
  if (ctx->gm_op == 2) RSPCHK(coarse_setup(ctx, go, Bgo, st));
  rsp::launch_gm_init(Bgo, o.max_gmres, o.gmres_rtol, st);
  rsp::launch_gm_zero(Bgo, w.dx, st);
  rsp::launch_gm_sumsq(Bgo, w.b, w.p1, st);
  rsp::launch_gm_start(Bgo, w.V, w.b, w.p1, 1, st);
  for (Inst* in : go) in->restarts = 0;
  std::vector<Inst*> cyc = go;
  int lslot = kLGo;
  for (;;) {
    GmBatch B = gm_of(ctx, w.ilist[lslot], (int)cyc.size());
    Items I = items_of(ctx, w.list[lslot], (int)ctx->hlist[lslot].size());
    I.skip = &w.gst[0].done;
    I.skip_stride = rsp::kGmDoneStride;
    const SubWork sw = sub_work(ctx, cyc, false);
    double L = 0;
    for (const Inst* in : cyc) L += 2.0 * in->n;
    for (int j = 0; j < m;) {
      const int chunk = std::min(ctx->gm_chunk, m - j), j0 = j;
      RSPCHK(launch_seq(ctx, GraphKey{SEQ_ARNOLDI, lslot, I.count, B.count, j0 * 1024 + chunk}, st,
                        [&](hipStream_t s) {
                          for (int q = j0; q < j0 + chunk; ++q) {
                            gm_apply(ctx, I, sw, cyc, B, w.V + (size_t)q * ldv, w.w, s, true, q);
                            Timed tm(ctx, KID_GMRES_ORTHO, s, ortho_flops(L, q), ortho_bytes(L, q), q);
                            const int mode = q == 0 ? 0 : q == j0 ? 2 : 1;
                            rsp::launch_gm_arnoldi(B, w.V, q, w.w, w.p1, w.p2, mode, s);
                            if (q == j0 + chunk - 1) rsp::launch_gm_finish(B, w.V, q + 1, w.p1, w.p2, s);
                          }
                        }));
      j += chunk;
      RSPCHK(read_gm_headers(ctx, st));
      if (ctx->prof) settle_gmres_timing(ctx, cyc);
      bool all = true;
      for (const Inst* in : cyc) all = all && ctx->hgm[in->slot].done;
      if (all) break;
    }
    rsp::launch_gm_update_x(B, w.V, w.dx, st);
    // instances that restart from r = b - F'(x) x
    std::vector<Inst*> next;
    for (Inst* in : cyc) {
      const GmState& h = ctx->hgm[in->slot];
      if (h.rel > h.rtol && h.used < o.max_gmres && h.steps > 0) next.push_back(in);
    }
    if (next.empty()) break;
    RSPCHK(upload_lists(ctx, kLCyc, next, st));
    lslot = kLCyc;
    const GmBatch Br = gm_of(ctx, w.ilist[kLCyc], (int)next.size());
    const Items Ir = items_of(ctx, w.list[kLCyc], (int)ctx->hlist[kLCyc].size());
    gm_apply(ctx, Ir, sub_work(ctx, next, false), next, Br, w.dx, w.w, st, false);
    rsp::launch_gm_residual(Br, w.b, w.w, w.r, st);
    rsp::launch_gm_sumsq(Br, w.r, w.p1, st);
    rsp::launch_gm_start(Br, w.V, w.r, w.p1, 0, st);
    HIPCHK(hipGetLastError());
    // an instance whose restart residual already meets the tolerance is stopped by
    // k_gm_start on the device, and the chunk's kernels skip it: no read-back here
    for (Inst* in : next) in->restarts += 1;
    cyc = next;
  }
  HIPCHK(hipGetLastError());
  for (Inst* in : go) {
    const GmState& h = ctx->hgm[in->slot];
    in->gm_used = h.used;
    in->gm_rel = h.rel;
    in->n_gmres += h.used;
    in->n_apply += h.used + in->restarts;
    double sfl = 0;
    for (int q = 0; q < in->part.S; ++q) {
      const int4 b = in->part.box[q];
      const double tx = b.y - b.x, ty = b.w - b.z;
      sfl += 2.0 * (2 * ty - 1) * 4 * tx * tx;
    }
    in->n_solve += (int64_t)in->part.S * (h.used + in->restarts);
    in->flops += sfl * (h.used + in->restarts);
    if (ctx->gm_op == 2) {
      const double N = 2.0 * in->part.S;
      in->flops += (28.0 * in->n + 2 * N * N) * (h.used + in->restarts);
    }
    if (!(h.rel <= h.rtol)) in->gm_stagnated = true;
  }
  return 0;
}

// Outputs of the instances that stopped: y, p, u = D_eps_min(p), the final global
// residual norm and the history.
int finish(rsp_context* ctx, const std::vector<Inst*>& fin, hipStream_t st) {
  Work& w = ctx->w;
  for (const Inst* in : fin) {
    const DevProblem& P = ctx->hprob[in->slot];
    const size_t n = in->n;
    const double* xi = ctx->x + 2 * in->noff;
    HIPCHK(hipMemcpyAsync(in->y, xi, 8 * n, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(in->p, xi + n, 8 * n, hipMemcpyDeviceToDevice, st));
    rsp::launch_control(P, xi + n, in->prob.eps_min, in->u, st);
    rsp::launch_global_residual(P, ctx->yd + in->noff, ctx->f + in->noff, xi, in->prob.eps_min,
                                w.w + 2 * in->noff, st);
  }
  HIPCHK(hipGetLastError());
  RSPCHK(upload_lists(ctx, kLFin, fin, st));
  RSPCHK(read_norms(ctx, kLFin, (int)fin.size(), w.w, st));
  const auto now = Clock::now();
  for (Inst* in : fin) {
    rsp_history* h = &in->hist;
    // an inexact GMRES solve only matters if the outer iteration then fails to converge
    if (!(in->Fn <= in->thr) && in->status == 0)
      in->status = in->gm_stagnated ? RSP_GMRES_STAGNATION : RSP_NOT_CONVERGED;
    // converged only after leaving the FP32 factors
    if (in->status == 0 && in->fallback_outer >= 0) in->status = RSP_REFINE_FALLBACK;
    h->status = in->status;
    h->fallback_outer = in->fallback_outer;
    h->outer = in->k;
    h->subdomains = in->part.S;
    h->factorizations = in->n_factor;
    h->local_solves = in->n_solve;
    h->gmres_total = in->n_gmres;
    h->newton_iterations = in->n_newton;
    h->jac_applies = in->n_apply;
    h->residual_final = ctx->hnorm[in->slot];
    h->flops = in->flops;
    h->ms_eval = in->ms_eval;
    h->ms_gmres = in->ms_gmres;
    h->ms_total = std::chrono::duration<double, std::milli>(now - in->t0).count();
    in->finished = true;
  }
  return 0;
}

double ms_since(Clock::time_point a) {
  return std::chrono::duration<double, std::milli>(Clock::now() - a).count();
}

}  // namespace

namespace rsp {

size_t batch_bytes(const rsp_problem* const* probs, int count, const rsp_options& o) {
  if (validate_options(&o) < 0 || count < 1) return 0;
  std::vector<Partition> parts(count);
  std::vector<const Partition*> pp;
  std::vector<size_t> ns;
  std::vector<long long> nc;
  for (int q = 0; q < count; ++q) {
    if (make_partition(probs[q], &parts[q]) < 0) return 0;
    pp.push_back(&parts[q]);
    ns.push_back((size_t)probs[q]->nx * probs[q]->ny);
    nc.push_back(probs[q]->coef ? coef_doubles(probs[q]->nx, probs[q]->ny) : 0);
  }
  return layout_bytes(geometry_of(pp, ns, nc), o);
}

int engine_place(rsp_context* ctx, const rsp_options& o, const std::vector<Inst*>& live, hipStream_t st) {
  RSPCHK(validate_options(&o));
  if (live.empty()) return fail(RSP_EINVAL, "no instance to place");
  std::vector<const Partition*> pp;
  std::vector<size_t> ns;
  std::vector<long long> ncv;
  for (const Inst* in : live) {
    pp.push_back(&in->part);
    ns.push_back(in->n);
    ncv.push_back(in->prob.coef ? coef_doubles(in->prob.nx, in->prob.ny) : 0);
  }
  const Geometry g = geometry_of(pp, ns, ncv);
  if (o.coarse && 2 * g.csx_max > rsp::kCoarseMaxNc)
    return fail(RSP_EINVAL, "the second level supports at most %d subdomains per row (got %d)",
                rsp::kCoarseMaxNc / 2, g.csx_max);
  Carve cg, cw;
  double *yd, *f, *x, *coef;
  Work w;
  carve_global(cg, g, &yd, &f, &x, &coef);
  carve_work(cw, g, o, &w);
  if (ctx->budget && cg.off + cw.off > ctx->budget)
    return fail(RSP_ENOMEM, "workspace needs %zu bytes, budget is %zu", cg.off + cw.off, ctx->budget);
  HIPCHK(hipSetDevice(ctx->device));
  bool migrate = false;
  for (const Inst* in : live) migrate = migrate || in->placed;
  const int tgt = migrate ? 1 - ctx->gcur : ctx->gcur;
  if (ctx->gcap[tgt] < cg.off) {
    if (ctx->gmem[tgt]) {
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(hipFree(ctx->gmem[tgt]));
    }
    ctx->gmem[tgt] = nullptr;
    ctx->gcap[tgt] = 0;
    hipError_t e = hipMalloc(&ctx->gmem[tgt], cg.off);
    if (e != hipSuccess) return fail(RSP_ENOMEM, "hipMalloc(%zu): %s", cg.off, hipGetErrorString(e));
    ctx->gcap[tgt] = cg.off;
  }
  Carve cg2;
  cg2.base = (char*)ctx->gmem[tgt];
  carve_global(cg2, g, &yd, &f, &x, &coef);
  // place the instances: move the state of those already placed, load new ones
  long long noff = 0, coff = 0;
  int sub0 = 0;
  for (size_t q = 0; q < live.size(); ++q) {
    Inst* in = live[q];
    const size_t n = in->n;
    const long long nc = ncv[q];
    if (in->placed) {
      HIPCHK(hipMemcpyAsync(yd + noff, ctx->yd + in->noff, 8 * n, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(f + noff, ctx->f + in->noff, 8 * n, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(x + 2 * noff, ctx->x + 2 * in->noff, 16 * n, hipMemcpyDeviceToDevice, st));
      if (nc) HIPCHK(hipMemcpyAsync(coef + coff, ctx->coef + in->coff, 8 * nc, hipMemcpyDeviceToDevice, st));
    } else {
      if (nc) {
        // the caller's coefficients, scaled by 1/h^2, into the layout
        DevProblem P = rsp::dev_problem(in->prob, 0, 0, 0, 0, 0);
        const long long nxf = (long long)(in->prob.nx + 1) * in->prob.ny;
        const long long nyf = (long long)in->prob.nx * (in->prob.ny + 1);
        auto al = [](long long v) { return (v + kAlignN - 1) / kAlignN * kAlignN; };
        rsp::launch_coef_load(P, in->prob.coef, coef + coff, coef + coff + al(nxf), coef + coff + al(nxf) + al(nyf),
                              st);
      }
      HIPCHK(hipMemcpyAsync(yd + noff, in->yd, 8 * n, hipMemcpyDeviceToDevice, st));
      if (in->f) HIPCHK(hipMemcpyAsync(f + noff, in->f, 8 * n, hipMemcpyDeviceToDevice, st));
      else HIPCHK(hipMemsetAsync(f + noff, 0, 8 * n, st));
      if (in->y0) {
        HIPCHK(hipMemcpyAsync(x + 2 * noff, in->y0, 8 * n, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(x + 2 * noff + n, in->p0, 8 * n, hipMemcpyDeviceToDevice, st));
      } else {
        HIPCHK(hipMemsetAsync(x + 2 * noff, 0, 16 * n, st));
      }
    }
    in->slot = (int)q;
    in->noff = noff;
    in->coff = nc ? coff : -1;
    in->sub0 = sub0;
    noff += ((long long)n + kAlignN - 1) / kAlignN * kAlignN;
    coff += nc;
    sub0 += in->part.S;
  }
  ctx->gcur = tgt;
  ctx->yd = yd;
  ctx->f = f;
  ctx->x = x;
  ctx->coef = coef;
  ctx->var = g.ncoef > 0;
  // work arena (contents are rebuilt by every outer iteration)
  if (ctx->wcap < cw.off) {
    HIPCHK(hipStreamSynchronize(st));
    if (ctx->wmem) HIPCHK(hipFree(ctx->wmem));
    ctx->wmem = nullptr;
    ctx->wcap = 0;
    hipError_t e = hipMalloc(&ctx->wmem, cw.off);
    if (e != hipSuccess) return fail(RSP_ENOMEM, "hipMalloc(%zu): %s", cw.off, hipGetErrorString(e));
    ctx->wcap = cw.off;
  }
  Carve cw2;
  cw2.base = (char*)ctx->wmem;
  carve_work(cw2, g, o, &ctx->w);
  ctx->geo = g;
  ctx->opts = o;
  ctx->fp32 = o.precision == RSP_FP32_REFINED;
  ctx->nref = ctx->fp32 ? o.max_refine : 0;
  ctx->gm_op = o.coarse ? 2 : 0;
  // tables
  ctx->hprob.assign(g.ninst, DevProblem{});
  ctx->hseg.assign(g.ninst, GmSeg{});
  ctx->gm_nbx = 1;
  int coarse_rect = 0;   // most coarse values the ring of one subdomain touches
  std::vector<int4> hbox, hcore;
  std::vector<int> hinst;
  long long sinv_off = 0, ainv_off = 0;
  for (const Inst* in : live) {
    DevProblem& P = ctx->hprob[in->slot];
    P = rsp::dev_problem(in->prob, in->noff, g.S, g.txm, g.tym, g.M);
    if (in->coff >= 0) {
      const long long nxf = (long long)(in->prob.nx + 1) * in->prob.ny;
      const long long nyf = (long long)in->prob.nx * (in->prob.ny + 1);
      auto al = [](long long v) { return (v + kAlignN - 1) / kAlignN * kAlignN; };
      P.cx = ctx->coef + in->coff;
      P.cy = P.cx + al(nxf);
      P.c0 = P.cy + al(nyf);
    }
    P.csx = in->part.sx;
    P.csy = in->part.sy;
    P.cbx = (in->prob.nx + in->part.sx - 1) / in->part.sx;
    P.cby = (in->prob.ny + in->part.sy - 1) / in->part.sy;
    P.sub0 = in->sub0;
    P.sinv_off = sinv_off;
    P.ainv_off = ainv_off;
    const long long nc = 2LL * in->part.sx, N = nc * in->part.sy;
    sinv_off += in->part.sy * nc * nc;
    ainv_off += N * N;
    ctx->hseg[in->slot].off = 2 * in->noff;
    ctx->hseg[in->slot].L = 2 * (long long)in->n;
    ctx->gm_nbx = std::max(ctx->gm_nbx, rsp::gm_blocks(2 * (long long)in->n));
    for (int q = 0; q < in->part.S; ++q) {
      int ex0, ey0, ew;
      coarse_rect = std::max(coarse_rect, rsp::apply_coarse_rect(in->part.box[q], in->prob.nx, in->prob.ny, P.cbx,
                                                                 P.cby, &ex0, &ey0, &ew));
      hbox.push_back(in->part.box[q]);
      hcore.push_back(in->part.core[q]);
      hinst.push_back(in->slot);
    }
  }
  ctx->coarse_in_apply = ctx->gm_op == 2 && ctx->nref == 0 && rsp::apply_one_launch(g.M, ctx->fp32) &&
                         coarse_rect <= rsp::kApplyCoarseMax;
  HIPCHK(hipMemcpyAsync(ctx->w.prob, ctx->hprob.data(), sizeof(DevProblem) * g.ninst, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ctx->w.seg, ctx->hseg.data(), sizeof(GmSeg) * g.ninst, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ctx->w.box, hbox.data(), sizeof(int4) * g.S, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ctx->w.core, hcore.data(), sizeof(int4) * g.S, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ctx->w.inst, hinst.data(), sizeof(int) * g.S, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(ctx->w.fallback, 0, sizeof(int) * g.S, st));
  HIPCHK(hipStreamSynchronize(st));   // host tables are temporaries; old arena no longer read
  for (Inst* in : live) in->placed = true;
  ctx->hstate.assign(g.S, SubState{});
  ctx->hgm.assign(g.ninst, GmState{});
  ctx->hnorm.assign(g.ninst, 0.0);
  return 0;
}

int engine_step(rsp_context* ctx, const std::vector<Inst*>& live, hipStream_t st) {
  const rsp_options& o = ctx->opts;
  std::vector<Inst*> ev;
  std::vector<char> cont;
  for (Inst* in : live) {
    if (in->finished || in->parked) continue;
    ev.push_back(in);
    cont.push_back(!in->started ? o.continuation != RSP_CONT_NONE : o.continuation == RSP_CONT_EVERY);
  }
  if (ev.empty()) return 0;
  auto t = Clock::now();
  std::vector<EvalStats> es;
  RSPCHK(run_eval(ctx, ev, cont, ctx->x, ctx->w.F, &es, st));
  RSPCHK(read_norms(ctx, kLEval, (int)ev.size(), ctx->w.F, st));
  double dt = ms_since(t);
  std::vector<Inst*> go, fin, park;
  for (size_t q = 0; q < ev.size(); ++q) {
    Inst* in = ev[q];
    in->ms_eval += dt;
    in->Fn = ctx->hnorm[in->slot];
    if (!in->started) {
      in->thr = std::max(o.tol_outer, o.tol_outer * in->Fn);
      in->started = true;
    }
    const int k = in->k;
    if (es[q].status == kSubNumeric || !std::isfinite(in->Fn)) {
      // NaN or Inf in a local residual or direction, or in the assembled residual
      in->status = fail(RSP_ENUMERIC, "a local residual, Newton direction or the RASPEN residual is not "
                                      "finite (NaN or Inf in the data, or a singular local Jacobian)");
      if (k <= RSP_HIST_MAX) in->hist.norm[k] = in->Fn;
      fin.push_back(in);
      continue;
    }
    if (ctx->fp32 && o.fallback_rho >= 0) {
      const bool local_fail = es[q].status == kSubNotConverged || es[q].status == kSubLineSearch;
      const bool open = !(in->Fn <= in->thr);
      // an outer step contracts by about the relative residual of its GMRES solve, so
      // both say whether the FP32 Jacobian action still gives a contraction by rho
      const bool stalled = open && ((k >= 1 && !(in->gm_rel <= o.fallback_rho)) ||
                                    (k >= 2 && !(in->Fn <= o.fallback_rho * in->Fn_prev)));
      if (local_fail || stalled) {
        park.push_back(in);
        continue;
      }
    }
    in->Fn_prev = in->Fn;
    in->status = std::max(in->status, es[q].status);
    if (k <= RSP_HIST_MAX) {
      rsp_history* h = &in->hist;
      h->norm[k] = in->Fn;
      h->inner_min[k] = es[q].inner_min;
      h->inner_max[k] = es[q].inner_max;
      h->inner_avg[k] = es[q].inner_avg;
      h->backtracks[k] = es[q].backtracks;
      if (k > 0) {
        h->gmres_its[k] = in->gm_used;
        h->gmres_rel[k] = in->gm_rel;
      }
    }
    if (!(in->Fn <= in->thr) && in->k - in->k_base < o.max_outer) go.push_back(in);
    else fin.push_back(in);
  }
  for (Inst* in : park) {
    // the FP32 factors were not good enough: save x^k in the outputs, to be laid out
    // again from there with FP64 factors (an evaluation at x^k is redone there)
    const double* xi = ctx->x + 2 * in->noff;
    HIPCHK(hipMemcpyAsync(in->y, xi, 8 * in->n, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(in->p, xi + in->n, 8 * in->n, hipMemcpyDeviceToDevice, st));
    in->y0 = in->y;
    in->p0 = in->p;
    in->placed = false;
    in->parked = true;
    in->fallback_outer = in->k;
    in->k_base = in->k;
    in->status = 0;
    in->gm_stagnated = false;
    if (in->k == 0) {   // x^0 itself: the first evaluation (and its snapshots) is redone
      in->started = false;
      in->hist.snapshots = 0;
    }
  }
  if (!fin.empty()) RSPCHK(finish(ctx, fin, st));
  if (!go.empty()) {
    // Newton systems F'(x^k) d = -F(x^k) by GMRES, then x^{k+1} = x^k + d (undamped)
    t = Clock::now();
    RSPCHK(upload_lists(ctx, kLGo, go, st));
    RSPCHK(run_gmres(ctx, go, st));
    const GmBatch B = gm_of(ctx, ctx->w.ilist[kLGo], (int)go.size());
    rsp::launch_gm_axpy(B, 1.0, ctx->w.dx, ctx->x, 1, st);
    HIPCHK(hipGetLastError());
    dt = ms_since(t);
    for (Inst* in : go) {
      in->ms_gmres += dt;
      in->k += 1;
    }
  }
  return 0;
}

// The monolithic methods of Section 4.1 for one placed instance: Algorithm 1 on the
// whole system F_eps(x) = 0, each Newton system F'_eps(x^k) d = -F_eps(x^k) solved by
// GMRES.  precond false (Newton_eps): GMRES on F'_eps(x^k) itself.  precond true
// (Newton_RAS,eps): GMRES preconditioned from the left with one-level RAS,
// M^{-1} = sum_i P~_i J_i^{-1} R_i,
// J_i = R_i F'_eps(x^k) P_i.  The local Jacobians are factored at R_i x^k with the
// current smoothing.  Because the spatial coupling of F' is the Laplacian only,
//   M^{-1} F'(x) d = d + sum_i P~_i J_i^{-1} B_i d,  B_i d = R_i diag(A, A)(I - P_i R_i) d,
// which is minus the Jacobian action of Algorithm 4 with these factors.  So GMRES runs
// on that action with right-hand side M^{-1} F, and its solution is the Newton direction.
// Backtracking on ||F_eps_k||, eps_{k+1} = max(gamma eps_k, eps_min); the loop also
// runs while eps_k > eps_min, at most max_outer + 1 steps.
int monolithic_newton(rsp_context* ctx, Inst* in, bool precond, hipStream_t st) {
  const rsp_options& o = ctx->opts;
  Work& w = ctx->w;
  const int M = ctx->geo.M;
  const std::vector<Inst*> one{in};
  RSPCHK(upload_lists(ctx, kLGo, one, st));
  const Items I = items_of(ctx, w.list[kLGo], (int)ctx->hlist[kLGo].size());
  const GmBatch B = gm_of(ctx, w.ilist[kLGo], 1);
  const SubWork all = sub_work(ctx, one, false);
  const double L = 2.0 * in->n;
  DevProblem& P = ctx->hprob[in->slot];
  const size_t off = 2 * in->noff;
  // ||F_eps(x)|| of the instance, F_eps(x) into out (x, out: batch vectors)
  auto residual = [&](const double* x, double eps, double* out, double* norm) -> int {
    {
      Timed t(ctx, KID_GLOBAL, st, 20.0 * L, 24.0 * L);   // x, y_d, f read, F written
      rsp::launch_global_residual(P, ctx->yd + in->noff, ctx->f + in->noff, x + off, eps, out + off, st);
    }
    HIPCHK(hipGetLastError());
    RSPCHK(read_norms(ctx, kLGo, 1, out, st));
    *norm = ctx->hnorm[in->slot];
    return 0;
  };
  double eps = o.continuation == RSP_CONT_NONE ? in->prob.eps_min : in->prob.eps0;
  double Fn = 0;
  RSPCHK(residual(ctx->x, eps, w.F, &Fn));
  in->started = true;
  in->thr = std::max(o.tol_outer, o.tol_outer * Fn);
  in->hist.norm[0] = Fn;
  if (!std::isfinite(Fn)) {   // NaN or Inf in the data or the start
    in->status = fail(RSP_ENUMERIC, "the residual of the start is not finite (NaN or Inf in the data)");
    in->Fn = Fn;
    return finish(ctx, one, st);
  }
  int k = 0;
  while ((!(Fn <= in->thr) || eps > in->prob.eps_min) && k <= o.max_outer) {
    auto t = Clock::now();
    // the smoothing of this step, read by the factor and the whole-system Jacobian
    P.eps_start = eps;
    RSPCHK(upload(ctx, w.prob + in->slot, &P, sizeof(DevProblem), st));
    if (precond) {
      // local Jacobians at x^k with smoothing eps_k
      {
        Timed tm(ctx, KID_RESTRICT, st, 0, all.halo_by * 2);
        rsp::launch_restrict_halo(I, ctx->x, w.tilex, st);
      }
      {
        Timed tm(ctx, KID_FACTOR, st, all.factor_fl, all.factor_by);
        rsp::launch_factor(I, M, w.tilex, nullptr, nullptr, -1.0, nullptr, 0.0, w.fac, ctx->fp32, w.g,
                           w.fallback, ctx->var, st);
      }
      // w.F <- -M^{-1} F_eps(x^k): GMRES then solves (action) d = M^{-1} F
      {
        Timed tm(ctx, KID_PRECOND, st, all.solve_fl, all.solve_by + 2 * all.tile_by + 16.0 * L);
        rsp::launch_restrict(I, w.F, w.t1, st);
        rsp::launch_block_solve(I, M, w.fac, ctx->fp32, w.t1, w.t2, st);
        rsp::launch_prolong(I, w.t2, nullptr, w.w, st);
        rsp::launch_gm_axpy(B, -1.0, w.w, w.F, 0, st);
      }
      HIPCHK(hipGetLastError());
      in->n_factor += in->part.S;
      in->flops += all.factor_fl + all.solve_fl;
    }
    // (no preconditioner: w.F holds F_eps(x^k) and GMRES solves F'(x^k) d = -F directly)
    in->ms_eval += ms_since(t);
    t = Clock::now();
    const int gm_op = ctx->gm_op;
    ctx->gm_op = precond ? 0 : 1;
    const int gr = run_gmres(ctx, one, st);
    ctx->gm_op = gm_op;
    RSPCHK(gr);
    in->ms_gmres += ms_since(t);
    // relaxed backtracking: alpha = 1, 1/2, ... until ||F_eps(x + alpha d)|| <= sigma ||F_eps(x)||
    double alpha = 1.0, rt = 0;
    int bt = 0;
    bool fail_ls = false;
    for (;;) {
      rsp::launch_gm_axpy(B, 1.0, ctx->x, w.b, 0, st);
      rsp::launch_gm_axpy(B, alpha, w.dx, w.b, 1, st);
      RSPCHK(residual(w.b, eps, w.w, &rt));
      if (rt <= o.sigma * Fn) break;
      alpha *= 0.5;
      bt += 1;
      if (alpha < o.alpha_min) {
        fail_ls = true;
        break;
      }
    }
    if (fail_ls) {
      in->status = std::max(in->status, (int)RSP_LINESEARCH_FAIL);
      if (k + 1 <= RSP_HIST_MAX) in->hist.backtracks[k + 1] = bt;
      break;
    }
    rsp::launch_gm_axpy(B, alpha, w.dx, ctx->x, 1, st);
    eps = std::max(in->prob.gamma * eps, in->prob.eps_min);
    k += 1;
    RSPCHK(residual(ctx->x, eps, w.F, &Fn));
    if (k <= RSP_HIST_MAX) {
      rsp_history* h = &in->hist;
      h->norm[k] = Fn;
      h->gmres_its[k] = in->gm_used;
      h->gmres_rel[k] = in->gm_rel;
      h->backtracks[k] = bt;
    }
  }
  in->k = k;
  in->Fn = Fn;
  if (in->status == 0 && (!(Fn <= in->thr) || eps > in->prob.eps_min))
    in->status = in->gm_stagnated ? RSP_GMRES_STAGNATION : RSP_NOT_CONVERGED;
  return finish(ctx, one, st);
}

}  // namespace rsp

namespace {

using rsp::engine_place;
using rsp::engine_step;

// Validates the arrays of a solve and builds its instances.
int make_instances(int count, const rsp_problem* probs, const double* const* yd, const double* const* f,
                   const double* const* y0, const double* const* p0, double* const* y, double* const* p,
                   double* const* u, std::vector<Inst>* out) {
  out->assign(count, Inst{});
  for (int q = 0; q < count; ++q) {
    if (!yd || !yd[q]) return fail(RSP_EINVAL, "instance %d: yd is NULL", q);
    if (!y || !p || !u || !y[q] || !p[q] || !u[q]) return fail(RSP_EINVAL, "instance %d: outputs y, p, u are required", q);
    const double* a = y0 ? y0[q] : nullptr;
    const double* b = p0 ? p0[q] : nullptr;
    if ((a == nullptr) != (b == nullptr)) return fail(RSP_EINVAL, "instance %d: give both y0 and p0 or neither", q);
    Inst& in = (*out)[q];
    int r = rsp::inst_init(&in, &probs[q]);
    if (r < 0) return r;
    in.yd = yd[q];
    in.f = f ? f[q] : nullptr;
    in.y0 = a;
    in.p0 = b;
    in.y = y[q];
    in.p = p[q];
    in.u = u[q];
  }
  return 0;
}

int solve_instances(rsp_context* ctx, const rsp_options* opts, std::vector<Inst>& insts, rsp_history* hist,
                    hipStream_t stream) {
  std::vector<Inst*> live;
  for (auto& in : insts) live.push_back(&in);
  RSPCHK(engine_place(ctx, *opts, live, stream));
  for (auto& in : insts) in.t0 = rsp::Clock::now();
  auto run = [&](const std::vector<Inst*>& set) -> int {
    bool more = true;
    while (more) {
      RSPCHK(engine_step(ctx, set, stream));
      more = false;
      for (const Inst* in : set) more = more || (!in->finished && !in->parked);
    }
    return 0;
  };
  RSPCHK(run(live));
  // instances that left the FP32 factors continue together with FP64 factors
  std::vector<Inst*> parked;
  for (Inst* in : live)
    if (in->parked) parked.push_back(in);
  if (!parked.empty()) {
    const rsp_options o64 = rsp::fallback_options(*opts);
    RSPCHK(engine_place(ctx, o64, parked, stream));
    for (Inst* in : parked) in->parked = false;
    RSPCHK(run(parked));
  }
  int worst = 0, hard = 0;
  for (size_t q = 0; q < insts.size(); ++q) {
    if (hist) hist[q] = insts[q].hist;
    worst = std::max(worst, insts[q].status);
    if (insts[q].status < 0 && hard == 0) hard = insts[q].status;
  }
  RSPCHK(resolve_events(ctx));
  return hard ? hard : worst;
}

}  // namespace

extern "C" {

int rsp_version(void) { return RSP_VERSION; }

const char* rsp_last_error(void) { return rsp::last_error(); }

int rsp_partition(const rsp_problem* prob, int32_t* S, int32_t* txm, int32_t* tym, int32_t* boxes) {
  Partition part;
  RSPCHK(rsp::make_partition(prob, &part));
  if (S) *S = part.S;
  if (txm) *txm = part.txm;
  if (tym) *tym = part.tym;
  if (boxes)
    for (int s = 0; s < part.S; ++s) {
      const int4 b = part.box[s], c = part.core[s];
      int32_t* o = boxes + 8 * s;
      o[0] = b.x; o[1] = b.y; o[2] = b.z; o[3] = b.w;
      o[4] = c.x; o[5] = c.y; o[6] = c.z; o[7] = c.w;
    }
  return 0;
}

size_t rsp_workspace_bytes(const rsp_problem* prob, const rsp_options* opts) {
  if (!prob || !opts) return 0;
  return rsp::batch_bytes(&prob, 1, *opts);
}

size_t rsp_batch_workspace_bytes(int count, const rsp_problem* probs, const rsp_options* opts) {
  if (count < 1 || !probs || !opts) return 0;
  std::vector<const rsp_problem*> pp;
  for (int q = 0; q < count; ++q) pp.push_back(&probs[q]);
  return rsp::batch_bytes(pp.data(), count, *opts);
}

int rsp_context_create(rsp_context** ctx, int device, size_t hbm_budget) {
  if (!ctx) return fail(RSP_EINVAL, "ctx is NULL");
  int n = 0;
  HIPCHK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(RSP_EINVAL, "device %d not present (%d devices)", device, n);
  rsp_context* c = new (std::nothrow) rsp_context();
  if (!c) return fail(RSP_ENOMEM, "out of host memory");
  c->device = device;
  c->budget = hbm_budget;
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c->n_cu < 1) {
    delete c;
    return fail(RSP_EHIP, "cannot read the compute-unit count of device %d", device);
  }
  *ctx = c;
  return 0;
}

int rsp_context_destroy(rsp_context* ctx) {
  if (!ctx) return 0;
  (void)hipSetDevice(ctx->device);
  (void)resolve_events(ctx);
  for (const Pending& p : ctx->pending) {
    ctx->ev_pool.push_back(p.a);
    ctx->ev_pool.push_back(p.b);
  }
  if (!ctx->gcache.empty()) (void)hipDeviceSynchronize();
  for (auto& kv : ctx->gcache) (void)hipGraphExecDestroy(kv.second);
  if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (void* m : ctx->gmem)
    if (m) (void)hipFree(m);
  if (ctx->wmem) (void)hipFree(ctx->wmem);
  if (ctx->pin) (void)hipHostFree(ctx->pin);
  if (ctx->wait_ev) (void)hipEventDestroy(ctx->wait_ev);
  delete ctx;
  return 0;
}

int rsp_setup(rsp_context* ctx, const rsp_problem* prob, const rsp_options* opts, const double* yd,
              const double* f, hipStream_t stream) {
  if (!ctx) return fail(RSP_EINVAL, "ctx is NULL");
  if (!yd) return fail(RSP_EINVAL, "yd is NULL");
  ctx->ready = false;
  RSPCHK(rsp::validate_options(opts));
  RSPCHK(rsp::inst_init(&ctx->single, prob));
  ctx->single.yd = yd;
  ctx->single.f = f;
  std::vector<Inst*> live{&ctx->single};
  RSPCHK(engine_place(ctx, *opts, live, stream));
  ctx->ready = true;
  return 0;
}

#define NEED_READY(ctx) \
  if (!(ctx) || !(ctx)->ready) return fail(RSP_EINVAL, "context has no problem (call rsp_setup)")

int rsp_residual(rsp_context* ctx, const double* x, double eps, double* out, hipStream_t stream) {
  NEED_READY(ctx);
  if (!(eps >= 0)) return fail(RSP_EINVAL, "eps must be >= 0");
  rsp::launch_global_residual(ctx->hprob[0], ctx->yd, ctx->f, x, eps, out, stream);
  HIPCHK(hipGetLastError());
  return 0;
}

int rsp_control(rsp_context* ctx, const double* p, double eps, double* u, hipStream_t stream) {
  NEED_READY(ctx);
  if (!(eps >= 0)) return fail(RSP_EINVAL, "eps must be >= 0");
  rsp::launch_control(ctx->hprob[0], p, eps, u, stream);
  HIPCHK(hipGetLastError());
  return 0;
}

int rsp_restrict(rsp_context* ctx, const double* x, double* tiles, hipStream_t stream) {
  NEED_READY(ctx);
  rsp::launch_restrict(all_items(ctx), x, tiles, stream);
  HIPCHK(hipGetLastError());
  return 0;
}

int rsp_prolong(rsp_context* ctx, const double* tiles, double* out, hipStream_t stream) {
  NEED_READY(ctx);
  rsp::launch_prolong(all_items(ctx), tiles, nullptr, out, stream);
  HIPCHK(hipGetLastError());
  return 0;
}

int rsp_local_residual(rsp_context* ctx, const double* x, const double* c, double eps, double* out,
                       double* norms, hipStream_t stream) {
  NEED_READY(ctx);
  if (!(eps >= 0)) return fail(RSP_EINVAL, "eps must be >= 0");
  const Items I = all_items(ctx);
  rsp::launch_restrict_halo(I, x, ctx->w.tilex, stream);
  rsp::launch_local_residual(I, ctx->w.tilex, ctx->yd, ctx->f, c, eps, out, norms, stream);
  HIPCHK(hipGetLastError());
  return 0;
}

int rsp_local_solve(rsp_context* ctx, const double* x, const double* c, double eps, const double* rhs,
                    double* z, hipStream_t stream) {
  NEED_READY(ctx);
  if (!(eps > 0)) return fail(RSP_EINVAL, "eps must be > 0");
  const Items I = all_items(ctx);
  rsp::launch_restrict_halo(I, x, ctx->w.tilex, stream);
  rsp::launch_factor(I, ctx->geo.M, ctx->w.tilex, c, nullptr, eps, nullptr, 0.0, ctx->w.fac, ctx->fp32,
                     ctx->w.g, ctx->w.fallback, ctx->var, stream);
  rsp::launch_block_solve(I, ctx->geo.M, ctx->w.fac, ctx->fp32, rhs, z, stream);
  HIPCHK(hipGetLastError());
  return 0;
}

int rsp_eval(rsp_context* ctx, const double* x, int continuation, double* out, double* norm,
             hipStream_t stream) {
  NEED_READY(ctx);
  std::vector<Inst*> set{&ctx->single};
  std::vector<char> cont{(char)(continuation != 0)};
  std::vector<EvalStats> es;
  RSPCHK(run_eval(ctx, set, cont, x, out, &es, stream));
  if (norm) {
    RSPCHK(read_norms(ctx, kLEval, 1, out, stream));
    *norm = ctx->hnorm[0];
  }
  if (es[0].status == rsp::kSubNumeric)
    return fail(RSP_ENUMERIC, "a local residual or Newton direction is not finite");
  return es[0].status;
}

int rsp_coarse_jac_apply(rsp_context* ctx, const double* x, const double* d, double* out, hipStream_t stream) {
  NEED_READY(ctx);
  if (!ctx->opts.coarse) return fail(RSP_EINVAL, "the context was set up without the second level");
  if (!x || !d || !out) return fail(RSP_EINVAL, "x, d and out are required");
  std::vector<Inst*> set{&ctx->single};
  RSPCHK(upload_lists(ctx, kLGo, set, stream));
  const Items I = all_items(ctx);
  Work& w = ctx->w;
  coarse_factorize(ctx, I, w.ilist[kLGo], set, x, stream);
  rsp::launch_coarse_project(I, 1, w.cpt, ctx->geo.ntot, d, w.cvec, stream);
  rsp::launch_coarse_solve(w.prob, w.ilist[kLGo], 1, coarse_max_n(set), nullptr, w.ainv, w.cvec, 1.0, w.evec, stream);
  jac_apply(ctx, I, sub_work(ctx, set, false), d, out, stream, -1, w.evec);
  HIPCHK(hipGetLastError());
  return 0;
}

int rsp_jac_apply(rsp_context* ctx, const double* d, double* out, hipStream_t stream) {
  NEED_READY(ctx);
  std::vector<Inst*> set{&ctx->single};
  jac_apply(ctx, all_items(ctx), sub_work(ctx, set, false), d, out, stream);
  HIPCHK(hipGetLastError());
  return 0;
}

int rsp_solve(rsp_context* ctx, const rsp_problem* prob, const rsp_options* opts, const double* yd,
              const double* f, const double* y0, const double* p0, double* y, double* p, double* u,
              rsp_history* hist, hipStream_t stream) {
  if (!ctx) return fail(RSP_EINVAL, "ctx is NULL");
  RSPCHK(rsp::validate_options(opts));
  if (!prob) return fail(RSP_EINVAL, "problem is NULL");
  ctx->ready = false;
  std::vector<Inst> insts;
  RSPCHK(make_instances(1, prob, &yd, &f, &y0, &p0, &y, &p, &u, &insts));
  insts[0].snap = opts->record_eps_snapshots > 0 ? opts->eps_snapshots : nullptr;
  insts[0].snap_max = opts->record_eps_snapshots;
  const int r = solve_instances(ctx, opts, insts, hist, stream);
  if (r >= 0) {
    // keep the problem bound for the single-problem calls, as after rsp_setup
    ctx->single = insts[0];
    ctx->ready = true;
  }
  return r;
}

int rsp_solve_newton_ras(rsp_context* ctx, const rsp_problem* prob, const rsp_options* opts, const double* yd,
                         const double* f, const double* y0, const double* p0, double* y, double* p, double* u,
                         rsp_history* hist, hipStream_t stream) {
  if (!ctx) return fail(RSP_EINVAL, "ctx is NULL");
  RSPCHK(rsp::validate_options(opts));
  if (!prob) return fail(RSP_EINVAL, "problem is NULL");
  if (opts->record_eps_snapshots) return fail(RSP_EINVAL, "eps snapshots are recorded by rsp_solve only");
  if (opts->coarse) return fail(RSP_EINVAL, "the second level applies to RASPEN (rsp_solve, batch, server)");
  ctx->ready = false;
  std::vector<Inst> insts;
  RSPCHK(make_instances(1, prob, &yd, &f, &y0, &p0, &y, &p, &u, &insts));
  std::vector<Inst*> live{&insts[0]};
  RSPCHK(engine_place(ctx, *opts, live, stream));
  insts[0].t0 = rsp::Clock::now();
  RSPCHK(rsp::monolithic_newton(ctx, &insts[0], true, stream));
  if (hist) *hist = insts[0].hist;
  RSPCHK(resolve_events(ctx));
  return insts[0].status;
}

int rsp_solve_newton(rsp_context* ctx, const rsp_problem* prob, const rsp_options* opts, const double* yd,
                     const double* f, const double* y0, const double* p0, double* y, double* p, double* u,
                     rsp_history* hist, hipStream_t stream) {
  if (!ctx) return fail(RSP_EINVAL, "ctx is NULL");
  RSPCHK(rsp::validate_options(opts));
  if (!prob) return fail(RSP_EINVAL, "problem is NULL");
  if (opts->record_eps_snapshots) return fail(RSP_EINVAL, "eps snapshots are recorded by rsp_solve only");
  if (opts->coarse) return fail(RSP_EINVAL, "the second level applies to RASPEN (rsp_solve, batch, server)");
  ctx->ready = false;
  std::vector<Inst> insts;
  RSPCHK(make_instances(1, prob, &yd, &f, &y0, &p0, &y, &p, &u, &insts));
  std::vector<Inst*> live{&insts[0]};
  RSPCHK(engine_place(ctx, *opts, live, stream));
  insts[0].t0 = rsp::Clock::now();
  RSPCHK(rsp::monolithic_newton(ctx, &insts[0], false, stream));
  if (hist) *hist = insts[0].hist;
  RSPCHK(resolve_events(ctx));
  return insts[0].status;
}

int rsp_solve_batch(rsp_context* ctx, int count, const rsp_problem* probs, const rsp_options* opts,
                    const double* const* yd, const double* const* f, const double* const* y0,
                    const double* const* p0, double* const* y, double* const* p, double* const* u,
                    rsp_history* hist, hipStream_t stream) {
  if (!ctx) return fail(RSP_EINVAL, "ctx is NULL");
  if (count < 1 || !probs) return fail(RSP_EINVAL, "need count >= 1 problems");
  RSPCHK(rsp::validate_options(opts));
  if (opts->record_eps_snapshots) return fail(RSP_EINVAL, "eps snapshots are recorded by rsp_solve only");
  ctx->ready = false;
  std::vector<Inst> insts;
  RSPCHK(make_instances(count, probs, yd, f, y0, p0, y, p, u, &insts));
  return solve_instances(ctx, opts, insts, hist, stream);
}

int rsp_set_profiling(rsp_context* ctx, int on) {
  if (!ctx) return fail(RSP_EINVAL, "ctx is NULL");
  ctx->prof = on != 0;
  return 0;
}

int rsp_set_profiling_sample(rsp_context* ctx, int every) {
  if (!ctx) return fail(RSP_EINVAL, "ctx is NULL");
  if (every < 1) return fail(RSP_EINVAL, "every must be >= 1 (got %d)", every);
  ctx->prof_every = every;
  ctx->prof_seq = 0;
  return 0;
}

int rsp_get_tuning(rsp_context* ctx, rsp_tuning* out) {
  if (!ctx || !out) return fail(RSP_EINVAL, "ctx and out are required");
  *out = rsp_tuning{};
  out->graphs = ctx->graphs;
  out->gm_chunk = ctx->gm_chunk;
  out->jac_form = ctx->jac_form;
  return 0;
}

int rsp_set_tuning(rsp_context* ctx, const rsp_tuning* t) {
  if (!ctx || !t) return fail(RSP_EINVAL, "ctx and tuning are required");
  if (t->graphs != 0 && t->graphs != 1) return fail(RSP_EINVAL, "graphs must be 0 or 1");
  if (t->gm_chunk < 1 || t->gm_chunk > kMaxRestart)
    return fail(RSP_EINVAL, "gm_chunk must be in [1, %d]", kMaxRestart);
  if (t->jac_form < 0 || t->jac_form > 2) return fail(RSP_EINVAL, "jac_form must be 0, 1 or 2");
  ctx->graphs = t->graphs;
  ctx->gm_chunk = t->gm_chunk;
  ctx->jac_form = t->jac_form;
  return 0;
}

int rsp_set_profiling_filter(rsp_context* ctx, const char* name) {
  if (!ctx) return fail(RSP_EINVAL, "ctx is NULL");
  if (!name || !*name) {
    ctx->prof_only = -1;
    return 0;
  }
  for (int k = 0; k < KID_N; ++k)
    if (std::strcmp(name, kKidName[k]) == 0) {
      ctx->prof_only = k;
      return 0;
    }
  return fail(RSP_EINVAL, "unknown kernel class '%s'", name);
}

int rsp_reset_kernel_stats(rsp_context* ctx) {
  if (!ctx) return fail(RSP_EINVAL, "ctx is NULL");
  RSPCHK(resolve_events(ctx));
  for (const Pending& p : ctx->pending) {   // unsettled timings of an interrupted GMRES chunk
    ctx->ev_pool.push_back(p.a);
    ctx->ev_pool.push_back(p.b);
  }
  ctx->pending.clear();
  for (auto& k : ctx->kstat) k = rsp_kernel_stat{};
  return 0;
}

int rsp_kernel_stats(rsp_context* ctx, rsp_kernel_stat* out, int max, int32_t* count) {
  if (!ctx) return fail(RSP_EINVAL, "ctx is NULL");
  RSPCHK(resolve_events(ctx));
  int n = 0;
  for (int k = 0; k < KID_N && n < max; ++k) {
    if (!out) break;
    out[n] = ctx->kstat[k];
    std::snprintf(out[n].name, sizeof out[n].name, "%s", kKidName[k]);
    ++n;
  }
  if (count) *count = out ? n : KID_N;
  return 0;
}

}  // extern "C"
