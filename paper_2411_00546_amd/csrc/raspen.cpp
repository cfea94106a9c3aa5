// Host side of the RASPEN library: C ABI, context and workspace, the partition of
// Section 4.2, and the drivers of Algorithms 1-4 (local Newton loop, evaluation
// of the RASPEN residual, Jacobian action, outer Newton-GMRES).  All arithmetic
// of the method runs in the HIP kernels; the host only sequences launches,
// reads back per-subdomain / per-iteration scalars and does the Givens updates
// of GMRES on the (restart+1) x restart Hessenberg matrix.
#include "raspen.h"

#include <algorithm>
#include <cstddef>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rsp_kernels.h"

using rsp::DevProblem;
using rsp::SubState;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

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

constexpr int kMaxRestart = 64;

struct Partition {
  int S = 0, txm = 0, tym = 0;
  std::vector<int4> box, core;   // (x0, x1, y0, y1) half-open
};

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
  return 0;
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
  if (out->txm > rsp::kMaxTile)
    return fail(RSP_EINVAL, "tile width %d exceeds the supported %d nodes", out->txm, rsp::kMaxTile);
  if (out->tym > rsp::kMaxTile)
    return fail(RSP_EINVAL, "tile height %d exceeds the supported %d nodes", out->tym, rsp::kMaxTile);
  return 0;
}

int line_block(int txm) { return ((2 * txm + 15) / 16) * 16; }

DevProblem make_dev(const rsp_problem* p, const Partition& part) {
  DevProblem P;
  P.nx = p->nx;
  P.ny = p->ny;
  P.phi = p->phi_kind;
  P.kappa = p->kappa;
  P.nu = p->nu;
  P.inv_nu = 1.0 / p->nu;
  P.mu = p->mu;
  const double hx = 1.0 / (p->nx + 1), hy = 1.0 / (p->ny + 1);
  P.hx2i = 1.0 / (hx * hx);
  P.hy2i = 1.0 / (hy * hy);
  P.diag0 = 2.0 * P.hx2i + 2.0 * P.hy2i;
  P.eps_min = p->eps_min;
  P.gamma = p->gamma;
  P.S = part.S;
  P.txm = part.txm;
  P.tym = part.tym;
  P.M = line_block(part.txm);
  return P;
}

// Sizes (in doubles unless noted) of every workspace buffer.
struct Layout {
  size_t n, L, tile, halo, fac, g, V, partial, gpart;
  size_t fac_elem;   // bytes per stored factor entry (8 FP64, 4 FP32)
  size_t bytes() const {
    return 8 * (2 * n /*yd,f*/ + 2 * L /*x,F*/ + halo + 5 * tile /*c,dir,res,t1,t2*/ + g +
                V + 4 * L /*w, b, dx, r*/ + partial + 4 * 80 /*h bufs*/ + 2 * gpart) +
           fac_elem * fac + sizeof(rsp::GmState);
  }
};

Layout make_layout(const DevProblem& P, const rsp_options* o) {
  Layout l;
  l.n = (size_t)P.nx * P.ny;
  l.L = 2 * l.n;
  l.tile = (size_t)P.S * 2 * P.txm * P.tym;
  l.halo = (size_t)P.S * 2 * (P.txm + 2) * (P.tym + 2);
  l.fac = (size_t)P.S * P.tym * P.M * P.M;
  l.g = (size_t)P.S * P.tym * P.M;
  l.V = (size_t)(o->gmres_restart + 1) * l.L;
  l.partial = (size_t)rsp::multidot_blocks(l.L) * 72;
  l.gpart = (size_t)rsp::kGmBlocks * rsp::kGmMaxVec;
  l.fac_elem = o->precision == RSP_FP32_REFINED ? 4 : 8;
  return l;
}

constexpr size_t kBuffers = 28;   // buffers carved from the workspace, each 256-byte aligned

size_t layout_bytes(const Layout& l, int S) {
  return l.bytes() + S * (sizeof(int4) * 2 + sizeof(SubState)) + kBuffers * 256;
}

// Kernel timing: HIP events around launches, resolved at synchronisation points.
enum Kid {
  KID_RESTRICT, KID_INIT, KID_FACTOR, KID_SOLVE_BWD, KID_LINESEARCH, KID_PROLONG, KID_RING,
  KID_BLOCK_SOLVE, KID_GMRES_ORTHO, KID_GLOBAL, KID_REFINE, KID_N
};
const char* const kKidName[KID_N] = {"restrict_halo", "newton_init", "factor", "solve_bwd",
                                     "linesearch", "prolong", "ring_rhs", "block_solve",
                                     "gmres_ortho", "global_residual", "newton_refine"};

struct Pending {
  int kid;
  hipEvent_t a, b;
  double flops, bytes;
};

}  // namespace

struct rsp_context {
  int device = 0;
  size_t budget = 0;
  bool ready = false;
  rsp_problem prob{};
  rsp_options opts{};
  Partition part;
  DevProblem P{};
  Layout lay{};
  void* mem = nullptr;
  size_t mem_bytes = 0;
  int4* box = nullptr;
  int4* core = nullptr;
  SubState* state = nullptr;
  double *yd = nullptr, *f = nullptr, *x = nullptr, *F = nullptr, *tilex = nullptr;
  double *c = nullptr, *dir = nullptr, *res = nullptr, *t1 = nullptr, *t2 = nullptr;
  void* fac = nullptr;
  double *g = nullptr, *V = nullptr, *w = nullptr, *b = nullptr, *dx = nullptr;
  double *partial = nullptr, *hbuf = nullptr, *r = nullptr, *gp1 = nullptr, *gp2 = nullptr;
  rsp::GmState* gst = nullptr;
  int fp32 = 0;       // FP32 line factors (mixed precision)
  int nref = 0;       // FP64 refinement steps per local solve with FP32 factors
  std::vector<SubState> hstate;
  // kernel timing
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<Pending> pending;
  rsp_kernel_stat kstat[KID_N]{};
  // counters of the current solve
  int64_t n_factor = 0, n_solve = 0, n_gmres = 0, n_newton = 0, n_apply = 0;
  double flops = 0;
  int64_t eval_inner_sum = 0;
};

namespace {

struct EvalStats {
  int status = 0, inner_min = 0, inner_max = 0, backtracks = 0;
  double inner_avg = 0;
};

int resolve_events(rsp_context* ctx) {
  for (auto& p : ctx->pending) {
    HIPCHK(hipEventSynchronize(p.b));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
    rsp_kernel_stat& k = ctx->kstat[p.kid];
    k.launches += 1;
    k.ms += ms;
    k.flops += p.flops;
    k.bytes += p.bytes;
    ctx->ev_pool.push_back(p.a);
    ctx->ev_pool.push_back(p.b);
  }
  ctx->pending.clear();
  return 0;
}

hipEvent_t event_get(rsp_context* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets the launches issued during its lifetime with events (when timing is on),
// attributing the given algorithmic flops and bytes to kernel `kid`.
struct Timed {
  rsp_context* c;
  int kid;
  hipStream_t st;
  double fl, by;
  hipEvent_t a = nullptr;
  Timed(rsp_context* c_, int kid_, hipStream_t st_, double fl_, double by_)
      : c(c_), kid(kid_), st(st_), fl(fl_), by(by_) {
    if (c->prof && (a = event_get(c)) != nullptr && hipEventRecord(a, st) != hipSuccess) a = nullptr;
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = event_get(c);
    if (!b || hipEventRecord(b, st) != hipSuccess) return;
    c->pending.push_back({kid, a, b, fl, by});
    if (c->pending.size() > 16384) (void)resolve_events(c);
  }
};

// Algorithmic work of the per-subdomain kernels (m = 2 tx line unknowns, ty lines).
struct SubWork {
  double factor_fl = 0, factor_by = 0, bwd_fl = 0, bwd_by = 0, solve_fl = 0, solve_by = 0;
  double tile_by = 0, halo_by = 0;
};

SubWork sub_work(const std::vector<int4>& boxes, const std::vector<SubState>* state, double fe = 8.0) {
  SubWork w;
  for (size_t s = 0; s < boxes.size(); ++s) {
    if (state && !(*state)[s].active) continue;
    const double tx = boxes[s].y - boxes[s].x, ty = boxes[s].w - boxes[s].z, m = 2 * tx;
    w.factor_fl += 16.0 * ty * tx * tx * tx;           // ty Gauss-Jordan inversions of m x m
    w.factor_by += fe * ty * m * m;                    // the inverses written once
    w.bwd_fl += 2.0 * (ty - 1) * m * m;
    w.bwd_by += fe * (ty - 1) * m * m;
    w.solve_fl += 2.0 * (2 * ty - 1) * m * m;          // forward + backward sweeps
    w.solve_by += fe * (2 * ty - 1) * m * m + 8.0 * 2 * m * ty;
    w.tile_by += 8.0 * m * ty;
    w.halo_by += 8.0 * 2 * (tx + 2) * (ty + 2);
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

// Algorithm 3 on the device: local Newton solves (Algorithm 1) for every subdomain,
// factorisation at x^(i), and the assembly F(x) = sum_i P~_i C_i(x) into `out`.
int run_eval(rsp_context* ctx, const double* x, bool continuation, double* out, EvalStats* es,
             hipStream_t st) {
  const DevProblem& P = ctx->P;
  const rsp_problem& pr = ctx->prob;
  const rsp_options& o = ctx->opts;
  const double eps0 = continuation ? pr.eps0 : pr.eps_min;
  const double fe = (double)ctx->lay.fac_elem;
  const SubWork all = sub_work(ctx->part.box, nullptr, fe);
  {
    Timed t(ctx, KID_RESTRICT, st, 0, all.halo_by * 2);
    rsp::launch_restrict_halo(P, ctx->box, x, ctx->tilex, st);
  }
  {
    Timed t(ctx, KID_INIT, st, 40.0 * all.tile_by / 8, all.halo_by + 3 * all.tile_by);
    rsp::launch_newton_init(P, ctx->box, ctx->tilex, ctx->yd, ctx->f, ctx->c, ctx->res, ctx->state,
                            eps0, o.tol_inner, o.max_inner, st);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(ctx->hstate.data(), ctx->state, sizeof(SubState) * P.S,
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const int ncont = continuation_steps(eps0, pr.eps_min, pr.gamma);
  int it = 0;
  int active = 0;
  for (auto& s : ctx->hstate) active += s.active;
  while (active && it < o.max_inner + 1) {
    // every subdomain needs the continuation steps: run them without looking, then
    // check after every step
    const int batch = std::max(1, std::min(ncont - it, o.max_inner + 1 - it));
    const SubWork w = sub_work(ctx->part.box, &ctx->hstate, fe);
    for (int b = 0; b < batch; ++b) {
      {
        Timed t(ctx, KID_FACTOR, st, w.factor_fl + w.bwd_fl / 2, w.factor_by);
        rsp::launch_factor(P, ctx->box, ctx->tilex, ctx->c, ctx->state, 0.0, ctx->res, -1.0,
                           ctx->fac, ctx->fp32, ctx->g, st);
      }
      {
        Timed t(ctx, KID_SOLVE_BWD, st, w.bwd_fl, w.bwd_by);
        rsp::launch_solve_bwd(P, ctx->box, ctx->state, ctx->fac, ctx->fp32, ctx->g, ctx->dir, st);
      }
      if (ctx->nref > 0) {
        Timed t(ctx, KID_REFINE, st, ctx->nref * (w.solve_fl + 20.0 * w.tile_by / 8),
                ctx->nref * (w.solve_by + 2 * w.tile_by));
        rsp::launch_newton_refine(P, ctx->box, ctx->tilex, ctx->c, ctx->state, ctx->fac, ctx->fp32,
                                  ctx->res, ctx->dir, ctx->nref, st);
      }
      {
        Timed t(ctx, KID_LINESEARCH, st, 40.0 * w.tile_by / 8, 6 * w.tile_by);
        rsp::launch_linesearch(P, ctx->box, ctx->tilex, ctx->yd, ctx->f, ctx->c, ctx->dir, ctx->res,
                               ctx->state, o.sigma, o.alpha_min, o.max_inner, st);
      }
    }
    HIPCHK(hipGetLastError());
    it += batch;
    HIPCHK(hipMemcpyAsync(ctx->hstate.data(), ctx->state, sizeof(SubState) * P.S,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    active = 0;
    for (auto& s : ctx->hstate) active += s.active;
  }
  int64_t ksum = 0;
  es->inner_min = 1 << 30;
  es->inner_max = 0;
  es->backtracks = 0;
  es->status = 0;
  double fl = 0;
  for (int s = 0; s < P.S; ++s) {
    const SubState& S = ctx->hstate[s];
    ksum += S.k;
    es->inner_min = std::min(es->inner_min, S.k);
    es->inner_max = std::max(es->inner_max, S.k);
    es->backtracks += S.backtracks;
    es->status = std::max(es->status, S.status);
    const double tx = ctx->part.box[s].y - ctx->part.box[s].x, ty = ctx->part.box[s].w - ctx->part.box[s].z;
    fl += S.k * (16.0 * ty * tx * tx * tx + 2.0 * (2 * ty - 1) * 4 * tx * tx);
  }
  es->inner_avg = (double)ksum / P.S;
  ctx->n_factor += ksum + P.S;
  ctx->n_solve += ksum;
  ctx->n_newton += ksum;
  ctx->flops += fl + all.factor_fl;
  // factor at x^(i) = x + P_i C_i(x) for Algorithm 4
  {
    Timed t(ctx, KID_FACTOR, st, all.factor_fl, all.factor_by);
    rsp::launch_factor(P, ctx->box, ctx->tilex, ctx->c, nullptr, pr.eps_min, nullptr, 0.0, ctx->fac,
                       ctx->fp32, ctx->g, st);
  }
  {
    Timed t(ctx, KID_PROLONG, st, 0, 8.0 * 2 * ctx->lay.L);
    rsp::launch_prolong(P, ctx->box, ctx->core, ctx->c, nullptr, out, st);
  }
  HIPCHK(hipGetLastError());
  return 0;
}

// Algorithm 4: out = -d + sum_i P~_i J_i^{-1} (hx^-2/hy^-2 weighted outside neighbours of d).
int run_jac_apply(rsp_context* ctx, const double* d, double* out, hipStream_t st,
                  const int* skip = nullptr) {
  const DevProblem& P = ctx->P;
  const SubWork w = sub_work(ctx->part.box, nullptr, (double)ctx->lay.fac_elem);
  {
    Timed t(ctx, KID_BLOCK_SOLVE, st, (1 + ctx->nref) * w.solve_fl,
            (1 + ctx->nref) * w.solve_by + 8.0 * 2 * ctx->lay.L);
    rsp::launch_jac_apply(P, ctx->box, ctx->core, ctx->fac, ctx->fp32, ctx->tilex, ctx->c, d, out, skip,
                          ctx->nref, st);
  }
  ctx->n_solve += P.S;
  ctx->n_apply += 1;
  ctx->flops += w.solve_fl;
  HIPCHK(hipGetLastError());
  return 0;
}

// |v|_2 on the device, read back (synchronises).
int dev_norm(rsp_context* ctx, const double* v, size_t L, double* out, hipStream_t st) {
  const int nb = rsp::multidot_blocks(L);
  rsp::launch_multidot(v, 0, 1, v, L, ctx->partial, st);
  rsp::launch_reduce_partials(ctx->partial, nb, 1, ctx->hbuf + 3 * 80, 0, st);
  double ss = 0;
  HIPCHK(hipMemcpyAsync(&ss, ctx->hbuf + 3 * 80, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *out = std::sqrt(ss);
  return 0;
}

// Restarted GMRES(m), x_0 = 0, on the device (kernels_gmres.hip): solves F'(x) dx = b.
// The host enqueues Arnoldi steps in chunks and reads the small state header back
// once per chunk; a stop flag set on the device turns the rest of a chunk into
// no-ops.  Returns RSP_GMRES_STAGNATION if max_gmres products did not reach rtol.
int run_gmres(rsp_context* ctx, const double* b, double* xs, int* used_out, double* rel_out,
              hipStream_t st) {
  constexpr int kChunk = 8;
  const size_t L = ctx->lay.L;
  const int m = ctx->opts.gmres_restart;
  const double rtol = ctx->opts.gmres_rtol;
  double* V = ctx->V;
  rsp::GmState hs{};
  const size_t hdr = offsetof(rsp::GmState, H);
  rsp::gm_init_state(ctx->gst, m, ctx->opts.max_gmres, rtol, st);
  HIPCHK(hipMemsetAsync(xs, 0, L * sizeof(double), st));
  rsp::launch_gm_sumsq(b, L, ctx->gp1, st);
  rsp::launch_gm_start(V, L, b, ctx->gst, ctx->gp1, 1, st);
  for (;;) {
    for (int j = 0; j < m;) {
      const int chunk = std::min(kChunk, m - j);
      for (int c = 0; c < chunk; ++c, ++j) {
        RSPCHK(run_jac_apply(ctx, V + (size_t)j * L, ctx->w, st, &ctx->gst->done));
        Timed tm(ctx, KID_GMRES_ORTHO, st, (double)L * (8.0 * (j + 1) + 3), 8.0 * L * (4.0 * j + 13));
        rsp::launch_gm_arnoldi(V, L, j, ctx->w, ctx->gst, ctx->gp1, ctx->gp2, st);
      }
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(&hs, ctx->gst, hdr, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (hs.done) break;
    }
    rsp::launch_gm_update_x(V, L, ctx->gst, xs, st);
    if (!(hs.rel > rtol) || hs.used >= ctx->opts.max_gmres || hs.steps == 0) break;
    // restart from r = b - F'(x) x
    RSPCHK(run_jac_apply(ctx, xs, ctx->w, st));
    rsp::launch_gm_residual(b, ctx->w, ctx->r, L, st);
    rsp::launch_gm_sumsq(ctx->r, L, ctx->gp1, st);
    rsp::launch_gm_start(V, L, ctx->r, ctx->gst, ctx->gp1, 0, st);
    HIPCHK(hipMemcpyAsync(&hs, ctx->gst, hdr, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hs.done) break;
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  ctx->n_gmres += hs.used;
  *used_out = hs.used;
  *rel_out = hs.rel;
  return hs.rel <= rtol ? 0 : RSP_GMRES_STAGNATION;
}

int ensure_setup(rsp_context* ctx, const rsp_problem* prob, const rsp_options* opts) {
  RSPCHK(validate_options(opts));
  Partition part;
  RSPCHK(make_partition(prob, &part));
  DevProblem P = make_dev(prob, part);
  Layout lay = make_layout(P, opts);
  const size_t bytes = layout_bytes(lay, P.S);
  if (ctx->budget && bytes > ctx->budget)
    return fail(RSP_ENOMEM, "workspace needs %zu bytes, budget is %zu", bytes, ctx->budget);
  HIPCHK(hipSetDevice(ctx->device));
  if (bytes > ctx->mem_bytes) {
    if (ctx->mem) HIPCHK(hipFree(ctx->mem));
    ctx->mem = nullptr;
    ctx->mem_bytes = 0;
    hipError_t e = hipMalloc(&ctx->mem, bytes);
    if (e != hipSuccess) return fail(RSP_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    ctx->mem_bytes = bytes;
  }
  char* p = (char*)ctx->mem;
  auto take = [&](size_t nbytes) {
    char* r = p;
    p += (nbytes + 255) / 256 * 256;
    return r;
  };
  ctx->box = (int4*)take(sizeof(int4) * P.S);
  ctx->core = (int4*)take(sizeof(int4) * P.S);
  ctx->state = (SubState*)take(sizeof(SubState) * P.S);
  ctx->yd = (double*)take(8 * lay.n);
  ctx->f = (double*)take(8 * lay.n);
  ctx->x = (double*)take(8 * lay.L);
  ctx->F = (double*)take(8 * lay.L);
  ctx->tilex = (double*)take(8 * lay.halo);
  ctx->c = (double*)take(8 * lay.tile);
  ctx->dir = (double*)take(8 * lay.tile);
  ctx->res = (double*)take(8 * lay.tile);
  ctx->t1 = (double*)take(8 * lay.tile);
  ctx->t2 = (double*)take(8 * lay.tile);
  ctx->fac = (void*)take(lay.fac_elem * lay.fac);
  ctx->g = (double*)take(8 * lay.g);
  ctx->V = (double*)take(8 * lay.V);
  ctx->w = (double*)take(8 * lay.L);
  ctx->b = (double*)take(8 * lay.L);
  ctx->dx = (double*)take(8 * lay.L);
  ctx->partial = (double*)take(8 * lay.partial);
  ctx->hbuf = (double*)take(8 * 4 * 80);
  ctx->r = (double*)take(8 * lay.L);
  ctx->gp1 = (double*)take(8 * lay.gpart);
  ctx->gp2 = (double*)take(8 * lay.gpart);
  ctx->gst = (rsp::GmState*)take(sizeof(rsp::GmState));
  if ((size_t)(p - (char*)ctx->mem) > ctx->mem_bytes)
    return fail(RSP_ENOMEM, "internal: workspace layout overflow");
  ctx->prob = *prob;
  ctx->opts = *opts;
  ctx->part = part;
  ctx->P = P;
  ctx->lay = lay;
  ctx->hstate.assign(P.S, SubState{});
  ctx->fp32 = opts->precision == RSP_FP32_REFINED;
  ctx->nref = ctx->fp32 ? opts->max_refine : 0;
  ctx->ready = true;
  return 0;
}

}  // namespace

extern "C" {

int rsp_version(void) { return RSP_VERSION; }

const char* rsp_last_error(void) { return g_err.c_str(); }

int rsp_partition(const rsp_problem* prob, int32_t* S, int32_t* txm, int32_t* tym, int32_t* boxes) {
  Partition part;
  RSPCHK(make_partition(prob, &part));
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
  Partition part;
  if (make_partition(prob, &part) < 0 || validate_options(opts) < 0) return 0;
  DevProblem P = make_dev(prob, part);
  Layout lay = make_layout(P, opts);
  return layout_bytes(lay, P.S);
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
  *ctx = c;
  return 0;
}

int rsp_context_destroy(rsp_context* ctx) {
  if (!ctx) return 0;
  (void)hipSetDevice(ctx->device);
  (void)resolve_events(ctx);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->mem) (void)hipFree(ctx->mem);
  delete ctx;
  return 0;
}

int rsp_setup(rsp_context* ctx, const rsp_problem* prob, const rsp_options* opts, const double* yd,
              const double* f, hipStream_t stream) {
  if (!ctx) return fail(RSP_EINVAL, "ctx is NULL");
  if (!yd) return fail(RSP_EINVAL, "yd is NULL");
  RSPCHK(ensure_setup(ctx, prob, opts));
  const size_t n = ctx->lay.n;
  HIPCHK(hipMemcpyAsync(ctx->box, ctx->part.box.data(), sizeof(int4) * ctx->P.S, hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync(ctx->core, ctx->part.core.data(), sizeof(int4) * ctx->P.S, hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync(ctx->yd, yd, 8 * n, hipMemcpyDeviceToDevice, stream));
  if (f) HIPCHK(hipMemcpyAsync(ctx->f, f, 8 * n, hipMemcpyDeviceToDevice, stream));
  else HIPCHK(hipMemsetAsync(ctx->f, 0, 8 * n, stream));
  HIPCHK(hipStreamSynchronize(stream));   // the partition vectors are host temporaries
  return 0;
}

#define NEED_READY(ctx) \
  if (!(ctx) || !(ctx)->ready) return fail(RSP_EINVAL, "context has no problem (call rsp_setup)")

int rsp_residual(rsp_context* ctx, const double* x, double eps, double* out, hipStream_t stream) {
  NEED_READY(ctx);
  if (!(eps >= 0)) return fail(RSP_EINVAL, "eps must be >= 0");
  rsp::launch_global_residual(ctx->P, ctx->yd, ctx->f, x, eps, out, stream);
  HIPCHK(hipGetLastError());
  return 0;
}

int rsp_control(rsp_context* ctx, const double* p, double eps, double* u, hipStream_t stream) {
  NEED_READY(ctx);
  if (!(eps >= 0)) return fail(RSP_EINVAL, "eps must be >= 0");
  rsp::launch_control(ctx->P, p, eps, u, stream);
  HIPCHK(hipGetLastError());
  return 0;
}

int rsp_restrict(rsp_context* ctx, const double* x, double* tiles, hipStream_t stream) {
  NEED_READY(ctx);
  rsp::launch_restrict(ctx->P, ctx->box, x, tiles, stream);
  HIPCHK(hipGetLastError());
  return 0;
}

int rsp_prolong(rsp_context* ctx, const double* tiles, double* out, hipStream_t stream) {
  NEED_READY(ctx);
  rsp::launch_prolong(ctx->P, ctx->box, ctx->core, tiles, nullptr, out, stream);
  HIPCHK(hipGetLastError());
  return 0;
}

int rsp_local_residual(rsp_context* ctx, const double* x, const double* c, double eps, double* out,
                       double* norms, hipStream_t stream) {
  NEED_READY(ctx);
  if (!(eps >= 0)) return fail(RSP_EINVAL, "eps must be >= 0");
  rsp::launch_restrict_halo(ctx->P, ctx->box, x, ctx->tilex, stream);
  rsp::launch_local_residual(ctx->P, ctx->box, ctx->tilex, ctx->yd, ctx->f, c, eps, out, norms, stream);
  HIPCHK(hipGetLastError());
  return 0;
}

int rsp_local_solve(rsp_context* ctx, const double* x, const double* c, double eps, const double* rhs,
                    double* z, hipStream_t stream) {
  NEED_READY(ctx);
  if (!(eps > 0)) return fail(RSP_EINVAL, "eps must be > 0");
  rsp::launch_restrict_halo(ctx->P, ctx->box, x, ctx->tilex, stream);
  rsp::launch_factor(ctx->P, ctx->box, ctx->tilex, c, nullptr, eps, nullptr, 0.0, ctx->fac, ctx->fp32,
                     ctx->g, stream);
  rsp::launch_block_solve(ctx->P, ctx->box, ctx->fac, ctx->fp32, rhs, z, stream);
  HIPCHK(hipGetLastError());
  return 0;
}

int rsp_eval(rsp_context* ctx, const double* x, int continuation, double* out, double* norm,
             hipStream_t stream) {
  NEED_READY(ctx);
  EvalStats es;
  RSPCHK(run_eval(ctx, x, continuation != 0, out, &es, stream));
  if (norm) RSPCHK(dev_norm(ctx, out, ctx->lay.L, norm, stream));
  return es.status;
}

int rsp_jac_apply(rsp_context* ctx, const double* d, double* out, hipStream_t stream) {
  NEED_READY(ctx);
  return run_jac_apply(ctx, d, out, stream);
}

int rsp_solve(rsp_context* ctx, const rsp_problem* prob, const rsp_options* opts, const double* yd,
              const double* f, const double* y0, const double* p0, double* y, double* p, double* u,
              rsp_history* hist, hipStream_t stream) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  if (!ctx) return fail(RSP_EINVAL, "ctx is NULL");
  if (!y || !p || !u) return fail(RSP_EINVAL, "outputs y, p, u are required");
  if ((y0 == nullptr) != (p0 == nullptr)) return fail(RSP_EINVAL, "give both y0 and p0 or neither");
  RSPCHK(rsp_setup(ctx, prob, opts, yd, f, stream));
  const size_t n = ctx->lay.n, L = ctx->lay.L;
  ctx->n_factor = ctx->n_solve = ctx->n_gmres = ctx->n_newton = ctx->n_apply = 0;
  ctx->flops = 0;
  rsp_history hloc;
  rsp_history* h = hist ? hist : &hloc;
  std::memset(h, 0, sizeof(*h));
  h->subdomains = ctx->P.S;
  if (y0) {
    HIPCHK(hipMemcpyAsync(ctx->x, y0, 8 * n, hipMemcpyDeviceToDevice, stream));
    HIPCHK(hipMemcpyAsync(ctx->x + n, p0, 8 * n, hipMemcpyDeviceToDevice, stream));
  } else {
    HIPCHK(hipMemsetAsync(ctx->x, 0, 8 * L, stream));
  }
  double ms_eval = 0, ms_gmres = 0;
  auto ms = [](clk::time_point a, clk::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
  };
  EvalStats es;
  auto te = clk::now();
  RSPCHK(run_eval(ctx, ctx->x, opts->continuation != RSP_CONT_NONE, ctx->F, &es, stream));
  double Fn = 0;
  RSPCHK(dev_norm(ctx, ctx->F, L, &Fn, stream));
  ms_eval += ms(te, clk::now());
  int status = es.status;
  h->norm[0] = Fn;
  h->inner_min[0] = es.inner_min;
  h->inner_max[0] = es.inner_max;
  h->inner_avg[0] = es.inner_avg;
  h->backtracks[0] = es.backtracks;
  const double thr = std::max(opts->tol_outer, opts->tol_outer * Fn);
  int k = 0;
  while (!(Fn <= thr) && k < opts->max_outer) {
    // Newton system F'(x^k) d = -F(x^k) by GMRES, then x^{k+1} = x^k + d (undamped)
    const auto tg = clk::now();
    rsp::launch_scale(-1.0, ctx->F, ctx->b, L, stream);
    int used = 0;
    double rel = 0;
    int gs = run_gmres(ctx, ctx->b, ctx->dx, &used, &rel, stream);
    if (gs < 0) return gs;
    if (gs > 0) status = std::max(status, gs);
    rsp::launch_axpy(1.0, ctx->dx, ctx->x, L, stream);
    ms_gmres += ms(tg, clk::now());
    ++k;
    te = clk::now();
    RSPCHK(run_eval(ctx, ctx->x, opts->continuation == RSP_CONT_EVERY, ctx->F, &es, stream));
    RSPCHK(dev_norm(ctx, ctx->F, L, &Fn, stream));
    ms_eval += ms(te, clk::now());
    status = std::max(status, es.status);
    if (k <= RSP_HIST_MAX) {
      h->norm[k] = Fn;
      h->gmres_its[k] = used;
      h->gmres_rel[k] = rel;
      h->inner_min[k] = es.inner_min;
      h->inner_max[k] = es.inner_max;
      h->inner_avg[k] = es.inner_avg;
      h->backtracks[k] = es.backtracks;
    }
  }
  if (!(Fn <= thr) && status == 0) status = RSP_NOT_CONVERGED;
  HIPCHK(hipMemcpyAsync(y, ctx->x, 8 * n, hipMemcpyDeviceToDevice, stream));
  HIPCHK(hipMemcpyAsync(p, ctx->x + n, 8 * n, hipMemcpyDeviceToDevice, stream));
  rsp::launch_control(ctx->P, ctx->x + n, prob->eps_min, u, stream);
  rsp::launch_global_residual(ctx->P, ctx->yd, ctx->f, ctx->x, prob->eps_min, ctx->w, stream);
  double rfin = 0;
  RSPCHK(dev_norm(ctx, ctx->w, L, &rfin, stream));
  h->status = status;
  h->outer = k;
  h->factorizations = ctx->n_factor;
  h->local_solves = ctx->n_solve;
  h->gmres_total = ctx->n_gmres;
  h->newton_iterations = ctx->n_newton;
  h->jac_applies = ctx->n_apply;
  h->residual_final = rfin;
  h->flops = ctx->flops;
  h->ms_eval = ms_eval;
  h->ms_gmres = ms_gmres;
  h->ms_total = ms(t0, clk::now());
  RSPCHK(resolve_events(ctx));
  return status;
}

int rsp_set_profiling(rsp_context* ctx, int on) {
  if (!ctx) return fail(RSP_EINVAL, "ctx is NULL");
  ctx->prof = on != 0;
  return 0;
}

int rsp_reset_kernel_stats(rsp_context* ctx) {
  if (!ctx) return fail(RSP_EINVAL, "ctx is NULL");
  RSPCHK(resolve_events(ctx));
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
