// Autotuner: measures whole solves of a sample problem under candidate execution
// settings and keeps the fastest.  It is a client of the public entry points
// (rsp_solve, rsp_solve_batch, rsp_set_tuning) and adds no device code.
//
// Searched, in this order (each stage keeps the winner of the previous ones):
//   1. graphs {0, 1} x Arnoldi chunk {4, 8, 16, restart}: no effect on results;
//   2. (RSP_TUNE_PARTITION) subdomain counts whose tiles, with the sample's
//      overlap, fit the line blocks of 48, 64 and 80 unknowns: the fixed point of
//      RASPEN does not depend on the partition, the work to reach it does;
//   3. (RSP_TUNE_BATCH) batches of 1, 2, 4, ... copies of the sample: the smallest
//      batch whose throughput is within 5 % of the best seen.
// Results are cached per (grid, partition, overlap, precision, restart, flags) for
// the life of the process.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "engine.h"
#include "raspen.h"

namespace {

using Clock = std::chrono::steady_clock;

struct TuneKey {
  int nx, ny, sx, sy, overlap, precision, restart, flags;
  bool operator<(const TuneKey& o) const {
    return std::tie(nx, ny, sx, sy, overlap, precision, restart, flags) <
           std::tie(o.nx, o.ny, o.sx, o.sy, o.overlap, o.precision, o.restart, o.flags);
  }
};

std::mutex g_mu;
std::map<TuneKey, rsp_tuning> g_cache;

// Device buffers for the outputs of up to `count` copies of an n-node problem.
struct Outputs {
  std::vector<double*> y, p, u;
  double* base = nullptr;
  ~Outputs() {
    if (base) (void)hipFree(base);
  }
  int alloc(int count, size_t n) {
    if (hipMalloc(&base, sizeof(double) * 3 * n * count) != hipSuccess) {
      base = nullptr;
      return rsp::fail(RSP_ENOMEM, "autotune: no device memory for %d output sets", count);
    }
    for (int q = 0; q < count; ++q) {
      y.push_back(base + (3 * q + 0) * n);
      p.push_back(base + (3 * q + 1) * n);
      u.push_back(base + (3 * q + 2) * n);
    }
    return 0;
  }
};

// Solves/s of `count` copies of the sample in one batch (count = 1: rsp_solve),
// from `reps` timed calls after one untimed call; < 0 on error, 0 if a copy did
// not converge.
double rate(rsp_context* ctx, const rsp_problem& pr, const rsp_options& o, const double* yd,
            const double* f, Outputs& out, int count, int reps, hipStream_t st) {
  std::vector<rsp_problem> probs(count, pr);
  std::vector<const double*> yds(count, yd), fs(count, f);
  std::vector<rsp_history> hist(count);
  auto once = [&]() -> int {
    if (count == 1)
      return rsp_solve(ctx, &pr, &o, yd, f, nullptr, nullptr, out.y[0], out.p[0], out.u[0], hist.data(), st);
    return rsp_solve_batch(ctx, count, probs.data(), &o, yds.data(), fs.data(), nullptr, nullptr,
                           out.y.data(), out.p.data(), out.u.data(), hist.data(), st);
  };
  int s = once();
  if (s < 0) return s;
  if (s != 0) return 0.0;
  if (hipStreamSynchronize(st) != hipSuccess) return RSP_EHIP;
  const auto t0 = Clock::now();
  for (int r = 0; r < reps; ++r) {
    s = once();
    if (s < 0) return s;
    if (s != 0) return 0.0;
  }
  if (hipStreamSynchronize(st) != hipSuccess) return RSP_EHIP;
  const double el = std::chrono::duration<double>(Clock::now() - t0).count();
  return el > 0 ? count * reps / el : 0.0;
}

}  // namespace

extern "C" {

int rsp_autotune(rsp_context* ctx, const rsp_problem* sample, const rsp_options* opts,
                 const double* yd, const double* f, int flags, rsp_tuning* out, hipStream_t stream) {
  if (!ctx || !sample || !opts || !yd || !out)
    return rsp::fail(RSP_EINVAL, "autotune: ctx, sample, opts, yd and out are required");
  if (flags & ~(RSP_TUNE_PARTITION | RSP_TUNE_BATCH))
    return rsp::fail(RSP_EINVAL, "autotune: unknown flags 0x%x", flags);
  {
    rsp::Inst probe;
    if (int e = rsp::inst_init(&probe, sample)) return e;
    if (int e = rsp::validate_options(opts)) return e;
  }
  const TuneKey key{sample->nx, sample->ny, sample->sx, sample->sy, sample->overlap, opts->precision,
                    opts->gmres_restart, flags};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      rsp_tuning cur;
      if (int e = rsp_get_tuning(ctx, &cur)) return e;
      *out = it->second;
      out->jac_form = cur.jac_form;   // not tuned: the context's own
      return rsp_set_tuning(ctx, out);
    }
  }
  const size_t n = (size_t)sample->nx * sample->ny;
  constexpr int kMaxCopies = 64;
  const int maxb = (flags & RSP_TUNE_BATCH) ? kMaxCopies : 1;
  Outputs bufs;
  if (int e = bufs.alloc(maxb, n)) return e;
  // about 0.3 s of timed solves per candidate, at least 2
  rsp_tuning best{};
  if (int e = rsp_get_tuning(ctx, &best)) return e;   // keeps the context's jac_form
  best.graphs = 0;
  best.gm_chunk = 8;
  if (int e = rsp_set_tuning(ctx, &best)) return e;
  double r0 = rate(ctx, *sample, *opts, yd, f, bufs, 1, 1, stream);
  if (r0 < 0) return (int)r0;
  if (r0 == 0) return rsp::fail(RSP_EINVAL, "autotune: the sample does not converge");
  const int reps = std::max(2, std::min(50, (int)(0.3 * r0)));

  // 1. execution settings
  best.solves_per_s = 0;
  const int chunks[] = {4, 8, 16, opts->gmres_restart};
  for (int g = 0; g <= 1; ++g)
    for (int c : chunks) {
      rsp_tuning t = best;
      t.graphs = g;
      t.gm_chunk = std::min(c, opts->gmres_restart);
      if (int e = rsp_set_tuning(ctx, &t)) return e;
      const double r = rate(ctx, *sample, *opts, yd, f, bufs, 1, reps, stream);
      if (r < 0) return (int)r;
      if (r > best.solves_per_s) {
        t.solves_per_s = r;
        best = t;
      }
    }
  if (int e = rsp_set_tuning(ctx, &best)) return e;
  best.sx = sample->sx;
  best.sy = sample->sy;

  // 2. subdomain counts: tiles of 48, 64, 80 line unknowns (width 24, 32, 40 with overlap)
  rsp_problem pr = *sample;
  if (flags & RSP_TUNE_PARTITION) {
    for (int width : {24, 32, 40}) {
      const int core = width - 2 * sample->overlap;
      if (core < 4) continue;
      rsp_problem c = *sample;
      c.sx = std::min(sample->nx, (sample->nx + core - 1) / core);
      c.sy = std::min(sample->ny, (sample->ny + core - 1) / core);
      if (c.sx == best.sx && c.sy == best.sy) continue;
      rsp::Inst probe;
      if (rsp::inst_init(&probe, &c) != 0) continue;   // not a valid partition
      const double r = rate(ctx, c, *opts, yd, f, bufs, 1, reps, stream);
      if (r < 0) return (int)r;
      if (r > best.solves_per_s) {
        best.solves_per_s = r;
        best.sx = c.sx;
        best.sy = c.sy;
      }
    }
    pr.sx = best.sx;
    pr.sy = best.sy;
  }

  // 3. batch size: copies of the (re-partitioned) sample
  best.max_batch = 1;
  if (flags & RSP_TUNE_BATCH) {
    double top = best.solves_per_s;
    std::vector<std::pair<int, double>> seen{{1, top}};
    for (int b = 2; b <= kMaxCopies; b *= 2) {
      std::vector<rsp_problem> probs(b, pr);
      const size_t need = rsp_batch_workspace_bytes(b, probs.data(), opts);
      size_t free_b = 0, total_b = 0;
      if (need == 0 || hipMemGetInfo(&free_b, &total_b) != hipSuccess || need > free_b / 2) break;
      const double r = rate(ctx, pr, *opts, yd, f, bufs, b, std::max(1, reps / b), stream);
      if (r < 0) return (int)r;
      seen.push_back({b, r});
      if (r < 1.05 * top) {   // saturated
        top = std::max(top, r);
        break;
      }
      top = r;
    }
    for (const auto& s : seen)
      if (s.second >= 0.95 * top) {
        best.max_batch = s.first;
        best.solves_per_s = s.second;
        break;
      }
  }
  if (int e = rsp_set_tuning(ctx, &best)) return e;
  *out = best;
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[key] = best;
  return 0;
}

}  // extern "C"
