// Serving loop: continuous batching of RASPEN solves on one device.
//
// A worker thread owns a context and a stream.  Between two outer iterations of
// the running batch (engine_step) it admits queued requests -- first come, first
// served, while the layout of the grown batch fits the memory budget and the batch
// limit -- and lays the batch out again (engine_place moves the state of the
// running instances).  Instances that meet their stopping test retire at the end
// of the iteration in which they do; their outputs are complete on the device
// when their ticket reads done.  Because every per-instance reduction has a fixed
// order, a request's result does not depend on which other requests shared its
// batch (when the padded line-block sizes agree).
#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "engine.h"

using rsp::Clock;
using rsp::Inst;
using rsp::fail;

namespace {

struct Request {
  uint64_t ticket = 0;
  Inst inst;
  int state = RSP_TICKET_QUEUED;
  int result = 0;                 // solve status, or a hard error (< 0)
  Clock::time_point t_submit, t_done;
};

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct rsp_server {
  rsp_server_options opts{};
  rsp_context* ctx = nullptr;
  rsp_context* ctx64 = nullptr;   // requests that left the FP32 factors (made on first use)
  hipStream_t stream = nullptr;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  // statistics (under mu)
  int64_t submitted = 0, completed = 0, failed = 0, running = 0, steps = 0, step_members = 0;
  std::vector<double> latencies;
  bool any_submit = false;
  Clock::time_point t_first, t_last;
  // kernel timing of the main batch (profile_every > 0), settled after each step
  std::vector<rsp_kernel_stat> kstat;
};

namespace {

// Bytes of a layout holding `live` plus `extra`.
size_t layout_need(const std::vector<Request*>& live, const std::vector<Request*>& adm, const Request* extra,
                   const rsp_options& o) {
  std::vector<const rsp_problem*> pp;
  for (const Request* r : live) pp.push_back(&r->inst.prob);
  for (const Request* r : adm) pp.push_back(&r->inst.prob);
  if (extra) pp.push_back(&extra->inst.prob);
  return rsp::batch_bytes(pp.data(), (int)pp.size(), o);
}

void complete(rsp_server* s, Request* r, int result) {
  // caller holds s->mu
  r->state = RSP_TICKET_DONE;
  r->result = result;
  r->t_done = Clock::now();
  if (result < 0) {
    s->failed += 1;
  } else {
    s->completed += 1;
    s->latencies.push_back(ms_between(r->t_submit, r->t_done));
  }
  s->t_last = r->t_done;
}

// Requests whose FP32 factors were not good enough (rsp_options.fallback_rho) leave
// the main batch parked and run to the end as a second batch with FP64 factors, in
// a context of their own (with the same budget), one outer iteration per round.
int step_fallback(rsp_server* s, std::vector<Request*>& fb, const std::vector<Request*>& fresh) {
  const rsp_options o64 = rsp::fallback_options(s->opts.opts);
  if (!s->ctx64) {
    int r = rsp_context_create(&s->ctx64, s->opts.device, s->opts.hbm_budget);
    if (r < 0) return r;
    if (s->opts.tune.gm_chunk != 0 && (r = rsp_set_tuning(s->ctx64, &s->opts.tune)) < 0) return r;
  }
  std::vector<Inst*> li;
  if (!fresh.empty()) {
    fb.insert(fb.end(), fresh.begin(), fresh.end());
    for (Request* r : fb) li.push_back(&r->inst);
    int e = rsp::engine_place(s->ctx64, o64, li, s->stream);
    if (e < 0) return e;
    for (Request* r : fresh) r->inst.parked = false;
    li.clear();
  }
  for (Request* r : fb) li.push_back(&r->inst);
  return li.empty() ? 0 : rsp::engine_step(s->ctx64, li, s->stream);
}

void worker_main(rsp_server* s) {
  (void)hipSetDevice(s->opts.device);
  std::vector<Request*> live, fb;
  const rsp_options& o = s->opts.opts;
  const size_t budget = s->opts.hbm_budget;
  for (;;) {
    std::vector<Request*> adm;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty() || !live.empty() || !fb.empty(); });
      if (live.empty() && fb.empty() && s->queue.empty() && s->stop) break;
      while (!s->queue.empty()) {
        if (s->opts.max_batch > 0 && (int)(live.size() + adm.size()) >= s->opts.max_batch) break;
        Request* r = s->queue.front();
        const size_t need = layout_need(live, adm, r, o);
        if (budget && need > budget) {
          if (live.empty() && adm.empty()) {
            // does not fit even alone
            s->queue.pop_front();
            complete(s, r, RSP_ENOMEM);
            s->cv_done.notify_all();
            continue;
          }
          break;   // wait for room
        }
        s->queue.pop_front();
        r->state = RSP_TICKET_RUNNING;
        adm.push_back(r);
      }
      s->running = (int64_t)(live.size() + adm.size());
    }
    int err = 0;
    if (!adm.empty()) {
      for (Request* r : adm) r->inst.t0 = Clock::now();
      live.insert(live.end(), adm.begin(), adm.end());
      std::vector<Inst*> li;
      for (Request* r : live) li.push_back(&r->inst);
      err = rsp::engine_place(s->ctx, o, li, s->stream);
    }
    if (err >= 0 && !live.empty()) {
      std::vector<Inst*> li;
      for (Request* r : live) li.push_back(&r->inst);
      err = rsp::engine_step(s->ctx, li, s->stream);
    }
    std::vector<Request*> still, parked;
    for (Request* r : live) {
      if (err >= 0 && r->inst.parked) parked.push_back(r);
      else still.push_back(r);
    }
    live.swap(still);
    still.clear();
    int err64 = 0;
    if (err >= 0 && (!fb.empty() || !parked.empty())) err64 = step_fallback(s, fb, parked);
    if (s->opts.profile_every > 0 && err >= 0) {
      int32_t nk = 0;
      std::vector<rsp_kernel_stat> ks(32);
      if (rsp_kernel_stats(s->ctx, ks.data(), (int)ks.size(), &nk) >= 0) {
        ks.resize(nk);
        std::lock_guard<std::mutex> lk(s->mu);
        s->kstat.swap(ks);
      }
    }
    std::vector<Request*> fb_still;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (!live.empty() || !fb.empty()) {
        s->steps += 1;
        s->step_members += (int64_t)(live.size() + fb.size());
      }
      for (Request* r : live) {
        if (err < 0) complete(s, r, err);
        else if (r->inst.finished) complete(s, r, r->inst.status);
        else still.push_back(r);
      }
      for (Request* r : fb) {
        if (err64 < 0) complete(s, r, err64);
        else if (r->inst.finished) complete(s, r, r->inst.status);
        else fb_still.push_back(r);
      }
      s->running = (int64_t)(still.size() + fb_still.size());
    }
    s->cv_done.notify_all();
    if (err < 0 || err64 < 0) (void)hipStreamSynchronize(s->stream);
    live.swap(still);
    fb.swap(fb_still);
  }
}

}  // namespace

extern "C" {

int rsp_server_create(rsp_server** out, const rsp_server_options* opts) {
  if (!out || !opts) return fail(RSP_EINVAL, "server and options are required");
  if (opts->max_batch < 0) return fail(RSP_EINVAL, "max_batch must be >= 0");
  int r = rsp::validate_options(&opts->opts);
  if (r < 0) return r;
  if (opts->opts.record_eps_snapshots) return fail(RSP_EINVAL, "eps snapshots are recorded by rsp_solve only");
  std::unique_ptr<rsp_server> s(new (std::nothrow) rsp_server());
  if (!s) return fail(RSP_ENOMEM, "out of host memory");
  s->opts = *opts;
  r = rsp_context_create(&s->ctx, opts->device, opts->hbm_budget);
  if (r < 0) return r;
  if (opts->tune.gm_chunk != 0 && (r = rsp_set_tuning(s->ctx, &opts->tune)) < 0) {
    rsp_context_destroy(s->ctx);
    return r;
  }
  if (opts->profile_every < 0) {
    rsp_context_destroy(s->ctx);
    return fail(RSP_EINVAL, "profile_every must be >= 0");
  }
  if (opts->profile_every > 0) {
    rsp_set_profiling(s->ctx, 1);
    rsp_set_profiling_filter(s->ctx, "block_solve");
    rsp_set_profiling_sample(s->ctx, opts->profile_every);
  }
  hipError_t e = hipSetDevice(opts->device);
  if (e == hipSuccess) e = hipStreamCreate(&s->stream);
  if (e != hipSuccess) {
    rsp_context_destroy(s->ctx);
    return fail(RSP_EHIP, "hipStreamCreate: %s", hipGetErrorString(e));
  }
  rsp_server* raw = s.get();
  try {
    s->worker = std::thread(worker_main, raw);
  } catch (...) {
    (void)hipStreamDestroy(s->stream);
    rsp_context_destroy(s->ctx);
    return fail(RSP_ENOMEM, "cannot start the worker thread");
  }
  *out = s.release();
  return 0;
}

int rsp_server_submit(rsp_server* s, const rsp_problem* prob, const double* yd, const double* f,
                      double* y, double* p, double* u, uint64_t* ticket) {
  if (!s || !ticket) return fail(RSP_EINVAL, "server and ticket are required");
  if (!yd || !y || !p || !u) return fail(RSP_EINVAL, "yd, y, p, u are required");
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return fail(RSP_ENOMEM, "out of host memory");
  int e = rsp::inst_init(&r->inst, prob);
  if (e < 0) return e;
  if (rsp::batch_bytes(&prob, 1, s->opts.opts) == 0) return fail(RSP_EINVAL, "problem cannot be laid out");
  r->inst.yd = yd;
  r->inst.f = f;
  r->inst.y = y;
  r->inst.p = p;
  r->inst.u = u;
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(RSP_EINVAL, "server is shutting down");
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    if (!s->any_submit) {
      s->any_submit = true;
      s->t_first = r->t_submit;
    }
    s->submitted += 1;
    s->queue.push_back(r.get());
    s->reqs.emplace(r->ticket, std::move(r));
  }
  s->cv_work.notify_one();
  return 0;
}

int rsp_server_poll(rsp_server* s, uint64_t ticket, int32_t* state) {
  if (!s || !state) return fail(RSP_EINVAL, "server and state are required");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(RSP_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  *state = it->second->state;
  return 0;
}

int rsp_server_wait(rsp_server* s, uint64_t ticket, double timeout_ms, rsp_history* hist) {
  if (!s) return fail(RSP_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(RSP_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second.get();
  auto done = [&] { return r->state == RSP_TICKET_DONE; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, done);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), done)) {
    return fail(RSP_EAGAIN, "ticket %llu not done within %.1f ms", (unsigned long long)ticket, timeout_ms);
  }
  const int result = r->result;
  if (hist) *hist = r->inst.hist;
  s->reqs.erase(it);
  if (result < 0) return fail(result, "request %llu failed (%d)", (unsigned long long)ticket, result);
  return result;
}

int rsp_server_stats(rsp_server* s, rsp_server_report* out) {
  if (!s || !out) return fail(RSP_EINVAL, "server and stats are required");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->queued = (int64_t)s->queue.size();
  out->running = s->running;
  out->steps = s->steps;
  out->mean_batch = s->steps ? (double)s->step_members / s->steps : 0.0;
  if (!s->latencies.empty()) {
    std::vector<double> l = s->latencies;
    std::sort(l.begin(), l.end());
    // nearest-rank percentiles
    auto pct = [&](double q) {
      size_t k = (size_t)std::ceil(q * l.size());
      k = std::min(std::max<size_t>(k, 1), l.size());
      return l[k - 1];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    double sum = 0;
    for (double v : l) sum += v;
    out->mean_ms = sum / l.size();
    const double span = ms_between(s->t_first, s->t_last);
    out->solves_per_s = span > 0 ? 1000.0 * s->completed / span : 0.0;
  }
  return 0;
}

int rsp_server_kernel_stats(rsp_server* s, rsp_kernel_stat* out, int max, int32_t* count) {
  if (!s) return fail(RSP_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  int n = 0;
  for (; out && n < max && n < (int)s->kstat.size(); ++n) out[n] = s->kstat[n];
  if (count) *count = out ? n : (int32_t)s->kstat.size();
  return 0;
}

int rsp_server_destroy(rsp_server* s) {
  if (!s) return 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->opts.device);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  rsp_context_destroy(s->ctx);
  if (s->ctx64) rsp_context_destroy(s->ctx64);
  delete s;
  return 0;
}

}  // extern "C"
