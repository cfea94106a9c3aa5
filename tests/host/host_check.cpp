// Host-side checks of libraspen's entry points that run without a GPU: the partition
// of Section 4.2, the workspace sizing used for serving admission, the validation of
// problems and options, and the error paths of the calls that need a device.  Built
// with AddressSanitizer and UndefinedBehaviorSanitizer on the host code (see
// paper_2411_00546_amd/build.py, build_host_check) and run by
// tests/test_host_sanitizers.py; exits non-zero on a failed check, and the sanitizers
// abort on the first report.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "raspen.h"

namespace {

int g_fail = 0;
int g_checks = 0;

#define CHECK(cond, ...)                                           \
  do {                                                             \
    ++g_checks;                                                    \
    if (!(cond)) {                                                 \
      ++g_fail;                                                    \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__);    \
      std::fprintf(stderr, __VA_ARGS__);                           \
      std::fprintf(stderr, "\n");                                  \
    }                                                              \
  } while (0)

rsp_problem problem(int nx, int ny, int sx, int sy, int overlap) {
  rsp_problem p;
  std::memset(&p, 0, sizeof p);
  p.nx = nx;
  p.ny = ny;
  p.phi_kind = RSP_PHI_CUBIC;
  p.kappa = 1.0;
  p.nu = 1e-2;
  p.mu = 1e-2;
  p.eps0 = 1.0;
  p.eps_min = 1e-6;
  p.gamma = 0.5;
  p.sx = sx;
  p.sy = sy;
  p.overlap = overlap;
  return p;
}

rsp_options options() {
  rsp_options o;
  std::memset(&o, 0, sizeof o);
  o.tol_outer = 1e-10;
  o.tol_inner = 1e-8;
  o.gmres_rtol = 1e-10;
  o.sigma = 1.1;
  o.alpha_min = std::ldexp(1.0, -30);
  o.gmres_restart = 30;
  o.max_outer = 50;
  o.max_inner = 200;
  o.max_gmres = 300;
  o.precision = RSP_FP64;
  o.max_refine = 1;
  o.continuation = RSP_CONT_FIRST;
  o.tol_inner_rel = -1.0;
  o.fallback_rho = 1.0;
  return o;
}

// The partition written out independently: boxes of width B = ceil(n / s) per
// direction, [j B, min((j + 1) B, n)), extended by `overlap` per side and clipped.
struct Expect {
  bool ok;
  int txm, tym;
};
Expect expect(const rsp_problem& p) {
  Expect e{true, 0, 0};
  auto dir = [&](int n, int s, int& w) {
    if (s < 1 || s > n) return false;
    const int B = (n + s - 1) / s;
    if ((s - 1) * B >= n) return false;   // the last box would be empty
    for (int j = 0; j < s; ++j) {
      const int lo = j * B, hi = std::min((j + 1) * B, n);
      w = std::max(w, std::min(n, hi + p.overlap) - std::max(0, lo - p.overlap));
    }
    return true;
  };
  e.ok = p.nx >= 1 && p.ny >= 1 && p.overlap >= 0 && dir(p.nx, p.sx, e.txm) && dir(p.ny, p.sy, e.tym);
  return e;
}

void check_partition(const rsp_problem& p, int max_tile) {
  int32_t S = -1, txm = -1, tym = -1;
  const int r = rsp_partition(&p, &S, &txm, &tym, nullptr);
  const Expect e = expect(p);
  const bool fits = e.ok && e.txm <= max_tile && e.tym <= max_tile;
  CHECK((r == 0) == fits, "partition %dx%d / %dx%d ov %d: code %d, expected %s", p.nx, p.ny, p.sx, p.sy,
        p.overlap, r, fits ? "ok" : "EINVAL");
  if (r != 0) {
    CHECK(r == RSP_EINVAL, "partition error code %d", r);
    CHECK(std::strlen(rsp_last_error()) > 0, "no error message");
    return;
  }
  CHECK(S == p.sx * p.sy && txm == e.txm && tym == e.tym, "S %d txm %d tym %d, expected %d %d %d", S, txm, tym,
        p.sx * p.sy, e.txm, e.tym);
  std::vector<int32_t> boxes(8 * (size_t)S + 8, -7);
  CHECK(rsp_partition(&p, &S, &txm, &tym, boxes.data()) == 0, "second call failed");
  CHECK(boxes[8 * (size_t)S] == -7, "wrote beyond 8 S entries");
  std::vector<int> cover((size_t)p.nx * p.ny, 0);
  for (int s = 0; s < S; ++s) {
    const int32_t* b = &boxes[8 * (size_t)s];
    // overlapping box contains the core, both inside the grid, the box is the core
    // extended by `overlap` and clipped
    CHECK(b[4] < b[5] && b[6] < b[7], "empty core %d", s);
    CHECK(b[0] == std::max(0, b[4] - p.overlap) && b[1] == std::min(p.nx, b[5] + p.overlap) &&
              b[2] == std::max(0, b[6] - p.overlap) && b[3] == std::min(p.ny, b[7] + p.overlap),
          "box %d is not the clipped extension of its core", s);
    CHECK(b[1] - b[0] <= txm && b[3] - b[2] <= tym, "box %d wider than the reported tile", s);
    for (int y = b[6]; y < b[7]; ++y)
      for (int x = b[4]; x < b[5]; ++x) cover[(size_t)y * p.nx + x] += 1;
  }
  int bad = 0;
  for (int v : cover) bad += v != 1;
  CHECK(bad == 0, "%d nodes not covered exactly once by the cores", bad);
}

void partitions(std::mt19937& rng) {
  // the supported tile: the widest overlapping box rsp_partition accepts
  int max_tile = 0;
  for (int w = 1; w <= 400; ++w) {
    rsp_problem p = problem(w, 1, 1, 1, 0);
    int32_t S, tx, ty;
    if (rsp_partition(&p, &S, &tx, &ty, nullptr) == 0) max_tile = w;
  }
  CHECK(max_tile >= 40, "largest accepted tile %d", max_tile);
  const int fixed[][5] = {{511, 511, 16, 16, 4}, {255, 255, 8, 8, 4}, {63, 63, 2, 2, 2}, {1, 1, 1, 1, 0},
                          {7, 5, 7, 5, 0},       {10, 10, 4, 4, 1},   {37, 29, 3, 4, 3}, {450, 450, 15, 15, 3}};
  for (const auto& f : fixed) check_partition(problem(f[0], f[1], f[2], f[3], f[4]), max_tile);
  std::uniform_int_distribution<int> n(1, 700), ov(0, 12);
  for (int it = 0; it < 400; ++it) {
    const int nx = n(rng), ny = n(rng);
    std::uniform_int_distribution<int> sx(1, std::min(nx + 2, 40)), sy(1, std::min(ny + 2, 40));
    check_partition(problem(nx, ny, sx(rng), sy(rng), ov(rng)), max_tile);
  }
  // degenerate arguments
  rsp_problem p = problem(37, 29, 3, 4, 3);
  int32_t S, tx, ty;
  CHECK(rsp_partition(nullptr, &S, &tx, &ty, nullptr) == RSP_EINVAL, "NULL problem accepted");
  for (int v : {0, -1}) {
    rsp_problem q = p;
    q.nx = v;
    CHECK(rsp_partition(&q, &S, &tx, &ty, nullptr) == RSP_EINVAL, "nx %d accepted", v);
    q = p;
    q.sy = v;
    CHECK(rsp_partition(&q, &S, &tx, &ty, nullptr) == RSP_EINVAL, "sy %d accepted", v);
  }
  rsp_problem q = p;
  q.overlap = -1;
  CHECK(rsp_partition(&q, &S, &tx, &ty, nullptr) == RSP_EINVAL, "negative overlap accepted");
}

void workspace(std::mt19937& rng) {
  const rsp_options o = options();
  // invalid problems and options lay out nothing
  rsp_problem p = problem(63, 63, 2, 2, 2);
  CHECK(rsp_workspace_bytes(&p, &o) > 0, "valid problem not laid out");
  CHECK(rsp_workspace_bytes(nullptr, &o) == 0 && rsp_workspace_bytes(&p, nullptr) == 0, "NULL laid out");
  const double bad_reals[] = {0.0, -1.0, std::nan("")};
  for (double v : bad_reals) {
    rsp_problem q = p;
    q.nu = v;
    CHECK(rsp_workspace_bytes(&q, &o) == 0, "nu %g laid out", v);
  }
  {
    rsp_problem q = p;
    q.eps_min = 2.0;
    CHECK(rsp_workspace_bytes(&q, &o) == 0, "eps_min > eps0 laid out");
    q = p;
    q.gamma = 1.0;
    CHECK(rsp_workspace_bytes(&q, &o) == 0, "gamma 1 laid out");
    q = p;
    q.phi_kind = 99;
    CHECK(rsp_workspace_bytes(&q, &o) == 0, "unknown phi laid out");
  }
  std::uniform_int_distribution<int> n(8, 600), ov(0, 6), rs(1, 64), coin(0, 1);
  for (int it = 0; it < 200; ++it) {
    const int nx = n(rng), ny = n(rng);
    rsp_problem q = problem(nx, ny, std::max(1, (nx + 31) / 32), std::max(1, (ny + 31) / 32), ov(rng));
    rsp_options a = o;
    a.gmres_restart = rs(rng);
    a.coarse = coin(rng);
    const size_t b64 = rsp_workspace_bytes(&q, &a);
    a.precision = RSP_FP32_REFINED;
    const size_t b32 = rsp_workspace_bytes(&q, &a);
    int32_t S, tx, ty;
    const bool ok = rsp_partition(&q, &S, &tx, &ty, nullptr) == 0;
    CHECK((b64 > 0) == ok && (b32 > 0) == ok, "laid out %zu / %zu, partition %d", b64, b32, (int)ok);
    if (!ok) continue;
    CHECK(b32 < b64, "FP32 factors (%zu bytes) not smaller than FP64 (%zu)", b32, b64);
    // a batch of one is the single layout; a batch holds at least its largest member
    rsp_problem qs[3] = {q, problem(63, 63, 2, 2, 2), problem(37, 29, 3, 4, 3)};
    CHECK(rsp_batch_workspace_bytes(1, qs, &a) == b32, "batch of one differs");
    const size_t b3 = rsp_batch_workspace_bytes(3, qs, &a);
    CHECK(b3 >= b32 && b3 >= rsp_workspace_bytes(&qs[1], &a), "batch smaller than a member");
  }
  rsp_problem qs[2] = {p, p};
  qs[1].nx = 0;
  CHECK(rsp_batch_workspace_bytes(2, qs, &o) == 0, "batch with an invalid member laid out");
  CHECK(rsp_batch_workspace_bytes(0, qs, &o) == 0 && rsp_batch_workspace_bytes(-3, qs, &o) == 0,
        "empty batch laid out");
}

// Calls that need a device: argument checks first, then the missing device reported as
// an error (this program runs where there is no GPU).
void device_calls() {
  rsp_problem p = problem(37, 29, 3, 4, 3);
  rsp_options o = options();
  rsp_context* ctx = reinterpret_cast<rsp_context*>(0x1);
  CHECK(rsp_context_create(nullptr, 0, 0) == RSP_EINVAL, "NULL context pointer accepted");
  const int r = rsp_context_create(&ctx, 0, 0);
  CHECK(r < 0 && ctx == reinterpret_cast<rsp_context*>(0x1), "context created without a device (%d)", r);
  CHECK(rsp_context_create(&ctx, -1, 0) < 0, "device -1 accepted");
  CHECK(rsp_context_destroy(nullptr) == 0, "destroying NULL failed");
  double y = 0, pp = 0, u = 0;
  rsp_history h;
  CHECK(rsp_solve(nullptr, &p, &o, &y, nullptr, nullptr, nullptr, &y, &pp, &u, &h, nullptr) == RSP_EINVAL,
        "solve without a context accepted");
  CHECK(rsp_setup(nullptr, &p, &o, &y, nullptr, nullptr) == RSP_EINVAL, "setup without a context accepted");
  // options are validated before any device is touched
  rsp_server_options so;
  std::memset(&so, 0, sizeof so);
  so.opts = o;
  so.opts.gmres_restart = 0;
  rsp_server* srv = nullptr;
  CHECK(rsp_server_create(&srv, &so) == RSP_EINVAL && srv == nullptr, "restart 0 accepted");
  so.opts = o;
  so.opts.precision = 7;
  CHECK(rsp_server_create(&srv, &so) == RSP_EINVAL, "precision 7 accepted");
  so.opts = o;
  so.opts.tol_outer = std::nan("");
  CHECK(rsp_server_create(&srv, &so) == RSP_EINVAL, "NaN tolerance accepted");
  so.opts = o;
  so.opts.coarse = 2;
  CHECK(rsp_server_create(&srv, &so) == RSP_EINVAL, "coarse 2 accepted");
  so.opts = o;
  so.max_batch = -1;
  CHECK(rsp_server_create(&srv, &so) == RSP_EINVAL, "max_batch -1 accepted");
  so.max_batch = 0;
  CHECK(rsp_server_create(&srv, &so) < 0 && srv == nullptr, "server created without a device");
  // the allocation-free residual checks its arguments before any device call
  double dummy[4] = {0, 0, 0, 0};
  CHECK(rsp_local_residual_noalloc(nullptr, dummy, dummy, dummy, dummy, 1.0, dummy, dummy, nullptr) == RSP_EINVAL,
        "NULL problem accepted");
  CHECK(rsp_local_residual_noalloc(&p, nullptr, dummy, dummy, dummy, 1.0, dummy, dummy, nullptr) == RSP_EINVAL,
        "NULL yd accepted");
  CHECK(rsp_local_residual_noalloc(&p, dummy, dummy, dummy, dummy, -1.0, dummy, dummy, nullptr) == RSP_EINVAL,
        "negative eps accepted");
  rsp_problem wide = problem(4000, 29, 1, 4, 3);
  CHECK(rsp_local_residual_noalloc(&wide, dummy, dummy, dummy, dummy, 1.0, dummy, dummy, nullptr) == RSP_EINVAL,
        "a tile wider than supported accepted");
}

// rsp_last_error is per thread.
void error_messages() {
  rsp_problem p = problem(37, 29, 3, 4, 3);
  p.nx = 0;
  int32_t S, tx, ty;
  CHECK(rsp_partition(&p, &S, &tx, &ty, nullptr) == RSP_EINVAL, "nx 0 accepted");
  const std::string mine = rsp_last_error();
  std::string other = "unset";
  std::thread t([&] {
    other = rsp_last_error();
    rsp_problem q = problem(37, 29, 3, 4, -5);
    (void)rsp_partition(&q, &S, &tx, &ty, nullptr);
  });
  t.join();
  CHECK(!mine.empty() && other.empty(), "error message shared between threads ('%s', '%s')", mine.c_str(),
        other.c_str());
  CHECK(mine == rsp_last_error(), "another thread changed this thread's message");
  CHECK(rsp_version() > 0, "version %d", rsp_version());
}

}  // namespace

int main() {
  std::mt19937 rng(20241101);
  partitions(rng);
  workspace(rng);
  device_calls();
  error_messages();
  std::printf("host_check: %d checks, %d failed\n", g_checks, g_fail);
  return g_fail == 0 ? 0 : 1;
}
