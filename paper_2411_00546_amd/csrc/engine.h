// Internal interface of the batch engine (raspen.cpp), shared with the serving
// loop (server.cpp).  A batch is a set of problem instances solved together: every
// launch of the hot path covers the subdomains of all of them (Algorithm 3 and 4
// kernels over a work list of items), and each instance runs its own Algorithm 2
// iteration (stopping test, GMRES, update) in lockstep with the others.
#pragma once
#include <chrono>
#include <cstdint>
#include <vector>

#include "raspen.h"
#include "rsp_kernels.h"

namespace rsp {

using Clock = std::chrono::steady_clock;

// Records `fmt` as the thread's last error and returns `code`.
int fail(int code, const char* fmt, ...);

struct Partition {
  int S = 0, txm = 0, tym = 0, sx = 0, sy = 0;
  std::vector<int4> box, core;   // (x0, x1, y0, y1) half-open
};

int validate_options(const rsp_options* o);
int validate_problem(const rsp_problem* p);
int make_partition(const rsp_problem* p, Partition* out);
// Padded line-block size of tiles up to txm wide: a multiple of 16 above 2 txm.
int line_block(int txm);
// Constants of an instance in the form the kernels read them (its arrays at offset
// noff; the batch's S, txm, tym and line-block size M).
DevProblem dev_problem(const rsp_problem& p, long long noff, int S, int txm, int tym, int M);

// One problem instance of a batch and its Algorithm 2 state.
struct Inst {
  rsp_problem prob{};
  Partition part;
  size_t n = 0;                                                            // nx ny
  const double *yd = nullptr, *f = nullptr, *y0 = nullptr, *p0 = nullptr;  // caller's inputs
  double *y = nullptr, *p = nullptr, *u = nullptr;                        // caller's outputs
  int slot = -1;          // instance index in the current layout
  long long noff = 0;     // offset of its [ny][nx] arrays in the batch arrays
  long long coff = -1;    // offset of its coefficient arrays of A (-1: A = -Laplacian)
  int sub0 = 0;           // its first item
  bool placed = false;    // x, y_d and f are in the current layout
  bool started = false;   // first evaluation done
  bool finished = false;  // outputs written, history complete
  int k = 0, status = 0, gm_used = 0, restarts = 0;
  bool gm_stagnated = false;   // some GMRES solve stopped at max_gmres above its tolerance
  double Fn = 0, thr = 0, gm_rel = 0;
  rsp_history hist{};
  int64_t n_factor = 0, n_solve = 0, n_gmres = 0, n_newton = 0, n_apply = 0;
  double flops = 0, ms_eval = 0, ms_gmres = 0;
  Clock::time_point t0;
  // FP32 -> FP64 fallback (rsp_options.fallback_rho)
  double Fn_prev = 0;        // |F(x^(k-1))|
  bool parked = false;       // left its FP32 layout; x^k saved in y, p (y0, p0 point there)
  int fallback_outer = -1;   // outer step k at the switch
  int k_base = 0;            // outer steps done before the current max_outer budget
  // snapshots x^0 + sum_i P~_i c_i^(k) of the first evaluation (rsp_solve)
  double* snap = nullptr;    // device [snap_max][2][ny][nx]
  int snap_max = 0;
};

// Validates the problem, partitions it and resets the solve state.
int inst_init(Inst* in, const rsp_problem* prob);
// Device bytes of a layout holding these problems (0 if one is invalid).
size_t batch_bytes(const rsp_problem* const* probs, int count, const rsp_options& o);
// Lays out `live` in the context's memory: instances already placed keep their
// state (x, y_d, f move to the new layout), new ones load their inputs.
int engine_place(rsp_context* ctx, const rsp_options& o, const std::vector<Inst*>& live,
                 hipStream_t st);
// One Algorithm 2 iteration for every unfinished instance of `live`: evaluation
// of F (Algorithm 3; continuation as the options say), the stopping test, and for
// those that go on GMRES on the Newton system (Algorithm 4 products) and the
// update.  Instances that stop get their outputs and history and are marked
// finished (their outputs are complete on return); the update of the others may
// still be running on the stream.
int engine_step(rsp_context* ctx, const std::vector<Inst*>& live, hipStream_t st);
// With FP32 line factors, an instance whose evaluation shows that they are not good
// enough (rsp_options.fallback_rho) is parked instead of going on: its iterate is
// copied into its outputs y, p (stream-ordered) and it becomes an unplaced instance
// that starts from there.  The caller lays parked instances out again with FP64
// factors (fallback_options) and steps them to the end.
rsp_options fallback_options(const rsp_options& o);

}  // namespace rsp
