// rsp_local_residual_noalloc: the local residuals K_i(c_i) of every subdomain of one
// problem (the same kernels and results as rsp_local_residual) without a context and
// without any device allocation.  Its staging buffers (the instance's constants, the
// subdomain boxes and the halo tiles of R_i x) live in a file-scope device array of
// kScratchBytes (with variable coefficients of A also their scaled copies).  The array's
// device address is resolved once per device
// (hipGetSymbolAddress) and only that address is passed to kernels and copies.
#include <algorithm>
#include <mutex>

#include "engine.h"

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // scratch's address on each device (null: not resolved)

// The instance's constants and the partition of Section 4.2: s boxes of width
// ceil(n / s) per direction, [j B, min((j + 1) B, n)), each extended by `overlap` nodes
// per side and clipped to the grid; subdomains numbered row-major, x fastest.
__global__ void k_noalloc_tables(rsp::DevProblem P, int sx, int sy, int overlap, rsp::DevProblem* prob,
                                 int4* box, int4* core, int* inst) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s == 0) *prob = P;
  if (s >= sx * sy) return;
  const int jx = s % sx, jy = s / sx;
  const int Bx = (P.nx + sx - 1) / sx, By = (P.ny + sy - 1) / sy;
  const int4 c = make_int4(jx * Bx, min((jx + 1) * Bx, P.nx), jy * By, min((jy + 1) * By, P.ny));
  core[s] = c;
  box[s] = make_int4(max(0, c.x - overlap), min(P.nx, c.y + overlap), max(0, c.z - overlap),
                     min(P.ny, c.w + overlap));
  inst[s] = 0;
}

// Largest overlapping tile extent along one direction; -1 when a box would be empty.
int tile_extent(int n, int s, int overlap) {
  if (s < 1 || s > n) return -1;
  const int B = (n + s - 1) / s;
  int w = 0;
  for (int j = 0; j < s; ++j) {
    const int lo = j * B, hi = std::min((j + 1) * B, n);
    if (lo >= hi) return -1;
    w = std::max(w, std::min(n, hi + overlap) - std::max(0, lo - overlap));
  }
  return w;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" int rsp_local_residual_noalloc(const rsp_problem* prob, const double* yd, const double* f,
                                          const double* x, const double* c, double eps, double* out,
                                          double* norms, hipStream_t stream) {
  using rsp::fail;
  int r = rsp::validate_problem(prob);
  if (r < 0) return r;
  if (!yd || !x || !c || !out || !norms) return fail(RSP_EINVAL, "yd, x, c, out and norms are required");
  if (!(eps >= 0)) return fail(RSP_EINVAL, "eps must be >= 0");
  const int txm = tile_extent(prob->nx, prob->sx, prob->overlap);
  const int tym = tile_extent(prob->ny, prob->sy, prob->overlap);
  if (txm < 0 || tym < 0) return fail(RSP_EINVAL, "the partition leaves an empty subdomain");
  if (txm > rsp::kMaxTile || tym > rsp::kMaxTile)
    return fail(RSP_EINVAL, "tile %d x %d exceeds the supported %d nodes", txm, tym, rsp::kMaxTile);
  const int S = prob->sx * prob->sy;
  // staging: constants, boxes, cores, instance indices, halo tiles [S][2][tym+2][txm+2]
  const size_t o_box = align256(sizeof(rsp::DevProblem));
  const size_t o_core = o_box + align256(sizeof(int4) * S);
  const size_t o_inst = o_core + align256(sizeof(int4) * S);
  const size_t o_tile = o_inst + align256(sizeof(int) * S);
  const size_t o_coef = o_tile + align256(sizeof(double) * S * 2 * (size_t)(txm + 2) * (tym + 2));
  const size_t nxf = (size_t)(prob->nx + 1) * prob->ny, nyf = (size_t)prob->nx * (prob->ny + 1);
  const size_t nn = (size_t)prob->nx * prob->ny;
  const size_t need = prob->coef ? o_coef + align256(8 * nxf) + align256(8 * nyf) + 8 * nn : o_coef;
  if (need > kScratchBytes)
    return fail(RSP_EINVAL, "needs %zu bytes of staging, the limit is %zu", need, kScratchBytes);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(RSP_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(RSP_EINVAL, "device %d beyond the supported %d", dev, kMaxDevices);
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) return fail(RSP_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      g_scratch[dev] = p;
    }
    base = static_cast<char*>(g_scratch[dev]);
  }
  rsp::DevProblem* P_d = reinterpret_cast<rsp::DevProblem*>(base);
  int4* box = reinterpret_cast<int4*>(base + o_box);
  int4* core = reinterpret_cast<int4*>(base + o_core);
  int* inst = reinterpret_cast<int*>(base + o_inst);
  double* tilex = reinterpret_cast<double*>(base + o_tile);
  rsp::DevProblem P = rsp::dev_problem(*prob, 0, S, txm, tym, rsp::line_block(txm));
  if (prob->coef) {
    double* cx = reinterpret_cast<double*>(base + o_coef);
    double* cy = reinterpret_cast<double*>(base + o_coef + align256(8 * nxf));
    double* c0 = reinterpret_cast<double*>(base + o_coef + align256(8 * nxf) + align256(8 * nyf));
    rsp::launch_coef_load(P, prob->coef, cx, cy, c0, stream);
    P.cx = cx;
    P.cy = cy;
    P.c0 = c0;
  }
  k_noalloc_tables<<<(S + 255) / 256, 256, 0, stream>>>(P, prob->sx, prob->sy, prob->overlap, P_d, box, core,
                                                         inst);
  rsp::Items I{};
  I.prob = P_d;
  I.inst = inst;
  I.box = box;
  I.core = core;
  I.count = S;
  rsp::launch_restrict_halo(I, x, tilex, stream);
  rsp::launch_local_residual(I, tilex, yd, f, c, eps, out, norms, stream);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(RSP_EHIP, "launch: %s", hipGetErrorString(e));
  return 0;
}
