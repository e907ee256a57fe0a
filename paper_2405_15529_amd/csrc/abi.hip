// abi.hip -- the C-ABI of include/pylom.h: context, options, workspace,
// argument validation, TSQR planning and the launch sequence of each call.
//
// POD / TSVD launch sequence (all on the context stream, no host sync):
//   leaf QR (+ fused mean removal)          Alg. 2, Alg. 1 local qr
//   tree combines, levels h = 1, 2, 4, ...  Alg. 1 reduce phase
//   Jacobi SVD of the root R + truncation   Eq. svdqr2, residual r
//   tree propagation, levels top .. 1       Alg. 1 broadcast phase
//   leaf apply U_i = Q_1i W_i               Eq. svdqr3 / Q_i = Q_1i Q_w
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <tuple>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/pylom.h"
#include "kernels.hpp"

using namespace pylom;

struct pylom_ctx_s {
  int device = -1;  // -1: host-only context (validation and planning only)
  hipStream_t stream = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int64_t block_rows = 0;
  int64_t max_sweeps = 60;
  int64_t ws_cap_mb = 0;
  int64_t blocked_from = 0;  // n at which the column-blocked TSQR takes over (0: automatic)
  int64_t narrow_leaves = 1;  // single-wave 32-row leaves for narrow problems with many leaves
  int64_t mixed_tree = 1;     // mixed column-blocked tree: 1 = FP32 below the final combine
  int64_t mixed_svd_tol = 1;  // mixed first SVD of R: 1 = rotation test at 2^-24, 0 = n 2^-53
  int64_t tree_pipeline = 8;  // column-blocked tree levels as a wavefront over this many lanes
  std::vector<hipEvent_t> tree_ev;  // (level, panel) completion events of that wavefront
  int* status_dev = nullptr;  // Jacobi status pairs (sweeps, barrier timeout) of the last call
  int status_valid = 0;
  int status_pairs = 1;        // 2 after a mixed-precision call (SVD of R + Gram eigen)
  int64_t timing = 0;         // number of per-call event slots (0 = off)
  std::vector<hipEvent_t> ev;  // timing x kEvPerSlot events
  std::vector<char> ev_mixed;  // per slot: recorded by a mixed-precision call
  int64_t ev_calls = 0;        // timed calls since the last read
  std::string last_error;
  // batched execution
  int ncu = 256;                 // compute units of the device
  int64_t streams = 4;           // concurrent streams of pylom_pod_batched
  std::vector<hipStream_t> lanes;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  hipStream_t cap = nullptr;     // origin stream of graph capture and replay
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // captured batches: key -> (graph, last use); at most kMaxGraphs are kept,
  // the least recently used is destroyed first
  std::unordered_map<uint64_t, std::pair<hipGraphExec_t, uint64_t>> graphs;
  uint64_t graph_clock = 0;
  // ordering of the multi-workgroup Jacobi launches of a batch across lanes
  // when their workgroups could not all be resident together
  std::vector<hipEvent_t> jac_ev;
  int64_t last_jac_chain = 0;  // whether the last batched call chained them
  // per-kernel timing (option "kernel_timing"): an event pair around every
  // launch of the single-problem calls, summed by role in pylom_kernel_times
  // out-of-core calls: copy streams and pinned host staging (two buffers each
  // way), grown on demand, freed with the context
  hipStream_t cs_in = nullptr, cs_out = nullptr;
  hipEvent_t ooc_ev[8] = {};
  void* pin_in[2] = {};
  void* pin_out[2] = {};
  size_t pin_bytes = 0;
  int64_t ooc_window_rows = 0;     // option "ooc_window_rows" (0: automatic)
  // option "work_queue": the TSQR phases as work-queue launches.  Switched
  // off: the queue launch of a stacked POD did not complete on the GPU (two
  // runs, the second after its spin loop was changed), with no cause found;
  // the option refuses 1 until one is.
  int64_t work_queue = 0;
  // measured leaf heights (pylom_autotune / pylom_tune_load): key -> (rows, ms)
  std::map<std::tuple<int, int, int, int64_t>, std::pair<int64_t, double>> tuned;
  int64_t ktiming = 0;
  bool kt_off = false;             // set while a batch is enqueued or captured
  std::vector<hipEvent_t> kev;     // event pool; pairs (start, end)
  size_t kev_next = 0;             // events used since the last read
  std::vector<std::pair<int, size_t>> kmarks;  // (role, start event index)
};

// Kernel roles of pylom_kernel_times (include/pylom.h lists them).
enum KernelRole {
  KR_WORK = 0,       // working copy of D (mean removal, type conversion)
  KR_LEAF_PANEL,     // leaf panel QRs (column-blocked)
  KR_LEAF_TRAIL,     // leaf trailing updates (column-blocked)
  KR_TREE_PANEL,     // tree panel QRs (column-blocked)
  KR_TREE_TRAIL,     // tree trailing updates (column-blocked)
  KR_SVD,            // SVD of R: Jacobi set-up, sweeps, finalize, truncation
  KR_PROPAGATE,      // down-tree propagation
  KR_LEAF_APPLY,     // U = Q [W; 0] per leaf, and U out
  KR_REFINE,         // mixed refinement: projection, Gram, eigenpairs, spectrum
  KR_FORM_U,         // mixed refinement: U = Z M
  KR_STACKED_LEAF,   // stacked leaf QR (with fused mean removal)
  KR_STACKED_TREE,   // stacked tree combines
  KR_COUNT
};
constexpr size_t kMaxKernelEvents = (size_t)1 << 16;

static int64_t kt_begin(pylom_ctx c, hipStream_t st) {
  if (!c->ktiming || c->kt_off || c->kev_next + 2 > kMaxKernelEvents) return -1;
  while (c->kev.size() < c->kev_next + 2) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      return -1;
    }
    c->kev.push_back(e);
  }
  const size_t t = c->kev_next;
  if (hipEventRecord(c->kev[t], st) != hipSuccess) {
    (void)hipGetLastError();
    return -1;
  }
  c->kev_next += 2;
  return (int64_t)t;
}
static void kt_end(pylom_ctx c, hipStream_t st, int64_t t, int role) {
  if (t < 0) return;
  if (hipEventRecord(c->kev[(size_t)t + 1], st) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  c->kmarks.emplace_back(role, (size_t)t);
}
// One launch under the kernel timer (stream `st` in scope).
#define KT(role, launch, where)                     \
  do {                                              \
    const int64_t _kt = kt_begin(c, st);            \
    HIPCHK(c, (launch), where);                     \
    kt_end(c, st, _kt, (role));                     \
  } while (0)

static void drop_graphs(pylom_ctx c) {
  for (auto& kv : c->graphs) hipGraphExecDestroy(kv.second.first);
  c->graphs.clear();
}

constexpr size_t kMaxGraphs = 16;  // captured batch graphs kept per context

static void evict_graphs(pylom_ctx c) {
  while (c->graphs.size() >= kMaxGraphs) {
    auto old = c->graphs.begin();
    for (auto it = c->graphs.begin(); it != c->graphs.end(); ++it)
      if (it->second.second < old->second.second) old = it;
    hipGraphExecDestroy(old->second.first);
    c->graphs.erase(old);
  }
}

static int fail(pylom_ctx c, int code, const char* msg) {
  if (c) c->last_error = msg;
  return code;
}

static int hip_fail(pylom_ctx c, hipError_t e, const char* where) {
  if (c) {
    c->last_error = std::string(where) + ": " + hipGetErrorString(e);
  }
  return PYLOM_EHIP;
}

#define HIPCHK(ctx, expr, where)                   \
  do {                                             \
    hipError_t _e = (expr);                        \
    if (_e != hipSuccess) return hip_fail(ctx, _e, where); \
  } while (0)

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kEvPerSlot = 8;  // timing events recorded per call
constexpr int64_t kMaxN = 2048;  // widest snapshot count the kernels take
constexpr int64_t kPW = 64;      // panel width of the column-blocked TSQR
constexpr int64_t kZcap = 1024;  // refinement width planned for the blocked mixed path
constexpr int64_t kTF = 256;     // elements of one 16 x 16 compact-WY T factor
constexpr int kPhases = 6;     // phases reported by pylom_phase_times

// ---------------------------------------------------------------------------
// fixed device scratch of the allocation-free entry point
// ---------------------------------------------------------------------------
// The split-K partial sums of pylom_matmul_noalloc live in this array, one
// copy per device, held until the process ends.  In host code its name is
// only a stand-in for the symbol: its device address is taken once per
// device, with that device current, at context creation (scratch_ptr[]),
// and only that address is ever handed to kernels.
constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];
static void* scratch_ptr[kMaxDevices] = {};
static std::mutex scratch_mu;

// With `device` current: the device address of its scratch copy.
static hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  scratch_ptr[device] = ptr;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" int pylom_create(pylom_ctx* out, int device) {
  if (!out) return PYLOM_EINVAL;
  *out = nullptr;
  pylom_ctx c = new pylom_ctx_s();
  if (device >= 0) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device >= count) {
      delete c;
      return PYLOM_ENODEV;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess ||
        std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
      delete c;
      return PYLOM_ENODEV;
    }
    if (hipSetDevice(device) != hipSuccess) {
      delete c;
      return PYLOM_ENODEV;
    }
    if (hipMalloc((void**)&c->status_dev, 256) != hipSuccess) {
      delete c;
      return PYLOM_ENOMEM;
    }
    if (scratch_setup(device) != hipSuccess) {
      (void)hipGetLastError();
      hipFree(c->status_dev);
      delete c;
      return PYLOM_ENODEV;
    }
    c->device = device;
    if (prop.multiProcessorCount > 0) c->ncu = prop.multiProcessorCount;
  }
  *out = c;
  return PYLOM_OK;
}

extern "C" int pylom_destroy(pylom_ctx c) {
  if (!c) return PYLOM_EINVAL;
  if (c->device >= 0) {
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    drop_graphs(c);
    for (hipStream_t q : c->lanes) hipStreamDestroy(q);
    for (hipEvent_t e : c->ev_join) hipEventDestroy(e);
    for (hipEvent_t e : c->jac_ev) hipEventDestroy(e);
    for (hipEvent_t e : c->tree_ev) hipEventDestroy(e);
    for (hipEvent_t e : c->kev) hipEventDestroy(e);
    for (hipEvent_t e : c->ooc_ev)
      if (e) hipEventDestroy(e);
    if (c->cs_in) hipStreamDestroy(c->cs_in);
    if (c->cs_out) hipStreamDestroy(c->cs_out);
    for (int k = 0; k < 2; ++k) {
      if (c->pin_in[k]) hipHostFree(c->pin_in[k]);
      if (c->pin_out[k]) hipHostFree(c->pin_out[k]);
    }
    if (c->ev_fork) hipEventDestroy(c->ev_fork);
    if (c->ev_in) hipEventDestroy(c->ev_in);
    if (c->ev_out) hipEventDestroy(c->ev_out);
    if (c->cap) hipStreamDestroy(c->cap);
    if (c->ws) hipFree(c->ws);
    if (c->status_dev) hipFree(c->status_dev);
    for (hipEvent_t e : c->ev)
      if (e) hipEventDestroy(e);
  }
  delete c;
  return PYLOM_OK;
}

extern "C" int pylom_set_stream(pylom_ctx c, void* s) {
  if (!c) return PYLOM_EINVAL;
  c->stream = (hipStream_t)s;
  return PYLOM_OK;
}

extern "C" int pylom_set_option(pylom_ctx c, const char* key, int64_t v) {
  if (!c || !key) return PYLOM_EINVAL;
  if (!std::strcmp(key, "block_rows")) {
    if (v < 0) return fail(c, PYLOM_EINVAL, "block_rows must be >= 0");
    c->block_rows = v;
  } else if (!std::strcmp(key, "max_sweeps")) {
    if (v < 0 || v > 1000) return fail(c, PYLOM_EINVAL, "max_sweeps must be in [0, 1000]");
    c->max_sweeps = v;
  } else if (!std::strcmp(key, "ws_cap_mb")) {
    if (v < 0) return fail(c, PYLOM_EINVAL, "ws_cap_mb must be >= 0");
    c->ws_cap_mb = v;
  } else if (!std::strcmp(key, "narrow_leaves")) {
    if (v != 0 && v != 1) return fail(c, PYLOM_EINVAL, "narrow_leaves must be 0 or 1");
    c->narrow_leaves = v;  // part of every batch graph key
  } else if (!std::strcmp(key, "blocked_from")) {
    if (v != 0 && (v < 2 || v > kMaxN + 1))
      return fail(c, PYLOM_EINVAL, "blocked_from must be 0 or in [2, 2049]");
    c->blocked_from = v;  // part of every batch graph key
  } else if (!std::strcmp(key, "mixed_tree")) {
    if (v != 0 && v != 1) return fail(c, PYLOM_EINVAL, "mixed_tree must be 0 or 1");
    c->mixed_tree = v;  // part of every batch graph key
  } else if (!std::strcmp(key, "tree_pipeline")) {
    if (v < 0 || v > 16) return fail(c, PYLOM_EINVAL, "tree_pipeline must be in [0, 16]");
    c->tree_pipeline = v;
  } else if (!std::strcmp(key, "mixed_svd_tol")) {
    if (v != 0 && v != 1) return fail(c, PYLOM_EINVAL, "mixed_svd_tol must be 0 or 1");
    c->mixed_svd_tol = v;  // part of every batch graph key
  } else if (!std::strcmp(key, "streams")) {
    if (v < 1 || v > 16) return fail(c, PYLOM_EINVAL, "streams must be in [1, 16]");
    c->streams = v;
  } else if (!std::strcmp(key, "work_queue")) {
    if (v != 0 && v != 1) return fail(c, PYLOM_EINVAL, "work_queue must be 0 or 1");
    if (v == 1)
      return fail(c, PYLOM_ENOTSUP,
                  "work_queue is switched off: its launch did not complete on the GPU");
    c->work_queue = v;
    drop_graphs(c);
  } else if (!std::strcmp(key, "ooc_window_rows")) {
    if (v < 0) return fail(c, PYLOM_EINVAL, "ooc_window_rows must be >= 0");
    c->ooc_window_rows = v;
  } else if (!std::strcmp(key, "kernel_timing")) {
    if (v != 0 && v != 1) return fail(c, PYLOM_EINVAL, "kernel_timing must be 0 or 1");
    c->ktiming = v;
    c->kev_next = 0;
    c->kmarks.clear();
  } else if (!std::strcmp(key, "timing")) {
    if (v < 0 || v > 4096) return fail(c, PYLOM_EINVAL, "timing must be in [0, 4096]");
    if (c->device >= 0) {
      hipSetDevice(c->device);
      hipStreamSynchronize(c->stream);
      for (hipEvent_t e : c->ev)
        if (e) hipEventDestroy(e);
      c->ev.assign((size_t)v * kEvPerSlot, nullptr);
      c->ev_mixed.assign((size_t)v, 0);
      for (auto& e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) return fail(c, PYLOM_EHIP, "hipEventCreate");
    }
    c->timing = v;
    c->ev_calls = 0;
  } else {
    return fail(c, PYLOM_EINVAL, "unknown option");
  }
  return PYLOM_OK;
}

extern "C" int pylom_get_option(pylom_ctx c, const char* key, int64_t* v) {
  if (!c || !key || !v) return PYLOM_EINVAL;
  if (!std::strcmp(key, "block_rows"))
    *v = c->block_rows;
  else if (!std::strcmp(key, "max_sweeps"))
    *v = c->max_sweeps;
  else if (!std::strcmp(key, "ws_cap_mb"))
    *v = c->ws_cap_mb;
  else if (!std::strcmp(key, "blocked_from"))
    *v = c->blocked_from;
  else if (!std::strcmp(key, "narrow_leaves"))
    *v = c->narrow_leaves;
  else if (!std::strcmp(key, "mixed_tree"))
    *v = c->mixed_tree;
  else if (!std::strcmp(key, "mixed_svd_tol"))
    *v = c->mixed_svd_tol;
  else if (!std::strcmp(key, "tree_pipeline"))
    *v = c->tree_pipeline;
  else if (!std::strcmp(key, "timing"))
    *v = c->timing;
  else if (!std::strcmp(key, "streams"))
    *v = c->streams;
  else if (!std::strcmp(key, "kernel_timing"))
    *v = c->ktiming;
  else if (!std::strcmp(key, "ooc_window_rows"))
    *v = c->ooc_window_rows;
  else if (!std::strcmp(key, "work_queue"))
    *v = c->work_queue;
  else if (!std::strcmp(key, "batch_jacobi_chained"))
    *v = c->last_jac_chain;
  else
    return fail(c, PYLOM_EINVAL, "unknown option");
  return PYLOM_OK;
}

extern "C" const char* pylom_strerror(int s) {
  switch (s) {
    case PYLOM_OK: return "success";
    case PYLOM_EINVAL: return "invalid argument";
    case PYLOM_ESHAPE: return "invalid shape or leading dimension";
    case PYLOM_EDTYPE: return "unsupported dtype / precision";
    case PYLOM_ENOMEM: return "workspace allocation failed or over the cap";
    case PYLOM_EHIP: return "HIP runtime error";
    case PYLOM_ENOTSUP: return "shape not supported by the kernels";
    case PYLOM_ENODEV: return "no usable gfx950 device";
    case PYLOM_WNOCONV: return "Jacobi SVD did not converge within max_sweeps";
    case PYLOM_WNONFINITE: return "a singular value is not finite (non-finite input)";
    default: return "unknown status";
  }
}

extern "C" const char* pylom_last_error(pylom_ctx c) {
  if (!c) return "null context";
  return c->last_error.c_str();
}

static int ensure_ws(pylom_ctx c, size_t bytes) {
  if (c->ws_cap_mb > 0 && bytes > (size_t)c->ws_cap_mb * (1u << 20))
    return fail(c, PYLOM_ENOMEM, "workspace over ws_cap_mb");
  if (bytes <= c->ws_bytes) return PYLOM_OK;
  if (c->ws) {
    hipStreamSynchronize(c->stream);
    for (hipStream_t q : c->lanes) hipStreamSynchronize(q);
    if (c->cap) hipStreamSynchronize(c->cap);
    drop_graphs(c);  // captured graphs point into the old workspace
    hipFree(c->ws);
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  if (hipMalloc(&c->ws, bytes) != hipSuccess) {
    c->ws = nullptr;
    (void)hipGetLastError();
    return fail(c, PYLOM_ENOMEM, "hipMalloc of the workspace failed");
  }
  c->ws_bytes = bytes;
  return PYLOM_OK;
}

// The workspace cap is checked with the plan, before anything else needs a
// device, so that an over-cap call fails the same way on every context.
static int cap_check(pylom_ctx c, size_t bytes) {
  if (c->ws_cap_mb > 0 && bytes > (size_t)c->ws_cap_mb * (1u << 20))
    return fail(c, PYLOM_ENOMEM, "workspace over ws_cap_mb");
  return PYLOM_OK;
}

extern "C" int pylom_reserve(pylom_ctx c, size_t bytes) {
  if (!c) return PYLOM_EINVAL;
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  hipSetDevice(c->device);
  return ensure_ws(c, bytes);
}

// ---------------------------------------------------------------------------
// planning
// ---------------------------------------------------------------------------
struct Plan {
  int64_t m, n, b, P, last_rows, nch_leaf, nch_tree, levels;
  QrGeom g;
  JacobiPlan jp;
  // workspace offsets (bytes)
  size_t oV, oTleaf, oR, oTtree, oW, oMean, oSig, oSvd, total;
  // work-queue counters of the stacked FP64 sequence (reduce, broadcast)
  size_t oQ1 = 0, oQ2 = 0, q1_bytes = 0, q2_bytes = 0;
  // mixed precision only: FP32 leaf R, first SVD, refinement buffers
  bool mixed;
  size_t oR32, oS0, oVT0, oNr0, oZ, oG, oPart, oLam, oWT, oUR2, oNr2, oM, oSvd2;
  size_t part_bytes;
  int64_t zcap;  // widest refinement subspace the workspace holds
  // column-blocked TSQR (wide problems): panels of kPW columns
  bool blocked;
  int64_t K, nch_l, nch_p, wcap;
  QrGeom gp, gpl;  // geometry of a full panel and of the last panel
  size_t oWk, oTl, oPSl, oTp, oPSp, oXu;
};

static int64_t level_pairs(int64_t P, int64_t h) { return (P - h + 2 * h - 1) / (2 * h); }

// Leaf height model.  The stacked QR of a leaf is a chain of ceil(b / s)
// chunks; each chunk factors n columns one after another (about 1.6k cycles
// of latency per column on one wave) plus one look-ahead tile per panel
// (about 5k cycles).  Leaves run one workgroup per CU, in waves over the
// device.  Tree level h holds level_pairs(P, h) combines, one workgroup each,
// so it too runs in waves over the device; one combine costs about half a
// chunk chain for each of its ceil(n / s) chunks, and every launch costs
// about 20k cycles.
// Whether a stacked plan of P leaves uses the narrow-leaf geometry: 32-row
// chunks in single-wave workgroups (3-6 panels, up to 8 for the FP32 leaves
// of the mixed path, at least two leaves per CU).  Measured on 3.6e7-row
// problems: 1.6x faster leaves at 3-4 panels; at 6 panels 1.3x (FP64) and
// 1.8x (FP32); at 8 panels 1.7x for FP32 but 16 % slower for FP64, where the
// single wave's serial trailing-tile MFMA work dominates; no gain at 1-2
// panels (already single-wave).
static bool narrow_plan(const pylom_ctx_s* c, int npanels, int64_t P, bool mixed) {
  return c->narrow_leaves && npanels >= 3 && npanels <= (mixed ? 8 : 6) &&
         P >= 2 * (int64_t)c->ncu;
}

static double leaf_model(const pylom_ctx_s* c, int64_t m, int64_t n, int64_t b, bool mixed) {
  QrGeom g;
  if (!qr_geom((int)n, 8, &g)) return 1e300;
  const int ncu = c->ncu;
  const double c_col = 1600.0, c_tile = 5000.0, c_launch = 20000.0;
  const double chain = (double)n * c_col + (double)g.npanels * c_tile;
  int64_t P = m / b;
  if (P < 1) P = 1;
  const int64_t last = m - (P - 1) * b;
  // leaves run in waves over the CUs: one four-wave workgroup per CU, or as
  // many single-wave narrow leaves as LDS holds (at most one per SIMD)
  double slots = (double)ncu;
  if (narrow_plan(c, g.npanels, P, mixed)) {
    g.s = 32;
    const double per_cu = std::floor(160.0 * 1024.0 / (double)qr_lds_bytes(g, 8));
    slots = (double)ncu * std::max(1.0, std::min(4.0, per_cu));
  }
  // every wave but the last holds b-row leaves; the last one holds the
  // remainder leaf too
  const double waves = std::ceil((double)P / slots);
  const double cb = std::ceil((double)b / g.s), cl = std::ceil((double)last / g.s);
  const double t_leaf = ((waves - 1.0) * cb + std::max(cb, cl)) * chain + c_launch;
  const double combine = std::ceil((double)n / g.s) * chain * 0.5;
  double t_tree = 0.0;
  for (int64_t h = 1; h < P; h *= 2)
    t_tree += std::ceil((double)level_pairs(P, h) / slots) * combine + c_launch;
  return t_leaf + t_tree;
}

static int64_t tune_block_rows(const pylom_ctx_s* c, int64_t m, int64_t n, bool mixed = false) {
  int64_t best = 0;
  double tbest = 0.0;
  for (int64_t b = 128; b <= 32768; b *= 2) {
    if (b < n) continue;
    const double t = leaf_model(c, m, n, b, mixed);
    if (best == 0 || t < tbest) {
      best = b;
      tbest = t;
    }
  }
  return best > 0 ? best : n;
}

// Leaf height of the column-blocked path: two leaves per CU (the panel
// factorisations run one workgroup per leaf, two per CU, their panel waves
// on different SIMDs), rows a multiple of the chunk.
static int64_t blocked_block_rows(int64_t m, int64_t n, int ncu) {
  const int64_t slots = 2 * (int64_t)(ncu > 0 ? ncu : 1);
  int64_t b = (m + slots - 1) / slots;
  if (b < n) b = n;
  return (b + kPW - 1) / kPW * kPW;
}

// Which TSQR serves an m x n problem.  An explicit "blocked_from" threshold
// decides alone.  The automatic choice (0) follows measurements of both paths
// on one MI355X: the column-blocked TSQR was 1.1-2x faster for 64 <= n <= 1024
// at up to 4M rows and 2.4x faster at 1.8e7 x 630, while the stacked QR was
// faster at 3.6e7 x 160 (many short leaves keep every CU busy and its
// workspace is smaller).  Instances of a batch follow the same rule.
static bool use_blocked(const pylom_ctx_s* c, int64_t m, int64_t n) {
  if (c->blocked_from > 0) return n >= c->blocked_from;
  return n >= 512 || (n >= 64 && m <= ((int64_t)8 << 20));
}

static int64_t tune_lookup(const pylom_ctx_s* c, bool blocked, bool mixed, int64_t m, int64_t n);

extern "C" int64_t pylom_tune_block_rows(pylom_ctx c, int64_t m, int64_t n) {
  if (!c || n < 1 || m < n || n > kMaxN) return PYLOM_EINVAL;
  const bool blk = use_blocked(c, m, n);
  const int64_t t = tune_lookup(c, blk, false, m, n);
  if (t > 0) return t < n ? n : t;
  if (blk) return blocked_block_rows(m, n, c->ncu);
  return tune_block_rows(c, m, n);
}

static int make_blocked_plan(pylom_ctx c, Plan* p, bool mixed);

// Key of the measured leaf-height table: path (1 = column-blocked), mixed
// precision, floor(log2 m), n rounded up to a multiple of 16.
static std::tuple<int, int, int, int64_t> tune_key(bool blocked, bool mixed, int64_t m,
                                                   int64_t n) {
  int lg = 0;
  while (((int64_t)1 << (lg + 1)) <= m) ++lg;
  return std::make_tuple(blocked ? 1 : 0, mixed ? 1 : 0, lg, (n + 15) / 16 * 16);
}
static int64_t tune_lookup(const pylom_ctx_s* c, bool blocked, bool mixed, int64_t m, int64_t n) {
  auto it = c->tuned.find(tune_key(blocked, mixed, m, n));
  return it == c->tuned.end() ? 0 : it->second.first;
}

static int make_plan(pylom_ctx c, int64_t m, int64_t n, bool store_q, Plan* p,
                     bool mixed = false) {
  if (n < 1 || m < n) return fail(c, PYLOM_ESHAPE, "need m >= n >= 1");
  if (n > kMaxN) return fail(c, PYLOM_ENOTSUP, "n > 2048 is not supported");
  p->mixed = mixed;
  p->blocked = false;
  p->zcap = n;
  if (mixed) store_q = false;
  p->m = m;
  p->n = n;
  if (use_blocked(c, m, n)) return make_blocked_plan(c, p, mixed);
  int64_t b = c->block_rows;
  if (b <= 0) b = tune_lookup(c, false, mixed, m, n);
  if (b <= 0) b = tune_block_rows(c, m, n, mixed);
  if (b < n) b = n;
  int64_t P = m / b;
  if (P < 1) P = 1;
  if (P > (1 << 30)) return fail(c, PYLOM_ENOTSUP, "too many leaves");
  p->b = b;
  p->P = P;
  p->last_rows = m - (P - 1) * b;
  if (!qr_geom((int)n, 8, &p->g)) return fail(c, PYLOM_ENOTSUP, "no chunk geometry");
  if (!jacobi_plan((int)n, &p->jp)) return fail(c, PYLOM_ENOTSUP, "no Jacobi plan");
  // Narrow problems with many leaves: 32-row chunks and single-wave
  // workgroups, so that several leaves share a CU (38 KB of LDS each at
  // n = 64), instead of one four-wave workgroup whose three trailing-tile
  // waves mostly wait on the panel wave (narrow_plan).
  if (narrow_plan(c, p->g.npanels, P, mixed)) {
    p->g.s = 32;
    p->g.nthr = 64;
  }
  const int64_t s = p->g.s, np = p->g.npanels;
  p->nch_leaf = (p->last_rows + s - 1) / s;
  p->nch_tree = (n + s - 1) / s;
  int64_t lv = 0;
  for (int64_t h = 1; h < P; h *= 2) ++lv;
  p->levels = lv;
  size_t off = 0;
  p->oV = off;
  if (store_q) off = align_up(off + sizeof(double) * (size_t)m * n);
  p->oTleaf = off;
  if (store_q) off = align_up(off + sizeof(double) * (size_t)P * p->nch_leaf * np * 256);
  p->oR = off;
  off = align_up(off + sizeof(double) * (size_t)P * n * n);
  p->oTtree = off;
  if (store_q) off = align_up(off + sizeof(double) * (size_t)P * p->nch_tree * np * 256);
  p->oW = off;
  off = align_up(off + sizeof(double) * (size_t)P * n * n);
  p->oMean = off;
  off = align_up(off + sizeof(double) * (size_t)m);
  p->oSig = off;
  off = align_up(off + sizeof(double) * (size_t)n);
  p->oSvd = off;
  off = align_up(off + jacobi_ws_bytes(p->jp, (int)c->max_sweeps));
  if (!mixed) {
    p->q1_bytes = queue_counter_bytes(1, P, 1);
    p->q2_bytes = queue_counter_bytes(1, P, (n + 15) / 16);
    p->oQ1 = off;
    off = align_up(off + p->q1_bytes);
    p->oQ2 = off;
    off = align_up(off + p->q2_bytes);
  }
  if (mixed) {
    // the refinement subspace k (<= n) is known only after the first SVD:
    // size every k-dependent buffer for the largest k
    size_t svd2 = 0, part = 0;
    for (int64_t k = 1; k <= n; ++k) {
      JacobiPlan jk;
      if (!jacobi_plan((int)k, &jk)) return fail(c, PYLOM_ENOTSUP, "no Jacobi plan");
      const size_t wb = jacobi_ws_bytes(jk, (int)c->max_sweeps);
      if (wb > svd2) svd2 = wb;
      const size_t pb = sizeof(double) * (size_t)matmul_tn_splits(m, k, k) * k * k;
      if (pb > part) part = pb;
    }
    p->part_bytes = part;
    p->oR32 = off;
    off = align_up(off + sizeof(float) * (size_t)p->P * n * n);
    p->oS0 = off;
    off = align_up(off + sizeof(double) * (size_t)n);
    p->oVT0 = off;
    off = align_up(off + sizeof(double) * (size_t)n * n);
    p->oNr0 = off;
    off = align_up(off + sizeof(int64_t));
    p->oZ = off;
    off = align_up(off + sizeof(double) * (size_t)m * n);
    p->oG = off;
    off = align_up(off + sizeof(double) * (size_t)n * n);
    p->oPart = off;
    off = align_up(off + part);
    p->oLam = off;
    off = align_up(off + sizeof(double) * (size_t)n);
    p->oWT = off;
    off = align_up(off + sizeof(double) * (size_t)n * n);
    p->oUR2 = off;
    off = align_up(off + sizeof(double) * (size_t)n * n);
    p->oNr2 = off;
    off = align_up(off + sizeof(int64_t));
    p->oM = off;
    off = align_up(off + sizeof(double) * (size_t)n * n);
    p->oSvd2 = off;
    off = align_up(off + svd2);
  }
  p->total = off;
  return PYLOM_OK;
}

// Wide problems (use_blocked): the leaves and the tree combines are
// column-blocked QRs (blocked.hip).  Workspace, in order: the working copy of
// D (compute type), the leaf T factors and panel states (per panel), the
// FP64 R of every leaf (tree state in place; the partner's triangle keeps
// the combine's reflectors), the tree T factors and panel states, the
// propagation W, and for FP64 the column-group buffer of the leaf apply; the
// mixed path adds its refinement buffers (Z for at most kZcap columns).
static int make_blocked_plan(pylom_ctx c, Plan* p, bool mixed) {
  const int64_t m = p->m, n = p->n;
  p->blocked = true;
  int64_t b = c->block_rows;
  if (b <= 0) b = tune_lookup(c, true, mixed, m, n);
  if (b <= 0) b = blocked_block_rows(m, n, c->ncu);
  if (b < n) b = n;
  int64_t P = m / b;
  if (P < 1) P = 1;
  if (P > 65535) return fail(c, PYLOM_ENOTSUP, "too many leaves for the blocked path");
  p->b = b;
  p->P = P;
  p->last_rows = m - (P - 1) * b;
  p->K = (n + kPW - 1) / kPW;
  const int es = mixed ? 4 : 8;
  if (!qr_geom((int)(n < kPW ? n : kPW), es, &p->gp) ||
      !qr_geom((int)(n - (p->K - 1) * kPW), es, &p->gpl) || p->gp.s != kPW || p->gpl.s != kPW)
    return fail(c, PYLOM_ENOTSUP, "no panel geometry");
  QrGeom g8;
  if (!qr_geom((int)(n - (p->K - 1) * kPW), 8, &g8) || g8.s != kPW)
    return fail(c, PYLOM_ENOTSUP, "no panel geometry");
  if (!jacobi_plan((int)n, &p->jp)) return fail(c, PYLOM_ENOTSUP, "no Jacobi plan");
  p->g = p->gp;
  p->nch_l = (p->last_rows + kPW - 1) / kPW;
  p->nch_p = (n + kPW - 1) / kPW;
  p->nch_leaf = p->nch_l;
  p->nch_tree = p->nch_p;
  int64_t lv = 0;
  for (int64_t h = 1; h < P; h *= 2) ++lv;
  p->levels = lv;
  const int64_t np_all = P - 1;
  const size_t tpp = (size_t)kTF;  // one T factor
  p->wcap = n < 256 ? n : 256;
  size_t off = 0;
  p->oV = p->oTleaf = p->oTtree = 0;
  p->oWk = off;
  off = align_up(off + (size_t)es * m * n);
  p->oTl = off;
  off = align_up(off + (size_t)es * p->K * P * p->nch_l * 4 * tpp);
  p->oPSl = off;
  off = align_up(off + (size_t)es * p->K * P * kPW * kPW);
  p->oR = off;
  off = align_up(off + sizeof(double) * (size_t)P * n * n);
  p->oTp = off;
  off = align_up(off + sizeof(double) * (size_t)p->K * np_all * p->nch_p * 4 * tpp);
  p->oPSp = off;
  off = align_up(off + sizeof(double) * (size_t)p->K * np_all * kPW * kPW);
  p->oW = off;
  off = align_up(off + sizeof(double) * (size_t)P * n * n);
  p->oMean = off;
  off = align_up(off + sizeof(double) * (size_t)m);
  p->oSig = off;
  off = align_up(off + sizeof(double) * (size_t)n);
  p->oSvd = off;
  off = align_up(off + jacobi_ws_bytes(p->jp, (int)c->max_sweeps));
  p->oXu = off;
  if (!mixed) {
    p->oXu = off;
    off = align_up(off + sizeof(double) * (size_t)m * p->wcap);
  } else {
    p->zcap = n < kZcap ? n : kZcap;
    size_t svd2 = 0, part = 0;
    for (int64_t k = 1; k <= p->zcap; ++k) {
      JacobiPlan jk;
      if (!jacobi_plan((int)k, &jk)) return fail(c, PYLOM_ENOTSUP, "no Jacobi plan");
      const size_t wb = jacobi_ws_bytes(jk, (int)c->max_sweeps);
      if (wb > svd2) svd2 = wb;
      const size_t pb = sizeof(double) * (size_t)matmul_tn_splits(m, k, k) * k * k;
      if (pb > part) part = pb;
    }
    const int64_t zc = p->zcap;
    p->part_bytes = part;
    p->oR32 = off;
    off = align_up(off + sizeof(float) * (size_t)P * n * n);
    p->oS0 = off;
    off = align_up(off + sizeof(double) * (size_t)n);
    p->oVT0 = off;
    off = align_up(off + sizeof(double) * (size_t)n * n);
    p->oNr0 = off;
    off = align_up(off + sizeof(int64_t));
    p->oZ = off;
    off = align_up(off + sizeof(double) * (size_t)m * zc);
    p->oG = off;
    off = align_up(off + sizeof(double) * (size_t)zc * zc);
    p->oPart = off;
    off = align_up(off + part);
    p->oLam = off;
    off = align_up(off + sizeof(double) * (size_t)zc);
    p->oWT = off;
    off = align_up(off + sizeof(double) * (size_t)zc * zc);
    p->oUR2 = off;
    off = align_up(off + sizeof(double) * (size_t)zc * zc);
    p->oNr2 = off;
    off = align_up(off + sizeof(int64_t));
    p->oM = off;
    off = align_up(off + sizeof(double) * (size_t)zc * zc);
    p->oSvd2 = off;
    off = align_up(off + svd2);
  }
  p->total = off;
  return PYLOM_OK;
}

extern "C" int pylom_workspace_query(pylom_ctx c, pylom_dtype dtype, pylom_prec prec, int64_t m,
                                     int64_t n, size_t* bytes) {
  if (!c || !bytes) return PYLOM_EINVAL;
  if (dtype != PYLOM_R64 && dtype != PYLOM_R32) return fail(c, PYLOM_EDTYPE, "dtype");
  if (prec != PYLOM_FP64 && prec != PYLOM_MIXED) return fail(c, PYLOM_EDTYPE, "precision");
  Plan p;
  int rc = make_plan(c, m, n, true, &p, prec == PYLOM_MIXED);
  if (rc) return rc;
  *bytes = p.total;
  return PYLOM_OK;
}

extern "C" int pylom_plan_query(pylom_ctx c, int64_t m, int64_t n, int64_t* leaves,
                                int64_t* block_rows, int64_t* chunk_rows, int64_t* levels) {
  if (!c) return PYLOM_EINVAL;
  Plan p;
  int rc = make_plan(c, m, n, true, &p);
  if (rc) return rc;
  if (leaves) *leaves = p.P;
  if (block_rows) *block_rows = p.b;
  if (chunk_rows) *chunk_rows = p.g.s;
  if (levels) *levels = p.levels;
  return PYLOM_OK;
}

extern "C" int64_t pylom_tree_plan(int64_t P, int64_t* out, int64_t cap) {
  if (P < 1 || (cap > 0 && !out)) return PYLOM_EINVAL;
  int64_t k = 0, level = 0;
  for (int64_t h = 1; h < P; h *= 2, ++level) {
    for (int64_t j = 0; j + h < P; j += 2 * h) {
      if (k < cap) {
        out[3 * k + 0] = level;
        out[3 * k + 1] = j;
        out[3 * k + 2] = j + h;
      }
      ++k;
    }
  }
  return k;
}

// ---------------------------------------------------------------------------
// shared TSQR-SVD sequence
// ---------------------------------------------------------------------------
static int check_common(pylom_ctx c, pylom_dtype dtype, pylom_prec prec) {
  if (!c) return PYLOM_EINVAL;
  if (dtype != PYLOM_R64 && dtype != PYLOM_R32) return fail(c, PYLOM_EDTYPE, "dtype must be R64 or R32");
  if (prec != PYLOM_FP64 && prec != PYLOM_MIXED) return fail(c, PYLOM_EDTYPE, "unknown precision");
  return PYLOM_OK;
}

// ---------------------------------------------------------------------------
// launch sequences, parameterised by stream / workspace / status so that the
// single-problem calls and the batched call share them
// ---------------------------------------------------------------------------
struct Exec {
  hipStream_t st;
  char* ws;             // this problem's workspace (Plan offsets)
  int* status;          // Jacobi status pair(s) of this problem (2 or 4 ints)
  bool coop;            // cooperative launch for the multi-workgroup Jacobi
  int max_sweeps;
  hipEvent_t* evs;      // timing events (kEvPerSlot) or nullptr
  int64_t* nr0;         // mixed precision: where N0 goes (nullptr: the workspace)
  char* keep;           // mixed precision: S0, VT0 and the mean, kept from phase 1 to
                        // phase 2 (nullptr: the workspace); layout keep_bytes()
  hipEvent_t* jac_ev;   // batch: events that chain the multi-workgroup Jacobi
  int64_t* jac_next;    //   launches across lanes (nullptr: no chaining)
  bool batched;         // an instance of a batch (the lanes are taken)
};

// A batch whose lanes could run more Jacobi workgroups at once than the
// device holds chains every multi-workgroup Jacobi launch after the previous
// one (in instance order, so the chain never points backwards in any lane):
// the grid barrier of each then waits only for workgroups that can be placed.
static int jac_before(pylom_ctx c, const Exec& x, const JacobiPlan& jp) {
  if (!x.jac_ev || jp.G <= 1 || *x.jac_next == 0) return PYLOM_OK;
  HIPCHK(c, hipStreamWaitEvent(x.st, x.jac_ev[*x.jac_next - 1], 0), "hipStreamWaitEvent");
  return PYLOM_OK;
}
static int jac_after(pylom_ctx c, const Exec& x, const JacobiPlan& jp) {
  if (!x.jac_ev || jp.G <= 1) return PYLOM_OK;
  HIPCHK(c, hipEventRecord(x.jac_ev[*x.jac_next], x.st), "hipEventRecord");
  ++*x.jac_next;
  return PYLOM_OK;
}
#define JAC_BEFORE(jp)                         \
  do {                                         \
    const int _r = jac_before(c, x, (jp));     \
    if (_r) return _r;                         \
  } while (0)
#define JAC_AFTER(jp)                          \
  do {                                         \
    const int _r = jac_after(c, x, (jp));      \
    if (_r) return _r;                         \
  } while (0)

// Jacobi plan of the first SVD of a mixed-precision call.  Its R comes from
// FP32 leaves, so the cosines of its column pairs are known only to about
// the FP32 unit roundoff; rotating further chases rounding noise of the FP32
// factorisation.  With option mixed_svd_tol = 1 the rotation test stops at
// 2^-24 instead of n 2^-53.  The leading right singular vectors only seed
// the Rayleigh-Ritz refinement against D, which sets the accuracy of the
// result, and forms U from D itself: the left factor U_R of R is not used,
// so the Jacobi does not accumulate it.
static JacobiPlan mixed_first_jp(const pylom_ctx_s* c, const JacobiPlan& jp) {
  JacobiPlan j = jp;
  if (c->mixed_svd_tol == 1) j.tol = 0x1p-24;
  j.no_ur = 1;
  return j;
}

// Phase-1 results of the mixed path that phase 2 reads: S0 (n), VT0 (n x n),
// mean (m), each 256-byte aligned.
static size_t keep_bytes(int64_t m, int64_t n) {
  return align_up(8 * (size_t)n) + align_up(8 * (size_t)n * n) + align_up(8 * (size_t)m);
}
static double* keep_S0(const Exec& x, const Plan& p) {
  return x.keep ? (double*)x.keep : (double*)(x.ws + p.oS0);
}
static double* keep_VT0(const Exec& x, const Plan& p) {
  return x.keep ? (double*)(x.keep + align_up(8 * (size_t)p.n)) : (double*)(x.ws + p.oVT0);
}
static double* keep_mean(const Exec& x, const Plan& p) {
  return x.keep ? (double*)(x.keep + align_up(8 * (size_t)p.n) + align_up(8 * (size_t)p.n * p.n))
                : (double*)(x.ws + p.oMean);
}

#define EVREC(j) \
  if (x.evs) HIPCHK(c, hipEventRecord(x.evs[j], x.st), "hipEventRecord")

static int enqueue_fp64_blocked(pylom_ctx c, const Exec& x, const Plan& p, pylom_dtype dtype,
                                const void* D, int64_t ldd, int remove_mean, double residual,
                                void* mean, void* U, int64_t ldu, double* S, double* VT,
                                int64_t ldvt, int64_t* n_r);
static int enqueue_mixed1_blocked(pylom_ctx c, const Exec& x, const Plan& p, const void* D,
                                  int64_t ldd, int remove_mean, double residual);

// FP64 POD / TSVD: Alg. 2 (mean) -> Alg. 1 (leaf QR, tree) -> Eq. svdqr2 ->
// propagation -> Eq. svdqr3.
static int enqueue_fp64(pylom_ctx c, const Exec& x, const Plan& p, pylom_dtype dtype,
                        const void* D, int64_t ldd, int remove_mean, double residual, void* mean,
                        void* U, int64_t ldu, double* S, double* VT, int64_t ldvt, int64_t* n_r) {
  if (p.blocked)
    return enqueue_fp64_blocked(c, x, p, dtype, D, ldd, remove_mean, residual, mean, U, ldu, S, VT,
                                ldvt, n_r);
  const int64_t m = p.m, n = p.n;
  double* V = (double*)(x.ws + p.oV);
  double* Tleaf = (double*)(x.ws + p.oTleaf);
  double* Rbuf = (double*)(x.ws + p.oR);
  double* Ttree = (double*)(x.ws + p.oTtree);
  double* W = (double*)(x.ws + p.oW);
  double* meanws = (double*)(x.ws + p.oMean);
  const int in64 = dtype == PYLOM_R64;
  hipStream_t st = x.st;
  EVREC(0);
  EVREC(1);
  // the leaf QRs and the tree combines: one work-queue launch when the
  // option is on and the plan has a tree, else one launch per level
  bool queued = false;
  if (c->work_queue && p.P > 1 && p.q1_bytes) {
    HIPCHK(c, launch_queue_reset(x.ws + p.oQ1, p.q1_bytes, st), "queue reset");
    const int64_t t = kt_begin(c, st);
    const hipError_t e = launch_qr_queue_f64(p.g, D, in64, ldd, m, p.b, p.P, remove_mean, meanws,
                                             V, Tleaf, p.nch_leaf, Rbuf, Ttree, p.nch_tree, 1,
                                             x.ws + p.oQ1, st, Batch());
    if (e == hipSuccess) {
      kt_end(c, st, t, KR_STACKED_LEAF);
      queued = true;
    } else if (e != hipErrorNotSupported) {
      return hip_fail(c, e, "leaf QR and tree (work queue)");
    }
  }
  if (!queued)
    KT(KR_STACKED_LEAF, launch_leaf_qr_f64(p.g, D, in64, ldd, m, p.b, p.P, remove_mean, meanws, V,
                                           Tleaf, p.nch_leaf, Rbuf, st), "leaf QR");
  EVREC(2);
  if (!queued)
    for (int64_t h = 1; h < p.P; h *= 2)
      KT(KR_STACKED_TREE, launch_tree_combine_f64(p.g, h, p.P, Rbuf, Ttree, p.nch_tree, 1, st),
         "tree combine");
  EVREC(3);
  JAC_BEFORE(p.jp);
  KT(KR_SVD, launch_small_svd(p.jp, Rbuf, x.max_sweeps, x.ws + p.oSvd, S, VT, ldvt, W, residual,
                              n_r, x.status, st, x.coop), "small SVD");
  JAC_AFTER(p.jp);
  EVREC(4);
  // the propagation of every level and the leaf applies: one work-queue
  // launch (or per level)
  bool bqueued = false;
  if (queued) {
    HIPCHK(c, launch_queue_reset(x.ws + p.oQ2, p.q2_bytes, st), "queue reset");
    const int64_t t = kt_begin(c, st);
    const hipError_t e = launch_apply_queue_f64(p.g, m, p.b, p.P, V, Tleaf, p.nch_leaf, Rbuf,
                                                Ttree, p.nch_tree, W, n, n_r, 0, n, U, in64, ldu,
                                                x.ws + p.oQ2, st, Batch());
    if (e == hipSuccess) {
      kt_end(c, st, t, KR_LEAF_APPLY);
      bqueued = true;
    } else if (e != hipErrorNotSupported) {
      return hip_fail(c, e, "propagation and apply (work queue)");
    }
    // a timed-out dependency wait of either queue is reported by pylom_check
    HIPCHK(c, launch_queue_err_merge(x.ws + p.oQ1, bqueued ? x.ws + p.oQ2 : nullptr,
                                     x.status + 1, st), "queue status");
  }
  int64_t top = 1;
  while (top * 2 < p.P) top *= 2;
  if (p.P > 1 && !bqueued)
    for (int64_t h = top; h >= 1; h /= 2)
      KT(KR_PROPAGATE, launch_apply_tree_f64(p.g, h, p.P, Rbuf, Ttree, p.nch_tree, W, n, n_r, n,
                                             st), "tree propagation");
  EVREC(5);
  if (!bqueued)
    KT(KR_LEAF_APPLY, launch_apply_leaf_f64(p.g, m, p.b, p.P, V, Tleaf, p.nch_leaf, W, n, n_r, n,
                                            U, in64, ldu, st), "leaf apply");
  if (remove_mean && mean) HIPCHK(c, launch_cast_out(meanws, mean, in64, m, st), "mean out");
  EVREC(6);
  return PYLOM_OK;
}

// ---- column-blocked sequences (use_blocked) -------------------------------
static size_t t_slot(const Plan& p, bool pairs) {  // T-factor elements per panel
  return (size_t)(pairs ? p.P - 1 : p.P) * (pairs ? p.nch_p : p.nch_l) * 4 * kTF;
}
static size_t ps_slot(const Plan& p, bool pairs) {  // panel-state elements per panel
  return (size_t)(pairs ? p.P - 1 : p.P) * kPW * kPW;
}

// Blocked QR of the P leaves of the working matrix (row stride n, zero
// initial state per panel); R of leaf l goes to Rout + l n^2 (row stride n).
template <typename T>
static int blocked_leaves(pylom_ctx c, hipStream_t st, const Plan& p, char* ws, T* Rout) {
  const int64_t n = p.n;
  T* Wk = (T*)(ws + p.oWk);
  const size_t tps = t_slot(p, false), pps = ps_slot(p, false);
  for (int64_t k = 0; k < p.K; ++k) {
    const int64_t c0 = k * kPW;
    const int kw = (int)((n - c0 < kPW) ? n - c0 : kPW);
    const QrGeom& g = (k == p.K - 1) ? p.gpl : p.gp;
    T* Tk = (T*)(ws + p.oTl) + k * tps;
    T* PSk = (T*)(ws + p.oPSl) + k * pps;
    KT(KR_LEAF_PANEL, launch_panel_qr<T>(g, Wk + c0, n, p.m, p.b, p.P, 0, Tk, p.nch_l, PSk, 1, st),
       "panel QR");
    if (c0 + kw < n) {
      PanelApplyArgs<T> a{};
      a.kw = kw; a.npan = g.npanels; a.nlv = p.P; a.b = p.b; a.m = p.m; a.rows_lim = 0;
      a.V = Wk + c0; a.ldv = n; a.Tf = Tk; a.nch = p.nch_l;
      a.X = Wk + c0 + kw; a.ldx = n; a.ncols = n - c0 - kw; a.nc_dev = nullptr; a.nc_off = 0;
      a.x_zero = 0; a.S = Rout + c0 * n + c0 + kw; a.s_leaf = n * n; a.s_ld = n;
      a.load_state = 0; a.store_state = 1; a.leaf_major = 0;
      KT(KR_LEAF_TRAIL, launch_panel_apply<T>(a, false, st), "trailing update");
    }
  }
  KT(KR_LEAF_PANEL, launch_assemble_r<T>((int)n, p.P, (T*)(ws + p.oPSl), (int64_t)pps, Rout,
                                         n * n, st), "R assembly");
  return PYLOM_OK;
}

static int ensure_lanes(pylom_ctx c, int64_t k);

// The reduction tree of Alg. 1 on the leaf R's at R (the FP64 ones at
// ws + oR, or FP32 ones), in place, over the levels h_lo <= h < h_hi: at
// level h, pair q combines R_j (j = 2hq, the state) with R_{j+h} (the
// chunks, rows 0..c0+kw at panel k); R_j becomes the combined R, R_{j+h}
// keeps the reflector tails.  The T factors and panel states of each level
// keep their own slots (the propagation reads them), whatever the range.
//
// With pipe (and option tree_pipeline = S > 1), the levels run as a
// wavefront: level i on lane i mod S, and panel k of level i waits only for
// panel k of level i - 1.  Panel k of a combine reads rows 0..c0+kw of its two
// operands, which are final once panel k of the level below has run, its
// trailing update written those rows right of the panel, and its diagonal
// block been assembled; later panels of the level below only touch rows
// below c0+kw of the states and the reflector tails, which this level never
// reads.  So every level assembles its R per panel.  Without pipe the levels
// run one after another on st0.
template <typename T>
static int blocked_tree(pylom_ctx c, hipStream_t st0, const Plan& p, char* ws, T* R,
                        int64_t h_lo = 1, int64_t h_hi = -1, bool pipe = false) {
  const int64_t n = p.n;
  if (h_hi < 0) h_hi = p.P;
  const size_t tps = t_slot(p, true), pps = ps_slot(p, true);
  int64_t base = 0;
  for (int64_t h = 1; h < h_lo; h *= 2) base += level_pairs(p.P, h);
  std::vector<int64_t> hs, bases;
  for (int64_t h = h_lo; h < p.P && h < h_hi; h *= 2) {
    hs.push_back(h);
    bases.push_back(base);
    base += level_pairs(p.P, h);
  }
  const int64_t L = (int64_t)hs.size();
  if (L == 0) return PYLOM_OK;
  const bool pl = pipe && c->tree_pipeline > 1 && L > 1;
  const int64_t S = pl ? std::min<int64_t>(L, c->tree_pipeline) : 1;
  if (pl) {
    const size_t need = (size_t)(L * p.K);
    while (c->tree_ev.size() < need) {
      hipEvent_t e = nullptr;
      HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
      c->tree_ev.push_back(e);
    }
    const int rc = ensure_lanes(c, S);
    if (rc) return rc;
    HIPCHK(c, hipEventRecord(c->ev_fork, st0), "hipEventRecord");
    for (int64_t l = 0; l < S; ++l)
      HIPCHK(c, hipStreamWaitEvent(c->lanes[(size_t)l], c->ev_fork, 0), "hipStreamWaitEvent");
  }
  for (int64_t li = 0; li < L; ++li) {
    const int64_t h = hs[(size_t)li];
    hipStream_t st = pl ? c->lanes[(size_t)(li % S)] : st0;
    const int64_t np = level_pairs(p.P, h);
    const int64_t rs = 2 * h * n * n;  // pair stride (elements)
    T* Rb = R + h * n * n;             // R_{j+h} of pair 0, as rows of stride n
    T* Tb = (T*)(ws + p.oTp) + bases[(size_t)li] * p.nch_p * 4 * kTF;
    T* PSb = (T*)(ws + p.oPSp) + bases[(size_t)li] * kPW * kPW;
    for (int64_t k = 0; k < p.K; ++k) {
      const int64_t c0 = k * kPW;
      const int kw = (int)((n - c0 < kPW) ? n - c0 : kPW);
      const QrGeom& g = (k == p.K - 1) ? p.gpl : p.gp;
      const int64_t rows_lim = c0 + kw;
      T* Tk = Tb + k * tps;
      T* PSk = PSb + k * pps;
      if (pl && li > 0)
        HIPCHK(c, hipStreamWaitEvent(st, c->tree_ev[(size_t)((li - 1) * p.K + k)], 0),
               "hipStreamWaitEvent");
      KT(KR_TREE_PANEL, launch_diag_load<T>((int)n, c0, kw, np, R, rs, PSk, st), "pair state");
      KT(KR_TREE_PANEL, launch_panel_qr<T>(g, Rb + c0, n, np * 2 * h * n, 2 * h * n, np,
                                           rows_lim, Tk, p.nch_p, PSk, 2, st),
         "pair panel QR");
      if (pl)
        KT(KR_TREE_PANEL, launch_assemble_r<T>((int)n, np, PSb, (int64_t)pps, R, rs, st, (int)c0,
                                               kw), "R assembly");
      if (c0 + kw < n) {
        PanelApplyArgs<T> a{};
        a.kw = kw; a.npan = g.npanels; a.nlv = np; a.b = 2 * h * n; a.m = np * 2 * h * n;
        a.rows_lim = rows_lim; a.V = Rb + c0; a.ldv = n; a.Tf = Tk; a.nch = p.nch_p;
        a.X = Rb + c0 + kw; a.ldx = n; a.ncols = n - c0 - kw; a.nc_dev = nullptr; a.nc_off = 0;
        a.x_zero = 0; a.S = R + c0 * n + c0 + kw; a.s_leaf = rs; a.s_ld = n;
        a.load_state = 1; a.store_state = 1; a.leaf_major = 0;
        KT(KR_TREE_TRAIL, launch_panel_apply<T>(a, false, st), "pair trailing update");
      }
      if (pl)
        HIPCHK(c, hipEventRecord(c->tree_ev[(size_t)(li * p.K + k)], st), "hipEventRecord");
    }
    if (!pl)
      KT(KR_TREE_PANEL, launch_assemble_r<T>((int)n, np, PSb, (int64_t)pps, R, rs, st),
         "R assembly");
  }
  if (pl)
    for (int64_t l = 0; l < S; ++l) {
      HIPCHK(c, hipEventRecord(c->ev_join[(size_t)l], c->lanes[(size_t)l]), "hipEventRecord");
      HIPCHK(c, hipStreamWaitEvent(st0, c->ev_join[(size_t)l], 0), "hipStreamWaitEvent");
    }
  return PYLOM_OK;
}

// Down-tree propagation: W_0 (ws + oW, n x ncols, row stride n) through every
// level's pair Q ([W_j; 0] -> [W_j; W_{j+h}], W_j updated in place),
// leaving W_j for every leaf j.  Columns >= *nc_dev are not touched (nc_dev
// may be null).
static int blocked_propagate(pylom_ctx c, hipStream_t st, const Plan& p, char* ws,
                             const int64_t* nc_dev, int64_t ncols) {
  const int64_t n = p.n;
  double* W = (double*)(ws + p.oW);
  const double* R = (const double*)(ws + p.oR);
  std::vector<int64_t> bases;
  int64_t base = 0;
  for (int64_t h = 1; h < p.P; h *= 2) {
    bases.push_back(base);
    base += level_pairs(p.P, h);
  }
  const size_t tps = t_slot(p, true);
  for (int64_t li = (int64_t)bases.size() - 1; li >= 0; --li) {
    const int64_t h = (int64_t)1 << li;
    const int64_t np = level_pairs(p.P, h);
    const double* Tb = (const double*)(ws + p.oTp) + bases[(size_t)li] * p.nch_p * 4 * kTF;
    for (int64_t k = p.K - 1; k >= 0; --k) {
      const int64_t c0 = k * kPW;
      const int kw = (int)((n - c0 < kPW) ? n - c0 : kPW);
      const QrGeom& g = (k == p.K - 1) ? p.gpl : p.gp;
      PanelApplyArgs<double> a{};
      a.kw = kw; a.npan = g.npanels; a.nlv = np; a.b = 2 * h * n; a.m = np * 2 * h * n;
      a.rows_lim = c0 + kw; a.V = R + h * n * n + c0; a.ldv = n; a.Tf = Tb + k * tps;
      a.nch = p.nch_p; a.X = W + h * n * n; a.ldx = n; a.ncols = ncols; a.nc_dev = nc_dev;
      a.nc_off = 0; a.x_zero = (k == p.K - 1); a.S = W + c0 * n; a.s_leaf = 2 * h * n * n;
      a.s_ld = n; a.load_state = 1; a.store_state = 1; a.leaf_major = 1;
      KT(KR_PROPAGATE, launch_panel_apply<double>(a, true, st), "tree propagation");
    }
  }
  return PYLOM_OK;
}

// U (m x ncols) = Q_leaf W_j for every leaf, in column groups of wcap through
// the FP64 buffer ws + oXu, stored in the output type.
static int blocked_leaf_apply(pylom_ctx c, hipStream_t st, const Plan& p, char* ws,
                              const int64_t* nc_dev, int64_t ncols, void* U, int out_f64,
                              int64_t ldu) {
  const int64_t n = p.n;
  double* W = (double*)(ws + p.oW);
  double* Xu = (double*)(ws + p.oXu);
  const double* Wk = (const double*)(ws + p.oWk);
  const double* Tl = (const double*)(ws + p.oTl);
  const size_t tps = t_slot(p, false);
  for (int64_t col0 = 0; col0 < ncols; col0 += p.wcap) {
    const int64_t ncg = (ncols - col0 < p.wcap) ? ncols - col0 : p.wcap;
    for (int64_t k = p.K - 1; k >= 0; --k) {
      const int64_t c0 = k * kPW;
      const int kw = (int)((n - c0 < kPW) ? n - c0 : kPW);
      const QrGeom& g = (k == p.K - 1) ? p.gpl : p.gp;
      PanelApplyArgs<double> a{};
      a.kw = kw; a.npan = g.npanels; a.nlv = p.P; a.b = p.b; a.m = p.m; a.rows_lim = 0;
      a.V = Wk + c0; a.ldv = n; a.Tf = Tl + k * tps; a.nch = p.nch_l;
      a.X = Xu; a.ldx = p.wcap; a.ncols = ncg; a.nc_dev = nc_dev; a.nc_off = col0;
      a.x_zero = (k == p.K - 1); a.S = W + c0 * n + col0; a.s_leaf = n * n; a.s_ld = n;
      a.load_state = 1; a.store_state = 0; a.leaf_major = 1;
      KT(KR_LEAF_APPLY, launch_panel_apply<double>(a, true, st), "leaf apply");
    }
    KT(KR_LEAF_APPLY, launch_copy_cols(out_f64, p.m, col0, ncg, ncols, nc_dev, Xu, p.wcap, U, ldu,
                                       st), "U out");
  }
  return PYLOM_OK;
}

static int enqueue_fp64_blocked(pylom_ctx c, const Exec& x, const Plan& p, pylom_dtype dtype,
                                const void* D, int64_t ldd, int remove_mean, double residual,
                                void* mean, void* U, int64_t ldu, double* S, double* VT,
                                int64_t ldvt, int64_t* n_r) {
  const int64_t m = p.m, n = p.n;
  double* Rbuf = (double*)(x.ws + p.oR);
  double* meanws = (double*)(x.ws + p.oMean);
  const int in64 = dtype == PYLOM_R64;
  hipStream_t st = x.st;
  EVREC(0);
  KT(KR_WORK, launch_make_work(in64, 1, m, (int)n, D, ldd, remove_mean, meanws, x.ws + p.oWk, st),
     "working copy");
  EVREC(1);
  int rc = blocked_leaves<double>(c, st, p, x.ws, Rbuf);
  if (rc) return rc;
  EVREC(2);
  rc = blocked_tree<double>(c, st, p, x.ws, Rbuf, 1, -1, !x.batched);
  if (rc) return rc;
  EVREC(3);
  JAC_BEFORE(p.jp);
  KT(KR_SVD, launch_small_svd(p.jp, Rbuf, x.max_sweeps, x.ws + p.oSvd, S, VT, ldvt,
                              (double*)(x.ws + p.oW), residual, n_r, x.status, st, x.coop),
     "small SVD");
  JAC_AFTER(p.jp);
  EVREC(4);
  rc = blocked_propagate(c, st, p, x.ws, n_r, n);
  if (rc) return rc;
  EVREC(5);
  rc = blocked_leaf_apply(c, st, p, x.ws, n_r, n, U, in64, ldu);
  if (rc) return rc;
  if (remove_mean && mean) HIPCHK(c, launch_cast_out(meanws, mean, in64, m, st), "mean out");
  EVREC(6);
  return PYLOM_OK;
}

static int enqueue_mixed1_blocked(pylom_ctx c, const Exec& x, const Plan& p, const void* D,
                                  int64_t ldd, int remove_mean, double residual) {
  const int64_t m = p.m, n = p.n;
  hipStream_t st = x.st;
  EVREC(0);
  KT(KR_WORK, launch_make_work(0, 0, m, (int)n, D, ldd, remove_mean, keep_mean(x, p),
                               x.ws + p.oWk, st), "working copy (FP32)");
  EVREC(1);
  float* R32 = (float*)(x.ws + p.oR32);
  double* R64 = (double*)(x.ws + p.oR);
  int rc = blocked_leaves<float>(c, st, p, x.ws, R32);
  if (rc) return rc;
  // tree: every level below the top in FP32 (option mixed_tree = 1) or none;
  // the final combine, the root R and its SVD in FP64
  int64_t top = 1;
  while (top * 2 < p.P) top *= 2;
  const int64_t h64 = (c->mixed_tree == 1 && p.P > 1) ? top : 1;
  if (h64 > 1) {
    EVREC(2);
    rc = blocked_tree<float>(c, st, p, x.ws, R32, 1, h64, !x.batched);
    if (rc) return rc;
    // the two operands of the final combine (R_0 and R_top)
    KT(KR_TREE_PANEL, launch_cast_f32_f64(R32, R64, n * n, st), "R to FP64");
    KT(KR_TREE_PANEL, launch_cast_f32_f64(R32 + h64 * n * n, R64 + h64 * n * n, n * n, st),
       "R to FP64");
  } else {
    KT(KR_LEAF_PANEL, launch_cast_f32_f64(R32, R64, p.P * n * n, st), "R to FP64");
    EVREC(2);
  }
  rc = blocked_tree<double>(c, st, p, x.ws, R64, h64, -1, !x.batched);
  if (rc) return rc;
  EVREC(3);
  JAC_BEFORE(p.jp);
  KT(KR_SVD, launch_small_svd(mixed_first_jp(c, p.jp), (double*)(x.ws + p.oR), x.max_sweeps,
                              x.ws + p.oSvd, keep_S0(x, p), keep_VT0(x, p), n,
                              (double*)(x.ws + p.oW), residual,
                              x.nr0 ? x.nr0 : (int64_t*)(x.ws + p.oNr0), x.status, st, x.coop),
     "small SVD");
  JAC_AFTER(p.jp);
  if (x.evs) HIPCHK(c, hipEventRecord(x.evs[7], st), "hipEventRecord");
  return PYLOM_OK;
}

// Mixed precision, phase 1: FP32 leaf QR (R only, mean fused), FP64 tree and
// SVD of R: S0, VT0 and N0 in the workspace.
static int enqueue_mixed1(pylom_ctx c, const Exec& x, const Plan& p, const void* D, int64_t ldd,
                          int remove_mean, double residual) {
  if (p.blocked) return enqueue_mixed1_blocked(c, x, p, D, ldd, remove_mean, residual);
  const int64_t m = p.m, n = p.n;
  hipStream_t st = x.st;
  EVREC(0);
  EVREC(1);
  KT(KR_STACKED_LEAF, launch_leaf_qr_f32(p.g, (const float*)D, ldd, m, p.b, p.P, remove_mean,
                                         keep_mean(x, p), (float*)(x.ws + p.oR32), st),
     "leaf QR (FP32)");
  KT(KR_STACKED_LEAF, launch_cast_f32_f64((const float*)(x.ws + p.oR32), (double*)(x.ws + p.oR),
                                          p.P * n * n, st), "R to FP64");
  EVREC(2);
  for (int64_t h = 1; h < p.P; h *= 2)
    KT(KR_STACKED_TREE, launch_tree_combine_f64(p.g, h, p.P, (double*)(x.ws + p.oR), nullptr,
                                                p.nch_tree, 0, st), "tree combine");
  EVREC(3);
  JAC_BEFORE(p.jp);
  KT(KR_SVD, launch_small_svd(mixed_first_jp(c, p.jp), (double*)(x.ws + p.oR), x.max_sweeps,
                              x.ws + p.oSvd, keep_S0(x, p), keep_VT0(x, p), n,
                              (double*)(x.ws + p.oW), residual,
                              x.nr0 ? x.nr0 : (int64_t*)(x.ws + p.oNr0), x.status, st, x.coop),
     "small SVD");
  JAC_AFTER(p.jp);
  // end of the first SVD (the host read-back of N0 follows)
  if (x.evs) HIPCHK(c, hipEventRecord(x.evs[7], st), "hipEventRecord");
  return PYLOM_OK;
}

static int64_t refine_width(int64_t nr0, int64_t n) {
  int64_t over = nr0 / 4;
  if (over < 8) over = 8;
  return (nr0 + over < n) ? nr0 + over : n;
}

// Mixed precision, phase 2 (after the host has read N0): Rayleigh-Ritz
// refinement on the k = refine_width(N0) leading right singular vectors.
static int enqueue_mixed2(pylom_ctx c, const Exec& x, const Plan& p, const void* D, int64_t ldd,
                          int remove_mean, double residual, void* mean, void* U, int64_t ldu,
                          double* S, double* VT, int64_t ldvt, int64_t* n_r, int64_t nr_first) {
  const int64_t m = p.m, n = p.n;
  hipStream_t st = x.st;
  double* S0 = keep_S0(x, p);
  double* meanws = keep_mean(x, p);
  EVREC(4);
  if (nr_first <= 0) {
    // all-zero spectrum: nothing to refine, no mode is kept
    HIPCHK(c, hipMemcpyAsync(S, S0, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, st),
           "S copy");
    HIPCHK(c, launch_set_i64(n_r, 0, st), "N_r");
    // no second SVD: its status pair reads (0 sweeps, no timeout)
    HIPCHK(c, launch_set_i64(reinterpret_cast<int64_t*>(x.status + 2), 0, st), "status");
    EVREC(5);
  } else {
    const int64_t k = refine_width(nr_first, n);
    if (k > p.zcap) return fail(c, PYLOM_ENOTSUP, "refinement width exceeds the planned workspace");
    JacobiPlan jk;
    if (!jacobi_plan((int)k, &jk)) return fail(c, PYLOM_ENOTSUP, "no Jacobi plan");
    const int64_t ns = matmul_tn_splits(m, k, k);
    if (sizeof(double) * (size_t)ns * k * k > p.part_bytes)
      return fail(c, PYLOM_ENOTSUP, "Gram partials exceed the planned workspace");
    double* Z = (double*)(x.ws + p.oZ);
    double* G = (double*)(x.ws + p.oG);
    double* lam = (double*)(x.ws + p.oLam);
    double* WT = (double*)(x.ws + p.oWT);
    double* M = (double*)(x.ws + p.oM);
    const double* VT0 = keep_VT0(x, p);
    KT(KR_REFINE, launch_rr_project(0, m, (int)n, (int)k, D, ldd, remove_mean ? meanws : nullptr,
                                    VT0, Z, st), "Rayleigh-Ritz projection");
    KT(KR_REFINE, launch_matmul_tn(1, m, k, k, Z, k, Z, k, G, k, (double*)(x.ws + p.oPart), ns, st),
       "Gram");
    JAC_BEFORE(jk);
    KT(KR_REFINE, launch_small_svd(jk, G, x.max_sweeps, x.ws + p.oSvd2, lam, WT, k,
                                   (double*)(x.ws + p.oUR2), 0.0, (int64_t*)(x.ws + p.oNr2),
                                   x.status + 2, st, x.coop), "Gram eigen-decomposition");
    JAC_AFTER(jk);
    KT(KR_REFINE, launch_rr_finish((int)n, (int)k, S0, lam, residual, S, n_r, WT, VT0, VT, ldvt,
                                   M, st), "refined spectrum");
    EVREC(5);
    KT(KR_FORM_U, launch_rr_form_u(0, m, (int)k, Z, M, n_r, U, ldu, st), "form U");
  }
  if (remove_mean && mean) HIPCHK(c, launch_cast_out(meanws, mean, 0, m, st), "mean out");
  EVREC(6);
  return PYLOM_OK;
}
#undef EVREC

static Exec ctx_exec(pylom_ctx c) {
  Exec x;
  x.st = c->stream;
  x.ws = (char*)c->ws;
  x.status = c->status_dev;
  x.coop = true;
  x.max_sweeps = (int)c->max_sweeps;
  const bool tm = c->timing > 0 && !c->ev.empty();
  x.evs = tm ? &c->ev[(size_t)(c->ev_calls % c->timing) * kEvPerSlot] : nullptr;
  x.nr0 = nullptr;
  x.keep = nullptr;
  x.jac_ev = nullptr;
  x.jac_next = nullptr;
  x.batched = false;
  return x;
}

// Mixed precision (FP32 storage): FP32 leaf QR (R only), FP64 tree and SVD of
// R, then the Rayleigh-Ritz refinement against the input on the k leading
// right singular vectors.  The host reads N0 once (one stream
// synchronisation) to size the refinement.
static int run_mixed(pylom_ctx c, pylom_dtype dtype, int64_t m, int64_t n, const void* D,
                     int64_t ldd, int remove_mean, double residual, void* mean, void* U,
                     int64_t ldu, double* S, double* VT, int64_t ldvt, int64_t* n_r) {
  if (dtype != PYLOM_R32) return fail(c, PYLOM_EDTYPE, "mixed precision needs R32 storage");
  Plan p;
  int rc = make_plan(c, m, n, false, &p, true);
  if (rc) return rc;
  if ((rc = cap_check(c, p.total))) return rc;
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
  rc = ensure_ws(c, p.total);
  if (rc) return rc;
  const Exec x = ctx_exec(c);
  if (x.evs) c->ev_mixed[(size_t)(c->ev_calls % c->timing)] = 1;
  rc = enqueue_mixed1(c, x, p, D, ldd, remove_mean, residual);
  if (rc) return rc;
  c->status_valid = 1;
  c->status_pairs = 1;
  int64_t nr_first = 0;
  HIPCHK(c, hipMemcpyAsync(&nr_first, x.ws + p.oNr0, sizeof(int64_t), hipMemcpyDeviceToHost, x.st),
         "N_r read-back");
  HIPCHK(c, hipStreamSynchronize(x.st), "hipStreamSynchronize");
  if (nr_first > 0) c->status_pairs = 2;
  rc = enqueue_mixed2(c, x, p, D, ldd, remove_mean, residual, mean, U, ldu, S, VT, ldvt, n_r,
                      nr_first);
  if (rc) return rc;
  if (x.evs) ++c->ev_calls;
  return PYLOM_OK;
}

static int run_tsvd(pylom_ctx c, pylom_dtype dtype, pylom_prec prec, int64_t m, int64_t n,
                    const void* D, int64_t ldd, int remove_mean, double residual, void* mean,
                    void* U, int64_t ldu, double* S, double* VT, int64_t ldvt, int64_t* n_r) {
  int rc = check_common(c, dtype, prec);
  if (rc) return rc;
  if (!D || !U || !S || !VT || !n_r) return fail(c, PYLOM_EINVAL, "null array argument");
  if (!(residual >= 0.0 && residual < 1.0)) return fail(c, PYLOM_EINVAL, "residual must be in [0, 1)");
  if (n < 1 || m < n) return fail(c, PYLOM_ESHAPE, "need m >= n >= 1");
  if (ldd < n || ldu < n || ldvt < n) return fail(c, PYLOM_ESHAPE, "leading dimension < n");
  if (prec == PYLOM_MIXED)
    return run_mixed(c, dtype, m, n, D, ldd, remove_mean, residual, mean, U, ldu, S, VT, ldvt, n_r);
  Plan p;
  rc = make_plan(c, m, n, true, &p);
  if (rc) return rc;
  if ((rc = cap_check(c, p.total))) return rc;
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
  rc = ensure_ws(c, p.total);
  if (rc) return rc;
  const Exec x = ctx_exec(c);
  if (x.evs) c->ev_mixed[(size_t)(c->ev_calls % c->timing)] = 0;
  rc = enqueue_fp64(c, x, p, dtype, D, ldd, remove_mean, residual, mean, U, ldu, S, VT, ldvt, n_r);
  if (rc) return rc;
  c->status_valid = 1;
  c->status_pairs = 1;
  if (x.evs) ++c->ev_calls;
  return PYLOM_OK;
}

// ---------------------------------------------------------------------------
// measured leaf heights
// ---------------------------------------------------------------------------
// Candidate leaf heights of an m x n problem on its path: the column-blocked
// path tries one to four leaves per CU (rows rounded up to 64), the stacked
// path the powers of two from 128 to 32768; each at least n, the analytic
// choice always included.
static std::vector<int64_t> tune_candidates(pylom_ctx c, bool blocked, bool mixed, int64_t m,
                                            int64_t n) {
  std::vector<int64_t> v;
  auto add = [&](int64_t b) {
    if (b < n) b = n;
    if (b > m) b = m;
    if (blocked && m / b > 65535) return;
    if (std::find(v.begin(), v.end(), b) == v.end()) v.push_back(b);
  };
  if (blocked) {
    for (int64_t k = 1; k <= 4; ++k) {
      const int64_t slots = k * (int64_t)c->ncu;
      add(((m + slots - 1) / slots + kPW - 1) / kPW * kPW);
    }
    add(blocked_block_rows(m, n, c->ncu));
  } else {
    for (int64_t b = 128; b <= 32768; b *= 2) add(b);
    add(tune_block_rows(c, m, n, mixed));
  }
  std::sort(v.begin(), v.end());
  return v;
}

extern "C" int pylom_autotune(pylom_ctx c, pylom_dtype dtype, pylom_prec prec, int64_t m,
                              int64_t n, const void* D, int64_t ldd, int remove_mean, int reps,
                              int64_t* best_rows, double* best_ms) {
  int rc = check_common(c, dtype, prec);
  if (rc) return rc;
  if (!D) return fail(c, PYLOM_EINVAL, "null array argument");
  if (n < 1 || m < n) return fail(c, PYLOM_ESHAPE, "need m >= n >= 1");
  if (ldd < n) return fail(c, PYLOM_ESHAPE, "leading dimension < n");
  if (reps < 1 || reps > 100) return fail(c, PYLOM_EINVAL, "reps must be in [1, 100]");
  if (prec == PYLOM_MIXED && dtype != PYLOM_R32)
    return fail(c, PYLOM_EDTYPE, "mixed precision needs R32 storage");
  if (n > kMaxN) return fail(c, PYLOM_ENOTSUP, "n > 2048 is not supported");
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
  const bool mixed = prec == PYLOM_MIXED;
  const bool blk = use_blocked(c, m, n);
  const int es = dtype == PYLOM_R64 ? 8 : 4;
  const std::vector<int64_t> cand = tune_candidates(c, blk, mixed, m, n);
  // outputs of the trial calls (tuning allocates; the calls it times do not)
  void* buf = nullptr;
  const size_t oU = 0, oS = align_up((size_t)es * m * n), oVT = oS + align_up(8 * (size_t)n),
               oNr = oVT + align_up(8 * (size_t)n * n), oMean = oNr + 256,
               tot = oMean + align_up((size_t)es * m);
  if (hipMalloc(&buf, tot) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, PYLOM_ENOMEM, "autotune outputs");
  }
  char* o = (char*)buf;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int64_t saved = c->block_rows;
  int64_t best = 0;
  double tbest = 0.0;
  rc = PYLOM_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = hip_fail(c, hipGetLastError(), "hipEventCreate");
  }
  for (size_t i = 0; rc == PYLOM_OK && i < cand.size(); ++i) {
    c->block_rows = cand[i];
    Plan pl;
    if (make_plan(c, m, n, !mixed, &pl, mixed) != PYLOM_OK) continue;  // not plannable
    if (c->ws_cap_mb > 0 && pl.total > (size_t)c->ws_cap_mb * (1u << 20)) continue;
    auto call = [&]() {
      return run_tsvd(c, dtype, prec, m, n, D, ldd, remove_mean, 0.01,
                      remove_mean ? o + oMean : nullptr, o + oU, n, (double*)(o + oS),
                      (double*)(o + oVT), n, (int64_t*)(o + oNr));
    };
    if ((rc = call()) < 0) break;  // warm-up: workspace, code objects
    hipError_t he = hipEventRecord(e0, c->stream);
    for (int r = 0; rc >= 0 && r < reps; ++r) rc = call();
    if (rc < 0) break;
    if (he == hipSuccess) he = hipEventRecord(e1, c->stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (he != hipSuccess) {
      rc = hip_fail(c, he, "autotune timing");
      break;
    }
    rc = PYLOM_OK;
    const double t = ms / reps;
    if (best == 0 || t < tbest) {
      best = cand[i];
      tbest = t;
    }
  }
  c->block_rows = saved;
  hipStreamSynchronize(c->stream);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(buf);
  if (rc < 0) return rc;
  if (best == 0) return fail(c, PYLOM_ENOTSUP, "no candidate leaf height could be planned");
  c->tuned[tune_key(blk, mixed, m, n)] = std::make_pair(best, tbest);
  if (best_rows) *best_rows = best;
  if (best_ms) *best_ms = tbest;
  return PYLOM_OK;
}

extern "C" int pylom_tune_save(pylom_ctx c, const char* path) {
  if (!c || !path) return PYLOM_EINVAL;
  std::ofstream f(path, std::ios::out | std::ios::trunc);
  if (!f) return fail(c, PYLOM_EINVAL, "cannot open the tuning file for writing");
  f << "{\"pylom_tuning\": 1, \"entries\": [";
  bool first = true;
  char line[256];
  for (const auto& kv : c->tuned) {
    std::snprintf(line, sizeof line,
                  "%s\n  {\"path\": \"%s\", \"precision\": \"%s\", \"m_log2\": %d, "
                  "\"n_bucket\": %lld, \"block_rows\": %lld, \"ms\": %.6g}",
                  first ? "" : ",", std::get<0>(kv.first) ? "blocked" : "stacked",
                  std::get<1>(kv.first) ? "mixed" : "fp64", std::get<2>(kv.first),
                  (long long)std::get<3>(kv.first), (long long)kv.second.first, kv.second.second);
    f << line;
    first = false;
  }
  f << "\n]}\n";
  if (!f) return fail(c, PYLOM_EINVAL, "writing the tuning file failed");
  return PYLOM_OK;
}

// Reads the value after "key": in one entry object (a string or a number).
static bool json_field(const std::string& obj, const char* key, std::string* out) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = obj.find(k);
  if (p == std::string::npos) return false;
  p = obj.find(':', p + k.size());
  if (p == std::string::npos) return false;
  ++p;
  while (p < obj.size() && (obj[p] == ' ' || obj[p] == '\t' || obj[p] == '\n')) ++p;
  if (p >= obj.size()) return false;
  if (obj[p] == '"') {
    const size_t q = obj.find('"', p + 1);
    if (q == std::string::npos) return false;
    *out = obj.substr(p + 1, q - p - 1);
    return true;
  }
  size_t q = p;
  while (q < obj.size() && obj[q] != ',' && obj[q] != '}' && obj[q] != ' ' && obj[q] != '\n') ++q;
  *out = obj.substr(p, q - p);
  return !out->empty();
}

extern "C" int pylom_tune_load(pylom_ctx c, const char* path) {
  if (!c || !path) return PYLOM_EINVAL;
  std::ifstream f(path);
  if (!f) return fail(c, PYLOM_EINVAL, "cannot open the tuning file");
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  if (text.find("\"pylom_tuning\"") == std::string::npos)
    return fail(c, PYLOM_EINVAL, "not a pylom tuning file");
  std::map<std::tuple<int, int, int, int64_t>, std::pair<int64_t, double>> got;
  size_t pos = text.find('[');
  while (pos != std::string::npos) {
    const size_t a = text.find('{', pos + 1);
    if (a == std::string::npos) break;
    const size_t b = text.find('}', a);
    if (b == std::string::npos) return fail(c, PYLOM_EINVAL, "malformed tuning entry");
    const std::string obj = text.substr(a, b - a + 1);
    std::string path_s, prec_s, lg_s, nb_s, br_s, ms_s;
    if (!json_field(obj, "path", &path_s) || !json_field(obj, "precision", &prec_s) ||
        !json_field(obj, "m_log2", &lg_s) || !json_field(obj, "n_bucket", &nb_s) ||
        !json_field(obj, "block_rows", &br_s))
      return fail(c, PYLOM_EINVAL, "malformed tuning entry");
    if ((path_s != "blocked" && path_s != "stacked") || (prec_s != "mixed" && prec_s != "fp64"))
      return fail(c, PYLOM_EINVAL, "malformed tuning entry");
    char* end = nullptr;
    const long lg = std::strtol(lg_s.c_str(), &end, 10);
    const long long nb = std::strtoll(nb_s.c_str(), &end, 10);
    const long long br = std::strtoll(br_s.c_str(), &end, 10);
    double ms = 0.0;
    if (json_field(obj, "ms", &ms_s)) ms = std::strtod(ms_s.c_str(), &end);
    if (lg < 0 || lg > 62 || nb < 16 || nb > kMaxN + 15 || br < 1)
      return fail(c, PYLOM_EINVAL, "tuning entry out of range");
    got[std::make_tuple(path_s == "blocked" ? 1 : 0, prec_s == "mixed" ? 1 : 0, (int)lg,
                        (int64_t)nb)] = std::make_pair((int64_t)br, ms);
    pos = b;
  }
  for (const auto& kv : got) c->tuned[kv.first] = kv.second;
  return (int)got.size();
}

// ---------------------------------------------------------------------------
// batched POD of uneven instances
// ---------------------------------------------------------------------------
static uint64_t fnv1a(uint64_t h, const void* data, size_t len) {
  const unsigned char* p = (const unsigned char*)data;
  for (size_t i = 0; i < len; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

static int ensure_lanes(pylom_ctx c, int64_t k) {
  while ((int64_t)c->lanes.size() < k) {
    hipStream_t q = nullptr;
    HIPCHK(c, hipStreamCreateWithFlags(&q, hipStreamNonBlocking), "hipStreamCreate");
    c->lanes.push_back(q);
    hipEvent_t e = nullptr;
    HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    c->ev_join.push_back(e);
  }
  if (!c->ev_fork) HIPCHK(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming), "hipEventCreate");
  if (!c->cap) HIPCHK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking), "hipStreamCreate");
  if (!c->ev_in) HIPCHK(c, hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming), "hipEventCreate");
  if (!c->ev_out) HIPCHK(c, hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming), "hipEventCreate");
  return PYLOM_OK;
}

struct BatchLayout {
  bool jac_chain = false;         // chain the multi-workgroup Jacobi launches (jac_before)
  std::vector<Plan> plans;
  std::vector<int> lane;          // lane of each problem
  std::vector<size_t> lane_off;   // workspace offset of each lane
  size_t oStatus, oNr0, total;
  std::vector<size_t> keep_off;   // mixed precision: per-instance phase-1 results
  int64_t K;
};

// One launch phase of the batch (0: FP64 whole path; 1, 2: mixed phases),
// forked from the context stream over the lanes and joined back.
static int batch_phase(pylom_ctx c, const BatchLayout& L, pylom_dtype dtype, int phase,
                       int64_t count, const pylom_problem* pr, const int64_t* nr_first,
                       bool capturing, hipStream_t origin) {
  char* ws = (char*)c->ws;
  int64_t jac_next = 0;
  HIPCHK(c, hipEventRecord(c->ev_fork, origin), "hipEventRecord");
  for (int64_t l = 0; l < L.K; ++l)
    HIPCHK(c, hipStreamWaitEvent(c->lanes[l], c->ev_fork, 0), "hipStreamWaitEvent");
  for (int64_t i = 0; i < count; ++i) {
    const int l = L.lane[i];
    Exec x;
    x.st = c->lanes[l];
    x.ws = ws + L.lane_off[l];
    x.status = (int*)(ws + L.oStatus) + 4 * i;
    x.coop = !capturing;
    x.max_sweeps = (int)c->max_sweeps;
    x.evs = nullptr;
    x.nr0 = (int64_t*)(ws + L.oNr0) + i;
    x.keep = L.keep_off.empty() ? nullptr : ws + L.keep_off[(size_t)i];
    x.jac_ev = L.jac_chain ? c->jac_ev.data() : nullptr;
    x.jac_next = L.jac_chain ? &jac_next : nullptr;
    x.batched = true;
    const pylom_problem& q = pr[i];
    int rc;
    if (phase == 0)
      rc = enqueue_fp64(c, x, L.plans[i], dtype, q.D, q.ldd, q.remove_mean ? 1 : 0, q.residual,
                        q.mean, q.U, q.ldu, q.S, q.VT, q.ldvt, q.n_r);
    else if (phase == 1)
      rc = enqueue_mixed1(c, x, L.plans[i], q.D, q.ldd, q.remove_mean ? 1 : 0, q.residual);
    else
      rc = enqueue_mixed2(c, x, L.plans[i], q.D, q.ldd, q.remove_mean ? 1 : 0, q.residual, q.mean,
                          q.U, q.ldu, q.S, q.VT, q.ldvt, q.n_r, nr_first[i]);
    if (rc) return rc;
  }
  for (int64_t l = 0; l < L.K; ++l) {
    HIPCHK(c, hipEventRecord(c->ev_join[l], c->lanes[l]), "hipEventRecord");
    HIPCHK(c, hipStreamWaitEvent(origin, c->ev_join[l], 0), "hipStreamWaitEvent");
  }
  if (phase != 1) {
    // reduced Jacobi status of the whole batch into the context's status
    HIPCHK(c, launch_status_reduce(count, (const int*)(ws + L.oStatus), 4, phase == 0 ? 1 : 2,
                                   c->status_dev, origin), "status");
  }
  return PYLOM_OK;
}

// Run one phase eagerly, or capture it once into a graph and replay it.
static int batch_run(pylom_ctx c, const BatchLayout& L, pylom_dtype dtype, int phase,
                     int64_t count, const pylom_problem* pr, const int64_t* nr_first,
                     bool use_graph, uint64_t key) {
  // per-kernel events are recorded for single-problem calls only
  struct KtOff {
    pylom_ctx c;
    explicit KtOff(pylom_ctx cc) : c(cc) { c->kt_off = true; }
    ~KtOff() { c->kt_off = false; }
  } kt_off(c);
  if (!use_graph) return batch_phase(c, L, dtype, phase, count, pr, nr_first, false, c->stream);
  // the graph is captured on, and replayed from, the context's own origin
  // stream, ordered after the caller's stream by events on both sides (the
  // caller's stream may be the legacy null stream, which cannot be captured)
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    evict_graphs(c);
    HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
    const int rc = batch_phase(c, L, dtype, phase, count, pr, nr_first, true, c->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap, &g);
    if (rc) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    hipGraphExec_t ge = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e2 != hipSuccess) return hip_fail(c, e2, "hipGraphInstantiate");
    it = c->graphs.emplace(key, std::make_pair(ge, (uint64_t)0)).first;
  }
  it->second.second = ++c->graph_clock;
  HIPCHK(c, hipEventRecord(c->ev_in, c->stream), "hipEventRecord");
  HIPCHK(c, hipStreamWaitEvent(c->cap, c->ev_in, 0), "hipStreamWaitEvent");
  HIPCHK(c, hipGraphLaunch(it->second.first, c->cap), "hipGraphLaunch");
  HIPCHK(c, hipEventRecord(c->ev_out, c->cap), "hipEventRecord");
  HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_out, 0), "hipStreamWaitEvent");
  return PYLOM_OK;
}

extern "C" int pylom_pod_batched(pylom_ctx c, pylom_dtype dtype, pylom_prec prec, int64_t count,
                                 const pylom_problem* pr, int use_graph) {
  int rc = check_common(c, dtype, prec);
  if (rc) return rc;
  if (count < 0 || (count > 0 && !pr)) return fail(c, PYLOM_EINVAL, "problems");
  if (count > (1 << 20)) return fail(c, PYLOM_ENOTSUP, "too many problems");
  if (prec == PYLOM_MIXED && dtype != PYLOM_R32)
    return fail(c, PYLOM_EDTYPE, "mixed precision needs R32 storage");
  const bool mixed = prec == PYLOM_MIXED;
  BatchLayout L;
  L.plans.resize((size_t)count);
  std::vector<double> cost((size_t)count);
  for (int64_t i = 0; i < count; ++i) {
    const pylom_problem& q = pr[i];
    if (!q.D || !q.U || !q.S || !q.VT || !q.n_r) return fail(c, PYLOM_EINVAL, "null array argument");
    if (!(q.residual >= 0.0 && q.residual < 1.0))
      return fail(c, PYLOM_EINVAL, "residual must be in [0, 1)");
    if (q.n < 1 || q.m < q.n) return fail(c, PYLOM_ESHAPE, "need m >= n >= 1");
    if (q.ldd < q.n || q.ldu < q.n || q.ldvt < q.n)
      return fail(c, PYLOM_ESHAPE, "leading dimension < n");
    rc = make_plan(c, q.m, q.n, !mixed, &L.plans[(size_t)i], mixed);
    if (rc) return rc;
    cost[(size_t)i] = leaf_model(c, q.m, q.n, L.plans[(size_t)i].b, mixed);
  }
  if (count == 0) return PYLOM_OK;
  // longest-processing-time assignment of instances to lanes
  L.K = std::min<int64_t>(c->streams, count);
  L.lane.assign((size_t)count, 0);
  std::vector<int64_t> order((size_t)count);
  for (int64_t i = 0; i < count; ++i) order[(size_t)i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return cost[(size_t)a] > cost[(size_t)b]; });
  std::vector<double> load((size_t)L.K, 0.0);
  std::vector<size_t> lane_ws((size_t)L.K, 0);
  for (int64_t i : order) {
    int64_t best = 0;
    for (int64_t l = 1; l < L.K; ++l)
      if (load[(size_t)l] < load[(size_t)best]) best = l;
    L.lane[(size_t)i] = (int)best;
    load[(size_t)best] += cost[(size_t)i];
    lane_ws[(size_t)best] = std::max(lane_ws[(size_t)best], L.plans[(size_t)i].total);
  }
  size_t off = 0;
  L.lane_off.resize((size_t)L.K);
  for (int64_t l = 0; l < L.K; ++l) {
    L.lane_off[(size_t)l] = off;
    off = align_up(off + lane_ws[(size_t)l]);
  }
  L.oStatus = off;
  off = align_up(off + sizeof(int) * 4 * (size_t)count);
  L.oNr0 = off;
  off = align_up(off + sizeof(int64_t) * (size_t)count);
  if (mixed) {
    // instances that share a lane also share its scratch, so what phase 2
    // reads from phase 1 is kept per instance
    L.keep_off.resize((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
      L.keep_off[(size_t)i] = off;
      off = align_up(off + keep_bytes(pr[i].m, pr[i].n));
    }
  }
  L.total = off;
  if ((rc = cap_check(c, L.total))) return rc;
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
  // Co-residency of the grid-barrier Jacobi: lanes run concurrently, so the
  // largest Jacobi grid of each lane may be live at once; when their sum
  // exceeds what the device holds, the Jacobi launches are chained instead.
  {
    std::vector<int64_t> lane_g((size_t)L.K, 0);
    int64_t per_cu = 1 << 20;
    for (int64_t i = 0; i < count; ++i) {
      const JacobiPlan& jp = L.plans[(size_t)i].jp;
      const int64_t wgs = (int64_t)jp.G * jp.ks;
      lane_g[(size_t)L.lane[(size_t)i]] = std::max<int64_t>(lane_g[(size_t)L.lane[(size_t)i]], wgs);
      if (wgs > 1) per_cu = std::min<int64_t>(per_cu, jacobi_resident_per_cu(jp));
    }
    int64_t gsum = 0;
    for (int64_t g : lane_g) gsum += (g > 1) ? g : 0;
    if (per_cu == (1 << 20)) per_cu = 1;
    L.jac_chain = L.K > 1 && gsum > (int64_t)c->ncu * std::max<int64_t>(per_cu, 1);
    c->last_jac_chain = L.jac_chain ? 1 : 0;
  }
  rc = ensure_ws(c, L.total);
  if (rc) return rc;
  rc = ensure_lanes(c, L.K);
  if (rc) return rc;
  if (L.jac_chain) {
    const size_t need = 2 * (size_t)count;
    while (c->jac_ev.size() < need) {
      hipEvent_t e = nullptr;
      HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
      c->jac_ev.push_back(e);
    }
  }
  // graph key: everything the captured launches depend on, field by field
  // (never the raw descriptor bytes, whose padding a C caller may leave
  // uninitialised)
  uint64_t key = 1469598103934665603ull;
  const int64_t hdr[11] = {(int64_t)dtype,    (int64_t)prec,    count,
                           L.K,              c->max_sweeps,    c->block_rows,
                           c->narrow_leaves, c->blocked_from,  c->mixed_tree,
                           c->mixed_svd_tol, L.jac_chain ? 1 : 0};
  key = fnv1a(key, hdr, sizeof(hdr));
  const void* wsp = c->ws;
  key = fnv1a(key, &wsp, sizeof(wsp));
  key = fnv1a(key, &c->stream, sizeof(c->stream));
  for (int64_t i = 0; i < count; ++i) {
    const pylom_problem& q = pr[i];
    int64_t rbits;
    std::memcpy(&rbits, &q.residual, sizeof(rbits));
    const int64_t f[14] = {q.m,         q.n,           (int64_t)(uintptr_t)q.D,    q.ldd,
                           q.remove_mean ? 1 : 0,      rbits,
                           (int64_t)(uintptr_t)q.mean, (int64_t)(uintptr_t)q.U,    q.ldu,
                           (int64_t)(uintptr_t)q.S,    (int64_t)(uintptr_t)q.VT,   q.ldvt,
                           (int64_t)(uintptr_t)q.n_r,  0};
    key = fnv1a(key, f, sizeof(f));
  }
  c->status_valid = 1;
  c->status_pairs = 1;
  if (!mixed)
    return batch_run(c, L, dtype, 0, count, pr, nullptr, use_graph != 0, fnv1a(key, "p0", 2));
  rc = batch_run(c, L, dtype, 1, count, pr, nullptr, use_graph != 0, fnv1a(key, "p1", 2));
  if (rc) return rc;
  std::vector<int64_t> nr0((size_t)count, 0);
  HIPCHK(c, hipMemcpyAsync(nr0.data(), (char*)c->ws + L.oNr0, sizeof(int64_t) * (size_t)count,
                           hipMemcpyDeviceToHost, c->stream), "N_r read-back");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  // phase 2 depends on the refinement widths, part of its key
  return batch_run(c, L, dtype, 2, count, pr, nr0.data(), use_graph != 0,
                   fnv1a(fnv1a(key, "p2", 2), nr0.data(), sizeof(int64_t) * (size_t)count));
}

extern "C" int pylom_pod(pylom_ctx c, pylom_dtype dtype, pylom_prec prec, int64_t m, int64_t n,
                         const void* D, int64_t ldd, int remove_mean, double residual, void* mean,
                         void* U, int64_t ldu, double* S, double* VT, int64_t ldvt, int64_t* n_r) {
  return run_tsvd(c, dtype, prec, m, n, D, ldd, remove_mean ? 1 : 0, residual, mean, U, ldu, S, VT,
                  ldvt, n_r);
}

extern "C" int pylom_tsvd(pylom_ctx c, pylom_dtype dtype, pylom_prec prec, int64_t m, int64_t n,
                          const void* A, int64_t lda, double residual, void* U, int64_t ldu,
                          double* S, double* VT, int64_t ldvt, int64_t* n_r) {
  return run_tsvd(c, dtype, prec, m, n, A, lda, 0, residual, nullptr, U, ldu, S, VT, ldvt, n_r);
}

extern "C" int pylom_tsqr(pylom_ctx c, pylom_dtype dtype, pylom_prec prec, int64_t m, int64_t n,
                          const void* A, int64_t lda, void* Q, int64_t ldq, double* R,
                          int64_t ldr) {
  int rc = check_common(c, dtype, prec);
  if (rc) return rc;
  if (!A || !R) return fail(c, PYLOM_EINVAL, "null array argument");
  if (n < 1 || m < n) return fail(c, PYLOM_ESHAPE, "need m >= n >= 1");
  if (lda < n || ldr < n || (Q && ldq < n)) return fail(c, PYLOM_ESHAPE, "leading dimension < n");
  Plan p;
  rc = make_plan(c, m, n, Q != nullptr, &p);
  if (rc) return rc;
  if ((rc = cap_check(c, p.total))) return rc;
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
  rc = ensure_ws(c, p.total);
  if (rc) return rc;
  char* ws = (char*)c->ws;
  const bool wq = Q != nullptr;
  if (p.blocked) {
    hipStream_t st = c->stream;
    const int in64 = dtype == PYLOM_R64;
    double* Rbuf = (double*)(ws + p.oR);
    double* signs = (double*)(ws + p.oSig);
    HIPCHK(c, launch_make_work(in64, 1, m, (int)n, A, lda, 0, nullptr, ws + p.oWk, st),
           "working copy");
    rc = blocked_leaves<double>(c, st, p, ws, Rbuf);
    if (rc) return rc;
    rc = blocked_tree<double>(c, st, p, ws, (double*)(ws + p.oR), 1, -1, true);
    if (rc) return rc;
    HIPCHK(c, launch_r_out(Rbuf, n, R, ldr, signs, st), "R out");
    if (wq) {
      HIPCHK(c, launch_eye((double*)(ws + p.oW), n, n, st), "identity");
      rc = blocked_propagate(c, st, p, ws, nullptr, n);
      if (rc) return rc;
      rc = blocked_leaf_apply(c, st, p, ws, nullptr, n, Q, in64, ldq);
      if (rc) return rc;
      HIPCHK(c, launch_q_signs(Q, in64, m, n, ldq, signs, st), "Q signs");
    }
    return PYLOM_OK;
  }
  double* V = wq ? (double*)(ws + p.oV) : nullptr;
  double* Tleaf = (double*)(ws + p.oTleaf);
  double* Rbuf = (double*)(ws + p.oR);
  double* Ttree = (double*)(ws + p.oTtree);
  double* W = (double*)(ws + p.oW);
  double* signs = (double*)(ws + p.oSig);
  hipStream_t st = c->stream;
  const int in64 = dtype == PYLOM_R64;
  HIPCHK(c, launch_leaf_qr_f64(p.g, A, in64, lda, m, p.b, p.P, 0, nullptr, V, Tleaf, p.nch_leaf,
                               Rbuf, st), "leaf QR");
  for (int64_t h = 1; h < p.P; h *= 2)
    HIPCHK(c, launch_tree_combine_f64(p.g, h, p.P, Rbuf, Ttree, p.nch_tree, wq ? 1 : 0, st),
           "tree combine");
  HIPCHK(c, launch_r_out(Rbuf, n, R, ldr, signs, st), "R out");
  if (wq) {
    HIPCHK(c, launch_eye(W, n, n, st), "identity");
    int64_t top = 1;
    while (top * 2 < p.P) top *= 2;
    if (p.P > 1)
      for (int64_t h = top; h >= 1; h /= 2)
        HIPCHK(c, launch_apply_tree_f64(p.g, h, p.P, Rbuf, Ttree, p.nch_tree, W, n, nullptr, n, st),
               "tree propagation");
    HIPCHK(c, launch_apply_leaf_f64(p.g, m, p.b, p.P, V, Tleaf, p.nch_leaf, W, n, nullptr, n, Q,
                                    in64, ldq, st), "leaf apply");
    HIPCHK(c, launch_q_signs(Q, in64, m, n, ldq, signs, st), "Q signs");
  }
  return PYLOM_OK;
}

extern "C" int pylom_matmul(pylom_ctx c, pylom_dtype dtype, pylom_prec prec, int trans_a,
                            int64_t m, int64_t p, int64_t q, const void* A, int64_t lda,
                            const void* B, int64_t ldb, void* C, int64_t ldc) {
  int rc = check_common(c, dtype, prec);
  if (rc) return rc;
  if (!A || !B || !C) return fail(c, PYLOM_EINVAL, "null array argument");
  if (m < 1 || p < 1 || q < 1) return fail(c, PYLOM_ESHAPE, "empty matrix");
  const int f64 = dtype == PYLOM_R64;
  if (trans_a) {
    if (lda < p || ldb < q || ldc < q) return fail(c, PYLOM_ESHAPE, "leading dimension");
    if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
    HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
    const int64_t ns = matmul_tn_splits(m, p, q);
    rc = ensure_ws(c, align_up(sizeof(double) * (size_t)ns * p * q));
    if (rc) return rc;
    HIPCHK(c, launch_matmul_tn(f64, m, p, q, A, lda, B, ldb, C, ldc, (double*)c->ws, ns, c->stream),
           "matmul tn");
  } else {
    if (lda < p || ldb < q || ldc < q) return fail(c, PYLOM_ESHAPE, "leading dimension");
    if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
    HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
    HIPCHK(c, launch_matmul_nn(f64, m, p, q, A, lda, B, ldb, C, ldc, c->stream), "matmul nn");
  }
  return PYLOM_OK;
}

// Alg. 4 as pylom_matmul, for callers that cannot allocate: the split-K
// partials of trans_a = 1 go to the device's fixed scratch (kScratchBytes),
// with fewer row splits when the usual count would not fit.  Every split
// writes its whole p x q partial, so nothing in the scratch needs clearing.
// Calls that overlap on one device race on the scratch.
extern "C" int pylom_matmul_noalloc(pylom_ctx c, pylom_dtype dtype, pylom_prec prec, int trans_a,
                                    int64_t m, int64_t p, int64_t q, const void* A, int64_t lda,
                                    const void* B, int64_t ldb, void* C, int64_t ldc) {
  int rc = check_common(c, dtype, prec);
  if (rc) return rc;
  if (!A || !B || !C) return fail(c, PYLOM_EINVAL, "null array argument");
  if (m < 1 || p < 1 || q < 1) return fail(c, PYLOM_ESHAPE, "empty matrix");
  if (lda < p || ldb < q || ldc < q) return fail(c, PYLOM_ESHAPE, "leading dimension");
  const int f64 = dtype == PYLOM_R64;
  const size_t one = sizeof(double) * (size_t)p * (size_t)q;
  if (trans_a && one > kScratchBytes)
    return fail(c, PYLOM_ENOMEM, "p x q partial sums exceed the 32 MiB static scratch");
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
  if (trans_a) {
    void* part = scratch_ptr[c->device];
    if (!part) return fail(c, PYLOM_ENODEV, "device scratch not set up");
    int64_t ns = matmul_tn_splits(m, p, q);
    const int64_t fit = (int64_t)(kScratchBytes / one);
    if (ns > fit) ns = fit;
    HIPCHK(c, launch_matmul_tn(f64, m, p, q, A, lda, B, ldb, C, ldc, (double*)part, ns, c->stream),
           "matmul tn");
  } else {
    HIPCHK(c, launch_matmul_nn(f64, m, p, q, A, lda, B, ldb, C, ldc, c->stream), "matmul nn");
  }
  return PYLOM_OK;
}

// ---------------------------------------------------------------------------
// exact DMD (Sec. 3.2, Alg. 3-5)
// ---------------------------------------------------------------------------
struct DmdLayout {
  size_t oRf, oR1, oS, oVT, oUR, oSvd, oNr, oAux, oPart, oA, oH0, oQv, oQtau, oWr, oWi, oHn, oW,
      oUb, oP, oQ, oB, oMu, oBo, oPerm, oBr, total;
};

// The R-only TSQR plan of all n snapshots first, then the DMD buffers, sized
// for the widest linear map the eigen-solver takes.
static int make_dmd_layout(pylom_ctx c, int64_t m, int64_t n, Plan* p, JacobiPlan* jp1,
                           DmdLayout* L) {
  const int64_t n1 = n - 1;
  int rc = make_plan(c, m, n, false, p);
  if (rc) return rc;
  if (!jacobi_plan((int)n1, jp1)) return fail(c, PYLOM_ENOTSUP, "no Jacobi plan");
  const int64_t kc = std::min<int64_t>(n1, kDmdMax);
  size_t off = align_up(p->total);
  auto take = [&off](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L->oRf = take(8 * (size_t)n * n);
  L->oR1 = take(8 * (size_t)n1 * n1);
  L->oS = take(8 * (size_t)n1);
  L->oVT = take(8 * (size_t)n1 * n1);
  L->oUR = take(8 * (size_t)n1 * n1);
  L->oSvd = take(jacobi_ws_bytes(*jp1, (int)c->max_sweeps));
  L->oNr = take(8);
  size_t part = 0;
  for (int64_t k = 1; k <= kc; ++k)
    part = std::max(part, 8 * (size_t)matmul_tn_splits(n1, k, n1) * k * n1);
  L->oAux = take(8 * (size_t)kc * n1);
  L->oPart = take(part);
  L->oA = take(8 * (size_t)kc * kc);
  L->oH0 = take(8 * (size_t)kc * kc);
  L->oQv = take(8 * (size_t)kc * kc);
  L->oQtau = take(8 * (size_t)kc);
  L->oWr = take(8 * (size_t)kc);
  L->oWi = take(8 * (size_t)kc);
  L->oHn = take(8);
  L->oW = take(16 * (size_t)kc * kc);
  L->oUb = take(16 * (size_t)kc * kc * kc);
  L->oP = take(16 * (size_t)kc * kc);
  L->oQ = take(16 * (size_t)kc);
  L->oB = take(16 * (size_t)kc);
  L->oMu = take(16 * (size_t)kc);
  L->oBo = take(16 * (size_t)kc);
  L->oPerm = take(4 * (size_t)kc);
  L->oBr = take(8 * (size_t)n1 * 2 * kc);
  L->total = off;
  return PYLOM_OK;
}

extern "C" int pylom_dmd_workspace_query(pylom_ctx c, pylom_dtype dtype, int64_t m, int64_t n,
                                         int remove_mean, size_t* bytes) {
  (void)remove_mean;
  if (!c || !bytes) return PYLOM_EINVAL;
  if (dtype != PYLOM_R64 && dtype != PYLOM_R32) return fail(c, PYLOM_EDTYPE, "dtype");
  if (n < 2 || m < n) return fail(c, PYLOM_ESHAPE, "need n >= 2 snapshots and m >= n");
  Plan p;
  JacobiPlan jp1;
  DmdLayout L;
  const int rc = make_dmd_layout(c, m, n, &p, &jp1, &L);
  if (rc) return rc;
  *bytes = L.total;
  return PYLOM_OK;
}

// Exact DMD.  The TS-SVD of Y1 and the product U^T Y2 of Alg. 3-4 come from
// one R-only TSQR of all n snapshots: with Y = Q_f R_f, the first n - 1
// columns of R_f are [R1; 0], so Y1 = Q_f[:, :n-1] R1, the SVD
// R1 = U_R S W^T gives U = Q_f[:, :n-1] U_R, and U^T Y2 = U_R^T R_f[:n-1, 1:]
// (exact; no reflector storage, no U, no pass over the data for U^T Y2).
// The QR's mean removal runs over all n snapshots, as the DMD mean does.
extern "C" int pylom_dmd(pylom_ctx c, pylom_dtype dtype, int64_t m, int64_t n, const void* D,
                         int64_t ldd, int remove_mean, double residual, double dt, void* phi,
                         int64_t ldphi, void* mu, void* b, double* freq, double* growth,
                         int64_t* n_r) {
  int rc = check_common(c, dtype, PYLOM_FP64);
  if (rc) return rc;
  if (!D || !phi || !mu || !b || !n_r) return fail(c, PYLOM_EINVAL, "null array argument");
  if (!(residual >= 0.0 && residual < 1.0)) return fail(c, PYLOM_EINVAL, "residual must be in [0, 1)");
  if (!(dt > 0.0)) return fail(c, PYLOM_EINVAL, "dt must be positive");
  if (n < 2 || m < n) return fail(c, PYLOM_ESHAPE, "need n >= 2 snapshots and m >= n");
  const int64_t n1 = n - 1, kc = std::min<int64_t>(n1, kDmdMax);
  if (ldd < n || ldphi < kc) return fail(c, PYLOM_ESHAPE, "leading dimension");
  Plan p;
  JacobiPlan jp1;
  DmdLayout L;
  rc = make_dmd_layout(c, m, n, &p, &jp1, &L);
  if (rc) return rc;
  if ((rc = cap_check(c, L.total))) return rc;
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
  rc = ensure_ws(c, L.total);
  if (rc) return rc;
  Exec x = ctx_exec(c);
  x.evs = nullptr;  // the phase ring times pod/tsvd calls only
  char* ws = x.ws;
  const hipStream_t st = x.st;
  const int in64 = dtype == PYLOM_R64;
  double* meanws = (double*)(ws + p.oMean);
  double* Rbuf = (double*)(ws + p.oR);
  // R-only TSQR of Y = D - mean 1^T (Alg. 2 + Alg. 1 reduce)
  if (p.blocked) {
    HIPCHK(c, launch_make_work(in64, 1, m, (int)n, D, ldd, remove_mean, meanws, ws + p.oWk, st),
           "working copy");
    rc = blocked_leaves<double>(c, st, p, ws, Rbuf);
    if (rc) return rc;
    rc = blocked_tree<double>(c, st, p, ws, (double*)(ws + p.oR), 1, -1, true);
    if (rc) return rc;
  } else {
    HIPCHK(c, launch_leaf_qr_f64(p.g, D, in64, ldd, m, p.b, p.P, remove_mean, meanws, nullptr,
                                 (double*)(ws + p.oTleaf), p.nch_leaf, Rbuf, st), "leaf QR");
    for (int64_t h = 1; h < p.P; h *= 2)
      HIPCHK(c, launch_tree_combine_f64(p.g, h, p.P, Rbuf, (double*)(ws + p.oTtree), p.nch_tree,
                                        0, st), "tree combine");
  }
  double* Rf = (double*)(ws + L.oRf);
  double* R1 = (double*)(ws + L.oR1);
  double* S = (double*)(ws + L.oS);
  double* VT = (double*)(ws + L.oVT);
  double* UR = (double*)(ws + L.oUR);
  int64_t* nr_dev = (int64_t*)(ws + L.oNr);
  HIPCHK(c, launch_r_out(Rbuf, n, Rf, n, nullptr, st), "R out");
  HIPCHK(c, launch_dmd_r1(n1, n, Rf, R1, st), "R1");
  // SVD of R1 = the SVD of Y1 (Eq. svdqr2) and truncation
  HIPCHK(c, launch_small_svd(jp1, R1, x.max_sweeps, ws + L.oSvd, S, VT, n1, UR, residual, nr_dev,
                             x.status, st, x.coop), "small SVD");
  c->status_valid = 1;
  c->status_pairs = 1;
  int64_t k = 0;
  std::vector<double> Sh((size_t)n1);
  HIPCHK(c, hipMemcpyAsync(&k, nr_dev, sizeof(int64_t), hipMemcpyDeviceToHost, st), "N_r read-back");
  HIPCHK(c, hipMemcpyAsync(Sh.data(), S, sizeof(double) * (size_t)n1, hipMemcpyDeviceToHost, st),
         "S read-back");
  HIPCHK(c, hipStreamSynchronize(st), "hipStreamSynchronize");
  if (k == 0) {
    HIPCHK(c, launch_set_i64(n_r, 0, st), "N_r");
    return PYLOM_OK;
  }
  if (k > kDmdMax) return fail(c, PYLOM_ENOTSUP, "DMD keeps at most 128 modes: raise the residual");
  if (!(Sh[(size_t)k - 1] > 0.0))
    return fail(c, PYLOM_ENOTSUP, "a retained singular value is zero: raise the residual");
  // U^T Y2 = U_R[:, :k]^T R_f[:n-1, 1:] (the product of Alg. 4 on the n - 1
  // rows that span Y1)
  HIPCHK(c, launch_matmul_tn(1, n1, k, n1, UR, n1, Rf + 1, n, ws + L.oAux, n1,
                             (double*)(ws + L.oPart), matmul_tn_splits(n1, k, n1), st), "U^T Y2");
  DmdSmallArgs a{};
  a.k = (int)k;
  a.n1 = (int)n1;
  a.dt = dt;
  a.aux = (const double*)(ws + L.oAux);
  a.VT = VT;
  a.ldvt = n1;
  a.S = S;
  a.A = (double*)(ws + L.oA);
  a.H0 = (double*)(ws + L.oH0);
  a.Qv = (double*)(ws + L.oQv);
  a.Qtau = (double*)(ws + L.oQtau);
  a.wr = (double*)(ws + L.oWr);
  a.wi = (double*)(ws + L.oWi);
  a.hnorm = (double*)(ws + L.oHn);
  a.status = x.status + 2;
  a.Ubuf = (double2*)(ws + L.oUb);
  a.W = (double2*)(ws + L.oW);
  a.P = (double2*)(ws + L.oP);
  a.q = (double2*)(ws + L.oQ);
  a.b = (double2*)(ws + L.oB);
  a.mu_out = (double2*)mu;
  a.b_out = (double2*)b;
  a.freq = freq;
  a.growth = growth;
  a.perm = (int*)(ws + L.oPerm);
  a.B = (double*)(ws + L.oBr);
  HIPCHK(c, launch_dmd_small(a, st), "DMD eigen-solve and amplitudes");
  c->status_pairs = 2;
  // phi = (D[:, 1:] - mean 1^T) B (Eq. dmdmodes), interleaved complex
  const void* D2 = in64 ? (const void*)((const double*)D + 1) : (const void*)((const float*)D + 1);
  HIPCHK(c, launch_tall_gemm_mu(in64, m, (int)n1, (int)(2 * k), D2, ldd,
                                remove_mean ? meanws : nullptr, a.B, 2 * k, (double*)phi,
                                2 * ldphi, st), "modes");
  HIPCHK(c, launch_set_i64(n_r, k, st), "N_r");
  return PYLOM_OK;
}

// ---------------------------------------------------------------------------
// out-of-core POD: row windows streamed from host memory (matrices larger
// than the device)
// ---------------------------------------------------------------------------
// The column-blocked TSQR of the whole matrix with the rows held in host
// memory.  Only the tree part (every leaf's R, the tree reflectors, the
// propagation W, the mean and the SVD workspace: O(P n^2 + m) bytes) lives in
// the device for the whole call; the rows pass through a window of wl leaves
// twice.  Pass 1 streams each window in, removes the mean, factors its leaves
// and keeps their R.  Then the tree, the SVD of R and the down-tree
// propagation run once.  Pass 2 streams each window in again, factors its
// leaves again (the same arithmetic on the same rows gives the same
// reflectors, so no reflector ever leaves the device) and forms its rows of
// U = Q [W; 0], which stream out.  The leaves, their R and every reflector
// are those of the in-device column-blocked path at the same leaf height:
// the results are identical.
struct OocLayout {
  Plan full;          // leaf geometry of the whole matrix and the tree part
  int64_t wl = 0;     // leaves per window
  int64_t nwin = 0;   // windows
  int64_t wrows = 0;  // rows of the largest window
  size_t oS = 0, oVT = 0, oNr = 0, oMeanOut = 0;
  size_t oDin[2] = {}, oUo[2] = {};
  size_t total = 0;
};

// Rows [r0, r1) and leaves [l0, l1) of window w.
static void ooc_window(const OocLayout& L, int64_t w, int64_t* r0, int64_t* r1, int64_t* l0,
                       int64_t* l1) {
  const Plan& p = L.full;
  *l0 = w * L.wl;
  *l1 = std::min(p.P, *l0 + L.wl);
  *r0 = *l0 * p.b;
  *r1 = (*l1 == p.P) ? p.m : *l1 * p.b;
}

static int make_ooc_layout(pylom_ctx c, int64_t m, int64_t n, int in64, OocLayout* L) {
  if (n < 1 || m < n) return fail(c, PYLOM_ESHAPE, "need m >= n >= 1");
  if (n > kMaxN) return fail(c, PYLOM_ENOTSUP, "n > 2048 is not supported");
  Plan& p = L->full;
  p.m = m;
  p.n = n;
  p.mixed = false;
  p.blocked = true;
  p.zcap = n;
  // default window: 2^20 rows (at least 4 n), at most the whole matrix
  int64_t wr = c->ooc_window_rows > 0 ? c->ooc_window_rows : ((int64_t)1 << 20);
  if (wr < 4 * n) wr = 4 * n;
  if (wr > m) wr = m;
  int64_t b = c->block_rows > 0 ? c->block_rows : blocked_block_rows(wr, n, c->ncu);
  if (b < n) b = n;
  if (b > wr) b = wr;
  int64_t P = m / b;
  if (P < 1) P = 1;
  if (P > 65535) return fail(c, PYLOM_ENOTSUP, "too many leaves: raise block_rows");
  p.b = b;
  p.P = P;
  p.last_rows = m - (P - 1) * b;
  p.K = (n + kPW - 1) / kPW;
  if (!qr_geom((int)(n < kPW ? n : kPW), 8, &p.gp) ||
      !qr_geom((int)(n - (p.K - 1) * kPW), 8, &p.gpl) || p.gp.s != kPW || p.gpl.s != kPW)
    return fail(c, PYLOM_ENOTSUP, "no panel geometry");
  if (!jacobi_plan((int)n, &p.jp)) return fail(c, PYLOM_ENOTSUP, "no Jacobi plan");
  p.g = p.gp;
  p.nch_l = (p.last_rows + kPW - 1) / kPW;  // the largest leaf sets the T-factor slots
  p.nch_p = (n + kPW - 1) / kPW;
  p.nch_leaf = p.nch_l;
  p.nch_tree = p.nch_p;
  int64_t lv = 0;
  for (int64_t h = 1; h < P; h *= 2) ++lv;
  p.levels = lv;
  p.wcap = n < 256 ? n : 256;
  L->wl = std::max<int64_t>(1, wr / b);
  L->nwin = (P + L->wl - 1) / L->wl;
  {
    int64_t r0, r1, l0, l1;
    ooc_window(*L, L->nwin - 1, &r0, &r1, &l0, &l1);
    L->wrows = std::max(L->wl * b, r1 - r0);
  }
  const int es = in64 ? 8 : 4;
  const size_t tps = (size_t)kTF;
  const int64_t np_all = P - 1;
  size_t off = 0;
  auto take = [&off](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  // tree part
  p.oR = take(8 * (size_t)P * n * n);
  p.oTp = take(8 * (size_t)p.K * np_all * p.nch_p * 4 * tps);
  p.oPSp = take(8 * (size_t)p.K * np_all * kPW * kPW);
  p.oW = take(8 * (size_t)P * n * n);
  p.oMean = take(8 * (size_t)m);
  p.oSig = take(8 * (size_t)n);
  p.oSvd = take(jacobi_ws_bytes(p.jp, (int)c->max_sweeps));
  L->oS = take(8 * (size_t)n);
  L->oVT = take(8 * (size_t)n * n);
  L->oNr = take(8);
  L->oMeanOut = take((size_t)es * m);
  // window part: working copy, leaf T factors and panel states, the FP64
  // column-group buffer of the apply, two input and two output windows
  p.oWk = take(8 * (size_t)L->wrows * n);
  p.oTl = take(8 * (size_t)p.K * L->wl * p.nch_l * 4 * tps);
  p.oPSl = take(8 * (size_t)p.K * L->wl * kPW * kPW);
  p.oXu = take(8 * (size_t)L->wrows * p.wcap);
  for (int k = 0; k < 2; ++k) L->oDin[k] = take((size_t)es * L->wrows * n);
  for (int k = 0; k < 2; ++k) L->oUo[k] = take((size_t)es * L->wrows * n);
  p.total = off;
  L->total = off;
  return PYLOM_OK;
}

// The plan of window w: its leaves and rows; R and W are those leaves' slots
// of the whole-matrix buffers.
static Plan ooc_window_plan(const OocLayout& L, int64_t w) {
  int64_t r0, r1, l0, l1;
  ooc_window(L, w, &r0, &r1, &l0, &l1);
  Plan pw = L.full;
  const int64_t n = pw.n;
  pw.m = r1 - r0;
  pw.P = l1 - l0;
  pw.last_rows = pw.m - (pw.P - 1) * pw.b;
  pw.oR = L.full.oR + 8 * (size_t)l0 * n * n;
  pw.oW = L.full.oW + 8 * (size_t)l0 * n * n;
  return pw;
}

// Host rows [r0, r1) of a row-major matrix with leading dimension ld
// (elements of es bytes) to or from a packed buffer of `cols` columns, on
// several host threads.
static void host_rows_copy(char* dst, int64_t ldd_dst, const char* src, int64_t ld_src,
                           int64_t rows, int64_t cols, int es) {
  const size_t row_bytes = (size_t)cols * es;
  const size_t total = row_bytes * (size_t)rows;
  unsigned nt = std::thread::hardware_concurrency();
  if (nt < 1) nt = 1;
  if (nt > 8) nt = 8;
  if (total < ((size_t)8 << 20)) nt = 1;
  auto work = [&](int64_t a, int64_t b) {
    if (ldd_dst == cols && ld_src == cols) {
      std::memcpy(dst + (size_t)a * row_bytes, src + (size_t)a * row_bytes,
                  (size_t)(b - a) * row_bytes);
      return;
    }
    for (int64_t r = a; r < b; ++r)
      std::memcpy(dst + (size_t)r * ldd_dst * es, src + (size_t)r * ld_src * es, row_bytes);
  };
  if (nt == 1) {
    work(0, rows);
    return;
  }
  std::vector<std::thread> th;
  const int64_t per = (rows + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    const int64_t a = t * per, b = std::min(rows, a + per);
    if (a < b) th.emplace_back(work, a, b);
  }
  for (auto& t : th) t.join();
}

static int ooc_resources(pylom_ctx c, size_t pin_bytes) {
  if (!c->cs_in)
    HIPCHK(c, hipStreamCreateWithFlags(&c->cs_in, hipStreamNonBlocking), "hipStreamCreate");
  if (!c->cs_out)
    HIPCHK(c, hipStreamCreateWithFlags(&c->cs_out, hipStreamNonBlocking), "hipStreamCreate");
  for (hipEvent_t& e : c->ooc_ev)
    if (!e) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
  if (c->pin_bytes < pin_bytes) {
    for (int k = 0; k < 2; ++k) {
      if (c->pin_in[k]) hipHostFree(c->pin_in[k]);
      if (c->pin_out[k]) hipHostFree(c->pin_out[k]);
      c->pin_in[k] = c->pin_out[k] = nullptr;
    }
    c->pin_bytes = 0;
    for (int k = 0; k < 2; ++k) {
      if (hipHostMalloc(&c->pin_in[k], pin_bytes, hipHostMallocDefault) != hipSuccess ||
          hipHostMalloc(&c->pin_out[k], pin_bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, PYLOM_ENOMEM, "pinned host staging allocation failed");
      }
    }
    c->pin_bytes = pin_bytes;
  }
  return PYLOM_OK;
}

extern "C" int pylom_ooc_workspace_query(pylom_ctx c, pylom_dtype dtype, int64_t m, int64_t n,
                                         size_t* bytes, int64_t* window_rows, int64_t* windows) {
  if (!c || !bytes) return PYLOM_EINVAL;
  if (dtype != PYLOM_R64 && dtype != PYLOM_R32) return fail(c, PYLOM_EDTYPE, "dtype");
  OocLayout L;
  const int rc = make_ooc_layout(c, m, n, dtype == PYLOM_R64, &L);
  if (rc) return rc;
  *bytes = L.total;
  if (window_rows) *window_rows = L.wl * L.full.b;
  if (windows) *windows = L.nwin;
  return PYLOM_OK;
}

extern "C" int pylom_pod_host(pylom_ctx c, pylom_dtype dtype, pylom_prec prec, int64_t m,
                              int64_t n, const void* D, int64_t ldd, int remove_mean,
                              double residual, void* mean, void* U, int64_t ldu, double* S,
                              double* VT, int64_t ldvt, int64_t* n_r) {
  int rc = check_common(c, dtype, prec);
  if (rc) return rc;
  if (prec != PYLOM_FP64) return fail(c, PYLOM_ENOTSUP, "the out-of-core path computes in FP64");
  if (!D || !U || !S || !VT || !n_r) return fail(c, PYLOM_EINVAL, "null array argument");
  if (!(residual >= 0.0 && residual < 1.0)) return fail(c, PYLOM_EINVAL, "residual must be in [0, 1)");
  if (n < 1 || m < n) return fail(c, PYLOM_ESHAPE, "need m >= n >= 1");
  if (ldd < n || ldu < n || ldvt < n) return fail(c, PYLOM_ESHAPE, "leading dimension < n");
  const int in64 = dtype == PYLOM_R64;
  const int es = in64 ? 8 : 4;
  OocLayout L;
  rc = make_ooc_layout(c, m, n, in64, &L);
  if (rc) return rc;
  if ((rc = cap_check(c, L.total))) return rc;
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
  rc = ensure_ws(c, L.total);
  if (rc) return rc;
  const size_t win_bytes = (size_t)es * L.wrows * n;
  rc = ooc_resources(c, win_bytes);
  if (rc) return rc;
  const Plan& p = L.full;
  char* ws = (char*)c->ws;
  hipStream_t st = c->stream;
  hipEvent_t* ev_h2d = c->ooc_ev;      // [2] window copied in
  hipEvent_t* ev_free = c->ooc_ev + 2; // [2] the device input window is free again
  hipEvent_t* ev_u = c->ooc_ev + 4;    // [2] U window formed
  hipEvent_t* ev_d2h = c->ooc_ev + 6;  // [2] U window copied out
  double* meanws = (double*)(ws + p.oMean);
  // the compute stream's earlier work precedes the copies
  HIPCHK(c, hipEventRecord(ev_free[0], st), "hipEventRecord");
  HIPCHK(c, hipEventRecord(ev_free[1], st), "hipEventRecord");
  HIPCHK(c, hipEventRecord(ev_h2d[0], st), "hipEventRecord");
  HIPCHK(c, hipEventRecord(ev_h2d[1], st), "hipEventRecord");
  HIPCHK(c, hipEventRecord(ev_d2h[0], st), "hipEventRecord");
  HIPCHK(c, hipEventRecord(ev_d2h[1], st), "hipEventRecord");

  // stage window w into device buffer k: the host copy into the pinned
  // buffer waits for that buffer's previous transfer; the transfer waits for
  // the compute that last read the device buffer
  auto stage_in = [&](int64_t w, int k) -> int {
    int64_t r0, r1, l0, l1;
    ooc_window(L, w, &r0, &r1, &l0, &l1);
    HIPCHK(c, hipEventSynchronize(ev_h2d[k]), "hipEventSynchronize");
    host_rows_copy((char*)c->pin_in[k], n, (const char*)D + (size_t)r0 * ldd * es, ldd, r1 - r0,
                   n, es);
    HIPCHK(c, hipStreamWaitEvent(c->cs_in, ev_free[k], 0), "hipStreamWaitEvent");
    HIPCHK(c, hipMemcpyAsync(ws + L.oDin[k], c->pin_in[k], (size_t)es * (r1 - r0) * n,
                             hipMemcpyHostToDevice, c->cs_in), "window in");
    HIPCHK(c, hipEventRecord(ev_h2d[k], c->cs_in), "hipEventRecord");
    HIPCHK(c, hipStreamWaitEvent(st, ev_h2d[k], 0), "hipStreamWaitEvent");
    return PYLOM_OK;
  };
  // leaf QR of window w from device buffer k (mean removal fused)
  auto factor = [&](int64_t w, int k) -> int {
    int64_t r0, r1, l0, l1;
    ooc_window(L, w, &r0, &r1, &l0, &l1);
    const Plan pw = ooc_window_plan(L, w);
    KT(KR_WORK, launch_make_work(in64, 1, r1 - r0, (int)n, ws + L.oDin[k], n, remove_mean,
                                 meanws + r0, ws + p.oWk, st), "working copy");
    HIPCHK(c, hipEventRecord(ev_free[k], st), "hipEventRecord");
    return blocked_leaves<double>(c, st, pw, ws, (double*)(ws + pw.oR));
  };

  // pass 1: every leaf's R
  for (int64_t w = 0; w < L.nwin; ++w) {
    const int k = (int)(w & 1);
    if ((rc = stage_in(w, k))) return rc;
    if ((rc = factor(w, k))) return rc;
  }
  // the tree, the SVD of the root R with truncation, the down-tree propagation
  rc = blocked_tree<double>(c, st, p, ws, (double*)(ws + p.oR), 1, -1, true);
  if (rc) return rc;
  double* Sd = (double*)(ws + L.oS);
  double* VTd = (double*)(ws + L.oVT);
  int64_t* nrd = (int64_t*)(ws + L.oNr);
  KT(KR_SVD, launch_small_svd(p.jp, (double*)(ws + p.oR), (int)c->max_sweeps, ws + p.oSvd, Sd,
                              VTd, n, (double*)(ws + p.oW), residual, nrd, c->status_dev, st,
                              true), "small SVD");
  c->status_valid = 1;
  c->status_pairs = 1;
  rc = blocked_propagate(c, st, p, ws, nrd, n);
  if (rc) return rc;
  int64_t nr = 0;
  HIPCHK(c, hipMemcpyAsync(&nr, nrd, sizeof(int64_t), hipMemcpyDeviceToHost, st), "N_r read-back");
  HIPCHK(c, hipStreamSynchronize(st), "hipStreamSynchronize");
  HIPCHK(c, hipMemcpy(S, Sd, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost), "S out");
  for (int64_t i = 0; i < nr; ++i)
    HIPCHK(c, hipMemcpy(VT + (size_t)i * ldvt, VTd + (size_t)i * n, sizeof(double) * (size_t)n,
                        hipMemcpyDeviceToHost), "VT out");
  *n_r = nr;
  if (remove_mean && mean) {
    HIPCHK(c, launch_cast_out(meanws, ws + L.oMeanOut, in64, m, st), "mean out");
    HIPCHK(c, hipStreamSynchronize(st), "hipStreamSynchronize");
    HIPCHK(c, hipMemcpy(mean, ws + L.oMeanOut, (size_t)es * m, hipMemcpyDeviceToHost), "mean out");
  }
  if (nr == 0) return PYLOM_OK;
  // pass 2: the leaves again, U = Q [W; 0] window by window
  auto drain = [&](int64_t w, int k) -> int {  // U rows of window w to the caller
    int64_t r0, r1, l0, l1;
    ooc_window(L, w, &r0, &r1, &l0, &l1);
    HIPCHK(c, hipEventSynchronize(ev_d2h[k]), "hipEventSynchronize");
    host_rows_copy((char*)U + (size_t)r0 * ldu * es, ldu, (const char*)c->pin_out[k], nr,
                   r1 - r0, nr, es);
    return PYLOM_OK;
  };
  for (int64_t w = 0; w < L.nwin; ++w) {
    const int k = (int)(w & 1);
    if ((rc = stage_in(w, k))) return rc;
    if ((rc = factor(w, k))) return rc;
    int64_t r0, r1, l0, l1;
    ooc_window(L, w, &r0, &r1, &l0, &l1);
    const Plan pw = ooc_window_plan(L, w);
    HIPCHK(c, hipStreamWaitEvent(st, ev_d2h[k], 0), "hipStreamWaitEvent");
    rc = blocked_leaf_apply(c, st, pw, ws, nullptr, nr, ws + L.oUo[k], in64, nr);
    if (rc) return rc;
    HIPCHK(c, hipEventRecord(ev_u[k], st), "hipEventRecord");
    if (w >= 2 && (rc = drain(w - 2, k))) return rc;  // frees pin_out[k]
    HIPCHK(c, hipStreamWaitEvent(c->cs_out, ev_u[k], 0), "hipStreamWaitEvent");
    HIPCHK(c, hipMemcpyAsync(c->pin_out[k], ws + L.oUo[k], (size_t)es * (r1 - r0) * nr,
                             hipMemcpyDeviceToHost, c->cs_out), "window out");
    HIPCHK(c, hipEventRecord(ev_d2h[k], c->cs_out), "hipEventRecord");
  }
  for (int64_t w = std::max<int64_t>(0, L.nwin - 2); w < L.nwin; ++w)
    if ((rc = drain(w, (int)(w & 1)))) return rc;
  // the context stream follows the copies
  HIPCHK(c, hipStreamSynchronize(c->cs_out), "hipStreamSynchronize");
  return PYLOM_OK;
}

// ---------------------------------------------------------------------------
// SPOD: FFT front end + one batch of realified TSQR-SVD problems
// ---------------------------------------------------------------------------
struct SpodPlan {
  int64_t m, nt, npwin, nolap, nb, nf, n, P, ldm;
  int e_f64;
  JacobiPlan jp;
  size_t oE, oTab, oScl, oRn, oVn, oVl, oWl, oRr, oSvd, oS, oVT, oUR, oNr, oSt, total;
  size_t svd_stride;
};

static int make_spod_plan(pylom_ctx c, pylom_dtype spectra, int64_t m, int64_t nt, int64_t npwin,
                          int64_t nolap, SpodPlan* p) {
  if (spectra != PYLOM_C64 && spectra != PYLOM_C128)
    return fail(c, PYLOM_EDTYPE, "spectra must be C64 or C128");
  if (npwin < 4 || npwin > 4096 || (npwin & (npwin - 1)))
    return fail(c, PYLOM_ENOTSUP, "npwin must be a power of two in [4, 4096]");
  if (nolap < 0 || nolap >= npwin) return fail(c, PYLOM_EINVAL, "need 0 <= nolap < npwin");
  if (nt < npwin) return fail(c, PYLOM_ESHAPE, "need nt >= npwin");
  const int64_t nb = (nt - nolap) / (npwin - nolap);
  if (nb < 1) return fail(c, PYLOM_ESHAPE, "no complete Welch block");
  if (nb > 16) return fail(c, PYLOM_ENOTSUP, "more than 16 Welch blocks");
  if (m < nb) return fail(c, PYLOM_ESHAPE, "need m >= number of blocks");
  p->m = m; p->nt = nt; p->npwin = npwin; p->nolap = nolap; p->nb = nb;
  p->nf = npwin / 2 + 1;
  p->n = 2 * nb;
  p->e_f64 = spectra == PYLOM_C128;
  p->P = ctsqr_leaves(m);
  p->ldm = (m + 63) / 64 * 64;
  if (p->P > 0x7fffffff) return fail(c, PYLOM_ESHAPE, "too many rows");
  if (!jacobi_plan((int)p->n, &p->jp) || p->jp.G != 1)
    return fail(c, PYLOM_ENOTSUP, "no single-workgroup Jacobi plan");
  p->svd_stride = jacobi_ws_stride(p->jp, (int)c->max_sweeps);
  const size_t es = p->e_f64 ? 8 : 4;
  const int64_t nf = p->nf, n = p->n;
  size_t off = 0;
  p->oE = off;     off = align_up(off + 2 * es * (size_t)nf * nb * p->ldm);
  p->oTab = off;   off = align_up(off + spod_table_bytes((int)npwin, p->e_f64));
  p->oScl = off;   off = align_up(off + 8);
  p->oRn = off;    off = align_up(off + ctsqr_node_bytes() * (size_t)nf * p->P);
  p->oVn = off;    off = align_up(off + ctsqr_vnode_bytes() * (size_t)nf * p->P);
  p->oVl = off;    off = align_up(off + ctsqr_leaf_v_bytes((int)nb, p->e_f64) * (size_t)nf * p->P);
  p->oWl = off;    off = align_up(off + ctsqr_node_bytes() * (size_t)nf * p->P);
  p->oRr = off;    off = align_up(off + 8 * (size_t)nf * n * n);
  p->oSvd = off;   off = align_up(off + p->svd_stride * (size_t)nf);
  p->oS = off;     off = align_up(off + 8 * (size_t)nf * n);
  p->oVT = off;    off = align_up(off + 8 * (size_t)nf * n * n);
  p->oUR = off;    off = align_up(off + 8 * (size_t)nf * n * n);
  p->oNr = off;    off = align_up(off + 8 * (size_t)nf);
  p->oSt = off;    off = align_up(off + 8 * (size_t)nf);
  p->total = off;
  return PYLOM_OK;
}

extern "C" int pylom_spod_query(pylom_ctx c, pylom_dtype spectra, int64_t m, int64_t nt,
                                int64_t npwin, int64_t nolap, int64_t* nblocks, int64_t* nfreq,
                                size_t* bytes) {
  if (!c) return PYLOM_EINVAL;
  SpodPlan p;
  const int rc = make_spod_plan(c, spectra, m, nt, npwin, nolap, &p);
  if (rc) return rc;
  if (nblocks) *nblocks = p.nb;
  if (nfreq) *nfreq = p.nf;
  if (bytes) *bytes = p.total;
  return PYLOM_OK;
}

extern "C" int pylom_spod(pylom_ctx c, pylom_dtype spectra, pylom_prec prec, int64_t m,
                          int64_t nt, const float* D, int64_t ldd, double dt, int64_t npwin,
                          int64_t nolap, int window, int remove_mean, void* modes, double* L,
                          double* freqs, int64_t* order) {
  if (!c) return PYLOM_EINVAL;
  if (prec != PYLOM_FP64) return fail(c, PYLOM_ENOTSUP, "SPOD runs the FP64 TSQR-SVD only");
  if (!D || !modes || !L) return fail(c, PYLOM_EINVAL, "null array argument");
  if (!(dt > 0.0)) return fail(c, PYLOM_EINVAL, "dt must be > 0");
  if (window != 0 && window != 1) return fail(c, PYLOM_EINVAL, "window must be 0 (Hann) or 1 (Hamming)");
  if (m < 1 || nt < 1) return fail(c, PYLOM_ESHAPE, "empty snapshot matrix");
  if (ldd < nt) return fail(c, PYLOM_ESHAPE, "leading dimension < nt");
  SpodPlan p;
  int rc = make_spod_plan(c, spectra, m, nt, npwin, nolap, &p);
  if (rc) return rc;
  if ((rc = cap_check(c, p.total))) return rc;
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
  rc = ensure_ws(c, p.total);
  if (rc) return rc;
  char* ws = (char*)c->ws;
  void* E = ws + p.oE;
  double* Rn = (double*)(ws + p.oRn);
  double* Vn = (double*)(ws + p.oVn);
  double* Rr = (double*)(ws + p.oRr);
  double* S = (double*)(ws + p.oS);
  double* VTb = (double*)(ws + p.oVT);
  double* URb = (double*)(ws + p.oUR);
  int64_t* nr = (int64_t*)(ws + p.oNr);
  int* st_each = (int*)(ws + p.oSt);
  hipStream_t st = c->stream;
  const int64_t n = p.n, nb = p.nb, nf = p.nf, P = p.P;
  const bool tm = c->timing > 0 && !c->ev.empty();
  hipEvent_t* evs = tm ? &c->ev[(size_t)(c->ev_calls % c->timing) * kEvPerSlot] : nullptr;
  if (tm) c->ev_mixed[(size_t)(c->ev_calls % c->timing)] = 0;
#define EVREC(j) \
  if (tm) HIPCHK(c, hipEventRecord(evs[j], st), "hipEventRecord")

  EVREC(0);
  HIPCHK(c, launch_spod_front(p.e_f64, m, nt, D, ldd, (int)npwin, (int)nolap, (int)nb, window,
                              remove_mean, ws + p.oTab, (double*)(ws + p.oScl), E, p.ldm, st),
         "SPOD front end");
  EVREC(1);
  void* Vl = ws + p.oVl;
  double* Wl = (double*)(ws + p.oWl);
  HIPCHK(c, launch_cleaf(p.e_f64, 0, (int)nb, m, p.ldm, P, nf, E, Rn, Vl, Wl, nullptr, nullptr,
                         st), "leaf QR");
  EVREC(2);
  for (int64_t h = 1; h < P; h *= 2)
    HIPCHK(c, launch_ctree_combine((int)nb, P, h, nf, Rn, Vn, st), "tree combine");
  EVREC(3);
  HIPCHK(c, launch_spod_root_realify((int)nb, P, nf, Rn, Rr, st), "root embedding");
  HIPCHK(c, launch_small_svd_batched(p.jp, nf, Rr, n * n, (int)c->max_sweeps, ws + p.oSvd, S, n,
                                     VTb, n, n * n, URb, n * n, 0.0, nr, st_each, c->status_dev,
                                     st), "batched SVD");
  c->status_valid = 1;
  c->status_pairs = 1;
  // the root blocks of Rn become the down-tree factors C
  HIPCHK(c, launch_spod_root_modes((int)nb, P, nf, S, VTb, URb, Rn, L, st), "root modes");
  EVREC(4);
  int64_t top = 1;
  while (top * 2 < P) top *= 2;
  if (P > 1)
    for (int64_t h = top; h >= 1; h /= 2)
      HIPCHK(c, launch_ctree_apply((int)nb, P, h, nf, Rn, Vn, st), "tree propagation");
  EVREC(5);
  HIPCHK(c, launch_cleaf(p.e_f64, 1, (int)nb, m, p.ldm, P, nf, nullptr, nullptr, Vl, Wl, Rn,
                         modes, st), "leaf apply");
  HIPCHK(c, launch_spod_order((int)nf, (int)nb, dt, (int)npwin, L, freqs, order, st), "order");
  EVREC(6);
#undef EVREC
  if (tm) ++c->ev_calls;
  return PYLOM_OK;
}

extern "C" int pylom_phase_times(pylom_ctx c, double* out, int cap) {
  if (!c || (cap > 0 && !out)) return PYLOM_EINVAL;
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  if (c->timing <= 0 || c->ev_calls == 0) return fail(c, PYLOM_EINVAL, "no timed call recorded");
  const int64_t nrec = c->ev_calls < c->timing ? c->ev_calls : c->timing;
  // events per slot: e0 call start, e1 after the front end (SPOD FFT, or the
  // working copy of the column-blocked path; none for the stacked POD),
  // e2..e6 after leaf QR, tree, SVD, propagation, apply; e7 (mixed
  // precision) after the first SVD, before the host read-back
  double acc[kPhases] = {0, 0, 0, 0, 0, 0};
  for (int64_t k = 0; k < nrec; ++k) {
    const int64_t slot = (c->ev_calls - 1 - k) % c->timing;
    hipEvent_t* e = &c->ev[(size_t)slot * kEvPerSlot];
    const bool mixed = c->ev_mixed[(size_t)slot] != 0;
    HIPCHK(c, hipEventSynchronize(e[6]), "hipEventSynchronize");
    for (int i = 0; i < kPhases; ++i) {
      float ms = 0.f;
      if (i == 2 && mixed)  // the first SVD ends at e7, before the host read-back
        HIPCHK(c, hipEventElapsedTime(&ms, e[3], e[7]), "hipEventElapsedTime");
      else if (i < 5)
        HIPCHK(c, hipEventElapsedTime(&ms, e[i + 1], e[i + 2]), "hipEventElapsedTime");
      else
        HIPCHK(c, hipEventElapsedTime(&ms, e[0], e[1]), "hipEventElapsedTime");
      acc[i] += ms;
    }
  }
  for (int i = 0; i < kPhases && i < cap; ++i) out[i] = acc[i] / (double)nrec;
  c->ev_calls = 0;
  return kPhases;
}

extern "C" int pylom_kernel_times(pylom_ctx c, double* ms, int64_t* launches, int cap) {
  if (!c || cap < 0 || (cap > 0 && (!ms || !launches))) return PYLOM_EINVAL;
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  if (!c->ktiming) return fail(c, PYLOM_EINVAL, "kernel_timing is off");
  HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
  double acc[KR_COUNT] = {};
  int64_t cnt[KR_COUNT] = {};
  for (const auto& mk : c->kmarks) {
    HIPCHK(c, hipEventSynchronize(c->kev[mk.second + 1]), "hipEventSynchronize");
    float t = 0.f;
    HIPCHK(c, hipEventElapsedTime(&t, c->kev[mk.second], c->kev[mk.second + 1]),
           "hipEventElapsedTime");
    acc[mk.first] += t;
    cnt[mk.first] += 1;
  }
  for (int i = 0; i < KR_COUNT && i < cap; ++i) {
    ms[i] = acc[i];
    launches[i] = cnt[i];
  }
  c->kmarks.clear();
  c->kev_next = 0;
  return KR_COUNT;
}

extern "C" int pylom_check(pylom_ctx c, int64_t* sweeps) {
  if (!c) return PYLOM_EINVAL;
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  if (!c->status_valid) {
    if (sweeps) *sweeps = 0;
    return PYLOM_OK;
  }
  int st[4] = {0, 0, 0, 0};
  HIPCHK(c, hipMemcpy(st, c->status_dev, sizeof(int) * 2 * c->status_pairs, hipMemcpyDeviceToHost),
         "status copy");
  if (sweeps) *sweeps = st[0];
  for (int k = 0; k < c->status_pairs; ++k) {
    if (st[2 * k + 1])
      return fail(c, PYLOM_EHIP, "a device-wide wait timed out (Jacobi grid barrier or work queue)");
    if (st[2 * k] == -2)
      return fail(c, PYLOM_WNONFINITE, "a singular value is not finite (non-finite input)");
  }
  for (int k = 0; k < c->status_pairs; ++k) {
    if (st[2 * k] < 0)
      return fail(c, PYLOM_WNOCONV,
                  k == 0 ? "Jacobi SVD did not converge"
                         : "second solve did not converge (Gram eigenpairs or DMD eigen/Cholesky)");
  }
  return PYLOM_OK;
}
