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

#include <cstdio>
#include <cstring>
#include <string>
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
  int* status_dev = nullptr;  // Jacobi status pairs (sweeps, barrier timeout) of the last call
  int status_valid = 0;
  int status_pairs = 1;        // 2 after a mixed-precision call (SVD of R + Gram eigen)
  int64_t timing = 0;         // number of per-call event slots (0 = off)
  std::vector<hipEvent_t> ev;  // timing x 6 events
  int64_t ev_calls = 0;        // timed calls since the last read
  std::string last_error;
};

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

constexpr int kEvPerSlot = 7;  // timing events recorded per call
constexpr int kPhases = 6;     // phases reported by pylom_phase_times

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
    c->device = device;
  }
  *out = c;
  return PYLOM_OK;
}

extern "C" int pylom_destroy(pylom_ctx c) {
  if (!c) return PYLOM_EINVAL;
  if (c->device >= 0) {
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
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
  } else if (!std::strcmp(key, "timing")) {
    if (v < 0 || v > 4096) return fail(c, PYLOM_EINVAL, "timing must be in [0, 4096]");
    if (c->device >= 0) {
      hipSetDevice(c->device);
      hipStreamSynchronize(c->stream);
      for (hipEvent_t e : c->ev)
        if (e) hipEventDestroy(e);
      c->ev.assign((size_t)v * kEvPerSlot, nullptr);
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
  else if (!std::strcmp(key, "timing"))
    *v = c->timing;
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
  // mixed precision only: FP32 leaf R, first SVD, refinement buffers
  bool mixed;
  size_t oR32, oS0, oVT0, oNr0, oZ, oG, oPart, oLam, oWT, oUR2, oNr2, oM, oSvd2;
  size_t part_bytes;
};

static int make_plan(pylom_ctx c, int64_t m, int64_t n, bool store_q, Plan* p,
                     bool mixed = false) {
  if (n < 1 || m < n) return fail(c, PYLOM_ESHAPE, "need m >= n >= 1");
  if (n > 1024) return fail(c, PYLOM_ENOTSUP, "n > 1024 is not supported");
  p->mixed = mixed;
  if (mixed) store_q = false;
  p->m = m;
  p->n = n;
  int64_t b = c->block_rows > 0 ? c->block_rows : 4096;
  if (b < n) b = n;
  int64_t P = m / b;
  if (P < 1) P = 1;
  if (P > (1 << 30)) return fail(c, PYLOM_ENOTSUP, "too many leaves");
  p->b = b;
  p->P = P;
  p->last_rows = m - (P - 1) * b;
  if (!qr_geom((int)n, 8, &p->g)) return fail(c, PYLOM_ENOTSUP, "no chunk geometry");
  if (!jacobi_plan((int)n, &p->jp)) return fail(c, PYLOM_ENOTSUP, "no Jacobi plan");
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

// Mixed precision (FP32 storage): FP32 leaf QR (R only), FP64 tree and SVD of
// R, then the Rayleigh-Ritz refinement against the input on the k leading
// right singular vectors, k = N_r0 + max(8, N_r0 / 4) (at most n).  The host
// reads N_r0 once (one stream synchronisation) to size the refinement.
static int run_mixed(pylom_ctx c, pylom_dtype dtype, int64_t m, int64_t n, const void* D,
                     int64_t ldd, int remove_mean, double residual, void* mean, void* U,
                     int64_t ldu, double* S, double* VT, int64_t ldvt, int64_t* n_r) {
  if (dtype != PYLOM_R32) return fail(c, PYLOM_EDTYPE, "mixed precision needs R32 storage");
  Plan p;
  int rc = make_plan(c, m, n, false, &p, true);
  if (rc) return rc;
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
  rc = ensure_ws(c, p.total);
  if (rc) return rc;
  char* ws = (char*)c->ws;
  double* Rbuf = (double*)(ws + p.oR);
  float* R32 = (float*)(ws + p.oR32);
  double* meanws = (double*)(ws + p.oMean);
  double* S0 = (double*)(ws + p.oS0);
  double* VT0 = (double*)(ws + p.oVT0);
  double* UR0 = (double*)(ws + p.oW);
  int64_t* nr0 = (int64_t*)(ws + p.oNr0);
  double* Z = (double*)(ws + p.oZ);
  double* G = (double*)(ws + p.oG);
  double* part = (double*)(ws + p.oPart);
  double* lam = (double*)(ws + p.oLam);
  double* WT = (double*)(ws + p.oWT);
  double* UR2 = (double*)(ws + p.oUR2);
  int64_t* nr2 = (int64_t*)(ws + p.oNr2);
  double* M = (double*)(ws + p.oM);
  hipStream_t st = c->stream;
  const bool tm = c->timing > 0 && !c->ev.empty();
  hipEvent_t* evs = tm ? &c->ev[(size_t)(c->ev_calls % c->timing) * kEvPerSlot] : nullptr;
#define EVREC(j) \
  if (tm) HIPCHK(c, hipEventRecord(evs[j], st), "hipEventRecord")

  EVREC(0);
  EVREC(1);
  HIPCHK(c, launch_leaf_qr_f32(p.g, (const float*)D, ldd, m, p.b, p.P, remove_mean, meanws, R32,
                               st), "leaf QR (FP32)");
  HIPCHK(c, launch_cast_f32_f64(R32, Rbuf, p.P * n * n, st), "R to FP64");
  EVREC(2);
  for (int64_t h = 1; h < p.P; h *= 2)
    HIPCHK(c, launch_tree_combine_f64(p.g, h, p.P, Rbuf, nullptr, p.nch_tree, 0, st),
           "tree combine");
  EVREC(3);
  HIPCHK(c, launch_small_svd(p.jp, Rbuf, (int)c->max_sweeps, ws + p.oSvd, S0, VT0, n, UR0,
                             residual, nr0, c->status_dev, st), "small SVD");
  c->status_valid = 1;
  c->status_pairs = 1;
  int64_t nr_first = 0;
  HIPCHK(c, hipMemcpyAsync(&nr_first, nr0, sizeof(int64_t), hipMemcpyDeviceToHost, st),
         "N_r read-back");
  HIPCHK(c, hipStreamSynchronize(st), "hipStreamSynchronize");
  EVREC(4);
  if (nr_first <= 0) {
    // all-zero spectrum: nothing to refine, no mode is kept
    HIPCHK(c, hipMemcpyAsync(S, S0, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, st),
           "S copy");
    HIPCHK(c, launch_set_i64(n_r, 0, st), "N_r");
  } else {
    int64_t over = nr_first / 4;
    if (over < 8) over = 8;
    const int64_t k = (nr_first + over < n) ? nr_first + over : n;
    JacobiPlan jk;
    if (!jacobi_plan((int)k, &jk)) return fail(c, PYLOM_ENOTSUP, "no Jacobi plan");
    const int64_t ns = matmul_tn_splits(m, k, k);
    if (sizeof(double) * (size_t)ns * k * k > p.part_bytes)
      return fail(c, PYLOM_ENOTSUP, "Gram partials exceed the planned workspace");
    HIPCHK(c, launch_rr_project(0, m, (int)n, (int)k, D, ldd, remove_mean ? meanws : nullptr, VT0,
                                Z, st), "Rayleigh-Ritz projection");
    HIPCHK(c, launch_matmul_tn(1, m, k, k, Z, k, Z, k, G, k, part, ns, st), "Gram");
    HIPCHK(c, launch_small_svd(jk, G, (int)c->max_sweeps, ws + p.oSvd2, lam, WT, k, UR2, 0.0, nr2,
                               c->status_dev + 2, st), "Gram eigen-decomposition");
    c->status_pairs = 2;
    HIPCHK(c, launch_rr_finish((int)n, (int)k, S0, lam, residual, S, n_r, WT, VT0, VT, ldvt, M,
                               st), "refined spectrum");
    EVREC(5);
    HIPCHK(c, launch_rr_form_u(0, m, (int)k, Z, M, n_r, U, ldu, st), "form U");
  }
  if (!(nr_first > 0) && tm) HIPCHK(c, hipEventRecord(evs[5], st), "hipEventRecord");
  if (remove_mean && mean) HIPCHK(c, launch_cast_out(meanws, mean, 0, m, st), "mean out");
  EVREC(6);
#undef EVREC
  if (tm) ++c->ev_calls;
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
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
  rc = ensure_ws(c, p.total);
  if (rc) return rc;
  char* ws = (char*)c->ws;
  double* V = (double*)(ws + p.oV);
  double* Tleaf = (double*)(ws + p.oTleaf);
  double* Rbuf = (double*)(ws + p.oR);
  double* Ttree = (double*)(ws + p.oTtree);
  double* W = (double*)(ws + p.oW);
  double* meanws = (double*)(ws + p.oMean);
  void* svdws = ws + p.oSvd;
  hipStream_t st = c->stream;
  const int in64 = dtype == PYLOM_R64;
  const bool tm = c->timing > 0 && !c->ev.empty();
  hipEvent_t* evs = tm ? &c->ev[(size_t)(c->ev_calls % c->timing) * kEvPerSlot] : nullptr;
#define EVREC(j) \
  if (tm) HIPCHK(c, hipEventRecord(evs[j], st), "hipEventRecord")

  EVREC(0);
  EVREC(1);
  HIPCHK(c, launch_leaf_qr_f64(p.g, D, in64, ldd, m, p.b, p.P, remove_mean, meanws, V, Tleaf,
                               p.nch_leaf, Rbuf, st), "leaf QR");
  EVREC(2);
  for (int64_t h = 1; h < p.P; h *= 2)
    HIPCHK(c, launch_tree_combine_f64(p.g, h, p.P, Rbuf, Ttree, p.nch_tree, 1, st), "tree combine");
  EVREC(3);
  HIPCHK(c, launch_small_svd(p.jp, Rbuf, (int)c->max_sweeps, svdws, S, VT, ldvt, W, residual, n_r,
                             c->status_dev, st), "small SVD");
  c->status_valid = 1;
  c->status_pairs = 1;
  EVREC(4);
  int64_t top = 1;
  while (top * 2 < p.P) top *= 2;
  if (p.P > 1)
    for (int64_t h = top; h >= 1; h /= 2)
      HIPCHK(c, launch_apply_tree_f64(p.g, h, p.P, Rbuf, Ttree, p.nch_tree, W, n, n_r, n, st),
             "tree propagation");
  EVREC(5);
  HIPCHK(c, launch_apply_leaf_f64(p.g, m, p.b, p.P, V, Tleaf, p.nch_leaf, W, n, n_r, n, U, in64,
                                  ldu, st), "leaf apply");
  if (remove_mean && mean) HIPCHK(c, launch_cast_out(meanws, mean, in64, m, st), "mean out");
  EVREC(6);
#undef EVREC
  if (tm) ++c->ev_calls;
  return PYLOM_OK;
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
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
  rc = ensure_ws(c, p.total);
  if (rc) return rc;
  char* ws = (char*)c->ws;
  const bool wq = Q != nullptr;
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

// ---------------------------------------------------------------------------
// SPOD: FFT front end + one batch of realified TSQR-SVD problems
// ---------------------------------------------------------------------------
struct SpodPlan {
  int64_t m, nt, npwin, nolap, nb, nf, n, M2, b, P, nch_leaf, nch_tree, levels;
  int e_f64;
  QrGeom g;
  JacobiPlan jp;
  size_t oE, oV, oTleaf, oR, oTtree, oW, oSvd, oS, oVT, oUR, oNr, oSt, oUe, total;
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
  p->M2 = 2 * m;
  p->e_f64 = spectra == PYLOM_C128;
  if (spod_fft_lds_bytes((int)npwin, (int)nb, p->e_f64 ? 8 : 4) > (size_t)160 * 1024)
    return fail(c, PYLOM_ENOTSUP, "npwin x blocks too large for the FFT staging");
  const int64_t n = p->n;
  int64_t b = c->block_rows > 0 ? c->block_rows : 4096;
  if (b < n) b = n;
  int64_t P = p->M2 / b;
  if (P < 1) P = 1;
  p->b = b;
  p->P = P;
  if (!qr_geom((int)n, 8, &p->g)) return fail(c, PYLOM_ENOTSUP, "no chunk geometry");
  if (!jacobi_plan((int)n, &p->jp) || p->jp.G != 1)
    return fail(c, PYLOM_ENOTSUP, "no single-workgroup Jacobi plan");
  const int64_t last = p->M2 - (P - 1) * b;
  const int64_t s = p->g.s, np = p->g.npanels, nf = p->nf;
  p->nch_leaf = (last + s - 1) / s;
  p->nch_tree = (n + s - 1) / s;
  int64_t lv = 0;
  for (int64_t h = 1; h < P; h *= 2) ++lv;
  p->levels = lv;
  p->svd_stride = jacobi_ws_stride(p->jp, (int)c->max_sweeps);
  const size_t es = p->e_f64 ? 8 : 4;
  size_t off = 0;
  p->oE = off;     off = align_up(off + es * (size_t)nf * p->M2 * n);
  p->oV = off;     off = align_up(off + 8 * (size_t)nf * p->M2 * n);
  p->oTleaf = off; off = align_up(off + 8 * (size_t)nf * P * p->nch_leaf * np * 256);
  p->oR = off;     off = align_up(off + 8 * (size_t)nf * P * n * n);
  p->oTtree = off; off = align_up(off + 8 * (size_t)nf * P * p->nch_tree * np * 256);
  p->oW = off;     off = align_up(off + 8 * (size_t)nf * P * n * n);
  p->oSvd = off;   off = align_up(off + p->svd_stride * (size_t)nf);
  p->oS = off;     off = align_up(off + 8 * (size_t)nf * n);
  p->oVT = off;    off = align_up(off + 8 * (size_t)nf * n * n);
  p->oUR = off;    off = align_up(off + 8 * (size_t)nf * n * n);
  p->oNr = off;    off = align_up(off + 8 * (size_t)nf);
  p->oSt = off;    off = align_up(off + 8 * (size_t)nf);
  p->oUe = off;    off = align_up(off + 8 * (size_t)nf * p->M2 * nb);
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
  if (c->device < 0) return fail(c, PYLOM_ENODEV, "host-only context");
  HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
  rc = ensure_ws(c, p.total);
  if (rc) return rc;
  char* ws = (char*)c->ws;
  void* E = ws + p.oE;
  double* V = (double*)(ws + p.oV);
  double* Tleaf = (double*)(ws + p.oTleaf);
  double* R = (double*)(ws + p.oR);
  double* Ttree = (double*)(ws + p.oTtree);
  double* W = (double*)(ws + p.oW);
  double* S = (double*)(ws + p.oS);
  double* VTb = (double*)(ws + p.oVT);
  double* URb = (double*)(ws + p.oUR);
  int64_t* nr = (int64_t*)(ws + p.oNr);
  int* st_each = (int*)(ws + p.oSt);
  double* Ue = (double*)(ws + p.oUe);
  hipStream_t st = c->stream;
  const int64_t n = p.n, nb = p.nb, nf = p.nf, M2 = p.M2, P = p.P, np = p.g.npanels;
  const bool tm = c->timing > 0 && !c->ev.empty();
  hipEvent_t* evs = tm ? &c->ev[(size_t)(c->ev_calls % c->timing) * kEvPerSlot] : nullptr;
#define EVREC(j) \
  if (tm) HIPCHK(c, hipEventRecord(evs[j], st), "hipEventRecord")

  EVREC(0);
  HIPCHK(c, launch_spod_fft(p.e_f64, m, nt, D, ldd, (int)npwin, (int)nolap, (int)nb, window,
                            remove_mean, E, n, M2 * n, st), "SPOD front end");
  EVREC(1);
  Batch bl;
  bl.count = nf;
  bl.sD = M2 * n;
  bl.sV = M2 * n;
  bl.sTleaf = P * p.nch_leaf * np * 256;
  bl.sR = P * n * n;
  bl.sTtree = P * p.nch_tree * np * 256;
  bl.sW = P * n * n;
  bl.sU = M2 * nb;
  HIPCHK(c, launch_leaf_qr_f64(p.g, E, p.e_f64, n, M2, p.b, P, 0, nullptr, V, Tleaf, p.nch_leaf, R,
                               st, bl), "leaf QR");
  EVREC(2);
  for (int64_t h = 1; h < P; h *= 2)
    HIPCHK(c, launch_tree_combine_f64(p.g, h, P, R, Ttree, p.nch_tree, 1, st, bl), "tree combine");
  EVREC(3);
  HIPCHK(c, launch_small_svd_batched(p.jp, nf, R, P * n * n, (int)c->max_sweeps, ws + p.oSvd, S, n,
                                     VTb, n, n * n, URb, n * n, 0.0, nr, st_each, c->status_dev,
                                     st), "batched SVD");
  c->status_valid = 1;
  c->status_pairs = 1;
  HIPCHK(c, launch_select_even((int)n, (int)nb, nf, URb, n * n, W, n, P * n * n, st), "root W");
  EVREC(4);
  int64_t top = 1;
  while (top * 2 < P) top *= 2;
  if (P > 1)
    for (int64_t h = top; h >= 1; h /= 2)
      HIPCHK(c, launch_apply_tree_f64(p.g, h, P, R, Ttree, p.nch_tree, W, n, nullptr, nb, st, bl),
             "tree propagation");
  EVREC(5);
  HIPCHK(c, launch_apply_leaf_f64(p.g, M2, p.b, P, V, Tleaf, p.nch_leaf, W, n, nullptr, nb, Ue, 1,
                                  nb, st, bl), "leaf apply");
  HIPCHK(c, launch_spod_modes(p.e_f64, m, (int)nb, nf, Ue, M2 * nb, VTb, n * n, S, n, modes, L, st),
         "modes");
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
  // events per slot: e0 call start, e1 after the front end (SPOD FFT; none
  // for POD), e2..e6 after leaf QR, tree, SVD, propagation, apply
  double acc[kPhases] = {0, 0, 0, 0, 0, 0};
  for (int64_t k = 0; k < nrec; ++k) {
    const int64_t slot = (c->ev_calls - 1 - k) % c->timing;
    hipEvent_t* e = &c->ev[(size_t)slot * kEvPerSlot];
    HIPCHK(c, hipEventSynchronize(e[kEvPerSlot - 1]), "hipEventSynchronize");
    for (int i = 0; i < kPhases; ++i) {
      float ms = 0.f;
      if (i < 5)
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
    if (st[2 * k + 1]) return fail(c, PYLOM_EHIP, "Jacobi grid barrier timed out");
    if (st[2 * k] < 0) return fail(c, PYLOM_WNOCONV, "Jacobi SVD did not converge");
  }
  return PYLOM_OK;
}
