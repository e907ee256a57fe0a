/*
 * pylom.h -- C-ABI of the MI355X (gfx950) POD / tall-skinny SVD library.
 *
 * The operations follow pyLOM (Eiximeno et al., "pyLOM: A HPC open source
 * reduced order model suite for fluid dynamics applications", arXiv
 * 2405.15529):
 *
 *   snapshot matrix  D (M x N, M grid points >> N snapshots), Sec. 3 intro;
 *   POD              Alg. 2 (optional temporal-mean removal) followed by the
 *                    TSQR-SVD of Alg. 1 and Eqs. svdqr1-svdqr3:
 *                      Y = Q [R; 0],  R = U_R S V^T,  U = Q U_R;
 *   energy           Sec. 3.1, cumulative energy sum_{i<=k} S_i^2 / sum S_i^2;
 *   truncation       residual r of Alg. 3, read as
 *                      N_r = min{k >= 1 : sum_{i>k} S_i^2 <= r sum_i S_i^2}
 *                    (r <= 0 keeps all N modes; an all-zero spectrum keeps 0);
 *   matmul           Alg. 4 (local products summed over the row partition);
 *   SPOD             Alg. 6 with the Frame-Towne SVD of Q_f / sqrt(nBlks).
 *
 * Conventions common to every entry point
 * ---------------------------------------
 *  - Matrices are ROW-MAJOR with an explicit leading dimension (elements
 *    between consecutive rows).  Rows are grid points, columns snapshots.
 *  - Every array argument is a DEVICE pointer owned by the caller (allocated
 *    with hipMalloc or by PyTorch), unless documented as host.  The library
 *    never frees or retains caller pointers after a call returns.
 *  - Calls are asynchronous and ordered on the context's stream; outputs are
 *    valid after that stream is synchronised.  No call synchronises the host
 *    except where documented.
 *  - Inputs are never written.  Outputs not listed as written are untouched.
 *  - Return value 0 = success.  Negative values are caller errors detected on
 *    the host before any device work is enqueued; positive values are
 *    numerical warnings (outputs are written).  pylom_strerror() names a
 *    code; pylom_last_error() returns the context's last message.
 *  - A context is not thread-safe; separate contexts are independent.  A
 *    context owns a device workspace that grows on demand (hipMalloc outside
 *    the call's stream work); pylom_workspace_query() + pylom_reserve() size
 *    it up front so that later calls allocate nothing.
 */
#ifndef PYLOM_H
#define PYLOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define PYLOM_OK 0
#define PYLOM_EINVAL (-1)   /* a pointer or scalar argument is invalid      */
#define PYLOM_ESHAPE (-2)   /* m < n, n < 1, leading dimension too small     */
#define PYLOM_EDTYPE (-3)   /* unsupported dtype / precision combination     */
#define PYLOM_ENOMEM (-4)   /* workspace allocation failed or over the cap   */
#define PYLOM_EHIP (-5)     /* HIP runtime error (message in last_error)     */
#define PYLOM_ENOTSUP (-6)  /* shape outside what the kernels support        */
#define PYLOM_ENODEV (-7)   /* no usable gfx950 device                       */
#define PYLOM_WNOCONV 1     /* Jacobi SVD hit max_sweeps before converging   */
#define PYLOM_WNONFINITE 2  /* a singular value is NaN or Inf: the input held
                               a non-finite value (outputs are written, and
                               hold NaN or Inf)                             */

/* ---- storage types ---- */
typedef enum {
  PYLOM_R32 = 1,  /* float                                    */
  PYLOM_R64 = 2,  /* double                                   */
  PYLOM_C64 = 3,  /* float complex, interleaved (re, im)      */
  PYLOM_C128 = 4  /* double complex, interleaved (re, im)     */
} pylom_dtype;

/* ---- compute precision ---- */
typedef enum {
  PYLOM_FP64 = 0,  /* every step in FP64 (FP32 inputs promoted on load)      */
  PYLOM_MIXED = 1  /* FP32 leaf QR, FP64 final tree combine + small SVD
                      (lower tree levels: see "mixed_tree"), FP64
                      Rayleigh-Ritz refinement against the input (R32
                      storage only) */
} pylom_prec;

typedef struct pylom_ctx_s* pylom_ctx;

/* Create a context on HIP device `device`.  Fails with PYLOM_ENODEV if the
 * device is missing or is not gfx950. The stream defaults to the null stream. */
int pylom_create(pylom_ctx* ctx, int device);
int pylom_destroy(pylom_ctx ctx);

/* Stream (a hipStream_t passed as void*) on which later calls are ordered. */
int pylom_set_stream(pylom_ctx ctx, void* hip_stream);

/* Options (int64 values):
 *   "block_rows"   leaf row-block height b of the TSQR (Alg. 1's local D_i);
 *                  0 = automatic (pylom_tune_block_rows; at least n).
 *   "max_sweeps"   Jacobi sweep limit (default 60).  0 makes every SVD call
 *                  return PYLOM_WNOCONV without sweeping (failure-path tests).
 *   "ws_cap_mb"    workspace cap in MiB (0 = unlimited); a call needing more
 *                  returns PYLOM_ENOMEM.
 *   "streams"      concurrent HIP streams of pylom_pod_batched (1..16,
 *                  default 4).
 *   "timing"       k > 0: record HIP events around the phases of every
 *                  pod/tsvd call in a ring of k call slots (read back with
 *                  pylom_phase_times); 0 = off (default).
 *   "work_queue"   0 (default, and the only value accepted): one launch per
 *                  phase and tree level.  1 would run the leaf QRs and tree
 *                  combines of the stacked FP64 TSQR as one persistent launch
 *                  draining a device task counter (and the propagation and
 *                  leaf applies likewise); it is switched off and returns
 *                  PYLOM_ENOTSUP, because that launch did not complete on the
 *                  GPU and its cause is not known.
 *   "ooc_window_rows" rows per window of pylom_pod_host (0 = automatic,
 *                  2^20; at least 4 n; rounded down to whole leaves).
 *   "kernel_timing" 1: record an event pair around every kernel launch of
 *                  the single-problem calls, read with pylom_kernel_times;
 *                  0 = off (default).
 *   "narrow_leaves" 1 (default): stacked-QR plans of 3 to 6 panels of 16
 *                  columns (33 <= n <= 96; up to 8 panels, n <= 128, for the
 *                  FP32 leaves of PYLOM_MIXED) with at least two leaves per
 *                  CU factor their leaves in 32-row chunks with single-wave
 *                  workgroups, several leaves per CU; 0: the default chunk
 *                  height with four-wave workgroups, one per CU.
 *   "blocked_from" n at which pod/tsvd/tsqr switch to the column-blocked
 *                  TSQR (2..2049), or 0 (default) for the automatic choice:
 *                  column-blocked when n >= 512, or when n >= 64 and
 *                  m <= 8,388,608; the stacked QR otherwise (instances of
 *                  pylom_pod_batched follow the same rule).  On the
 *                  column-blocked path every leaf and every tree combine is a
 *                  blocked Householder QR over panels of 64 columns (the
 *                  local QR of Alg. 1 as LAPACK blocks it), the leaf height
 *                  defaults to ceil(m / (2 CUs)) rounded up to 64, and the
 *                  working copy of D, the reflectors of every panel and the
 *                  tree pairs stay in the workspace.  The stacked QR factors
 *                  at most 1024 columns.
 *   "mixed_tree"   1 (default): a PYLOM_MIXED call on the column-blocked
 *                  path combines the FP32 leaf R factors in FP32 on every
 *                  tree level below the last one (Alg. 1 reduce); the final
 *                  combine, the root R and its SVD run in FP64.  0: the whole
 *                  tree in FP64.  The Rayleigh-Ritz refinement against D
 *                  sets the accuracy of the result either way.  The stacked
 *                  path always combines in FP64.
 *   "tree_pipeline" S in [0, 16], default 8: on the column-blocked path
 *                  the levels of the R-tree (Alg. 1 reduce) run as a
 *                  wavefront over up to S library streams: panel k of level
 *                  h starts once panel k of level h/2 is done, not once that
 *                  whole level is.  The arithmetic and the results are the
 *                  same as with 0 or 1, which run the levels one after
 *                  another on the context stream.  Instances of
 *                  pylom_pod_batched always run their levels one after
 *                  another on their own stream.
 *   "mixed_svd_tol" 1 (default): the first SVD of R in a PYLOM_MIXED call
 *                  (Eq. svdqr2 on the R of the FP32 leaves) treats a column
 *                  pair as orthogonal once its cosine is at most 2^-24, the
 *                  FP32 unit roundoff that bounds what that R determines;
 *                  its leading right singular vectors only seed the
 *                  Rayleigh-Ritz refinement.  0: the FP64 threshold
 *                  n 2^-53 of every other SVD of R.
 * Read-only (pylom_get_option):
 *   "batch_jacobi_chained"  1 if the last pylom_pod_batched call ordered its
 *                  multi-workgroup Jacobi launches one after another across
 *                  streams (their grid barriers need every workgroup resident;
 *                  the batch chains them when the largest Jacobi grid of each
 *                  stream would not fit on the device together), else 0.
 * Unknown keys return PYLOM_EINVAL. */
int pylom_set_option(pylom_ctx ctx, const char* key, int64_t value);
int pylom_get_option(pylom_ctx ctx, const char* key, int64_t* value);

/* Workspace bytes a pod/tsvd/tsqr call of this shape needs (host only). */
int pylom_workspace_query(pylom_ctx ctx, pylom_dtype dtype, pylom_prec prec, int64_t m, int64_t n,
                          size_t* bytes);
/* Grow the context workspace to at least `bytes` now. */
int pylom_reserve(pylom_ctx ctx, size_t bytes);

const char* pylom_strerror(int status);
const char* pylom_last_error(pylom_ctx ctx);

/* POD of the snapshot matrix (Alg. 2 -> Alg. 1 -> Eqs. svdqr1-3).
 *
 *   D      m x n, leading dimension ldd >= n, dtype PYLOM_R64 or PYLOM_R32.
 *   remove_mean  nonzero: Y = D - mean 1^T with mean_j = (1/n) sum_t D[j,t]
 *          (Alg. 2); zero: Y = D.
 *   residual     truncation residual r (0.01 keeps 99 % of the energy).
 *   mean   m entries of the storage type, or NULL; written when remove_mean.
 *   U      m x n capacity (ldu >= n), storage type; the first N_r columns are
 *          written (spatial modes, orthonormal).
 *   S      n doubles, all n singular values, descending.
 *   VT     n x n capacity (ldvt >= n), doubles; the first N_r rows are
 *          written; row i holds mode i's temporal coefficients (Sec. 3.1).
 *   n_r    one int64 in device memory: N_r.
 * Sign convention: each (u_i, v_i) is signed so that the largest-magnitude
 * entry of v_i (lowest index on ties) is positive.  Requires m >= n >= 1 and
 * n <= 2048 (on the column-blocked TSQR, see "blocked_from", the modes of an
 * exactly zero singular value of an exactly rank-deficient panel may come out
 * as zero columns of U).
 * PYLOM_MIXED (D must be R32): FP32 leaf QR without reflector storage, FP64
 * tree (below its final combine FP32 on the column-blocked path, see
 * "mixed_tree") and SVD of R, then a Rayleigh-Ritz refinement against D in FP64 on the
 * k = min(n, N0 + max(8, N0/4)) leading right singular vectors V_k of that SVD
 * (N0 = its truncation): Z = (D - mean 1^T) V_k, the Jacobi eigenpairs
 * (lambda, w) of Z^T Z give S[i] = sqrt(lambda_i) (i < k; S[i] for i >= k is
 * the unrefined value), v_i = V_k w_i, u_i = Z w_i / S[i]; N_r <= k.  The call
 * synchronises the stream once, after the first SVD, to read N0.  Modes with
 * S[i] = 0 get a zero U column.  On the column-blocked path the working copy
 * of D is FP32 and k may not exceed 1024 (PYLOM_ENOTSUP otherwise).
 * Returns PYLOM_WNOCONV (>0, outputs written) if the Jacobi SVD did not
 * converge within max_sweeps -- this is only known after the stream is
 * synchronised, so the return value of an asynchronous call is 0 and the
 * warning is reported by the next pylom_check() call. */
int pylom_pod(pylom_ctx ctx, pylom_dtype dtype, pylom_prec prec, int64_t m, int64_t n,
              const void* D, int64_t ldd, int remove_mean, double residual, void* mean, void* U,
              int64_t ldu, double* S, double* VT, int64_t ldvt, int64_t* n_r);

/* Out-of-core POD (Alg. 2 -> Alg. 1 -> Eqs. svdqr1-3) of a snapshot matrix
 * held in HOST memory, for matrices larger than the device: the arguments of
 * pylom_pod with D, mean, U, S, VT and n_r all HOST pointers (D need not be
 * pinned).  FP64 compute (PYLOM_FP64; R64 or R32 storage, promoted on load).
 * The rows stream through the device in windows of whole leaves (option
 * "ooc_window_rows", default 2^20 rows, at least 4 n; the leaf height is the
 * "block_rows" option, else two leaves per CU per window), each window
 * twice: pass 1 removes the mean and factors the window's leaves into their
 * R (Alg. 1 local QR); the binary tree of Alg. 1, the SVD of R, the
 * truncation and the down-tree propagation then run once on the device;
 * pass 2 factors each window's leaves again (the same arithmetic, so the
 * same reflectors) and forms its rows of U = Q [W; 0], which stream back.
 * Only O(P n^2 + m) bytes (P = leaves) stay resident, plus the windows.
 * The leaves, the tree and every reflector are those of the column-blocked
 * path (see "blocked_from") at the same leaf height, so the results equal
 * those of pylom_pod there.  Transfers run on two copy streams through
 * pinned staging buffers that the context allocates (two windows each way);
 * host-side copies between the caller's rows and that staging use up to 8
 * host threads.  Synchronous: returns when U, S, VT, mean and n_r are
 * written.  Workspace: pylom_ooc_workspace_query. */
int pylom_pod_host(pylom_ctx ctx, pylom_dtype dtype, pylom_prec prec, int64_t m, int64_t n,
                   const void* D, int64_t ldd, int remove_mean, double residual, void* mean,
                   void* U, int64_t ldu, double* S, double* VT, int64_t ldvt, int64_t* n_r);
/* Device workspace bytes of a pylom_pod_host call of this shape, the rows of
 * a full window and the number of windows (host only; the last two may be
 * NULL). */
int pylom_ooc_workspace_query(pylom_ctx ctx, pylom_dtype dtype, int64_t m, int64_t n,
                              size_t* bytes, int64_t* window_rows, int64_t* windows);

/* Tall-skinny SVD without mean removal (pylom_pod with remove_mean = 0, as
 * DMD's Alg. 3 applies it to Y[:, :-1]).  Arguments as pylom_pod. */
int pylom_tsvd(pylom_ctx ctx, pylom_dtype dtype, pylom_prec prec, int64_t m, int64_t n,
               const void* A, int64_t lda, double residual, void* U, int64_t ldu, double* S,
               double* VT, int64_t ldvt, int64_t* n_r);

/* TSQR (Alg. 1): A = Q R.
 *   R  n x n doubles (ldr >= n), upper triangular with diag(R) >= 0, always
 *      written.
 *   Q  m x n (ldq >= n) of the storage type, or NULL to skip forming Q.
 * FP64 compute; dtype PYLOM_R64 or PYLOM_R32 (promoted on load).  Q has
 * orthonormal columns; for an exactly rank-deficient A the columns attached
 * to a zero diagonal entry of R are not determined. */
int pylom_tsqr(pylom_ctx ctx, pylom_dtype dtype, pylom_prec prec, int64_t m, int64_t n,
               const void* A, int64_t lda, void* Q, int64_t ldq, double* R, int64_t ldr);

/* Alg. 4 on one GPU (the all_reduce becomes a device reduction over row
 * blocks):  trans_a = 1:  C (p x q) = A^T B,  A m x p, B m x q;
 *           trans_a = 0:  C (m x q) = A B,    A m x p, B p x q.
 * dtype PYLOM_R64 (FP64 MFMA) or PYLOM_R32 (FP32 inputs; FP32 MFMA with FP64
 * cross-block accumulation when trans_a = 1).  C has the storage type. */
int pylom_matmul(pylom_ctx ctx, pylom_dtype dtype, pylom_prec prec, int trans_a, int64_t m,
                 int64_t p, int64_t q, const void* A, int64_t lda, const void* B, int64_t ldb,
                 void* C, int64_t ldc);

/* pylom_matmul for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments and results as pylom_matmul; it calls no hipMalloc, hipFree
 * or allocating library routine.  For trans_a = 1 the split-K partial sums
 * go to a fixed 32 MiB device array of the library (one per device, held
 * until the process ends; every call on a device shares it and it keeps the
 * last call's contents, none of which a call reads), with fewer row splits
 * when the usual count would not fit, so results may differ from
 * pylom_matmul in the rounding of the cross-split sum.  p * q * 8 bytes over
 * 32 MiB returns PYLOM_ENOMEM before any launch.  Calls that overlap on one
 * device (several streams or host threads) race on that array. */
int pylom_matmul_noalloc(pylom_ctx ctx, pylom_dtype dtype, pylom_prec prec, int trans_a, int64_t m,
                         int64_t p, int64_t q, const void* A, int64_t lda, const void* B,
                         int64_t ldb, void* C, int64_t ldc);

/* One instance of a batched POD (the arguments of pylom_pod). */
typedef struct {
  int64_t m, n;        /* shape, m >= n >= 1, n <= 2048 (as pylom_pod)      */
  const void* D;       /* m x n snapshots (storage type of the batch), ldd   */
  int64_t ldd;
  int remove_mean;     /* Alg. 2 mean removal                                 */
  double residual;     /* truncation residual r in [0, 1)                     */
  void* mean;          /* m entries of the storage type, or NULL              */
  void* U;             /* m x n capacity, ldu >= n                            */
  int64_t ldu;
  double* S;           /* n                                                   */
  double* VT;          /* n x n capacity, ldvt >= n                           */
  int64_t ldvt;
  int64_t* n_r;        /* one int64 (device)                                  */
} pylom_problem;

/* A batch of POD instances of uneven shapes (Alg. 2 + Alg. 1 + Eqs. svdqr1-3
 * for each), with the same dtype and precision.  `problems` is a host array
 * of `count` descriptors; every pointer inside is a device pointer, as for
 * pylom_pod, and the results are those of `count` pylom_pod calls.
 * Each instance takes the TSQR of the "blocked_from" rule (stacked or
 * column-blocked) and its leaf height is the "block_rows" option when set,
 * else the library's autotuned choice (see pylom_tune_block_rows).  Instances
 * run their tree levels one after another on their own stream.  Instances are
 * spread over "streams" (option, default 4) concurrent HIP streams with
 * workspaces of their own, forked from and joined back into the context
 * stream.  use_graph != 0 captures the whole launch sequence into a HIP graph
 * on the first call with a given problem list (pointers and shapes) and
 * replays it on later calls (no per-kernel launch cost); PYLOM_MIXED batches
 * run as two graphs around one host read-back of every instance's N0.
 * All validation happens before any launch; PYLOM_WNOCONV is reported by
 * pylom_check if any instance's Jacobi SVD did not converge. */
int pylom_pod_batched(pylom_ctx ctx, pylom_dtype dtype, pylom_prec prec, int64_t count,
                      const pylom_problem* problems, int use_graph);

/* The leaf height b chosen for an m x n problem when "block_rows" is 0: the
 * minimiser, over b in {128, 256, ..., 32768} with b >= n, of a latency model
 * of the stacked QR (leaf critical path of ceil(b / s) chunks; leaves in
 * waves over the compute units, one per CU, or several single-wave narrow
 * leaves per CU, see "narrow_leaves"; the remainder leaf in the last wave;
 * ceil(log2 P) tree levels, each in waves of its combines, and one launch
 * per level).  FP64 plans.  Where the column-blocked TSQR serves the shape (see
 * "blocked_from"), ceil(m / (2 CUs)) rounded up to a multiple of 64 (at
 * least n).  Host only; n <= 2048. */
int64_t pylom_tune_block_rows(pylom_ctx ctx, int64_t m, int64_t n);

/* Measured leaf height (the "block-row shape" of the TSQR) for an m x n
 * pylom_pod of this dtype, precision and mean removal: times pylom_pod on D
 * (device, m x n, ldd) with each candidate leaf height of the path the
 * context would take (column-blocked: one to four leaves per CU; stacked:
 * 128 ... 32768 rows; the analytic choice always included), `reps` timed
 * calls each after one warm-up, 99 % energy, on the context stream with HIP
 * events, and records the fastest in the context's table under the key
 * (path, precision, floor(log2 m), n rounded up to 16).  While "block_rows"
 * is 0, every later call whose shape falls under a recorded key uses that
 * height.  Writes the height and its mean milliseconds (either pointer may
 * be NULL).  Allocates its own trial outputs; synchronises the stream. */
int pylom_autotune(pylom_ctx ctx, pylom_dtype dtype, pylom_prec prec, int64_t m, int64_t n,
                   const void* D, int64_t ldd, int remove_mean, int reps, int64_t* best_rows,
                   double* best_ms);
/* The context's measured table as a JSON file at `path` (host path):
 *   {"pylom_tuning": 1, "entries": [{"path": "blocked"|"stacked",
 *    "precision": "fp64"|"mixed", "m_log2": L, "n_bucket": N,
 *    "block_rows": B, "ms": T}, ...]} */
int pylom_tune_save(pylom_ctx ctx, const char* path);
/* Merges the entries of such a file into the context's table; returns the
 * number of entries read, or PYLOM_EINVAL for a missing or malformed file
 * (the table is then unchanged).  Works on host-only contexts too. */
int pylom_tune_load(pylom_ctx ctx, const char* path);

/* SPOD (Alg. 6; Sec. 2.3, Eq. csdimp with the SVD of the spectral matrix).
 *
 *   D       m x nt FP32 snapshots (rows = points, ldd >= nt), device.
 *   spectra PYLOM_C64: FFT and spectral storage in FP32, modes complex64;
 *           PYLOM_C128: FFT and storage in FP64, modes complex128.
 *   prec    PYLOM_FP64 (the TSQR-SVD of every frequency runs in FP64).
 *   npwin   block length, a power of two in [4, 4096]; nolap overlap
 *           (0 <= nolap < npwin); nBlks = (nt - nolap) / (npwin - nolap),
 *           1 <= nBlks <= 16; block b starts at sample b (npwin - nolap).
 *   window  0 = Hann, 1 = Hamming (the paper's), both
 *           a0 - a1 cos(2 pi j / (npwin - 1)), j = 0..npwin-1.
 *   remove_mean  subtract each point's temporal mean over all nt samples.
 * Per point and block: q_f = c_f DFT_f(w x) / sum(w) / sqrt(nBlks) for
 * f = 0..npwin/2 (nfreq values), DFT_f(x) = sum_j x_j exp(-2 pi i j f/npwin),
 * c_f = 2 for 0 < f < npwin/2 and 1 otherwise.  For every frequency the thin
 * SVD Q_f = U_f S_f V_f^H of the m x nBlks matrix (all nBlks modes kept) is
 * computed by the TSQR-SVD of its real 2m x 2nBlks realification, all
 * frequencies in one batch.
 * Outputs (device): modes  nfreq x m x nBlks complex (interleaved re, im),
 *           modes[f][p][c] = U_f[p][c], each mode's phase fixed so that the
 *           largest-|.| entry of v_c (lowest index on ties) is real > 0;
 *         L      nfreq x nBlks doubles, L[f][c] = S_f[c]^2, descending in c;
 *         freqs  nfreq doubles f / (dt npwin), or NULL;
 *         order  nfreq int64, the frequencies sorted by L[f][0] descending
 *                (ties by ascending f), or NULL.
 * The Jacobi status is reported by pylom_check (largest sweep count). */
int pylom_spod(pylom_ctx ctx, pylom_dtype spectra, pylom_prec prec, int64_t m, int64_t nt,
               const float* D, int64_t ldd, double dt, int64_t npwin, int64_t nolap, int window,
               int remove_mean, void* modes, double* L, double* freqs, int64_t* order);

/* Exact DMD (Sec. 3.2, the exact DMD of Tu et al.; Alg. 3 with the product
 * of Alg. 4 and the amplitudes of Alg. 5, Jovanovic et al.).
 *
 *   D       m x n snapshots (rows = points, ldd >= n), PYLOM_R64 or PYLOM_R32
 *           (promoted to FP64), device; n >= 2 and m >= n.
 *   remove_mean  nonzero: Y = D - mean 1^T with the mean over all n
 *           snapshots; zero: Y = D.  Y1 = Y[:, :n-1], Y2 = Y[:, 1:].
 *   residual  truncation of the TS-SVD of Y1 = U S W^T, as for pylom_pod.
 *   dt      snapshot spacing (> 0), for the frequencies and growth rates.
 *   phi     m x ldphi complex128 (interleaved re, im), ldphi >= min(n-1, 128);
 *           columns 0..N_r-1 receive the exact DMD modes
 *           phi_i = Y2 W S^-1 w_i / mu_i (Eq. dmdmodes).
 *   mu, b   min(n-1, 128) complex128 each: the eigenvalues of the linear map
 *           A = U^T Y2 W S^-1 and the amplitudes minimising
 *           |S W^T - w diag(b) V_and|_F (V_and[i][t] = mu_i^t, t < n-1).
 *   freq, growth  min(n-1, 128) doubles each, or NULL: arg(mu) / (2 pi dt)
 *           (Eq. freq) and log|mu| / dt.
 *   n_r     one int64 in device memory: N_r.
 * Every modal output is ordered by |b| descending (ties: Im(mu) descending,
 * then eigenvalue index).  Each eigenvector w_i has unit 2-norm with its
 * largest-magnitude entry real and positive.  All arithmetic is FP64; every
 * step runs on the device: one R-only TSQR of Y = Q_f R_f gives both the
 * TS-SVD of Y1 (the SVD of R1 = R_f[:n-1, :n-1], since Y1 = Q_f[:, :n-1] R1)
 * and U^T Y2 = U_R^T R_f[:n-1, 1:]; then the Householder-Hessenberg
 * reduction, Francis double-shift QR, complex inverse iteration, the
 * Cholesky solve of Alg. 5 and the mode GEMM.  The call synchronises once,
 * to read N_r.
 * Errors: PYLOM_ESHAPE (shapes, leading dimensions), PYLOM_EINVAL (null
 * arrays, residual outside [0, 1), dt <= 0), PYLOM_ENOTSUP when the
 * truncation keeps more than 128 modes or a zero singular value (raise the
 * residual).  N_r = 0 (Y1 = 0) writes n_r only.  A QR sweep limit or a
 * Cholesky pivot <= 0 is reported by pylom_check as PYLOM_WNOCONV.  The
 * workspace is that of an R-only TSQR of an m x n matrix plus O(n^2). */
int pylom_dmd(pylom_ctx ctx, pylom_dtype dtype, int64_t m, int64_t n, const void* D, int64_t ldd,
              int remove_mean, double residual, double dt, void* phi, int64_t ldphi, void* mu,
              void* b, double* freq, double* growth, int64_t* n_r);
/* Workspace bytes of a pylom_dmd call of this shape (host only). */
int pylom_dmd_workspace_query(pylom_ctx ctx, pylom_dtype dtype, int64_t m, int64_t n,
                              int remove_mean, size_t* bytes);

/* Number of Welch blocks and frequencies, and the workspace bytes, of a
 * pylom_spod call of this shape (host only). */
int pylom_spod_query(pylom_ctx ctx, pylom_dtype spectra, int64_t m, int64_t nt, int64_t npwin,
                     int64_t nolap, int64_t* nblocks, int64_t* nfreq, size_t* bytes);

/* Host-side copy of the in-device binary reduction tree of Alg. 1 for P
 * leaves: writes up to `cap` triples (level, receiver, sender) in execution
 * order into `out` (host memory, 3*cap int64) and returns the number of
 * combines (P - 1), or a negative status.  At level l (blevel = 2^l), node j
 * with j mod 2^(l+1) == 0 absorbs node j + 2^l when that node exists. */
int64_t pylom_tree_plan(int64_t P, int64_t* out, int64_t cap);

/* Leaf geometry chosen for a pod/tsvd/tsqr call of this shape: leaves,
 * rows per leaf (the last leaf takes the remainder), chunk rows, tree levels.
 * Host only. */
int pylom_plan_query(pylom_ctx ctx, int64_t m, int64_t n, int64_t* leaves, int64_t* block_rows,
                     int64_t* chunk_rows, int64_t* levels);

/* Mean phase durations (milliseconds) over the timed pod/tsvd/spod calls
 * made since the previous read (at most the last k, k = the "timing"
 * option):
 *   out[0] leaf QR (+ fused mean removal)
 *   out[1] tree combines
 *   out[2] small SVD + truncation
 *   out[3] tree propagation
 *   out[4] leaf apply U = Q_1i W_i (+ mean output; for SPOD also the modes,
 *          energies and frequency order)
 *   out[5] the front end: the SPOD windowed FFT, or the working copy of D
 *          on the column-blocked path; 0 for the stacked pod/tsvd.
 * For PYLOM_MIXED calls out[3] is the refinement (projection
 * Z = (D - mean 1^T) V_k, Gram, its eigen-solve, refined spectrum) and out[4]
 * forms U = Z M; the host read-back of N0 between them is in neither.
 * `out` is a host array of `cap` doubles; returns the number of phases (6)
 * or a negative status.  Waits for the recorded events, then starts a new
 * averaging window. */
int pylom_phase_times(pylom_ctx ctx, double* out, int cap);

/* Per-kernel durations (option "kernel_timing" = 1: an event pair around
 * every launch of the pod/tsvd/tsqr calls on this context; batched calls are
 * not timed).  Sums, over the launches made since the previous read, of the
 * milliseconds of each kernel role, and the launch counts:
 *   0 working copy of D (mean removal, type conversion)
 *   1 leaf panel QRs (column-blocked TSQR; with the R assembly and cast)
 *   2 leaf trailing updates (column-blocked TSQR)
 *   3 tree panel QRs (column-blocked TSQR; pair states and R assembly)
 *   4 tree trailing updates (column-blocked TSQR)
 *   5 SVD of R (Jacobi set-up, sweeps, finalize and truncation)
 *   6 down-tree propagation
 *   7 leaf apply U = Q [W; 0] and U out
 *   8 mixed refinement (projection, Gram, its eigenpairs, refined spectrum)
 *   9 mixed refinement U = Z M
 *  10 stacked leaf QR (and the FP32 to FP64 cast of its R)
 *  11 stacked tree combines
 * `ms` and `launches` are host arrays of `cap` entries; returns the number of
 * roles (12) or a negative status.  Waits for the recorded events. */
int pylom_kernel_times(pylom_ctx ctx, double* ms, int64_t* launches, int cap);

/* After a stream synchronisation: the deferred numerical status of the last
 * pod/tsvd/spod/dmd/batched call on this context (0, PYLOM_WNOCONV, or
 * PYLOM_WNONFINITE, which takes precedence) and its sweep count.  A grid
 * barrier that timed out returns PYLOM_EHIP.  Synchronises the context's
 * stream. */
int pylom_check(pylom_ctx ctx, int64_t* sweeps);

#ifdef __cplusplus
}
#endif
#endif /* PYLOM_H */
