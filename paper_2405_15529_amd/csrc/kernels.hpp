// kernels.hpp -- host-side launchers of the gfx950 kernels (implemented in the
// .hip files next to the kernels; used by the C-ABI layer in abi.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pylom {

// Geometry of one stacked-QR problem family (leaves or tree combines).
struct QrGeom {
  int n;        // columns
  int s;        // chunk rows staged in LDS (multiple of 16)
  int ldc;      // LDS row stride of the chunk (odd)
  int npanels;  // ceil(n / 16)
  int nthr;     // threads of a QR workgroup (0: 64 for at most two panels, else 256)
};

// A batch of same-shape problems (blockIdx.y = problem): element strides
// between the buffers of consecutive problems.  count = 1 is one problem.
struct Batch {
  int64_t count = 1;
  int64_t sD = 0, sMean = 0, sV = 0, sTleaf = 0, sR = 0, sTtree = 0, sW = 0, sU = 0;
};

// Chunk rows and LDS stride for n columns of element size `esize`; returns
// false if n is too wide for the single-workgroup stacked QR.
bool qr_geom(int n, int esize, QrGeom* g);
size_t qr_lds_bytes(const QrGeom& g, int esize);
size_t apply_lds_bytes(const QrGeom& g, int esize);

// ---- column-blocked TSQR for wide problems (blocked.hip) ----------------------
// One panel (kw <= 64 columns, starting at Wk) of every leaf of a working
// matrix with row stride ldw: the stacked QR with every chunk structured,
// from a zero state (state_mode 1) or from the upper-triangular state given
// in Rstate (state_mode 2); reflector tails overwrite the panel in place, T
// factors go to Tf[((l nch + c) npan + p) 256], the kw x kw state of leaf l
// to Rstate + l kw^2.  At most rows_lim rows per leaf take part (0: all).
template <typename T>
hipError_t launch_panel_qr(const QrGeom& g, T* Wk, int64_t ldw, int64_t m, int64_t b, int64_t P,
                           int64_t rows_lim, T* Tf, int64_t nch, T* Rstate, int state_mode,
                           hipStream_t st);

template <typename T>
struct PanelApplyArgs {
  int kw, npan;                 // panel width and its 16-column sub-panels
  int64_t nlv, b, m, rows_lim;  // leaves, leaf row stride, total rows, row cap (0: none)
  const T* V;                   // reflector tails (row stride ldv), rows as X
  int64_t ldv;
  const T* Tf;                  // T factors, nch chunks per leaf
  int64_t nch;
  T* X;                         // rows updated in place (row stride ldx)
  int64_t ldx;
  int64_t ncols;                // columns of X (and of the state)
  const int64_t* nc_dev;        // optional device bound: columns < *nc_dev - nc_off
  int64_t nc_off;
  int x_zero;                   // the rows of X start at zero and are not read
  T* S;                         // state of leaf l: S + l s_leaf, row stride s_ld
  int64_t s_leaf, s_ld;
  int load_state;               // the state starts from S (else zero)
  int store_state;              // the final state is written to S
  int leaf_major;               // grid x = leaves (for launches with few live tiles)
};
size_t panel_apply_lds_bytes(int esize);
// fwd = false: [state; X] <- Q_k^T [state; X] (trailing update);
// fwd = true: [state; X] <- Q_k [state; X] (modes, propagation).
template <typename T>
hipError_t launch_panel_apply(const PanelApplyArgs<T>& a, bool fwd, hipStream_t st);
// Copies the kw x kw diagonal block at (c0, c0) of R_j (j = 2 h q, upper
// part, zeros below) into PS + q kw^2 for each of npairs tree pairs.
template <typename T>
hipError_t launch_diag_load(int n, int64_t c0, int kw, int64_t npairs, const T* R,
                            int64_t rstride, T* PS, hipStream_t st);
hipError_t launch_make_work(int in_f64, int out_f64, int64_t m, int n, const void* D, int64_t ldd,
                            int remove_mean, double* mean_out, void* W, hipStream_t st);
// Rows r0 .. r0 + rows - 1 of R (rows < 0: through row n - 1).
template <typename T>
hipError_t launch_assemble_r(int n, int64_t nprob, const T* PSt, int64_t pstride, T* R,
                             int64_t rstride, hipStream_t st, int r0 = 0, int rows = -1);
hipError_t launch_copy_cols(int out_f64, int64_t m, int64_t col0, int64_t ncg, int64_t ncols,
                            const int64_t* nc_dev, const double* X, int64_t ldx, void* U,
                            int64_t ldu, hipStream_t st);

// ---- leaf QR (Alg. 1, local qr of each row block) ----------------------------
// One workgroup per leaf j: rows [j*b, j*b + b) (the last leaf takes the
// remainder), optional fused mean removal (Alg. 2) into mean_ws (double, m).
// Writes R_j to Rbuf + j*n*n (n x n row-major), reflectors to V (m x n) and
// per-(chunk, panel) T factors to Tleaf when V != nullptr.
// in_f64: input is double (else float).  Compute type: double.
hipError_t launch_leaf_qr_f64(const QrGeom& g, const void* D, int in_f64, int64_t ldd, int64_t m,
                              int64_t b, int64_t P, int remove_mean, double* mean_ws, double* V,
                              double* Tleaf, int64_t nch_leaf, double* Rbuf, hipStream_t st,
                              const Batch& bt = Batch());
// FP32 compute leaf QR (mixed precision): R only (no reflectors), R_j written
// in FP32 to Rbuf32 + j*n*n.
hipError_t launch_leaf_qr_f32(const QrGeom& g, const float* D, int64_t ldd, int64_t m, int64_t b,
                              int64_t P, int remove_mean, double* mean_ws, float* Rbuf32,
                              hipStream_t st, const Batch& bt = Batch());

// ---- tree combine (Alg. 1 reduce phase): node j absorbs node j+h ------------
// for every j = 0, 2h, 4h, ... with j + h < P.  In place: R_j <- R of
// [R_j; R_{j+h}]; Rbuf + (j+h)*n*n <- reflectors; Ttree <- T factors (if
// store_q).
hipError_t launch_tree_combine_f64(const QrGeom& g, int64_t h, int64_t P, double* Rbuf,
                                   double* Ttree, int64_t nch_tree, int store_q, hipStream_t st,
                                   const Batch& bt = Batch());

// ---- work queues: a whole batch's TSQR phase in one persistent launch -------
// Task numbering and counters of k_qr_queue / k_apply_queue (tsqr.hip).
constexpr int kMaxQueueLevels = 32;
struct QrQueue {
  int64_t P;                              // leaves per problem
  int nlev;                               // tree levels
  int64_t lvl_off[kMaxQueueLevels + 2];   // first task of each level, then the total
  unsigned long long* next;               // task counter (zero before the launch)
  unsigned int* cnt;                      // count * P node counters (zero before the launch)
  int* err;                               // set if a dependency wait timed out
};
struct ApplyQueue {
  int64_t P;
  int nlev;
  int64_t ntiles;                         // 16-column tiles of W
  int64_t ncols;                          // columns, when nr is null
  const int64_t* nr;                      // per-problem column counts (device) or null
  int64_t nr_stride;
  int64_t lvl_off[kMaxQueueLevels + 2];   // top level first, the leaves last
  unsigned long long* next;
  unsigned int* cnt;                      // count * P * ntiles counters
  int* err;
};
// Bytes of the counter region of one queue launch over `count` problems of P
// leaves (the task counter at byte 0, the timeout flag at byte 64, node
// counters from byte 256), to be zeroed by launch_queue_reset before it.
size_t queue_counter_bytes(int64_t count, int64_t P, int64_t ntiles);
hipError_t launch_queue_reset(void* counters, size_t bytes, hipStream_t st);
// *flag = 1 if the timeout flag of either counter region (the second may be
// null) is set.
hipError_t launch_queue_err_merge(const void* counters1, const void* counters2, int* flag,
                                  hipStream_t st);
// The reduce phase (every leaf QR and every tree combine of `bt.count`
// problems, FP64 compute) as one work-queue launch; same arguments as
// launch_leaf_qr_f64 + launch_tree_combine_f64.  counters: a zeroed region of
// queue_counter_bytes(bt.count, P, 1).  Returns hipErrorNotSupported when the
// shape does not fit the queue kernel.
hipError_t launch_qr_queue_f64(const QrGeom& g, const void* D, int in_f64, int64_t ldd, int64_t m,
                               int64_t b, int64_t P, int remove_mean, double* mean_ws, double* V,
                               double* Tleaf, int64_t nch_leaf, double* Rbuf, double* Ttree,
                               int64_t nch_tree, int store_q, void* counters, hipStream_t st,
                               const Batch& bt);
// The broadcast phase (every propagation level, then every leaf apply) as
// one work-queue launch; arguments as launch_apply_tree_f64 +
// launch_apply_leaf_f64 (nr: one device count per problem, stride nr_stride,
// or null for ncols).  counters: a zeroed region of
// queue_counter_bytes(bt.count, P, ceil(ncols / 16)).
hipError_t launch_apply_queue_f64(const QrGeom& g, int64_t m, int64_t b, int64_t P,
                                  const double* V, const double* Tleaf, int64_t nch_leaf,
                                  const double* Rbuf, const double* Ttree, int64_t nch_tree,
                                  double* W, int64_t ldw, const int64_t* nr, int64_t nr_stride,
                                  int64_t ncols, void* U, int out_f64, int64_t ldu, void* counters,
                                  hipStream_t st, const Batch& bt);

// ---- apply (Alg. 1 broadcast phase + Q_i = Q_1i Q_w, Eq. svdqr3) -----------
// Leaf mode: U rows of leaf j = Q_1j [W_j; 0]; combine mode (level h):
// [W_j; W_{j+h}] = Q2 [W_j; 0].  Only the first ncols (or *nr) columns.
hipError_t launch_apply_leaf_f64(const QrGeom& g, int64_t m, int64_t b, int64_t P,
                                 const double* V, const double* Tleaf, int64_t nch_leaf,
                                 const double* W, int64_t ldw, const int64_t* nr, int64_t ncols,
                                 void* U, int out_f64, int64_t ldu, hipStream_t st,
                                 const Batch& bt = Batch());
hipError_t launch_apply_tree_f64(const QrGeom& g, int64_t h, int64_t P, const double* Rbuf,
                                 const double* Ttree, int64_t nch_tree, double* W, int64_t ldw,
                                 const int64_t* nr, int64_t ncols, hipStream_t st,
                                 const Batch& bt = Batch());

// ---- small SVD (Eq. svdqr2) ------------------------------------------------
struct JacobiPlan {
  int n, npad, w, G, lpp, xcd_stride;
  int block;  // 1: block Jacobi of 16-column blocks (n > 256)
  int ks;     // workgroups per block pair (block Jacobi; grid = G * ks)
  double tol = 0.0;  // rotation threshold on the cosine of a column pair (0: n 2^-53)
  int no_ur = 0;     // 1: the caller needs no U_R (launch_small_svd then leaves UR unwritten)
};
bool jacobi_plan(int n, JacobiPlan* p);
double jacobi_tol(const JacobiPlan& p);
size_t jacobi_ws_bytes(const JacobiPlan& p, int max_sweeps);
// Workgroups of this plan's Jacobi kernel that one CU holds at once (the
// occupancy query; 1 if it fails).
int jacobi_resident_per_cu(const JacobiPlan& p);
// Full SVD of R (n x n row-major, FP64) into S (n, descending), VT (n x n
// row-major, ldvt), UR (n x n row-major, ld n; the left factor, sign
// convention applied) and N_r (device) for residual r; status[0] = sweeps
// (-1 if not converged, -2 if a singular value is not finite: a non-finite
// input), status[1] = barrier timeout flag.  With p.no_ur, UR is not written
// and the Jacobi does not accumulate it.
// coop = false uses a plain launch (for stream capture).
hipError_t launch_small_svd(const JacobiPlan& p, const double* R, int max_sweeps, void* ws,
                            double* S, double* VT, int64_t ldvt, double* UR, double residual,
                            int64_t* nr, int* status, hipStream_t st, bool coop = true);

// Same for `count` problems of one size n <= 32 (one workgroup each; G == 1):
// problem k reads R + k*sR, uses the workspace slice ws + k*jacobi_ws_stride,
// writes S + k*sS, VT + k*sVT, UR + k*sUR, nr[k] and status_each[2k..2k+1];
// status[0..1] receives the reduced status (max sweeps, or the lowest
// negative code, -2 before -1; timeout flag).
size_t jacobi_ws_stride(const JacobiPlan& p, int max_sweeps);
hipError_t launch_small_svd_batched(const JacobiPlan& p, int64_t count, const double* R,
                                    int64_t sR, int max_sweeps, void* ws, double* S, int64_t sS,
                                    double* VT, int64_t ldvt, int64_t sVT, double* UR,
                                    int64_t sUR, double residual, int64_t* nr, int* status_each,
                                    int* status, hipStream_t st);

// status[0..1] <- reduction of `count` records of `stride` ints, each holding
// `pairs` (sweeps, timeout) pairs.
hipError_t launch_status_reduce(int64_t count, const int* st_each, int stride, int pairs,
                                int* status, hipStream_t st);

// ---- misc ------------------------------------------------------------------
hipError_t launch_cast_out(const double* src, void* dst, int dst_f64, int64_t count, hipStream_t st);
hipError_t launch_eye(double* W, int64_t n, int64_t ldw, hipStream_t st);
hipError_t launch_r_out(const double* Rroot, int64_t n, double* R, int64_t ldr, double* signs,
                        hipStream_t st);
hipError_t launch_q_signs(void* Q, int q_f64, int64_t m, int64_t n, int64_t ldq,
                          const double* signs, hipStream_t st);
hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t st);

// ---- matmul (Alg. 4) --------------------------------------------------------
hipError_t launch_matmul_tn(int f64, int64_t m, int64_t p, int64_t q, const void* A, int64_t lda,
                            const void* B, int64_t ldb, void* C, int64_t ldc, double* partial,
                            int64_t nsplit, hipStream_t st);
int64_t matmul_tn_splits(int64_t m, int64_t p, int64_t q);
hipError_t launch_matmul_nn(int f64, int64_t m, int64_t p, int64_t q, const void* A, int64_t lda,
                            const void* B, int64_t ldb, void* C, int64_t ldc, hipStream_t st);

// ---- exact DMD (Sec. 3.2, Alg. 3-5) ----------------------------------------
constexpr int kDmdMax = 128;  // widest linear map A (N_r) the eigen-solver takes
struct DmdSmallArgs {
  int k, n1;              // N_r, N - 1
  double dt;
  const double* aux;      // U^T Y2, k x n1 (ld n1)
  const double* VT;       // right singular vectors as rows, ld ldvt
  int64_t ldvt;
  const double* S;        // singular values
  double *A, *H0, *Qv, *Qtau, *wr, *wi, *hnorm;  // k x k, k x k, k x k, k, k, k, 1
  int* status;            // (sweeps or -1, 0)
  double2* Ubuf;          // k x k x k
  double2* W;             // eigenvectors, k x k (column i = eigenvalue i)
  double2 *P, *q, *b;     // k x k, k, k
  double2 *mu_out, *b_out;  // k each, ordered
  double *freq, *growth;  // k each (may be null)
  int* perm;              // k
  double* B;              // n1 x 2k, interleaved complex
};
size_t dmd_eig_lds_bytes(int k);
// Linear map, eigendecomposition, amplitudes, ordering and the right factor
// of the modes (every step after U^T Y2 and before phi = Y2 B).
hipError_t launch_dmd_small(const DmdSmallArgs& a, hipStream_t st);
// C (m x nc, ld ldc, FP64) = (A - mu 1^T) (m x K, ld lda; FP64 or FP32, mu
// may be null) B (K x nc, ld ldb), FP64 MFMA.
hipError_t launch_tall_gemm_mu(int in_f64, int64_t m, int K, int nc, const void* A, int64_t lda,
                               const double* mu, const double* B, int64_t ldb, double* C,
                               int64_t ldc, hipStream_t st);
// R1 (n1 x n1, row stride n1) = the leading n1 x n1 block of R (row stride n).
hipError_t launch_dmd_r1(int64_t n1, int64_t n, const double* R, double* R1, hipStream_t st);

// ---- mixed precision: Rayleigh-Ritz refinement against the input ------------
hipError_t launch_cast_f32_f64(const float* src, double* dst, int64_t count, hipStream_t st);
// Z (m x k, ld k) = (A - mu 1^T) V_k with V_k[t][j] = VT0[j * n + t].
hipError_t launch_rr_project(int in_f64, int64_t m, int n, int k, const void* A, int64_t lda,
                             const double* mu, const double* VT0, double* Z, hipStream_t st);
// S, N_r (capped at k), VT rows c < N_r and M (k x k) from the Gram eigenpairs.
hipError_t launch_rr_finish(int n, int k, const double* S0, const double* lam, double residual,
                            double* S, int64_t* nr, const double* WT, const double* VT0,
                            double* VT, int64_t ldvt, double* M, hipStream_t st);
// U[:, c] = Z M[:, c] for c < N_r.
hipError_t launch_rr_form_u(int out_f64, int64_t m, int k, const double* Z, const double* M,
                            const int64_t* nr, void* U, int64_t ldu, hipStream_t st);

// ---- SPOD (Alg. 6): front end, complex TSQR back end ------------------------
size_t spod_table_bytes(int npwin, int t_f64);
// Twiddle/window tables (tab, spod_table_bytes) and scl[0], then the windowed
// one-sided FFT of every Welch block of every point of D (m x nt, FP32): the
// spectral matrix of frequency f is column-major, column blk at complex
// element (f * nb + blk) * ldm of E (complex128 if t_f64, else complex64).
hipError_t launch_spod_front(int t_f64, int64_t m, int64_t nt, const float* D, int64_t ldd,
                             int npwin, int nolap, int nb, int window, int remove_mean, void* tab,
                             double* scl, void* E, int64_t ldm, hipStream_t st);
hipError_t launch_spod_root_realify(int nb, int64_t P, int64_t nf, const double* Rn, double* Rr,
                                    hipStream_t st);
hipError_t launch_spod_root_modes(int nb, int64_t P, int64_t nf, const double* S, const double* VT,
                                  const double* UR, double* Cn, double* L, hipStream_t st);
hipError_t launch_spod_order(int nf, int nb, double dt, int npwin, const double* L, double* freqs,
                             int64_t* order, hipStream_t st);

// ---- complex TSQR of the spectral matrices (ctsqr.hip) -------------------------
// 128-row leaves (one wave each): P = ctsqr_leaves(m) per frequency.  Tree
// node blocks are ctsqr_node_bytes (16 x 16 complex FP64), reflector blocks
// ctsqr_vnode_bytes; both arrays are [nf][P].
int64_t ctsqr_leaves(int64_t m);
size_t ctsqr_node_bytes();
size_t ctsqr_vnode_bytes();
// Per-leaf storage of the factor pass: Vl holds ctsqr_leaf_v_bytes per leaf
// (the reflectors, complex T = t_f64 ? double : float), Wl one node block.
size_t ctsqr_leaf_v_bytes(int nb, int t_f64);
// apply = 0: R of every leaf into Rn, its reflectors into Vl and
// W = T V_top^H into Wl.  apply = 1: modes[f][p][c] = (Q_leaf [C_leaf; 0])[p][c]
// (complex T) with C_leaf the node block of Cn.
hipError_t launch_cleaf(int t_f64, int apply, int nb, int64_t m, int64_t ldm, int64_t P,
                        int64_t nf, const void* E, double* Rn, void* Vl, double* Wl,
                        const double* Cn, void* modes, hipStream_t st);
// Level h of the binary reduction tree (every frequency): node j = 2hc absorbs
// node j + h; the combine's reflectors go to Vn[j + h].
hipError_t launch_ctree_combine(int nb, int64_t P, int64_t h, int64_t nf, double* Rn,
                                double* Vn, hipStream_t st);
// Level h down the tree: [C_j; C_{j+h}] = Q_(j, j+h) [C_j; 0].
hipError_t launch_ctree_apply(int nb, int64_t P, int64_t h, int64_t nf, double* Cn,
                              const double* Vn, hipStream_t st);

}  // namespace pylom
