// svd.hip -- SVD of the small n x n triangular factor R (Eq. svdqr2), FP64.
//
// One-sided (Hestenes) Jacobi applied to X = R^T: the columns of X (the rows
// of R) are rotated pairwise until all pairs are orthogonal to
// tol = n * 2^-53 (relative; a plan may carry a looser threshold, see
// jacobi_tol).  With X J = W (J the accumulated rotations),
// R = J W^T = J diag(sigma) (W diag(1/sigma))^T, so sigma_j = |w_j|,
// U_R = J and V = W diag(1/sigma).  Working on R^T instead of R converges in
// far fewer sweeps for triangular factors (9 instead of 29 on a 256 x 256 R
// with a 1e8 spread of singular values), the effect of the second QR
// preconditioning of Drmac and Veselic obtained here for free, and it yields
// U_R as a product of rotations (exactly orthogonal).  Pair rotation
// (Rutishauser): zeta = (|b|^2 - |a|^2) / (2 a.b),
// t = sign(zeta) / (|zeta| + sqrt(1+zeta^2)), c = 1/sqrt(1+t^2), s = c t,
// a' = c a - s b, b' = s a + c b, with |a'|^2 = |a|^2 - t a.b and
// |b'|^2 = |b|^2 + t a.b carried along (recomputed at every block step and
// after any rotation whose update cancels).
//
// Parallel layout: the npad >= n columns are cut into 2G blocks of w
// columns.  G workgroups (one CU each) form a round-robin tournament over the
// blocks: at every step each workgroup owns two blocks and rotates all w*w
// cross pairs (w rounds; group i keeps column a_i in registers while the
// b-columns circulate through LDS), and once per sweep it also rotates the
// pairs inside its two starting blocks.  Blocks live in global memory between
// steps; steps are separated by a device-wide barrier (bounded spin: a
// timeout sets an error flag instead of hanging).  When G <= 32 the
// participating workgroups are spread over launch slots so that the hardware's
// round-robin placement puts them on one XCD (one shared L2).
#include "common.hpp"
#include "kernels.hpp"

namespace pylom {

constexpr int JT = 256;     // threads per Jacobi workgroup
constexpr int JRPL = 16;    // max column rows per lane
constexpr int BJB = 16;     // column block of the block Jacobi
// Widths above this use the block Jacobi (k_bjacobi): at n = 1808 the
// pairwise tournament needs 451 barrier steps per sweep over 4-column blocks.
constexpr int kBlockJacobiFrom = 256;

// Rotation threshold of a plan: the plan's own, else n 2^-53 (a pair counts
// as orthogonal once its cosine is at the level of the rounding of n-term
// FP64 dot products).
double jacobi_tol(const JacobiPlan& p) { return p.tol > 0.0 ? p.tol : (double)p.n * 0x1p-53; }

bool jacobi_plan(int n, JacobiPlan* p) {
  if (n < 1 || n > 2048) return false;
  p->tol = 0.0;
  p->no_ur = 0;
  p->block = 0;
  p->ks = 1;
  if (n > kBlockJacobiFrom) {
    // block tournament: 2G blocks of 16 columns, G workgroups
    p->n = n;
    p->w = BJB;
    p->npad = (n + 2 * BJB - 1) / (2 * BJB) * (2 * BJB);
    p->G = p->npad / (2 * BJB);
    p->lpp = 64;
    p->xcd_stride = 1;
    p->block = 1;
    // workgroups per block pair (rows split in ks parts): at most 240
    // workgroups in all, one per CU
    p->ks = 240 / p->G < 4 ? (240 / p->G < 1 ? 1 : 240 / p->G) : 4;
    return true;
  }
  // block width w (even, 4..16): a pair is handled by 256/w lanes of one wave,
  // each holding at most JRPL rows of a column.  16 up to n = 256: measured
  // on one MI355X (the SVD phase of FP64 POD), n = 256 takes 6.3 ms at
  // w = 16, 8.9 at w = 8 and 17.3 at w = 4; fewer, wider blocks win because
  // every tournament step ends in a grid barrier.
  int w = 16;
  if (n <= 2 * w) {
    int half = (n + 1) / 2;
    int ww = 4;
    while (ww < half) ww <<= 1;
    w = ww;
  }
  const int G = (n + 2 * w - 1) / (2 * w);
  p->n = n;
  p->w = w;
  p->G = G;
  p->npad = 2 * G * w;
  p->lpp = JT / w;
  p->xcd_stride = (G <= 32) ? 8 : 1;
  return p->lpp <= 64 && (n + p->lpp - 1) / p->lpp <= JRPL;
}

struct JacobiWs {
  double* A;          // npad columns x n rows (column-major)
  double* V;          // npad columns x n rows
  unsigned int* bar;  // barrier counter
  int* flags;         // rotations per sweep; then (block Jacobi) the pair counters
  int* pairc;
  double* gp;         // block Jacobi: posted partial Gram matrices
};

// Ints of the flags area: rotation counts of max_sweeps + 1 sweeps, then one
// counter per block pair 16 ints apart (all zeroed by the setup kernel).
static int jacobi_pair_off(int max_sweeps) { return (max_sweeps + 1 + 15) / 16 * 16; }
static int jacobi_nflags(const JacobiPlan& p, int max_sweeps) {
  return p.block ? jacobi_pair_off(max_sweeps) + 16 * p.G : max_sweeps + 1;
}

static JacobiWs jacobi_ws(const JacobiPlan& p, int max_sweeps, void* ws) {
  JacobiWs w;
  char* c = (char*)ws;
  w.A = (double*)c;
  c += sizeof(double) * (size_t)p.npad * p.n;
  w.V = (double*)c;
  c += sizeof(double) * (size_t)p.npad * p.n;
  w.bar = (unsigned int*)c;  // global counter, deflation maximum, eight group counters
  c += 1024;
  w.flags = (int*)c;
  w.pairc = w.flags + jacobi_pair_off(max_sweeps);
  c += (sizeof(int) * (size_t)(jacobi_nflags(p, max_sweeps) + 64) + 255) & ~(size_t)255;
  w.gp = (double*)c;
  return w;
}

size_t jacobi_ws_bytes(const JacobiPlan& p, int max_sweeps) {
  size_t b = sizeof(double) * 2 * (size_t)p.npad * p.n + 1024 +
             ((sizeof(int) * (size_t)(jacobi_nflags(p, max_sweeps) + 64) + 255) & ~(size_t)255);
  if (p.block) b += sizeof(double) * 3 * 256 * (size_t)p.G * p.ks;
  return b;
}

// ---- setup: A <- R^T (column j = row j of R), V <- I, counters <- 0 ---------
__global__ void k_jacobi_setup(int n, int npad, const double* __restrict__ R, double* A,
                               double* V, unsigned int* bar, int* flags, int nflags, int* status,
                               int status0, int64_t sR, int64_t sWs) {
  if (blockIdx.y) {
    // batch: problem blockIdx.y has its own R (stride sR doubles) and its own
    // workspace slice (stride sWs bytes)
    const int64_t pb = blockIdx.y;
    R += pb * sR;
    A = (double*)((char*)A + pb * sWs);
    V = (double*)((char*)V + pb * sWs);
    bar = (unsigned int*)((char*)bar + pb * sWs);
    flags = (int*)((char*)flags + pb * sWs);
    status += 2 * pb;
  }
  const int64_t total = (int64_t)npad * n;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx / n), i = (int)(idx % n);
    A[idx] = (j < n) ? R[(int64_t)j * n + i] : 0.0;
    V[idx] = (i == j) ? 1.0 : 0.0;
  }
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < nflags; k += blockDim.x) flags[k] = 0;
    if (threadIdx.x < 8)
      *reinterpret_cast<unsigned int*>(reinterpret_cast<char*>(bar) + 128 + 64 * threadIdx.x) = 0u;
    if (threadIdx.x == 0) {
      *bar = 0u;
      *reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(bar) + 64) = 0ull;
      status[0] = status0;
      status[1] = 0;
    }
  }
}

// Device-wide barrier of the G participating workgroups (participant index
// gi).  Two levels: participants arrive on eight group counters (gi & 7,
// separate 64-byte lines after the global counter and the deflation word),
// and only the last arriver of each group increments the global counter, so
// a barrier costs eight global atomics instead of G.  The spin is bounded:
// a timeout, or a timeout already flagged by any workgroup, sets the error
// flag and stops waiting, so a failed barrier ends the kernel quickly
// instead of stalling every later one.
__device__ __forceinline__ void grid_barrier(unsigned int* bar, unsigned int G, unsigned int gi,
                                             unsigned int& epoch, int* status) {
  __syncthreads();
  if (threadIdx.x == 0) {
    ++epoch;
    const unsigned int ng = G < 8u ? G : 8u;
    const unsigned int grp = gi & 7u;
    const unsigned int gs = (G - grp + 7u) / 8u;  // participants in this group
    unsigned int* cnt =
        reinterpret_cast<unsigned int*>(reinterpret_cast<char*>(bar) + 128 + 64 * grp);
    __threadfence();
    const unsigned int prev = atomicAdd(cnt, 1u);
    if (prev == epoch * gs - 1u) {
      __threadfence();
      atomicAdd(bar, 1u);
    }
    const unsigned int target = epoch * ng;
    unsigned long long spins = 0;
    // relaxed polls: an acquire load invalidates this XCD's L2 on every
    // iteration, under workgroups still loading and storing their columns
    // for this step; the fence after the loop is the acquire
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if ((++spins & 1023ull) == 0 &&
          (spins > (1ull << 24) ||
           __hip_atomic_load(status + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
        atomicExch(status + 1, 1);
        break;
      }
    }
    __threadfence();
  }
  __syncthreads();
}

// Sum over an LPP-lane group (LPP = 16, 32 or 64): DPP rotations inside the
// 16-lane row, then the row-pair swaps.
template <int LPP>
__device__ __forceinline__ double gsum(double x) {
  x += dpp<0x128>(x);
  x += dpp<0x124>(x);
  x += dpp<0x122>(x);
  x += dpp<0x121>(x);
  if (LPP >= 32) x = perm16_pairsum(x);
  if (LPP >= 64) x = perm32_pairsum(x);
  return x;
}

// block index of player i (0..2G-1) at tournament step st (circle method)
__device__ __forceinline__ int rr_player(int i, int st, int nplayers) {
  if (i == 0) return 0;
  return ((i - 1 + st) % (nplayers - 1)) + 1;
}

template <int LPP, int JR>
__device__ __forceinline__ double col_norm2(const double (&a)[JR], int rpl) {
  double x = 0.0;
#pragma unroll
  for (int k = 0; k < JR; ++k)
    if (k < rpl) x += a[k] * a[k];
  return gsum<LPP>(x);
}

// Rotate the pair (a, b) held by an LPP-lane group (RPL rows per lane each)
// if it is not yet orthogonal; norms na, nb are updated.  Returns 1 if rotated.
template <int LPP, int JR>
__device__ __forceinline__ int jacobi_pair(double (&a)[JR], double (&va)[JR], double (&b)[JR],
                                           double (&vb)[JR], double& na, double& nb, int rpl_a,
                                           int rpl_v, double tol) {
  double g = 0.0;
#pragma unroll
  for (int k = 0; k < JR; ++k)
    if (k < rpl_a) g += a[k] * b[k];
  g = gsum<LPP>(g);
  if (!(na > 0.0) || !(nb > 0.0)) return 0;
  if (fabs(g) <= tol * sqrt(na) * sqrt(nb)) return 0;
  const double zeta = (nb - na) / (2.0 * g);
  const double az = fabs(zeta);
  // |zeta| > 1e150 (columns of very different tiny norms, as rank-deficient
  // R produces): zeta^2 would overflow and t become 0, an identity rotation
  // that still counts as one and stalls convergence; there t = 1/(2|zeta|)
  // to full precision
  double t = (az > 1e150) ? 0.5 / az : 1.0 / (az + sqrt(1.0 + zeta * zeta));
  if (!(t > 0.0)) return 0;  // zeta = inf: no representable rotation
  if (zeta < 0.0) t = -t;
  const double c = 1.0 / sqrt(1.0 + t * t);
  const double s = c * t;
#pragma unroll
  for (int k = 0; k < JR; ++k) {
    if (k < rpl_a) {
      const double x = a[k], y = b[k];
      a[k] = c * x - s * y;
      b[k] = s * x + c * y;
    }
    if (k < rpl_v) {
      const double x = va[k], y = vb[k];
      va[k] = c * x - s * y;
      vb[k] = s * x + c * y;
    }
  }
  const double na2 = na - t * g, nb2 = nb + t * g;
  if (na2 < 0.5 * na || nb2 < 0.5 * nb) {
    // the update cancels (a column nearly parallel to a much longer one, as
    // in rank-deficient R): carried norms would lose all accuracy and stall
    // the convergence test, so recompute both from the rotated columns.
    // The branch is uniform over the group (its inputs are group sums).
    na = col_norm2<LPP, JR>(a, rpl_a);
    nb = col_norm2<LPP, JR>(b, rpl_a);
  } else {
    na = na2;
    nb = nb2;
  }
  return 1;
}

template <int LPP, int JR>
__device__ __forceinline__ void load_col(double (&x)[JR], const double* __restrict__ col, int rows,
                                         int sub) {
#pragma unroll
  for (int k = 0; k < JR; ++k) {
    const int r = sub + LPP * k;
    x[k] = (r < rows) ? col[r] : 0.0;
  }
}

template <int LPP, int JR>
__device__ __forceinline__ void store_col(const double (&x)[JR], double* __restrict__ col, int rows,
                                          int sub) {
#pragma unroll
  for (int k = 0; k < JR; ++k) {
    const int r = sub + LPP * k;
    if (r < rows) col[r] = x[k];
  }
}

struct JacobiArgs {
  int n, npad, w, G, xcd_stride, max_sweeps;
  int uv;      // 1: accumulate the rotations into V (U_R); 0: V is not touched
  double tol;  // rotation test: |a_p . a_q| > tol |a_p| |a_q|
  double* A;
  double* V;
  unsigned int* bar;
  int* flags;
  int* status;
  int64_t sWs;  // batch: workspace slice stride in bytes (problem = blockIdx.y)
};

template <int LPP, int JR>
__global__ __launch_bounds__(JT) void k_jacobi(JacobiArgs a) {
  if (blockIdx.x % a.xcd_stride) return;
  if (blockIdx.y) {
    const int64_t pb = blockIdx.y;
    a.A = (double*)((char*)a.A + pb * a.sWs);
    a.V = (double*)((char*)a.V + pb * a.sWs);
    a.bar = (unsigned int*)((char*)a.bar + pb * a.sWs);
    a.flags = (int*)((char*)a.flags + pb * a.sWs);
    a.status += 2 * pb;
  }
  // circulating b columns (A and V parts), double-buffered
  constexpr int NBUF = 2;
  __shared__ double xbuf[NBUF][JT * 2 * JR];
  __shared__ double xnorm[2][JT / 2];
  __shared__ int rot_count;
  const int g = blockIdx.x / a.xcd_stride;
  const int tid = threadIdx.x;
  const int w = a.w, n = a.n;
  const int grp = tid / LPP, sub = tid % LPP;
  const int rpl = (n + LPP - 1) / LPP;
  const double tol = a.tol;
  const int rv = a.uv ? rpl : 0;  // V rows per lane that the rotations update
  const int nplayers = 2 * a.G;
  unsigned int epoch = 0;
  double ca[JR], cva[JR], cb[JR], cvb[JR];
  int sweep_done = -1;
  // Deflation: columns of R^T (rows of R) whose norm is at most 2^-53 times
  // the largest are rounding noise (rank-deficient input leaves them graded
  // down to the underflow range, where Jacobi would spend dozens of sweeps
  // orthogonalising them); they are set to zero, a perturbation of R within
  // the QR's own backward error.  The maximum is combined with an atomic max
  // on the bit pattern (non-negative doubles order like integers), which
  // does not depend on the order of arrival.
  {
    unsigned long long* cmax =
        reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(a.bar) + 64);
    const int blk0 = rr_player(g, 0, nplayers), blk1 = rr_player(nplayers - 1 - g, 0, nplayers);
    double nr2[2];
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
      const int jc = (hb ? blk1 : blk0) * w + grp;
      load_col<LPP, JR>(ca, a.A + (int64_t)jc * n, n, sub);
      nr2[hb] = col_norm2<LPP, JR>(ca, rpl);
    }
    if (sub == 0)
      atomicMax(cmax, (unsigned long long)__double_as_longlong(nr2[0] > nr2[1] ? nr2[0] : nr2[1]));
    grid_barrier(a.bar, (unsigned int)a.G, (unsigned int)g, epoch, a.status);
    const double mx = __longlong_as_double(
        (long long)__hip_atomic_load(cmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const double thr2 = mx * 0x1p-106;
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
      if (nr2[hb] > 0.0 && nr2[hb] <= thr2) {
        const int jc = (hb ? blk1 : blk0) * w + grp;
#pragma unroll
        for (int k = 0; k < JR; ++k) ca[k] = 0.0;
        store_col<LPP, JR>(ca, a.A + (int64_t)jc * n, n, sub);
      }
    }
    __syncthreads();
  }
  for (int sw = 0; sw < a.max_sweeps; ++sw) {
    if (tid == 0) rot_count = 0;
    __syncthreads();
    int myrot = 0;
    // ---- pairs inside my two starting blocks (round-robin of w columns)
    {
      const int blk_a = rr_player(g, 0, nplayers), blk_b = rr_player(nplayers - 1 - g, 0, nplayers);
      const int half = w / 2;
      const int which = (grp < half) ? blk_a : blk_b;
      const int pi = (grp < half) ? grp : grp - half;
      for (int q = 0; q < w - 1; ++q) {
        const int c1 = rr_player(pi, q, w), c2 = rr_player(w - 1 - pi, q, w);
        const int j1 = which * w + c1, j2 = which * w + c2;
        load_col<LPP, JR>(ca, a.A + (int64_t)j1 * n, n, sub);
        load_col<LPP, JR>(cb, a.A + (int64_t)j2 * n, n, sub);
        if (a.uv) {
          load_col<LPP, JR>(cva, a.V + (int64_t)j1 * n, n, sub);
          load_col<LPP, JR>(cvb, a.V + (int64_t)j2 * n, n, sub);
        }
        double na = col_norm2<LPP, JR>(ca, rpl), nb = col_norm2<LPP, JR>(cb, rpl);
        myrot += jacobi_pair<LPP, JR>(ca, cva, cb, cvb, na, nb, rpl, rv, tol);
        store_col<LPP, JR>(ca, a.A + (int64_t)j1 * n, n, sub);
        store_col<LPP, JR>(cb, a.A + (int64_t)j2 * n, n, sub);
        if (a.uv) {
          store_col<LPP, JR>(cva, a.V + (int64_t)j1 * n, n, sub);
          store_col<LPP, JR>(cvb, a.V + (int64_t)j2 * n, n, sub);
        }
        __syncthreads();
      }
    }
    // ---- cross-block steps of the tournament
    for (int st = 0; st < nplayers - 1; ++st) {
      const int blk_a = rr_player(g, st, nplayers), blk_b = rr_player(nplayers - 1 - g, st, nplayers);
      const int ja = blk_a * w + grp;
      load_col<LPP, JR>(ca, a.A + (int64_t)ja * n, n, sub);
      load_col<LPP, JR>(cb, a.A + (int64_t)(blk_b * w + grp) * n, n, sub);
      if (a.uv) {
        load_col<LPP, JR>(cva, a.V + (int64_t)ja * n, n, sub);
        load_col<LPP, JR>(cvb, a.V + (int64_t)(blk_b * w + grp) * n, n, sub);
      }
      double na = col_norm2<LPP, JR>(ca, rpl), nb = col_norm2<LPP, JR>(cb, rpl);
      for (int q = 0; q < w; ++q) {
        myrot += jacobi_pair<LPP, JR>(ca, cva, cb, cvb, na, nb, rpl, rv, tol);
        if (q < w - 1) {
          // pass my b column to group grp-1, take the one of group grp+1; with
          // two alternating buffers one barrier per round suffices
          double* xb = xbuf[q & 1];
          // k-major slots: consecutive lanes touch consecutive doubles
#pragma unroll
          for (int k = 0; k < JR; ++k) xb[k * JT + tid] = cb[k];
          if (a.uv) {
#pragma unroll
            for (int k = 0; k < JR; ++k) xb[(JR + k) * JT + tid] = cvb[k];
          }
          if (sub == 0) xnorm[q & 1][grp] = nb;
          __syncthreads();
          const int src = (grp + 1) % w;
#pragma unroll
          for (int k = 0; k < JR; ++k) cb[k] = xb[k * JT + src * LPP + sub];
          if (a.uv) {
#pragma unroll
            for (int k = 0; k < JR; ++k) cvb[k] = xb[(JR + k) * JT + src * LPP + sub];
          }
          nb = xnorm[q & 1][src];
        }
      }
      store_col<LPP, JR>(ca, a.A + (int64_t)ja * n, n, sub);
      const int jb = blk_b * w + (grp + w - 1) % w;
      store_col<LPP, JR>(cb, a.A + (int64_t)jb * n, n, sub);
      if (a.uv) {
        store_col<LPP, JR>(cva, a.V + (int64_t)ja * n, n, sub);
        store_col<LPP, JR>(cvb, a.V + (int64_t)jb * n, n, sub);
      }
      if (st == nplayers - 2) {
        // count rotations of this sweep before the last barrier
        if (sub == 0 && myrot) atomicAdd(&rot_count, myrot);
        __syncthreads();
        if (tid == 0 && rot_count) atomicAdd(a.flags + sw, rot_count);
      }
      grid_barrier(a.bar, (unsigned int)a.G, (unsigned int)g, epoch, a.status);
    }
    const int total = __hip_atomic_load(a.flags + sw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (total == 0) {
      sweep_done = sw + 1;
      break;
    }
  }
  if (g == 0 && tid == 0) a.status[0] = sweep_done;
}

// ---- block one-sided Jacobi (n > 256) ----------------------------------------
// The columns of X = R^T are cut into 2G blocks of 16.  G block pairs play
// the round-robin tournament of the pairwise kernel over blocks, one
// device-wide barrier per step; each pair is served by ks workgroups, one
// per quarter of the rows.  At a step the workgroups of pair g own the 32
// columns X_p = [X_I X_J]:
//   1. each forms the Gram matrix of its rows, M_k = X_p,k^T X_p,k (FP64
//      MFMA), and posts it; after a barrier of the ks workgroups each sums
//      them in the same order, M = sum_k M_k;
//   2. each runs the same rounds of two-sided rotations on M in LDS
//      (16 disjoint pairs per round: the 256 pairs across the two blocks in
//      16 rounds, and at the first step of a sweep also the pairs inside
//      each block in 15 rounds before them; each is the pair rotation of
//      jacobi_pair, decided by the same relative test m_pq^2 > tol^2 m_pp
//      m_qq, with m_pp - t m_pq and m_qq + t m_pq as the new diagonal and an
//      exact zero at (p, q)), accumulating the orthogonal W (32 x 32);
//      identical inputs give identical W in every workgroup;
//   3. each applies W to its rows: X_p <- X_p W, V_p <- V_p W (FP64 MFMA).
// Every step starts from a fresh Gram matrix of the current columns, so each
// rotation decision rests on dot products as accurate as the pairwise ones;
// a step whose Gram matrix passes the test for every pair leaves its columns
// untouched.  A sweep in which no step rotated ends the iteration.
struct BJArgs {
  int n, npad, G, ks, max_sweeps;
  double tol;  // rotation test, as in the pairwise kernel
  double* A;
  double* V;
  unsigned int* bar;
  int* flags;
  int* pairc;   // one counter per block pair, 16 ints apart
  double* gp;   // posted partial Gram matrices: [G][ks][3 * 256]
  int* status;
};

// Barrier of the ks workgroups of one block pair (bounded spin, as the grid
// barrier).
__device__ __forceinline__ void pair_barrier(int* cnt, int ks, int& pep, int* status) {
  __syncthreads();
  if (threadIdx.x == 0) {
    ++pep;
    __threadfence();
    atomicAdd(cnt, 1);
    const int target = pep * ks;
    unsigned long long spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 1023ull) == 0 &&
          (spins > (1ull << 24) ||
           __hip_atomic_load(status + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
        atomicExch(status + 1, 1);
        break;
      }
    }
    __threadfence();
  }
  __syncthreads();
}

// Pair k (< 16) of round rd of a step: the within-block rounds (15, first
// step of a sweep) pair the columns of each block among themselves (8 pairs
// in block I, 8 in block J); the cross rounds (16) pair column k of block I
// with column (k + rd) mod 16 of block J.
__device__ __forceinline__ void bj_pair(int k, int rd, bool within, int& p, int& q) {
  if (within) {
    const int kk = k & 7, off = k < 8 ? 0 : 16;
    p = off + rr_player(kk, rd, 16);
    q = off + rr_player(15 - kk, rd, 16);
  } else {
    p = k;
    q = 16 + ((k + rd) & 15);
  }
}

// c = (1 + t^2)^(-1/2): hardware reciprocal square root refined by two
// Newton steps.
__device__ __forceinline__ double rot_cos(double t) {
  const double x = fma(t, t, 1.0);
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  y = y * fma(-0.5 * x * y, y, 1.5);
  return y;
}

// UV: the rotations are accumulated into V (J, the left factor U_R of R);
// without UV, V is left as it is (callers that need only sigma and V of R).
template <bool UV>
__global__ __launch_bounds__(256) void k_bjacobi(BJArgs a) {
  typedef Mfma<double>::v4 v4;
  constexpr int LD = 33;
  __shared__ double Ms[32 * LD];
  __shared__ double Ws[32 * LD];
  __shared__ double part[4][3][256];
  __shared__ double rcs[16][6];  // c, s, t, m_pq, m_pp, m_qq of pair k in this round
  __shared__ int step_rot, rot_count;
  const int g = blockIdx.x / a.ks, kq = blockIdx.x % a.ks;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, g4 = lane >> 4;
  const int n = a.n, ks = a.ks;
  const double tol = a.tol, tol2 = tol * tol;
  const int nplayers = 2 * a.G;
  const unsigned int nwg = (unsigned int)(a.G * ks);
  // this workgroup's rows: 16-row tiles [t0, t1)
  const int ntiles = (n + 15) / 16, tq = (ntiles + ks - 1) / ks;
  const int t0 = kq * tq < ntiles ? kq * tq : ntiles;
  const int t1 = t0 + tq < ntiles ? t0 + tq : ntiles;
  const int rlo = 16 * t0, rhi = 16 * t1 < n ? 16 * t1 : n;
  int* pcnt = a.pairc + 16 * g;
  double* mypart = a.gp + ((int64_t)g * ks + kq) * (3 * 256);
  unsigned int epoch = 0;
  int pep = 0;
  int sweep_done = -1;
  // deflation of rounding-noise columns, as in the pairwise kernel (the first
  // workgroup of each pair, 8 threads per column of its starting blocks)
  {
    unsigned long long* cmax =
        reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(a.bar) + 64);
    const int b0 = rr_player(g, 0, nplayers), b1 = rr_player(nplayers - 1 - g, 0, nplayers);
    const int c = tid >> 3, sub = tid & 7;
    const int jc = (c < 16 ? b0 : b1) * BJB + (c & 15);
    double x = 0.0;
    if (kq == 0) {
      const double* col = a.A + (int64_t)jc * n;
      for (int r = sub; r < n; r += 8) x += col[r] * col[r];
    }
    x = group_sum<8>(x);
    if (kq == 0 && sub == 0) atomicMax(cmax, (unsigned long long)__double_as_longlong(x));
    grid_barrier(a.bar, nwg, (unsigned int)blockIdx.x, epoch, a.status);
    const double mx = __longlong_as_double(
        (long long)__hip_atomic_load(cmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (kq == 0 && x > 0.0 && x <= mx * 0x1p-106) {
      double* cw = a.A + (int64_t)jc * n;
      for (int r = sub; r < n; r += 8) cw[r] = 0.0;
    }
    grid_barrier(a.bar, nwg, (unsigned int)blockIdx.x, epoch, a.status);
  }
  for (int sw = 0; sw < a.max_sweeps; ++sw) {
    if (tid == 0) rot_count = 0;
    for (int st = 0; st < nplayers - 1; ++st) {
      const int bI = rr_player(g, st, nplayers), bJ = rr_player(nplayers - 1 - g, st, nplayers);
      // ---- partial Gram matrix of rows [rlo, rhi): wave w takes the 4-row
      // steps w, w + 4, ...; three 16 x 16 tiles M_II, M_IJ, M_JJ
      {
        const double* xa = a.A + (int64_t)(bI * BJB + i16) * n;
        const double* xb = a.A + (int64_t)(bJ * BJB + i16) * n;
        v4 t00 = vzero4<double>(), t01 = vzero4<double>(), t11 = vzero4<double>();
        const int nst = rhi - rlo - 4 * wave > 0 ? (rhi - rlo - 4 * wave + 15) / 16 : 0;
        for (int s0 = 0; s0 < nst; s0 += 16) {
          double u[16], v[16];
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            const int r = rlo + 16 * (s0 + k) + 4 * wave + g4;
            const bool ok = s0 + k < nst && r < rhi;
            u[k] = ok ? xa[r] : 0.0;
            v[k] = ok ? xb[r] : 0.0;
          }
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            t00 = Mfma<double>::op(u[k], u[k], t00);
            t01 = Mfma<double>::op(u[k], v[k], t01);
            t11 = Mfma<double>::op(v[k], v[k], t11);
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = Mfma<double>::drow(g4, q) * 16 + i16;
          part[wave][0][e] = t00[q];
          part[wave][1][e] = t01[q];
          part[wave][2][e] = t11[q];
        }
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < 3; ++t)
        mypart[t * 256 + tid] = (part[0][t][tid] + part[1][t][tid]) + (part[2][t][tid] + part[3][t][tid]);
      pair_barrier(pcnt, ks, pep, a.status);
      if (tid == 0) step_rot = 0;
      {
        const double* gp0 = a.gp + (int64_t)g * ks * (3 * 256);
        // the ks <= 4 partial Gram matrices, all loads issued before the
        // sums (in the fixed order k = 0, 1, ...)
        double pv[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int t = 0; t < 3; ++t) pv[k][t] = (k < ks) ? gp0[k * (3 * 256) + t * 256 + tid] : 0.0;
        double m[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int t = 0; t < 3; ++t) m[t] = (k < ks) ? m[t] + pv[k][t] : m[t];
        const int i = tid >> 4, j = tid & 15;
        Ms[i * LD + j] = m[0];
        Ms[i * LD + 16 + j] = m[1];
        Ms[(16 + j) * LD + i] = m[1];
        Ms[(16 + i) * LD + 16 + j] = m[2];
#pragma unroll
        for (int e = tid; e < 32 * 32; e += 256) Ws[(e >> 5) * LD + (e & 31)] = (e >> 5) == (e & 31) ? 1.0 : 0.0;
      }
      __syncthreads();
      // does any pair of this step need a rotation?  (the cross pairs; at
      // the first step of a sweep also the pairs inside each block)
      const bool first = st == 0;
      {
        int need = 0;
        for (int e = tid; e < 32 * 32; e += 256) {
          const int i = e >> 5, j = e & 31;
          if (i < j && (first || (i < 16 && j >= 16))) {
            const double mii = Ms[i * LD + i], mjj = Ms[j * LD + j], mij = Ms[i * LD + j];
            if (mii > 0.0 && mjj > 0.0 && mij * mij > tol2 * mii * mjj) need = 1;
          }
        }
        if (need) step_rot = 1;
      }
      __syncthreads();
      if (step_rot) {
        int myrot = 0;
        // ---- one cyclic sweep of two-sided rotations on M, accumulated in W
        const int ra = tid >> 4, cb = tid & 15;  // 2 x 2 block (row pair ra, column pair cb)
        const int nrounds = first ? 31 : 16;
        for (int rdi = 0; rdi < nrounds; ++rdi) {
          const bool within = first && rdi < 15;
          const int rd = within ? rdi : (first ? rdi - 15 : rdi);
          if (tid < 16) {
            int p, q;
            bj_pair(tid, rd, within, p, q);
            const double mpp = Ms[p * LD + p], mqq = Ms[q * LD + q], mpq = Ms[p * LD + q];
            double c = 1.0, sn = 0.0, t = 0.0;
            if (mpp > 0.0 && mqq > 0.0 && mpq * mpq > tol2 * mpp * mqq) {
              // the pair rotation: t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2))
              // with zeta = (m_qq - m_pp) / (2 m_pq), written as
              // 2 m_pq sign(d) / (|d| + sqrt(d^2 + 4 m_pq^2)), d = m_qq - m_pp
              const double d = mqq - mpp;
              const double rr = sqrt(fma(d, d, 4.0 * mpq * mpq));
              double tt = 2.0 * mpq / (fabs(d) + rr);
              if (d < 0.0) tt = -tt;
              if (tt != 0.0 && isfinite(tt)) {
                c = rot_cos(tt);
                sn = c * tt;
                t = tt;
                ++myrot;
              }
            }
            rcs[tid][0] = c;
            rcs[tid][1] = sn;
            rcs[tid][2] = t;
            rcs[tid][3] = mpq;
            rcs[tid][4] = mpp;
            rcs[tid][5] = mqq;
          }
          __syncthreads();
          {
            // rows (p_a, q_a) and columns (p_b, q_b) of M: both sides at once
            int pa, qa, pb, qb;
            bj_pair(ra, rd, within, pa, qa);
            bj_pair(cb, rd, within, pb, qb);
            const double ca = rcs[ra][0], sa = rcs[ra][1];
            const double cc = rcs[cb][0], sc = rcs[cb][1];
            if (ra == cb) {
              if (rcs[ra][2] != 0.0) {
                const double t = rcs[ra][2], mpq = rcs[ra][3];
                Ms[pa * LD + pa] = rcs[ra][4] - t * mpq;
                Ms[qa * LD + qa] = rcs[ra][5] + t * mpq;
                Ms[pa * LD + qa] = 0.0;
                Ms[qa * LD + pa] = 0.0;
              }
            } else if (rcs[ra][2] != 0.0 || rcs[cb][2] != 0.0) {
              const double xpp = Ms[pa * LD + pb], xpq = Ms[pa * LD + qb];
              const double xqp = Ms[qa * LD + pb], xqq = Ms[qa * LD + qb];
              const double ypp = ca * xpp - sa * xqp, ypq = ca * xpq - sa * xqq;
              const double yqp = sa * xpp + ca * xqp, yqq = sa * xpq + ca * xqq;
              Ms[pa * LD + pb] = cc * ypp - sc * ypq;
              Ms[pa * LD + qb] = sc * ypp + cc * ypq;
              Ms[qa * LD + pb] = cc * yqp - sc * yqq;
              Ms[qa * LD + qb] = sc * yqp + cc * yqq;
            }
            // W <- W J: rows (p_a, q_a), columns (p_b, q_b)
            if (rcs[cb][2] != 0.0) {
              const double wpp = Ws[pa * LD + pb], wpq = Ws[pa * LD + qb];
              const double wqp = Ws[qa * LD + pb], wqq = Ws[qa * LD + qb];
              Ws[pa * LD + pb] = cc * wpp - sc * wpq;
              Ws[pa * LD + qb] = sc * wpp + cc * wpq;
              Ws[qa * LD + pb] = cc * wqp - sc * wqq;
              Ws[qa * LD + qb] = sc * wqp + cc * wqq;
            }
          }
          __syncthreads();
        }
        if (kq == 0 && myrot) atomicAdd(&rot_count, myrot);
        // ---- X_p <- X_p W and (UV) V_p <- V_p W on this workgroup's tiles; wave w
        // takes the tiles t0 + w, t0 + w + 4, ...; B operand W[4 s + g4][16 h + i16]
        double wb[2][8];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int s4 = 0; s4 < 8; ++s4) wb[h][s4] = Ws[(4 * s4 + g4) * LD + 16 * h + i16];
        int64_t coff[8];
#pragma unroll
        for (int s4 = 0; s4 < 8; ++s4) {
          const int cl = 4 * s4 + g4;
          coff[s4] = (int64_t)((cl < 16 ? bI : bJ) * BJB + (cl & 15)) * n;
        }
        // up to TMX tiles of the wave are loaded from both buffers before any
        // product or store: one memory round trip for the step, and no wait
        // for loads issued after stores (a single counter tracks both, in
        // issue order)
        constexpr int TMX = 8;
        constexpr int NBUF = UV ? 2 : 1;
        for (int base = t0 + wave; base < t1; base += 4 * TMX) {
          double xv[NBUF][TMX][8];
#pragma unroll
          for (int buf = 0; buf < NBUF; ++buf) {
            const double* X = buf ? a.V : a.A;
#pragma unroll
            for (int jt = 0; jt < TMX; ++jt) {
              const int tl = base + 4 * jt, rr = 16 * tl + i16;
              const bool ok = tl < t1 && rr < n;
#pragma unroll
              for (int s4 = 0; s4 < 8; ++s4) xv[buf][jt][s4] = ok ? X[coff[s4] + rr] : 0.0;
            }
          }
#pragma unroll
          for (int buf = 0; buf < NBUF; ++buf) {
            double* X = buf ? a.V : a.A;
#pragma unroll
            for (int jt = 0; jt < TMX; ++jt) {
              const int tl = base + 4 * jt;
              if (tl < t1) {
                v4 o0 = vzero4<double>(), o1 = vzero4<double>();
#pragma unroll
                for (int s4 = 0; s4 < 8; ++s4) {
                  o0 = Mfma<double>::op(xv[buf][jt][s4], wb[0][s4], o0);
                  o1 = Mfma<double>::op(xv[buf][jt][s4], wb[1][s4], o1);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  const int row = 16 * tl + Mfma<double>::drow(g4, q);
                  if (row < n) {
                    X[(int64_t)(bI * BJB + i16) * n + row] = o0[q];
                    X[(int64_t)(bJ * BJB + i16) * n + row] = o1[q];
                  }
                }
              }
            }
          }
        }
      }
      if (st == nplayers - 2) {
        __syncthreads();
        if (tid == 0 && rot_count) atomicAdd(a.flags + sw, rot_count);
      }
      grid_barrier(a.bar, nwg, (unsigned int)blockIdx.x, epoch, a.status);
    }
    const int total = __hip_atomic_load(a.flags + sw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (total == 0) {
      sweep_done = sw + 1;
      break;
    }
  }
  if (blockIdx.x == 0 && tid == 0) a.status[0] = sweep_done;
}

// ---- finalize: sigma, sort, sign convention, outputs, truncation ------------
// A holds W (columns w_j, sigma_j = |w_j|, v_j = w_j / sigma_j); V holds J
// (u_j = column j).  Each pair is signed so that the largest-magnitude entry
// of v_j (lowest index on ties) is positive.  A zero sigma leaves v_j = 0.
// A singular value that is not finite (NaN or Inf in the input propagates
// into R, and the Jacobi rotates no pair whose norms are not positive) sets
// status[0] = -2.
constexpr int FT = 1024;
__global__ __launch_bounds__(FT) void k_svd_finalize(int n, const double* __restrict__ A,
                                                     const double* __restrict__ V, double* S,
                                                     double* VT, int64_t ldvt, double* UR,
                                                     double residual, int64_t* nr, int64_t sWs,
                                                     int64_t sS, int64_t sVT, int64_t sUR,
                                                     int* status) {
  if (blockIdx.y) {
    const int64_t pb = blockIdx.y;
    A = (const double*)((const char*)A + pb * sWs);
    V = (const double*)((const char*)V + pb * sWs);
    S += pb * sS;
    VT += pb * sVT;
    if (UR) UR += pb * sUR;
    nr += pb;
    status += 2 * pb;
  }
  __shared__ int nonfinite;
  if (threadIdx.x == 0) nonfinite = 0;
  __shared__ double sig[2048];
  __shared__ double sgn[2048];
  __shared__ int rank[2048];
  __shared__ double tail[2049];
  const int tid = threadIdx.x;
  for (int j = tid; j < n; j += FT) {
    const double* col = A + (int64_t)j * n;
    double x = 0.0;
    int arg = 0;
    double best = -1.0;
    for (int i = 0; i < n; ++i) {
      x += col[i] * col[i];
      const double av = fabs(col[i]);
      if (av > best) {
        best = av;
        arg = i;
      }
    }
    sig[j] = sqrt(x);
    sgn[j] = (col[arg] < 0.0) ? -1.0 : 1.0;
    if (!isfinite(sig[j])) nonfinite = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0 && nonfinite) status[0] = -2;
  for (int j = tid; j < n; j += FT) {
    const double sj = sig[j];
    int r = 0;
    for (int i = 0; i < n; ++i) r += (sig[i] > sj) || (sig[i] == sj && i < j);
    rank[j] = r;
  }
  __syncthreads();
  for (int j = tid; j < n; j += FT) S[rank[j]] = sig[j];
  for (int64_t idx = tid; idx < (int64_t)n * n; idx += FT) {
    const int j = (int)(idx / n), i = (int)(idx % n);
    const int rj = rank[j];
    const double sj = sig[j];
    VT[(int64_t)rj * ldvt + i] = (sj > 0.0) ? sgn[j] * A[(int64_t)j * n + i] / sj : 0.0;
    if (UR) UR[(int64_t)i * n + rj] = sgn[j] * V[(int64_t)j * n + i];
  }
  __syncthreads();
  if (tid == 0) {
    // tail sums from the smallest value upward
    tail[n] = 0.0;
    for (int k = n - 1; k >= 0; --k) tail[k] = tail[k + 1] + S[k] * S[k];
    const double total = tail[0];
    int64_t keep = n;
    if (!(residual > 0.0)) {
      keep = n;
    } else if (total == 0.0) {
      keep = 0;
    } else {
      for (int k = 1; k <= n; ++k)
        if (tail[k] <= residual * total) {
          keep = k;
          break;
        }
    }
    *nr = keep;
  }
}

// n = 1: sigma = |r|, u = v = sign
__global__ void k_svd_one(const double* R, double* S, double* VT, double* UR, double residual,
                          int64_t* nr, int* status) {
  const double r = R[0];
  S[0] = fabs(r);
  VT[0] = 1.0;
  UR[0] = (r < 0.0) ? -1.0 : 1.0;
  *nr = (residual > 0.0 && r == 0.0) ? 0 : 1;
  status[0] = isfinite(r) ? 1 : -2;
  status[1] = 0;
}

hipError_t launch_small_svd(const JacobiPlan& p, const double* R, int max_sweeps, void* ws,
                            double* S, double* VT, int64_t ldvt, double* UR, double residual,
                            int64_t* nr, int* status, hipStream_t st, bool coop) {
  if (p.n == 1) {
    hipLaunchKernelGGL(k_svd_one, dim3(1), dim3(1), 0, st, R, S, VT, UR, residual, nr, status);
    return hipGetLastError();
  }
  JacobiWs w = jacobi_ws(p, max_sweeps, ws);
  const int nflags = jacobi_nflags(p, max_sweeps);
  hipLaunchKernelGGL(k_jacobi_setup, dim3(64), dim3(256), 0, st, p.n, p.npad, R, w.A, w.V, w.bar,
                     w.flags, nflags, status, max_sweeps > 0 ? 0 : -1, (int64_t)0, (int64_t)0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (max_sweeps > 0 && p.block) {
    BJArgs b;
    b.n = p.n; b.npad = p.npad; b.G = p.G; b.ks = p.ks; b.max_sweeps = max_sweeps;
    b.tol = jacobi_tol(p); b.A = w.A;
    b.V = w.V; b.bar = w.bar; b.flags = w.flags; b.pairc = w.pairc; b.gp = w.gp;
    b.status = status;
    void* args[] = {&b};
    const void* fn = p.no_ur ? (const void*)k_bjacobi<false> : (const void*)k_bjacobi<true>;
    const dim3 grid((unsigned)(p.G * p.ks));
    e = coop ? hipLaunchCooperativeKernel(fn, grid, dim3(256), args, 0, st)
             : hipLaunchKernel(fn, grid, dim3(256), args, 0, st);
    if (e != hipSuccess) return e;
  } else if (max_sweeps > 0) {
    JacobiArgs a;
    a.n = p.n; a.npad = p.npad; a.w = p.w; a.G = p.G; a.xcd_stride = p.xcd_stride;
    a.max_sweeps = max_sweeps; a.uv = p.no_ur ? 0 : 1; a.tol = jacobi_tol(p); a.A = w.A;
    a.V = w.V; a.bar = w.bar;
    a.flags = w.flags;
    a.status = status;
    a.sWs = 0;
    void* args[] = {&a};
    const dim3 grid(p.G * p.xcd_stride), block(JT);
    const void* fn = nullptr;
    switch (p.lpp) {
      case 16: fn = (const void*)k_jacobi<16, 16>; break;
      case 32: fn = (const void*)k_jacobi<32, 16>; break;
      case 64: fn = (const void*)k_jacobi<64, 16>; break;
      default: return hipErrorInvalidValue;
    }
    if (coop && p.G > 1) {
      e = hipLaunchCooperativeKernel(fn, grid, block, args, 0, st);
    } else {
      // plain launch (one workgroup, or inside stream capture, where a
      // cooperative launch cannot be recorded).  The G workgroups (8 at
      // n = 256, each holding 128 KB of LDS) become
      // resident as earlier work drains, since nothing else they wait for
      // holds a CU; the batched call chains its Jacobi launches across lanes
      // whenever their grids could not all be resident together.  Should
      // co-residency fail anyway, the bounded-spin barrier sets the error
      // flag (PYLOM_EHIP from pylom_check) instead of hanging.
      e = hipLaunchKernel(fn, grid, block, args, 0, st);
    }
    if (e != hipSuccess) return e;
  }
  // without U_R (no_ur) the block Jacobi leaves V unrotated: nothing to write
  hipLaunchKernelGGL(k_svd_finalize, dim3(1), dim3(FT), 0, st, p.n, w.A, w.V, S, VT, ldvt,
                     p.no_ur ? nullptr : UR, residual, nr, (int64_t)0, (int64_t)0, (int64_t)0,
                     (int64_t)0, status);
  return hipGetLastError();
}

int jacobi_resident_per_cu(const JacobiPlan& p) {
  const void* fn = nullptr;
  if (p.block) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_bjacobi<true>, 256, 0) !=
            hipSuccess ||
        nb < 1) {
      (void)hipGetLastError();
      return 1;
    }
    return nb;
  }
  switch (p.lpp) {
    case 16: fn = (const void*)k_jacobi<16, 16>; break;
    case 32: fn = (const void*)k_jacobi<32, 16>; break;
    case 64: fn = (const void*)k_jacobi<64, 16>; break;
    default: return 1;
  }
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, JT, 0) != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    return 1;
  }
  return nb;
}

size_t jacobi_ws_stride(const JacobiPlan& p, int max_sweeps) {
  return (jacobi_ws_bytes(p, max_sweeps) + 255) & ~(size_t)255;
}

// Status of a batch: sweeps = the largest count, -1 if any problem did not
// converge; the barrier flag is the OR over problems.
__global__ void k_status_reduce(int64_t count, const int* __restrict__ st, int stride, int pairs,
                                int* out) {
  __shared__ int smax, sneg, stmo;
  if (threadIdx.x == 0) {
    smax = 0;
    sneg = 0;
    stmo = 0;
  }
  __syncthreads();
  for (int64_t k = threadIdx.x; k < count; k += blockDim.x) {
    for (int q = 0; q < pairs; ++q) {
      const int sw = st[k * stride + 2 * q];
      if (sw < 0) atomicMin(&sneg, sw);
      else atomicMax(&smax, sw);
      if (st[k * stride + 2 * q + 1]) atomicOr(&stmo, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = sneg ? sneg : smax;
    out[1] = stmo;
  }
}

hipError_t launch_small_svd_batched(const JacobiPlan& p, int64_t count, const double* R,
                                    int64_t sR, int max_sweeps, void* ws, double* S, int64_t sS,
                                    double* VT, int64_t ldvt, int64_t sVT, double* UR,
                                    int64_t sUR, double residual, int64_t* nr, int* status_each,
                                    int* status, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (p.G != 1 || p.n < 2 || count > 65535) return hipErrorInvalidValue;
  const int64_t wsb = (int64_t)jacobi_ws_stride(p, max_sweeps);
  JacobiWs w = jacobi_ws(p, max_sweeps, ws);
  const int nflags = max_sweeps + 1;
  hipLaunchKernelGGL(k_jacobi_setup, dim3(8, (unsigned)count), dim3(256), 0, st, p.n, p.npad, R,
                     w.A, w.V, w.bar, w.flags, nflags, status_each, max_sweeps > 0 ? 0 : -1, sR,
                     wsb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (max_sweeps > 0) {
    // one workgroup per problem: no device-wide barrier is involved, so a
    // plain launch is enough
    JacobiArgs a;
    a.n = p.n; a.npad = p.npad; a.w = p.w; a.G = 1; a.xcd_stride = 1;
    a.max_sweeps = max_sweeps; a.uv = p.no_ur ? 0 : 1; a.tol = jacobi_tol(p); a.A = w.A;
    a.V = w.V; a.bar = w.bar;
    a.flags = w.flags;
    a.status = status_each;
    a.sWs = wsb;
    const dim3 grid(1, (unsigned)count), block(JT);
    if ((p.n + p.lpp - 1) / p.lpp > 16) return hipErrorInvalidValue;
    switch (p.lpp) {
      case 16: hipLaunchKernelGGL((k_jacobi<16, 16>), grid, block, 0, st, a); break;
      case 32: hipLaunchKernelGGL((k_jacobi<32, 16>), grid, block, 0, st, a); break;
      case 64: hipLaunchKernelGGL((k_jacobi<64, 16>), grid, block, 0, st, a); break;
      default: return hipErrorInvalidValue;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_svd_finalize, dim3(1, (unsigned)count), dim3(FT), 0, st, p.n, w.A, w.V, S,
                     VT, ldvt, UR, residual, nr, wsb, sS, sVT, sUR, status_each);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_status_reduce, dim3(1), dim3(256), 0, st, count, status_each, 2, 1, status);
  return hipGetLastError();
}

hipError_t launch_status_reduce(int64_t count, const int* st_each, int stride, int pairs,
                                int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_status_reduce, dim3(1), dim3(256), 0, st, count, st_each, stride, pairs,
                     status);
  return hipGetLastError();
}

}  // namespace pylom
