// tsqr.hip -- the TSQR of Alg. 1 on one gfx950 GPU.
//
// One kernel, `k_stacked_qr`, does both the local QR of every row block (the
// leaves) and every combine of the binary reduction tree.  Both are the same
// operation: a Householder QR of a stacked matrix [R; C], where R is the
// n x n upper-triangular "state" and C a block of further rows.  A leaf starts
// with an empty state and streams its row block through LDS in chunks of s
// rows; a combine starts with R_j as the state and streams R_{j+h} (the
// partner's triangle, the lower half of the 2N x N buffer of Alg. 1) through
// the same path, skipping the panels left of each chunk where R_{j+h} is
// zero.  Each chunk is read from HBM once and its reflectors written once; the
// state stays in global memory (L2 / MALL resident) and only its 16 active
// rows per panel move.
//
// Inside a chunk the columns are processed in panels of 16: one wave factors
// the panel with wave64 shuffle reductions and builds its compact-WY T factor
// (H_1..H_16 = I - V T V^T), then all four waves apply Q_p^T to the trailing
// columns with FP64 (or FP32) MFMA 16x16x4.
//
// Reflector storage ("filling" rows): while the state of a leaf is not yet
// full (f < n rows filled), the head of the reflector of column k >= f is
// chunk row k - f (an ordinary Householder inside the chunk), and that row
// becomes state row k at the end of the chunk; once f = n every head is the
// state row k.  So the leaf's rows are consumed in order and Q_1i is an exact
// orthogonal factor of the leaf.
//
// `k_stacked_apply` walks the same chunks and panels backwards to form
// Q [W; 0] (Eq. svdqr3 for a leaf, the broadcast step of Alg. 1 for a tree
// node): the state tile X (n x 16) stays in LDS, the chunk rows Z accumulate
// the output.
#include "common.hpp"
#include "kernels.hpp"

namespace pylom {

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
static const size_t kQrLdsBudget = 156 * 1024;  // bytes usable by one workgroup

size_t qr_lds_bytes(const QrGeom& g, int esize) {
  size_t e = (size_t)g.s * g.ldc + (size_t)g.s * VPLD + (size_t)NB * TLD + 4 * (size_t)NB * YLD;
  return e * esize;
}

bool qr_geom(int n, int esize, QrGeom* g) {
  if (n < 1) return false;
  g->n = n;
  g->ldc = (n % 2 == 1) ? n : n + 1;
  g->npanels = (n + NB - 1) / NB;
  int best = 0;
  for (int s = 16; s <= 64; s += 16) {  // one chunk row per lane of the panel wave
    QrGeom t = *g;
    t.s = s;
    if (qr_lds_bytes(t, esize) <= kQrLdsBudget) best = s;
  }
  if (best == 0) return false;
  g->s = best;
  return true;
}

size_t apply_lds_bytes(const QrGeom& g, int esize) {
  // X (n x 17), Z (s x 17), Vp (s x 17), Tm (16 x 17), 4 partial Y + 4 own Y.
  size_t e = (size_t)g.n * 17 + 2 * (size_t)g.s * 17 + (size_t)NB * TLD + 8 * (size_t)NB * YLD;
  return e * esize;
}

// ---------------------------------------------------------------------------
// kernel arguments
// ---------------------------------------------------------------------------
template <typename T, typename TI>
struct QrArgs {
  int n, s, ldc, npanels;
  int mode;     // 0 = leaf, 1 = combine
  int store_q;  // write reflectors and T factors
  // leaf
  const TI* D;
  int64_t ldd, m, b, P;
  int remove_mean;
  double* mean_ws;
  T* V;
  T* Tleaf;
  int64_t nch_leaf;
  // combine
  int64_t h;
  T* Ttree;
  int64_t nch_tree;
  // both
  T* Rbuf;
};

// ---------------------------------------------------------------------------
// panel factorisation (one wave)
// ---------------------------------------------------------------------------
// Factors columns k0..k0+kw-1 of the stacked matrix.  Structured panel
// (!internal): the head of column k is state row k, held as the 16x16 diagonal
// block rd (lane jj keeps column jj), the tail is the whole chunk column.
// Internal panel (leaf filling): the head is chunk row h = k - f.
// On exit: C holds the reflector tails (and, for internal panels, the new R
// rows), Vp the exact reflectors (0 / 1 / tail), Tm the T factor, and the
// state's diagonal block is updated (structured).
template <typename T, int RPL>
__device__ __forceinline__ void factor_panel(T* __restrict__ C, int ldc, int s, T* __restrict__ Vp,
                             T* __restrict__ Tm, T* __restrict__ state, int n, int k0, int kw,
                             bool internal, int f, int lane) {
  T p[RPL][NB];
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int r = lane + 64 * i;
#pragma unroll
    for (int kk = 0; kk < NB; ++kk) p[i][kk] = (r < s && kk < kw) ? C[r * ldc + k0 + kk] : T(0);
  }
  T rd[NB];
#pragma unroll
  for (int kk = 0; kk < NB; ++kk)
    rd[kk] = (!internal && lane < kw && kk <= lane) ? state[(int64_t)(k0 + kk) * n + k0 + lane] : T(0);
  T tr[NB];
#pragma unroll
  for (int jj = 0; jj < NB; ++jj) tr[jj] = T(0);

#pragma unroll
  for (int kk = 0; kk < NB; ++kk) {
    if (kk < kw) {
      const int h = internal ? (k0 + kk - f) : -1;
      T alpha;
      if (!internal) {
        alpha = readlane(rd[kk], kk);
      } else {
        T hv = p[0][kk];
#pragma unroll
        for (int i = 1; i < RPL; ++i)
          if ((h >> 6) == i) hv = p[i][kk];
        alpha = readlane(hv, h & 63);
      }
      T x2 = T(0);
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int r = lane + 64 * i;
        if (!internal || r > h) x2 += p[i][kk] * p[i][kk];
      }
      const T sig = wave_sum(x2);
      T tau, beta, scal;
      if (sig == T(0)) {
        tau = T(0);
        beta = alpha;
        scal = T(0);
      } else {
        const T nrm = sqrt(alpha * alpha + sig);
        beta = (alpha >= T(0)) ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = T(1) / (alpha - beta);
      }
      T v[RPL];
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int r = lane + 64 * i;
        if (internal) {
          v[i] = (r < h) ? T(0) : ((r == h) ? T(1) : p[i][kk] * scal);
          if (r == h)
            p[i][kk] = beta;
          else if (r > h)
            p[i][kk] = v[i];
        } else {
          v[i] = p[i][kk] * scal;
          p[i][kk] = v[i];
        }
      }
      if (!internal && lane == kk) rd[kk] = beta;
      // partial products: Gram with earlier reflectors (T factor), and
      // v^T [head; column] for the remaining panel columns
      T part[NB];
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) {
        T acc = T(0);
        if (jj < kk) {
          const int hj = internal ? (k0 + jj - f) : -1;
#pragma unroll
          for (int i = 0; i < RPL; ++i) {
            const int r = lane + 64 * i;
            T vj = internal ? ((r < hj) ? T(0) : ((r == hj) ? T(1) : p[i][jj])) : p[i][jj];
            acc += vj * v[i];
          }
        } else if (jj > kk) {
#pragma unroll
          for (int i = 0; i < RPL; ++i) acc += v[i] * p[i][jj];
          if (!internal && lane == jj) acc += rd[kk];
        }
        part[jj] = acc;
      }
      T w[NB];
      wave_reduce16(part, w, lane);
      // T(0:kk, kk) = -tau T(0:kk, 0:kk) (V(:,0:kk)^T v_kk),  T(kk,kk) = tau
      T tcol = T(0);
#pragma unroll
      for (int l = 0; l < kk; ++l) tcol += tr[l] * w[l];
      if (lane < kk)
        tr[kk] = -tau * tcol;
      else if (lane == kk)
        tr[kk] = tau;
      // apply H_kk^T to the remaining panel columns
#pragma unroll
      for (int jj = kk + 1; jj < NB; ++jj) {
        const T tw = tau * w[jj];
#pragma unroll
        for (int i = 0; i < RPL; ++i) p[i][jj] -= tw * v[i];
        if (!internal && lane == jj) rd[kk] -= tw;
      }
    }
  }
  // write back: C (tails and R rows), exact reflectors, T, state diagonal block
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int r = lane + 64 * i;
    if (r < s) {
#pragma unroll
      for (int kk = 0; kk < NB; ++kk) {
        T vx = T(0);
        if (kk < kw) {
          C[r * ldc + k0 + kk] = p[i][kk];
          if (internal) {
            const int hk = k0 + kk - f;
            vx = (r < hk) ? T(0) : ((r == hk) ? T(1) : p[i][kk]);
          } else {
            vx = p[i][kk];
          }
        }
        Vp[r * VPLD + kk] = vx;
      }
    }
  }
  if (lane < NB) {
#pragma unroll
    for (int jj = 0; jj < NB; ++jj) Tm[lane * TLD + jj] = tr[jj];
  }
  if (!internal && lane < kw) {
#pragma unroll
    for (int kk = 0; kk < NB; ++kk)
      if (kk <= lane && kk < kw) state[(int64_t)(k0 + kk) * n + k0 + lane] = rd[kk];
  }
}

// ---------------------------------------------------------------------------
// trailing update: [head; C(:, trail)] <- Q_p^T [head; C(:, trail)]
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void trailing_update(T* __restrict__ C, int ldc, int s, const T* __restrict__ Vp,
                                const T* __restrict__ Tm, T* __restrict__ Yw, T* __restrict__ state,
                                int n, int k0, int kw, bool internal, int wave, int lane) {
  typedef typename Mfma<T>::v4 v4;
  const int cb = k0 + kw;
  const int ntiles = (n - cb + 15) / 16;
  const int i16 = lane & 15, g4 = lane >> 4;
  for (int t = wave; t < ntiles; t += 4) {
    const int col = cb + 16 * t + i16;
    const bool colok = col < n;
    v4 y = vzero4<T>();
    for (int kb = 0; kb < s / 4; ++kb) {
      const int r = 4 * kb + g4;
      const T av = Vp[r * VPLD + i16];
      const T bv = colok ? C[r * ldc + col] : T(0);
      y = Mfma<T>::op(av, bv, y);
    }
    T head[4] = {T(0), T(0), T(0), T(0)};
    if (!internal) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = Mfma<T>::drow(g4, q);
        if (colok && i < kw) head[q] = state[(int64_t)(k0 + i) * n + col];
        y[q] += head[q];
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) Yw[(Mfma<T>::drow(g4, q)) * YLD + i16] = y[q];
    wave_lds_sync();
    v4 z = vzero4<T>();
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const int k = 4 * kb + g4;
      z = Mfma<T>::op(Tm[k * TLD + i16], Yw[k * YLD + i16], z);  // (T^T Y)
    }
    if (!internal) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = Mfma<T>::drow(g4, q);
        if (colok && i < kw) state[(int64_t)(k0 + i) * n + col] = head[q] - z[q];
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q) Yw[(Mfma<T>::drow(g4, q)) * YLD + i16] = z[q];
    wave_lds_sync();
    for (int mt = 0; mt < s / 16; ++mt) {
      v4 u = vzero4<T>();
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const int k = 4 * kb + g4;
        u = Mfma<T>::op(Vp[(16 * mt + i16) * VPLD + k], Yw[k * YLD + i16], u);
      }
      if (colok) {
#pragma unroll
        for (int q = 0; q < 4; ++q) C[(16 * mt + Mfma<T>::drow(g4, q)) * ldc + col] -= u[q];
      }
    }
    wave_lds_sync();
  }
}

// ---------------------------------------------------------------------------
// chunk loads
// ---------------------------------------------------------------------------
template <typename T, typename TI>
__device__ __forceinline__ void load_chunk(T* __restrict__ C, int ldc, int s, int sc, int n,
                           const TI* __restrict__ src, int64_t ld_src, int remove_mean,
                           double* __restrict__ mean_out, int wave, int lane) {
  for (int i = wave; i < s; i += 4) {
    if (i >= sc) {
      for (int col = lane; col < n; col += 64) C[i * ldc + col] = T(0);
      continue;
    }
    const TI* row = src + (int64_t)i * ld_src;
    if (remove_mean) {
      double acc = 0.0;
      for (int col = lane; col < n; col += 64) acc += (double)row[col];
      acc = wave_sum(acc);
      const double mu = acc / (double)n;
      for (int col = lane; col < n; col += 64) C[i * ldc + col] = (T)((double)row[col] - mu);
      if (lane == 0 && mean_out) mean_out[i] = mu;
    } else {
      for (int col = lane; col < n; col += 64) C[i * ldc + col] = (T)row[col];
    }
  }
}

// ---------------------------------------------------------------------------
// the stacked QR kernel (leaf or combine)
// ---------------------------------------------------------------------------
template <typename T, typename TI, int RPL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_stacked_qr(QrArgs<T, TI> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = a.n, s = a.s, ldc = a.ldc, npan = a.npanels;
  T* C = reinterpret_cast<T*>(smem);
  T* Vp = C + (size_t)s * ldc;
  T* Tm = Vp + (size_t)s * VPLD;
  T* Yb = Tm + NB * TLD;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool leaf = (a.mode == 0);

  const TI* srcI = nullptr;
  const T* srcT = nullptr;
  int64_t ld_src, rows, row0 = 0;
  T* vout;
  T* state;
  T* tout;
  if (leaf) {
    const int64_t j = blockIdx.x;
    row0 = j * a.b;
    rows = (j == a.P - 1) ? (a.m - row0) : a.b;
    srcI = a.D + row0 * a.ldd;
    ld_src = a.ldd;
    vout = a.store_q ? a.V + row0 * n : nullptr;
    state = a.Rbuf + j * (int64_t)n * n;
    tout = a.store_q ? a.Tleaf + j * a.nch_leaf * npan * (NB * NB) : nullptr;
  } else {
    const int64_t j = (int64_t)blockIdx.x * 2 * a.h;
    const int64_t jb = j + a.h;
    srcT = a.Rbuf + jb * (int64_t)n * n;
    ld_src = n;
    rows = n;
    vout = a.store_q ? const_cast<T*>(srcT) : nullptr;
    state = a.Rbuf + j * (int64_t)n * n;
    tout = a.store_q ? a.Ttree + jb * a.nch_tree * npan * (NB * NB) : nullptr;
  }
  const int nch = (int)((rows + s - 1) / s);
  int f = leaf ? 0 : n;
  for (int c = 0; c < nch; ++c) {
    const int64_t r0 = (int64_t)c * s;
    const int sc = (int)((rows - r0) < s ? (rows - r0) : s);
    if (leaf)
      load_chunk<T, TI>(C, ldc, s, sc, n, srcI + r0 * ld_src, ld_src, a.remove_mean,
                        a.mean_ws ? a.mean_ws + row0 + r0 : nullptr, wave, lane);
    else
      load_chunk<T, T>(C, ldc, s, sc, n, srcT + r0 * ld_src, ld_src, 0, nullptr, wave, lane);
    __syncthreads();
    int p_lo, p_hi;
    if (leaf) {
      const int lim = (f + sc < n) ? f + sc : n;
      p_lo = 0;
      p_hi = (lim + NB - 1) / NB;
    } else {
      p_lo = (int)(r0 / NB);
      p_hi = npan;
    }
    for (int p = p_lo; p < p_hi; ++p) {
      const int k0 = p * NB;
      const int kw = (n - k0 < NB) ? n - k0 : NB;
      const bool internal = leaf && (k0 >= f);
      if (wave == 0) {
        factor_panel<T, RPL>(C, ldc, s, Vp, Tm, state, n, k0, kw, internal, f, lane);
        if (tout) {
          T* tp = tout + ((int64_t)c * npan + p) * (NB * NB);
          for (int e = lane; e < NB * NB; e += 64) tp[e] = Tm[(e / NB) * TLD + (e % NB)];
        }
      }
      __syncthreads();
      trailing_update<T>(C, ldc, s, Vp, Tm, Yb + wave * NB * YLD, state, n, k0, kw, internal,
                         wave, lane);
      __syncthreads();
    }
    if (leaf && f < n) {
      const int nf = (sc < n - f) ? sc : n - f;
      for (int idx = tid; idx < nf * n; idx += 256) {
        const int i = idx / n, col = idx - (idx / n) * n;
        state[(int64_t)(f + i) * n + col] = (col >= f + i) ? C[i * ldc + col] : T(0);
      }
    }
    if (vout) {
      for (int idx = tid; idx < sc * n; idx += 256) {
        const int i = idx / n, col = idx - (idx / n) * n;
        vout[(r0 + i) * n + col] = C[i * ldc + col];
      }
    }
    __syncthreads();
    if (leaf) f = (f + sc < n) ? f + sc : n;
  }
}

// ---------------------------------------------------------------------------
// apply kernel: Q [W; 0], walking chunks and panels backwards
// ---------------------------------------------------------------------------
template <typename T, typename TO>
struct ApplyArgs {
  int n, s, npanels, mode;  // mode 0 = leaf, 1 = combine
  const int64_t* nr;
  int64_t ncols;
  // leaf
  int64_t m, b, P;
  const T* V;
  const T* Tleaf;
  int64_t nch_leaf;
  TO* U;
  int64_t ldu;
  // combine
  int64_t h;
  const T* Rbuf;
  const T* Ttree;
  int64_t nch_tree;
  // state tiles
  T* W;
  int64_t ldw;
};

template <typename T, typename TO>
__global__ __launch_bounds__(256) void k_stacked_apply(ApplyArgs<T, TO> a) {
  typedef typename Mfma<T>::v4 v4;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = a.n, s = a.s, npan = a.npanels;
  const int64_t ncols = a.nr ? *a.nr : a.ncols;
  const int ntiles = (int)((a.ncols + 15) / 16);
  const int tile = blockIdx.x % ntiles;
  const int64_t prob = blockIdx.x / ntiles;
  if ((int64_t)tile * 16 >= ncols) return;
  const int c0 = tile * 16;
  const bool leaf = (a.mode == 0);

  T* X = reinterpret_cast<T*>(smem);  // n x 17
  T* Z = X + (size_t)n * 17;          // s x 17
  T* Vp = Z + (size_t)s * 17;         // s x 17
  T* Tm = Vp + (size_t)s * 17;        // 16 x 17
  T* Yp = Tm + NB * TLD;              // 4 x 16 x 17 partials
  T* Yo = Yp + 4 * NB * YLD;          // 4 x 16 x 17 per-wave Y
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, g4 = lane >> 4;
  T* Yw = Yo + wave * NB * YLD;

  int64_t rows, row0 = 0;
  const T* Vsrc;
  const T* Tsrc;
  T* Wx;  // state source
  int64_t nch;
  if (leaf) {
    row0 = prob * a.b;
    rows = (prob == a.P - 1) ? (a.m - row0) : a.b;
    Vsrc = a.V + row0 * n;
    Tsrc = a.Tleaf + prob * a.nch_leaf * npan * (NB * NB);
    Wx = a.W + prob * (int64_t)n * a.ldw;
  } else {
    const int64_t j = prob * 2 * a.h, jb = j + a.h;
    rows = n;
    Vsrc = a.Rbuf + jb * (int64_t)n * n;
    Tsrc = a.Ttree + jb * a.nch_tree * npan * (NB * NB);
    Wx = a.W + j * (int64_t)n * a.ldw;
    row0 = jb;  // destination node
  }
  nch = (rows + s - 1) / s;
  // state tile
  for (int idx = tid; idx < n * 16; idx += 256) {
    const int i = idx >> 4, cc = idx & 15;
    X[i * 17 + cc] = (c0 + cc < ncols) ? Wx[(int64_t)i * a.ldw + c0 + cc] : T(0);
  }
  __syncthreads();
  const int ntr = s / 16;
  for (int64_t c = nch - 1; c >= 0; --c) {
    const int64_t r0 = c * s;
    const int sc = (int)((rows - r0) < s ? (rows - r0) : s);
    const int f = leaf ? (int)((r0 < n) ? r0 : n) : n;
    const int nf = (leaf && f < n) ? ((sc < n - f) ? sc : n - f) : 0;
    for (int idx = tid; idx < s * 16; idx += 256) {
      const int r = idx >> 4, cc = idx & 15;
      Z[r * 17 + cc] = (r < nf) ? X[(f + r) * 17 + cc] : T(0);
    }
    int p_lo, p_hi;
    if (leaf) {
      const int lim = (f + sc < n) ? f + sc : n;
      p_lo = 0;
      p_hi = (lim + NB - 1) / NB;
    } else {
      p_lo = (int)(r0 / NB);
      p_hi = npan;
    }
    for (int p = p_hi - 1; p >= p_lo; --p) {
      const int k0 = p * NB;
      const int kw = (n - k0 < NB) ? n - k0 : NB;
      const bool internal = leaf && (k0 >= f);
      // stage exact reflectors and T
      for (int idx = tid; idx < s * NB; idx += 256) {
        const int r = idx >> 4, kk = idx & 15;
        T vx = T(0);
        if (r < sc && kk < kw) {
          const T raw = Vsrc[(r0 + r) * n + k0 + kk];
          if (internal) {
            const int hk = k0 + kk - f;
            vx = (r < hk) ? T(0) : ((r == hk) ? T(1) : raw);
          } else {
            vx = raw;
          }
        }
        Vp[r * 17 + kk] = vx;
      }
      {
        const T* tp = Tsrc + (c * npan + p) * (NB * NB);
        const int e = tid;  // 256 = 16 x 16
        Tm[(e >> 4) * TLD + (e & 15)] = tp[e];
      }
      __syncthreads();
      // partial Y = V^T Z over this wave's row tiles
      v4 y = vzero4<T>();
      for (int mt = wave; mt < ntr; mt += 4) {
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
          const int r = 16 * mt + 4 * kb + g4;
          y = Mfma<T>::op(Vp[r * 17 + i16], Z[r * 17 + i16], y);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) Yp[wave * NB * YLD + (Mfma<T>::drow(g4, q)) * YLD + i16] = y[q];
      __syncthreads();
      // full Y (every wave, redundantly), then T Y
      T yf[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = Mfma<T>::drow(g4, q);
        T acc = Yp[i * YLD + i16] + Yp[NB * YLD + i * YLD + i16] + Yp[2 * NB * YLD + i * YLD + i16] +
                Yp[3 * NB * YLD + i * YLD + i16];
        if (!internal && i < kw) acc += X[(k0 + i) * 17 + i16];
        yf[q] = acc;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) Yw[(Mfma<T>::drow(g4, q)) * YLD + i16] = yf[q];
      wave_lds_sync();
      v4 ty = vzero4<T>();
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const int k = 4 * kb + g4;
        ty = Mfma<T>::op(Tm[i16 * TLD + k], Yw[k * YLD + i16], ty);  // (T Y)
      }
      wave_lds_sync();
#pragma unroll
      for (int q = 0; q < 4; ++q) Yw[(Mfma<T>::drow(g4, q)) * YLD + i16] = ty[q];
      wave_lds_sync();
      for (int mt = wave; mt < ntr; mt += 4) {
        v4 u = vzero4<T>();
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
          const int k = 4 * kb + g4;
          u = Mfma<T>::op(Vp[(16 * mt + i16) * 17 + k], Yw[k * YLD + i16], u);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Z[(16 * mt + Mfma<T>::drow(g4, q)) * 17 + i16] -= u[q];
      }
      __syncthreads();
      // every wave has read the head rows of X for this panel: update them now
      if (!internal && wave == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = Mfma<T>::drow(g4, q);
          if (i < kw) X[(k0 + i) * 17 + i16] -= ty[q];
        }
      }
    }
    __syncthreads();
    // chunk rows are final
    if (leaf) {
      for (int idx = tid; idx < sc * 16; idx += 256) {
        const int r = idx >> 4, cc = idx & 15;
        if (c0 + cc < ncols) a.U[(row0 + r0 + r) * a.ldu + c0 + cc] = (TO)Z[r * 17 + cc];
      }
    } else {
      T* Wd = a.W + row0 * (int64_t)n * a.ldw;
      for (int idx = tid; idx < sc * 16; idx += 256) {
        const int r = idx >> 4, cc = idx & 15;
        if (c0 + cc < ncols) Wd[(r0 + r) * a.ldw + c0 + cc] = Z[r * 17 + cc];
      }
    }
    __syncthreads();
  }
  if (!leaf) {
    for (int idx = tid; idx < n * 16; idx += 256) {
      const int i = idx >> 4, cc = idx & 15;
      if (c0 + cc < ncols) Wx[(int64_t)i * a.ldw + c0 + cc] = X[i * 17 + cc];
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, typename TI, int RPL>
static hipError_t launch_qr_t(const QrArgs<T, TI>& a, int grid, size_t lds, hipStream_t st) {
  hipError_t e = hipFuncSetAttribute((const void*)k_stacked_qr<T, TI, RPL>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_stacked_qr<T, TI, RPL>), dim3(grid), dim3(256), lds, st, a);
  return hipGetLastError();
}

template <typename T, typename TI>
static hipError_t launch_qr_any(const QrArgs<T, TI>& a, int grid, size_t lds, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  if (a.s > 64) return hipErrorInvalidValue;
  return launch_qr_t<T, TI, 1>(a, grid, lds, st);
}

hipError_t launch_leaf_qr_f64(const QrGeom& g, const void* D, int in_f64, int64_t ldd, int64_t m,
                              int64_t b, int64_t P, int remove_mean, double* mean_ws, double* V,
                              double* Tleaf, int64_t nch_leaf, double* Rbuf, hipStream_t st) {
  const size_t lds = qr_lds_bytes(g, 8);
  if (in_f64) {
    QrArgs<double, double> a{};
    a.n = g.n; a.s = g.s; a.ldc = g.ldc; a.npanels = g.npanels; a.mode = 0;
    a.store_q = V != nullptr;
    a.D = (const double*)D; a.ldd = ldd; a.m = m; a.b = b; a.P = P;
    a.remove_mean = remove_mean; a.mean_ws = mean_ws; a.V = V; a.Tleaf = Tleaf;
    a.nch_leaf = nch_leaf; a.Rbuf = Rbuf;
    return launch_qr_any(a, (int)P, lds, st);
  }
  QrArgs<double, float> a{};
  a.n = g.n; a.s = g.s; a.ldc = g.ldc; a.npanels = g.npanels; a.mode = 0;
  a.store_q = V != nullptr;
  a.D = (const float*)D; a.ldd = ldd; a.m = m; a.b = b; a.P = P;
  a.remove_mean = remove_mean; a.mean_ws = mean_ws; a.V = V; a.Tleaf = Tleaf;
  a.nch_leaf = nch_leaf; a.Rbuf = Rbuf;
  return launch_qr_any(a, (int)P, lds, st);
}

hipError_t launch_leaf_qr_f32(const QrGeom& g, const float* D, int64_t ldd, int64_t m, int64_t b,
                              int64_t P, int remove_mean, double* mean_ws, float* Rbuf32,
                              hipStream_t st) {
  QrArgs<float, float> a{};
  a.n = g.n; a.s = g.s; a.ldc = g.ldc; a.npanels = g.npanels; a.mode = 0; a.store_q = 0;
  a.D = D; a.ldd = ldd; a.m = m; a.b = b; a.P = P;
  a.remove_mean = remove_mean; a.mean_ws = mean_ws; a.Rbuf = Rbuf32;
  return launch_qr_any(a, (int)P, qr_lds_bytes(g, 4), st);
}

hipError_t launch_tree_combine_f64(const QrGeom& g, int64_t h, int64_t P, double* Rbuf,
                                   double* Ttree, int64_t nch_tree, int store_q, hipStream_t st) {
  QrArgs<double, double> a{};
  a.n = g.n; a.s = g.s; a.ldc = g.ldc; a.npanels = g.npanels; a.mode = 1;
  a.store_q = store_q; a.h = h; a.Ttree = Ttree; a.nch_tree = nch_tree; a.Rbuf = Rbuf;
  // combines at this level: j = 0, 2h, 4h, ... with j + h < P
  const int64_t ncomb = (P - h + 2 * h - 1) / (2 * h);
  return launch_qr_any(a, (int)ncomb, qr_lds_bytes(g, 8), st);
}

template <typename TO>
static hipError_t launch_apply_t(const ApplyArgs<double, TO>& a, int grid, size_t lds,
                                 hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)k_stacked_apply<double, TO>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_stacked_apply<double, TO>), dim3(grid), dim3(256), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_apply_leaf_f64(const QrGeom& g, int64_t m, int64_t b, int64_t P,
                                 const double* V, const double* Tleaf, int64_t nch_leaf,
                                 const double* W, int64_t ldw, const int64_t* nr, int64_t ncols,
                                 void* U, int out_f64, int64_t ldu, hipStream_t st) {
  const int ntiles = (int)((ncols + 15) / 16);
  const size_t lds = apply_lds_bytes(g, 8);
  if (out_f64) {
    ApplyArgs<double, double> a{};
    a.n = g.n; a.s = g.s; a.npanels = g.npanels; a.mode = 0; a.nr = nr; a.ncols = ncols;
    a.m = m; a.b = b; a.P = P; a.V = V; a.Tleaf = Tleaf; a.nch_leaf = nch_leaf;
    a.U = (double*)U; a.ldu = ldu; a.W = const_cast<double*>(W); a.ldw = ldw;
    return launch_apply_t(a, (int)(P * ntiles), lds, st);
  }
  ApplyArgs<double, float> a{};
  a.n = g.n; a.s = g.s; a.npanels = g.npanels; a.mode = 0; a.nr = nr; a.ncols = ncols;
  a.m = m; a.b = b; a.P = P; a.V = V; a.Tleaf = Tleaf; a.nch_leaf = nch_leaf;
  a.U = (float*)U; a.ldu = ldu; a.W = const_cast<double*>(W); a.ldw = ldw;
  return launch_apply_t(a, (int)(P * ntiles), lds, st);
}

hipError_t launch_apply_tree_f64(const QrGeom& g, int64_t h, int64_t P, const double* Rbuf,
                                 const double* Ttree, int64_t nch_tree, double* W, int64_t ldw,
                                 const int64_t* nr, int64_t ncols, hipStream_t st) {
  const int ntiles = (int)((ncols + 15) / 16);
  const int64_t ncomb = (P - h + 2 * h - 1) / (2 * h);
  ApplyArgs<double, double> a{};
  a.n = g.n; a.s = g.s; a.npanels = g.npanels; a.mode = 1; a.nr = nr; a.ncols = ncols;
  a.h = h; a.Rbuf = Rbuf; a.Ttree = Ttree; a.nch_tree = nch_tree; a.W = W; a.ldw = ldw;
  return launch_apply_t(a, (int)(ncomb * ntiles), apply_lds_bytes(g, 8), st);
}

}  // namespace pylom
