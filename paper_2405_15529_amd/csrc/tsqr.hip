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
#include <type_traits>
#include "common.hpp"
#include "kernels.hpp"

namespace pylom {

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
static const size_t kQrLdsBudget = 160 * 1024;  // bytes of LDS per workgroup (gfx950)

// LDS of the QR kernel: chunk C (s x ldc), two reflector panels Vp (s x 17),
// two T factors (16 x 16), four 16 x 16 Y tiles (the panel wave's also holds
// its Gram matrix), the diagonal block Rd (16 x 17), the broadcast column vb
// (64) and the 16 tau.
size_t qr_lds_bytes(const QrGeom& g, int esize) {
  size_t e = (size_t)g.s * g.ldc + 2 * (size_t)g.s * VPLD + 2 * (size_t)NB * NB +
             4 * (size_t)NB * NB + (size_t)NB * TLD + 64 + 16;
  return e * esize;
}

bool qr_geom(int n, int esize, QrGeom* g) {
  if (n < 1) return false;
  g->n = n;
  g->ldc = n;  // column-per-lane panel access and MFMA operand walks are row-contiguous
  g->npanels = (n + NB - 1) / NB;
  g->nthr = 0;
  int best = 0;
  for (int s = 16; s <= 64; s += 16) {
    QrGeom t = *g;
    t.s = s;
    if (qr_lds_bytes(t, esize) <= kQrLdsBudget) best = s;
  }
  if (best == 0) return false;
  g->s = best;
  return true;
}

size_t apply_lds_bytes(const QrGeom& g, int esize) {
  // X (n x 17), Z (s x 17), Vp (s x 17), Tm (16 x 17), 4 partial Y (each
  // wave keeps the full Y and T Y in registers).
  size_t e = (size_t)g.n * 17 + 2 * (size_t)g.s * 17 + (size_t)NB * TLD + 4 * (size_t)NB * YLD;
  return e * esize;
}

// ---------------------------------------------------------------------------
// kernel arguments
// ---------------------------------------------------------------------------
// Thresholds below which a Householder column is renormalised with an exact
// power-of-two scale before its norm is formed (x2: squared tail norm; root:
// |head|; max_exp: the largest scale exponent that is representable).
template <typename T>
struct Tiny;
template <>
struct Tiny<double> {
  static constexpr double x2 = 0x1p-960, root = 0x1p-480;
  static constexpr int max_exp = 1022;  // largest representable scale 2^k
};
template <>
struct Tiny<float> {
  static constexpr float x2 = 0x1p-100f, root = 0x1p-50f;
  static constexpr int max_exp = 126;
};

template <typename T, typename TI>
struct QrArgs {
  int n, s, ldc, npanels;
  int nthr;     // workgroup threads (0: 64 for at most two panels, else 256)
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
  // batch strides (elements), problem = blockIdx.y
  int64_t bsD, bsMean, bsV, bsTleaf, bsR, bsTtree;
  // column-blocked use (a panel of a wider matrix): state_mode 1 starts the
  // leaf state at zero, 2 takes it as given in Rbuf; either way every chunk
  // is a structured [state; chunk] step (no filling rows).  Reflectors are
  // written with row stride ldv (0: n); at most rows_lim rows of each leaf
  // take part (0: all)
  int state_mode;
  int64_t ldv, rows_lim;
};

// ---------------------------------------------------------------------------
// panel factorisation (one wave)
// ---------------------------------------------------------------------------
// Factors columns k0..k0+kw-1 of the stacked matrix.  Structured panel
// (!INTERNAL): the head of column k is state row k (the 16x16 diagonal block,
// staged in LDS as Rd), the tail is the whole chunk column.  Internal panel
// (INTERNAL, leaf filling): the head is chunk row h = k - f.
//
// Layout: lane l = 16 g + j holds column j of the panel for the chunk rows
// r = g + 4 t (t < RT = s/4), so a column norm or a column dot product is an
// in-lane sum plus two row-pair swaps.  The reflector of the current column
// is broadcast through LDS (vb).  One fused pass gives both v_k^T [head;
// column j] for j > k (the update coefficients) and the Gram entries
// v_j^T v_k for j < k (from which the compact-WY T factor is built).
//
// On exit: C holds the reflector tails (and, for internal panels, the new R
// rows), Vp the exact reflectors (0 / 1 / tail), Tm the T factor, and the
// state's diagonal block is written back (structured).
template <typename T, int RT, bool INTERNAL>
__device__ __forceinline__ void factor_panel(T* __restrict__ C, int ldc, T* __restrict__ Vp,
                                             T* __restrict__ Tm, T* __restrict__ state, int n,
                                             int k0, int kw, int f, int lane,
                                             const T (&rd4)[4], T* __restrict__ Rd,
                                             T* __restrict__ Gm, T* __restrict__ vb,
                                             T* __restrict__ taus) {
  const int j = lane & 15, g = lane >> 4;
  T p[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) p[t] = (j < kw) ? C[(g + 4 * t) * ldc + k0 + j] : T(0);
  if (!INTERNAL) {
#pragma unroll
    for (int u = 0; u < 4; ++u) Rd[(g * 4 + u) * TLD + j] = rd4[u];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) Gm[(g * 4 + u) * NB + j] = T(0);
  wave_lds_sync();
#pragma unroll 1
  for (int kk = 0; kk < kw; ++kk) {
    const int h = INTERNAL ? (k0 + kk - f) : -1;
    T alpha;
    if (!INTERNAL) {
      alpha = Rd[kk * TLD + kk];
    } else {
      T x = T(0);
#pragma unroll
      for (int t = 0; t < RT; ++t)
        if (t == (h >> 2)) x = p[t];
      alpha = readlane(x, ((h & 3) << 4) + kk);
    }
    // squared norm of the tail of column kk (four independent partial sums:
    // the in-lane part of the column chain)
    T x2;
    {
      T xq[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int r = g + 4 * t;
        if (!INTERNAL || r > h) xq[t & 3] += p[t] * p[t];
      }
      x2 = (xq[0] + xq[1]) + (xq[2] + xq[3]);
    }
    x2 = perm32_pairsum(perm16_pairsum(x2));
    T sig = readlane(x2, kk);
    T tau, beta, scal;
    T sc = T(1);  // power-of-two rescaling of a tiny column (exact)
    if (sig < Tiny<T>::x2 && fabs(alpha) < Tiny<T>::root) {
      // both the head and the tail are tiny (rank-deficient input leaves
      // columns of rounding noise that shrink geometrically): squares in
      // the subnormal range keep few significant bits and tau would no
      // longer match v, so the column is scaled by the power of two that
      // brings max(|alpha|, |x|) into [0.5, 1) before its norm is formed
      // (as LAPACK's reflector generator does).  Wave-uniform branch: sig
      // and alpha are broadcast values.
      T amax = T(0);
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int r = g + 4 * t;
        if (!INTERNAL || r > h) amax = fmax(amax, fabs(p[t]));
      }
      amax = perm32_pairmax(perm16_pairmax(amax));
      amax = fmax(readlane(amax, kk), fabs(alpha));
      if (amax > T(0)) {
        int e;
        frexp(amax, &e);  // amax = f 2^e, f in [0.5, 1)
        sc = ldexp(T(1), (-e < Tiny<T>::max_exp) ? -e : Tiny<T>::max_exp);
      }
      T xs2 = T(0);
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int r = g + 4 * t;
        const T xs = p[t] * sc;
        if (!INTERNAL || r > h) xs2 += xs * xs;
      }
      xs2 = perm32_pairsum(perm16_pairsum(xs2));
      sig = readlane(xs2, kk);
    }
    if (sig == T(0)) {
      tau = T(0);
      beta = alpha;
      scal = T(0);
    } else {
      // scaled head as and norm nrm >= max(|as|, |x sc|): v = (x sc) / (as - bs)
      // has entries of magnitude <= 1, whatever the scale
      const T as = alpha * sc;
      const T nrm = sqrt(as * as + sig);
      const T bs = (as >= T(0)) ? -nrm : nrm;
      tau = (bs - as) / bs;
      scal = T(1) / (as - bs);
      beta = bs / sc;
    }
    // reflector of column kk: exact values to vb, stored values back into p
    if (j == kk) {
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int r = g + 4 * t;
        T vx;
        if (INTERNAL) {
          vx = (r < h) ? T(0) : ((r == h) ? T(1) : (p[t] * sc) * scal);
          p[t] = (r == h) ? beta : ((r > h) ? vx : p[t]);
        } else {
          vx = (p[t] * sc) * scal;
          p[t] = vx;
        }
        vb[g * RT + t] = vx;
      }
      if (g == 0) taus[kk] = tau;
    }
    if (!INTERNAL && lane == 0) Rd[kk * TLD + kk] = beta;
    wave_lds_sync();
    T v[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) v[t] = vb[g * RT + t];
    // fused pass: j > kk -> v^T [head; column j];  j < kk -> v_j^T v
    const int hj = INTERNAL ? (k0 + j - f) : -1;
    T d;
    {
      T dq[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int r = g + 4 * t;
        T cj = p[t];
        if (INTERNAL && j < kk) cj = (r < hj) ? T(0) : ((r == hj) ? T(1) : p[t]);
        dq[t & 3] += cj * v[t];
      }
      d = (dq[0] + dq[1]) + (dq[2] + dq[3]);
    }
    if (!INTERNAL && j > kk && g == 0) d += Rd[kk * TLD + j];
    d = perm32_pairsum(perm16_pairsum(d));
    if (j < kk && g == 0) Gm[kk * NB + j] = d;
    if (j > kk) {
      const T tw = tau * d;
#pragma unroll
      for (int t = 0; t < RT; ++t) p[t] -= tw * v[t];
      if (!INTERNAL && g == 0) Rd[kk * TLD + j] -= tw;
    }
    wave_lds_sync();
  }
  // compact-WY T by recursive doubling: with T = diag(tau) for blocks of
  // size 1, each level joins adjacent diagonal blocks A, B of size bs,
  //   T(A,B) = -T(A,A) G(A,B) T(B,B)      (G = V^T V, Gm holds G^T),
  // which is T_new = M - M Gb M with M the current block-diagonal T and Gb
  // the G entries of the (A,B) blocks: two 16x16 MFMA products per level.
  {
    typedef typename Mfma<T>::v4 v4;
    const int i16 = lane & 15, g4 = lane >> 4;
    T* Pb = Rd;  // the diagonal block is back in registers' callers: reuse as scratch
    // Rd still holds the diagonal block of R; write it back first
    if (!INTERNAL) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = g * 4 + u;
        if (kk <= j && j < kw) state[(int64_t)(k0 + kk) * n + k0 + j] = Rd[kk * TLD + j];
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = Mfma<T>::drow(g4, q);
      Tm[r * NB + i16] = (r == i16 && r < kw) ? taus[r] : T(0);
    }
    wave_lds_sync();
#pragma unroll
    for (int bs = 1; bs < NB; bs *= 2) {
      // P = M Gb
      v4 acc = vzero4<T>();
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const int k = 4 * kb + g4;
        const bool msk = (k / (2 * bs) == i16 / (2 * bs)) && (k % (2 * bs) < bs) &&
                         (i16 % (2 * bs) >= bs);
        const T gb = msk ? Gm[i16 * NB + k] : T(0);
        acc = Mfma<T>::op(Tm[i16 * NB + k], gb, acc);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) Pb[Mfma<T>::drow(g4, q) * TLD + i16] = acc[q];
      wave_lds_sync();
      // T -= P M
      v4 acc2 = vzero4<T>();
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const int k = 4 * kb + g4;
        acc2 = Mfma<T>::op(Pb[i16 * TLD + k], Tm[k * NB + i16], acc2);
      }
      wave_lds_sync();
#pragma unroll
      for (int q = 0; q < 4; ++q) Tm[Mfma<T>::drow(g4, q) * NB + i16] -= acc2[q];
      wave_lds_sync();
    }
  }
  // write back: C (tails and R rows), exact reflectors, state diagonal block
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int r = g + 4 * t;
    T vx = T(0);
    if (j < kw) {
      C[r * ldc + k0 + j] = p[t];
      if (INTERNAL) {
        const int hk = k0 + j - f;
        vx = (r < hk) ? T(0) : ((r == hk) ? T(1) : p[t]);
      } else {
        vx = p[t];
      }
    }
    Vp[r * VPLD + j] = vx;
  }
  wave_lds_sync();
}

// Diagonal block of the state for the panel starting at k0: lane 16 g + j
// holds rows 4 g .. 4 g + 3 of column j (upper triangle only).
template <typename T>
__device__ __forceinline__ void load_diag4(T (&rd)[4], const T* __restrict__ state, int n, int k0,
                                           int lane) {
  const int j = lane & 15, g = lane >> 4;
  const int kw = (n - k0 < NB) ? n - k0 : NB;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int kk = g * 4 + u;
    rd[u] = (j < kw && kk <= j) ? state[(int64_t)(k0 + kk) * n + k0 + j] : T(0);
  }
}

// Head values (state rows k0..k0+15, the 16 columns from col0) in MFMA D
// layout.
template <typename T>
__device__ __forceinline__ void load_head4(T (&hd)[4], const T* __restrict__ state, int n, int k0,
                                           int kw, int col0, int lane) {
  const int i16 = lane & 15, g4 = lane >> 4;
  const int col = col0 + i16;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = Mfma<T>::drow(g4, q);
    hd[q] = (col < n && i < kw) ? state[(int64_t)(k0 + i) * n + col] : T(0);
  }
}

// ---------------------------------------------------------------------------
// one trailing tile: [head; C(:, col0:col0+16)] <- Q_p^T [head; C(...)]
// ---------------------------------------------------------------------------
// HEADREG: the head rows stay in registers (head is updated in place and
// the state is not touched).
template <typename T, int RT, bool HEADREG = false>
__device__ __forceinline__ void tile_update(T* __restrict__ C, int ldc, const T* __restrict__ Vp,
                                            const T* __restrict__ Tm, T* __restrict__ Yw,
                                            T* __restrict__ state, int n, int k0, int kw,
                                            bool internal, int col0, T (&head)[4], int lane) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int S = 4 * RT;  // chunk rows
  const int i16 = lane & 15, g4 = lane >> 4;
  const int col = col0 + i16;
  const bool colok = col < n;
  // Y = V^T C(:, tile): operands batched, two independent accumulators
  v4 y0 = vzero4<T>(), y1 = vzero4<T>();
#pragma unroll
  for (int kb0 = 0; kb0 < S / 4; kb0 += 4) {
    T av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = 4 * (kb0 + u) + g4;
      av[u] = Vp[r * VPLD + i16];
      bv[u] = colok ? C[r * ldc + col] : T(0);
    }
    y0 = Mfma<T>::op(av[0], bv[0], y0);
    y1 = Mfma<T>::op(av[1], bv[1], y1);
    y0 = Mfma<T>::op(av[2], bv[2], y0);
    y1 = Mfma<T>::op(av[3], bv[3], y1);
  }
  T y[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) y[q] = y0[q] + y1[q] + (internal ? T(0) : head[q]);
  // In the FP64 16x16x4 layout, accumulator q of lane (i16, g4) holds row
  // 4q + g4, column i16: exactly the B operand that lane supplies at step
  // kb = q, so Y and T^T Y feed the next products from registers.  The FP32
  // layout (rows 4 g4 + q) goes through the wave's LDS tile instead.
  constexpr bool REG = sizeof(T) == 8;
  if (!REG) {
#pragma unroll
    for (int q = 0; q < 4; ++q) Yw[(Mfma<T>::drow(g4, q)) * NB + i16] = y[q];
    wave_lds_sync();
  }
  v4 z = vzero4<T>();
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    const int k = 4 * kb + g4;
    z = Mfma<T>::op(Tm[k * NB + i16], REG ? y[kb] : Yw[k * NB + i16], z);  // (T^T Y)
  }
  if (HEADREG) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = Mfma<T>::drow(g4, q);
      head[q] = (colok && i < kw) ? head[q] - z[q] : head[q];
    }
  } else if (!internal) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = Mfma<T>::drow(g4, q);
      if (colok && i < kw) state[(int64_t)(k0 + i) * n + col] = head[q] - z[q];
    }
  }
  // C(:, tile) -= V Z: the S/16 row tiles are independent accumulations
  T zb[4];
  if (REG) {
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) zb[kb] = z[kb];
  } else {
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q) Yw[(Mfma<T>::drow(g4, q)) * NB + i16] = z[q];
    wave_lds_sync();
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) zb[kb] = Yw[(4 * kb + g4) * NB + i16];
  }
  v4 u[S / 16];
  T a[S / 16][4];
#pragma unroll
  for (int m = 0; m < S / 16; ++m)
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) a[m][kb] = Vp[(16 * m + i16) * VPLD + 4 * kb + g4];
#pragma unroll
  for (int m = 0; m < S / 16; ++m) u[m] = vzero4<T>();
#pragma unroll
  for (int kb = 0; kb < 4; ++kb)
#pragma unroll
    for (int m = 0; m < S / 16; ++m) u[m] = Mfma<T>::op(a[m][kb], zb[kb], u[m]);
  if (colok) {
#pragma unroll
    for (int m = 0; m < S / 16; ++m)
#pragma unroll
      for (int q = 0; q < 4; ++q) C[(16 * m + Mfma<T>::drow(g4, q)) * ldc + col] -= u[m][q];
  }
  wave_lds_sync();
}

// ---------------------------------------------------------------------------
// Structured panel (the head of column k0+kk is state row k0+kk, the tail is
// all s chunk rows), written for a short per-column critical path:
//  - every lane keeps its column's raw values and the scale that turns them
//    into the reflector, so the register tile is never rewritten per column,
//    and the update weight is simply zero for columns at or left of kk;
//  - the head rows come from the prefetched diagonal block in registers (the
//    lane that holds an entry adds it to its partial sum) and the new R rows
//    and tau stay there until the state is written back;
//  - 1/sqrt and 1/x use the hardware estimates refined by Newton steps (one
//    in FP32, two in FP64), and the power-of-two rescale is undone by a
//    multiplication with its exact inverse;
//  - column kk is final when its step starts, so it is broadcast raw through
//    an LDS vector (laid out without bank conflicts) before anything else,
//    and the raw products x_kk^T x_j are formed beside its norm; the
//    reflector scale 1/(alpha - beta) is wave-uniform and is applied once to
//    each product and once to each update weight, so only the Householder
//    scalars lie between the two reductions and the update;
//  - the Gram values v_i^T v_k (i < k) of the same pass are kept in LDS, and
//    the compact-WY factor is formed once after the loop as
//    T = (diag(1/tau) + striu(V^T V))^{-1}, the triangular inverse that the
//    column recurrence T(:c, c) = -tau_c T(:c, :c) V(:, :c)^T v_c also
//    computes: lane c back-substitutes column c.
__device__ __forceinline__ double hw_rcp(double x) { return __builtin_amdgcn_rcp(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double hw_rsq(double x) { return __builtin_amdgcn_rsq(x); }
__device__ __forceinline__ float hw_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
// Newton steps: the FP32 estimates are within about one ulp (one step
// reaches rounding level); the FP64 ones carry about 23 bits (two steps).
template <typename T>
__device__ __forceinline__ T rcp_nr(T x) {
  T r = hw_rcp(x);
  r = r * (T(2) - x * r);
  if constexpr (sizeof(T) == 8) r = r * (T(2) - x * r);
  return r;
}
template <typename T>
__device__ __forceinline__ T rsq_nr(T x) {
  T y = hw_rsq(x);
  y = y * (T(1.5) - T(0.5) * x * y * y);
  if constexpr (sizeof(T) == 8) y = y * (T(1.5) - T(0.5) * x * y * y);
  return y;
}

// Core of the structured panel factorisation: p holds the tail rows g + 4t
// of column j (lane 16 g + j) and rfin the head rows 4g .. 4g+3 (the
// diagonal block of the state); on exit p, mysc and myscal give the
// reflector tails v_j = (p mysc) myscal, rfin the R rows and Tm the T factor.
template <typename T, int RT>
__device__ __forceinline__ void factor_core(T (&p)[RT], T& mysc, T& myscal, T (&rfin)[4],
                                            T* __restrict__ Tm, int kw, int lane,
                                            T* __restrict__ Gm, T* __restrict__ vb) {
  const int j = lane & 15, g = lane >> 4;
  mysc = T(1);
  myscal = T(0);
  T mytau = T(0);  // tau_j, on the lanes of column j
  const T rd0[4] = {rfin[0], rfin[1], rfin[2], rfin[3]};  // head rows at entry
  // Gram scratch S(i, k) = v_i^T v_k at Gm[i NB + k] for i < k < kw; every
  // other entry stays zero
#pragma unroll
  for (int u = 0; u < 4; ++u) Gm[lane * 4 + u] = T(0);
#pragma unroll 1
  for (int kb = 0; kb < kw; kb += 4) {
    const bool owner = g == (kb >> 2);  // this lane holds head row kk (kb <= kk < kb + 4)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = kb + u;
      if (kk >= kw) break;
      const T rsel = rd0[u];  // head row kk, column j, on the owner lanes
      // column kk is final: broadcast it first, so that the LDS round trip
      // overlaps the norm
      if (j == kk) {
#pragma unroll
        for (int t = 0; t < RT; ++t) vb[t * 4 + g] = p[t];
      }
      wave_lds_sync();
      T w[RT];  // x_kk, and x_kk sc after a rescale: the reflector's tail is w scal
#pragma unroll
      for (int t = 0; t < RT; ++t) w[t] = vb[t * 4 + g];
      const T alpha = readlane(rsel, 4 * kb + kk);
      // squared norm of column kk's tail (all s chunk rows) and, independent
      // of it, the raw products x_kk^T x_j and head row kk of column j
      T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
#pragma unroll
      for (int t = 0; t < RT; t += 4) {
        a0 += p[t] * p[t];
        if (t + 1 < RT) a1 += p[t + 1] * p[t + 1];
        if (t + 2 < RT) a2 += p[t + 2] * p[t + 2];
        if (t + 3 < RT) a3 += p[t + 3] * p[t + 3];
      }
      T d0 = T(0), d1 = T(0), d2 = T(0), d3 = T(0);
#pragma unroll
      for (int t = 0; t < RT; t += 4) {
        d0 += p[t] * w[t];
        if (t + 1 < RT) d1 += p[t + 1] * w[t + 1];
        if (t + 2 < RT) d2 += p[t + 2] * w[t + 2];
        if (t + 3 < RT) d3 += p[t + 3] * w[t + 3];
      }
      T x2 = perm32_pairsum(perm16_pairsum((a0 + a1) + (a2 + a3)));
      T dw = perm32_pairsum(perm16_pairsum((d0 + d1) + (d2 + d3)));
      const T hd = perm32_pairsum(perm16_pairsum((owner && j > kk) ? rsel : T(0)));
      T sig = readlane(x2, kk);
      T sc = T(1), isc = T(1);
      if (__builtin_expect(sig < Tiny<T>::x2 && fabs(alpha) < Tiny<T>::root, 0)) {
        // tiny head and tail (rank-deficient input): rescale by the power of
        // two that brings max(|alpha|, |x|) into [0.5, 1) before forming the
        // norm, so that no square falls into the subnormal range, and form
        // the products again from the rescaled column
        T amax = T(0);
#pragma unroll
        for (int t = 0; t < RT; ++t) amax = fmax(amax, fabs(p[t]));
        amax = perm32_pairmax(perm16_pairmax(amax));
        amax = fmax(readlane(amax, kk), fabs(alpha));
        if (amax > T(0)) {
          int e;
          frexp(amax, &e);
          const int k = (-e < Tiny<T>::max_exp) ? -e : Tiny<T>::max_exp;
          sc = ldexp(T(1), k);
          isc = ldexp(T(1), -k);
        }
        T xs2 = T(0), dd = T(0);
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          const T xs = p[t] * sc;
          xs2 += xs * xs;
          w[t] *= sc;
          dd += p[t] * w[t];
        }
        xs2 = perm32_pairsum(perm16_pairsum(xs2));
        dw = perm32_pairsum(perm16_pairsum(dd));
        sig = readlane(xs2, kk);
      }
      // a = as^2 + sig is a normal number unless sig = 0 (>= 2^-960, or
      // >= 1/4 after a rescale): y = 1/sqrt(a), |beta_s| = a y, 1/beta_s =
      // -+y, tau = (bs - as)/bs = 1 - as/bs, scal = 1/(as - bs); sig = 0
      // gives the identity (tau = 0, beta = alpha)
      const bool ident = sig == T(0);
      const T as = alpha * sc;
      const T a = ident ? T(1) : as * as + sig;
      const T y = rsq_nr(a);
      const T nrm = a * y;
      const bool pos = as >= T(0);
      const T bs = pos ? -nrm : nrm;
      const T ibs = pos ? -y : y;
      const T tau = ident ? T(0) : T(1) - as * ibs;
      const T scal = ident ? T(0) : rcp_nr(as - bs);
      const T beta = ident ? alpha : bs * isc;
      mysc = (j == kk) ? sc : mysc;
      myscal = (j == kk) ? scal : myscal;
      mytau = (j == kk) ? tau : mytau;
      // d_j = v_kk^T [head; x_j]: v^T [head row kk; column j] for j > kk, and
      // x_j^T v_kk for j < kk (x_j = the raw column, v_j = x_j mysc myscal)
      const T d = scal * dw + hd;
      if (j < kk && g == 0) Gm[j * NB + kk] = (d * mysc) * myscal;
      const T tw = (j > kk) ? tau * d : T(0);
      const T tws = tw * scal;
#pragma unroll
      for (int t = 0; t < RT; ++t) p[t] -= tws * w[t];
      // R row kk: beta on the diagonal, the updated head entries right of it
      rfin[u] = owner ? ((j == kk) ? beta : ((j > kk) ? rsel - tw : rfin[u])) : rfin[u];
      wave_lds_sync();
    }
  }
  // T = (diag(1/tau) + striu(V^T V))^{-1}, column c = j by back substitution
  // from the bottom row: T(c, c) = tau_c, T(i, c) = -tau_i sum_{k > i}
  // S(i, k) T(k, c); rows and columns at or beyond kw are zero (S is zero
  // there, so no stale value enters a sum)
  {
    T tv[NB];
#pragma unroll
    for (int i = NB - 1; i >= 0; --i) {
      T sacc = T(0);
#pragma unroll
      for (int k = NB - 1; k > i; --k) sacc += Gm[i * NB + k] * tv[k];
      const T ti = readlane(mytau, i);
      tv[i] = (i >= kw) ? T(0) : ((i == j) ? ti : ((i < j) ? -ti * sacc : T(0)));
    }
    // lane 16 g + j writes rows 4g .. 4g+3 of column j
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T val = (g == 0) ? tv[u] : (g == 1) ? tv[4 + u] : (g == 2) ? tv[8 + u] : tv[12 + u];
      Tm[(4 * g + u) * NB + j] = val;
    }
  }
}

// Structured panel of the stacked QR: columns k0 .. k0+kw-1 of the chunk C
// under the state's diagonal block (prefetched in rd4).  On exit C and Vp
// hold the exact reflectors, Tm the T factor, and the state its new rows.
template <typename T, int RT>
__device__ __forceinline__ void factor_panel_structured(
    T* __restrict__ C, int ldc, T* __restrict__ Vp, T* __restrict__ Tm, T* __restrict__ state,
    int n, int k0, int kw, int lane, const T (&rd4)[4], T* __restrict__ Gm,
    T* __restrict__ vb) {
  const int j = lane & 15, g = lane >> 4;
  T p[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) p[t] = (j < kw) ? C[(g + 4 * t) * ldc + k0 + j] : T(0);
  T mysc, myscal;
  T rfin[4] = {rd4[0], rd4[1], rd4[2], rd4[3]};
  factor_core<T, RT>(p, mysc, myscal, rfin, Tm, kw, lane, Gm, vb);
  // the state diagonal block (R rows of this panel), then C and the exact
  // reflectors (structured: the chunk rows of column j hold v_j)
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int kk = g * 4 + u;
    if (kk <= j && j < kw) state[(int64_t)(k0 + kk) * n + k0 + j] = rfin[u];
  }
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int r = g + 4 * t;
    const T vx = (p[t] * mysc) * myscal;
    if (j < kw) C[r * ldc + k0 + j] = vx;
    Vp[r * VPLD + j] = (j < kw) ? vx : T(0);
  }
  wave_lds_sync();
}

// ---------------------------------------------------------------------------
// chunk loads, with optional row-mean removal (Alg. 2)
template <int LB, int NCOL, typename T, typename TI>
__device__ __forceinline__ void load_rows(T* __restrict__ C, int ldc, int s, int sc, int n,
                                          const TI* __restrict__ src, int64_t ld_src,
                                          int remove_mean, double* __restrict__ mean_out,
                                          int wave, int lane, int nw) {
  for (int i0 = wave; i0 < s; i0 += nw * LB) {
    TI x[LB][NCOL];
#pragma unroll
    for (int b = 0; b < LB; ++b) {
      const int i = i0 + nw * b;
#pragma unroll
      for (int c = 0; c < NCOL; ++c) {
        const int col = lane + 64 * c;
        x[b][c] = (i < sc && col < n) ? src[(int64_t)i * ld_src + col] : TI(0);
      }
    }
#pragma unroll
    for (int b = 0; b < LB; ++b) {
      const int i = i0 + nw * b;
      if (i >= s) continue;
      double mu = 0.0;
      if (remove_mean && i < sc) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < NCOL; ++c) acc += (double)x[b][c];
        acc = wave_sum_fast(acc);
        mu = acc / (double)n;
        if (lane == 0 && mean_out) mean_out[i] = mu;
      }
#pragma unroll
      for (int c = 0; c < NCOL; ++c) {
        const int col = lane + 64 * c;
        if (col < n) C[i * ldc + col] = (i < sc) ? (T)((double)x[b][c] - mu) : T(0);
      }
    }
  }
}

// Rows i = wave, wave + nw, ... of the chunk (nw waves); each batch issues
// all its loads before any is consumed: 16 rows per wave for rows of at most
// 64 values (a 64-row chunk of four waves in one round trip), 4 rows of up
// to 256 values otherwise.
template <typename T, typename TI>
__device__ __forceinline__ void load_chunk(T* __restrict__ C, int ldc, int s, int sc, int n,
                                           const TI* __restrict__ src, int64_t ld_src,
                                           int remove_mean, double* __restrict__ mean_out,
                                           int wave, int lane, int nw) {
  if (n <= 64) {
    load_rows<16, 1, T, TI>(C, ldc, s, sc, n, src, ld_src, remove_mean, mean_out, wave, lane, nw);
    return;
  }
  if (n <= 256) {
    load_rows<4, 4, T, TI>(C, ldc, s, sc, n, src, ld_src, remove_mean, mean_out, wave, lane, nw);
    return;
  }
  for (int i = wave; i < s; i += nw) {
    if (i >= sc) {
      for (int col = lane; col < n; col += 64) C[i * ldc + col] = T(0);
      continue;
    }
    const TI* row = src + (int64_t)i * ld_src;
    if (remove_mean) {
      double acc = 0.0;
      for (int col = lane; col < n; col += 64) acc += (double)row[col];
      acc = wave_sum_fast(acc);
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
// Per chunk the panels are pipelined: in step p, wave 0 first applies panel
// p-1 to the 16 columns of panel p (look-ahead) and then factors panel p,
// while waves 1..3 apply panel p-1 to the remaining trailing columns.  The
// reflectors and T of consecutive panels alternate between two LDS buffers.
// Small-chunk prefetch of the stacked QR (variant 3): the loads of the next
// chunk are in flight while the current one is factored, instead of a chain
// of dependent load rounds at the start of every chunk (a single-wave
// workgroup needs 16 of them for 64 rows).  Element e = tid + t nthr of the
// chunk (row e / n, column e % n) goes to register t; rows past the leaf are
// zero.
constexpr int kPfn = 32;
template <typename TI, int N>
__device__ __forceinline__ void chunk_prefetch(TI (&pfv)[N], const TI* __restrict__ src,
                                               int64_t ld_src, int c, int64_t rows, int S, int n,
                                               int tid, int nthr) {
  const int64_t r0 = (int64_t)c * S;
  const int lim = (int)(((rows - r0) < S ? (rows - r0) : S) * n);
  int j = tid - (tid / n) * n;
  const int di = nthr / n, dj = nthr - (nthr / n) * n;
  // one walking pointer: consecutive elements of a thread are nthr apart
  const TI* ptr = src + (r0 + tid / n) * ld_src + j;
  const int64_t step = (int64_t)di * ld_src + dj, wrap = ld_src - n;
#pragma unroll
  for (int t = 0; t < N; ++t) {
    pfv[t] = (tid + t * nthr < lim) ? *ptr : TI(0);
    ptr += step;
    j += dj;
    if (j >= n) {
      j -= n;
      ptr += wrap;
    }
  }
}
template <typename T, typename TI, int N>
__device__ __forceinline__ void chunk_commit(const TI (&pfv)[N], T* __restrict__ C, int ldc, int S,
                                             int n, int tid, int nthr) {
  int i = tid / n, j = tid - (tid / n) * n;
  const int di = nthr / n, dj = nthr - (nthr / n) * n;
#pragma unroll
  for (int t = 0; t < N; ++t) {
    if (tid + t * nthr < S * n) C[i * ldc + j] = (T)pfv[t];
    j += dj;
    i += di;
    if (j >= n) {
      j -= n;
      ++i;
    }
  }
}

// Variants: VAR 0 fills the leaf state from the first chunks (stacked
// leaves); VAR 3 does the same and prefetches small chunks (see pf below);
// VAR 1, 2 and 4 compile the filling path out (tree combines and
// column-blocked panels never fill).  VAR 2 is register-limited to two waves
// per SIMD, so that two workgroups share a CU, and the wave that factors the
// panels rotates with the workgroup index, so that the panel waves of
// co-resident workgroups sit on different SIMDs.  VAR 4 is VAR 2 for grids
// of at most one workgroup per CU: with one wave per SIMD it keeps its
// overflow registers in AGPRs instead of scratch memory.
// One leaf (a.mode 0, leaf bx) or one combine (a.mode 1, pair bx at level
// a.h) of problem by, by the whole workgroup; smem is the dynamic LDS.
template <typename T, typename TI, int RT, int VAR>
__device__ __forceinline__ void stacked_qr_task(QrArgs<T, TI> a, int64_t bx, int64_t by,
                                                unsigned char* smem) {
  constexpr bool FILL = VAR == 0 || VAR == 3;
  constexpr bool PF = VAR == 3;
  if (by) {
    const int64_t pb = by;
    if (a.D) a.D += pb * a.bsD;
    if (a.mean_ws) a.mean_ws += pb * a.bsMean;
    if (a.V) a.V += pb * a.bsV;
    if (a.Tleaf) a.Tleaf += pb * a.bsTleaf;
    if (a.Ttree) a.Ttree += pb * a.bsTtree;
    a.Rbuf += pb * a.bsR;
  }
  constexpr int S = 4 * RT;
  const int n = a.n, ldc = a.ldc, npan = a.npanels;
  T* C = reinterpret_cast<T*>(smem);
  T* Vp0 = C + (size_t)S * ldc;
  T* Tm0 = Vp0 + 2 * (size_t)S * VPLD;
  T* Yb = Tm0 + 2 * NB * NB;
  T* Rd = Yb + 4 * NB * NB;
  T* vb = Rd + NB * TLD;
  T* taus = vb + 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = (int)(blockDim.x >> 6);  // 4, or 1 for narrow problems
  // panel wave pw; wr = 0 for it, 1..3 for the trailing-tile waves
  const int pw = ((VAR == 2 || VAR == 4) && nw == 4) ? (int)(((bx >> 3) + (bx >> 8)) & 3) : 0;
  const int wr = (wave - pw) & 3;
  T* Gm = Yb + pw * NB * NB;  // the panel wave's Y tile doubles as its Gram scratch
  const bool leaf = (a.mode == 0);
  const int64_t ldv = (leaf && a.ldv > 0) ? a.ldv : n;
  T* Yw = Yb + wave * NB * NB;

  const TI* srcI = nullptr;
  const T* srcT = nullptr;
  int64_t ld_src, rows, row0 = 0;
  T* vout;
  T* state;
  T* tout;
  if (leaf) {
    const int64_t jl = bx;
    row0 = jl * a.b;
    rows = (jl == a.P - 1) ? (a.m - row0) : a.b;
    if (a.rows_lim > 0 && rows > a.rows_lim) rows = a.rows_lim;
    srcI = a.D + row0 * a.ldd;
    ld_src = a.ldd;
    vout = a.store_q ? a.V + row0 * ldv : nullptr;
    state = a.Rbuf + jl * (int64_t)n * n;
    tout = a.store_q ? a.Tleaf + jl * a.nch_leaf * npan * (NB * NB) : nullptr;
  } else {
    const int64_t jn = bx * 2 * a.h;
    const int64_t jb = jn + a.h;
    srcT = a.Rbuf + jb * (int64_t)n * n;
    ld_src = n;
    rows = n;
    vout = a.store_q ? const_cast<T*>(srcT) : nullptr;
    state = a.Rbuf + jn * (int64_t)n * n;
    tout = a.store_q ? a.Ttree + jb * a.nch_tree * npan * (NB * NB) : nullptr;
  }
  const int nch = (int)((rows + S - 1) / S);
  int f = (FILL && leaf && a.state_mode == 0) ? 0 : n;
  if (leaf && a.state_mode == 1) {
    for (int idx = tid; idx < n * n; idx += (int)blockDim.x) state[idx] = T(0);
    __syncthreads();
  }
  // VAR 3 (leaves without mean removal whose chunk is at most kPfn values
  // per thread) prefetches the next chunk into registers (chunk_prefetch).
  // (only leaves read srcI: a work-queue launch runs combines in the same
  // variant)
  TI pfv[PF ? kPfn : 1];
  if constexpr (PF) {
    if (leaf) chunk_prefetch<TI, kPfn>(pfv, srcI, ld_src, 0, rows, S, n, tid, (int)blockDim.x);
  }
  for (int c = 0; c < nch; ++c) {
    const int64_t r0 = (int64_t)c * S;
    const int sc = (int)((rows - r0) < S ? (rows - r0) : S);
    bool staged = false;
    if constexpr (PF) {
      if (leaf) {
        chunk_commit<T, TI, kPfn>(pfv, C, ldc, S, n, tid, (int)blockDim.x);
        if (c + 1 < nch)
          chunk_prefetch<TI, kPfn>(pfv, srcI, ld_src, c + 1, rows, S, n, tid, (int)blockDim.x);
        staged = true;
      }
    }
    if (!staged) {
      if (leaf)
        load_chunk<T, TI>(C, ldc, S, sc, n, srcI + r0 * ld_src, ld_src, a.remove_mean,
                          a.mean_ws ? a.mean_ws + row0 + r0 : nullptr, wave, lane, nw);
      else
        load_chunk<T, T>(C, ldc, S, sc, n, srcT + r0 * ld_src, ld_src, 0, nullptr, wave, lane, nw);
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
    // panel wave prefetches: diagonal block of the first panel
    T rd4[4] = {T(0), T(0), T(0), T(0)};
    T hd4[4] = {T(0), T(0), T(0), T(0)};
    if (wr == 0 && !(FILL && leaf && p_lo * NB >= f)) load_diag4<T>(rd4, state, n, p_lo * NB, lane);
    __syncthreads();
    for (int p = p_lo; p <= p_hi; ++p) {
      const int kp = (p - 1) * NB;  // previous panel (its reflectors are applied now)
      const int kwp = (n - kp < NB) ? n - kp : NB;
      const bool int_prev = FILL && leaf && (kp >= f);
      T* Vprev = Vp0 + ((p - 1) & 1) * S * VPLD;
      T* Tprev = Tm0 + ((p - 1) & 1) * NB * NB;
      if (wr == 0) {
        if (p > p_lo && p < npan)
          tile_update<T, RT>(C, ldc, Vprev, Tprev, Yw, state, n, kp, kwp, int_prev, p * NB, hd4,
                             lane);
        if (p < p_hi) {
          const int k0 = p * NB;
          const int kw = (n - k0 < NB) ? n - k0 : NB;
          const bool internal = FILL && leaf && (k0 >= f);
          T* Vcur = Vp0 + (p & 1) * S * VPLD;
          T* Tcur = Tm0 + (p & 1) * NB * NB;
          // prefetch for the next step: head values of this panel's rows over the
          // next panel's columns, and the next panel's diagonal block
          T rd_next[4] = {T(0), T(0), T(0), T(0)};
          if (!internal && p + 1 < npan) load_head4<T>(hd4, state, n, k0, kw, (p + 1) * NB, lane);
          if (p + 1 < p_hi && !(FILL && leaf && (p + 1) * NB >= f))
            load_diag4<T>(rd_next, state, n, (p + 1) * NB, lane);
          if (internal)
            factor_panel<T, RT, true>(C, ldc, Vcur, Tcur, state, n, k0, kw, f, lane, rd4, Rd, Gm,
                                      vb, taus);
          else
            factor_panel_structured<T, RT>(C, ldc, Vcur, Tcur, state, n, k0, kw, lane, rd4, Gm,
                                           vb);
          if (tout) {
            T* tp = tout + ((int64_t)c * npan + p) * (NB * NB);
#pragma unroll
            for (int e = 0; e < 4; ++e) tp[lane + 64 * e] = Tcur[lane + 64 * e];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) rd4[u] = rd_next[u];
        }
        if (nw == 1 && p > p_lo) {
          // single-wave workgroup (narrow problems, several leaves per CU):
          // this wave also applies panel p-1 to the remaining tiles
          for (int t = p + 1; t < npan; ++t) {
            T hd[4] = {T(0), T(0), T(0), T(0)};
            if (!int_prev) load_head4<T>(hd, state, n, kp, kwp, t * NB, lane);
            tile_update<T, RT>(C, ldc, Vprev, Tprev, Yw, state, n, kp, kwp, int_prev, t * NB, hd,
                               lane);
          }
        }
      } else if (p > p_lo) {
        for (int t = p + wr; t < npan; t += 3) {
          T hd[4] = {T(0), T(0), T(0), T(0)};
          if (!int_prev) load_head4<T>(hd, state, n, kp, kwp, t * NB, lane);
          tile_update<T, RT>(C, ldc, Vprev, Tprev, Yw, state, n, kp, kwp, int_prev, t * NB, hd,
                             lane);
        }
      }
      __syncthreads();
    }
    if (FILL && leaf && f < n) {
      const int nf = (sc < n - f) ? sc : n - f;
      for (int idx = tid; idx < nf * n; idx += (int)blockDim.x) {
        const int i = idx / n, col = idx - (idx / n) * n;
        state[(int64_t)(f + i) * n + col] = (col >= f + i) ? C[i * ldc + col] : T(0);
      }
    }
    if (vout) {
      for (int idx = tid; idx < sc * n; idx += (int)blockDim.x) {
        const int i = idx / n, col = idx - (idx / n) * n;
        vout[(r0 + i) * ldv + col] = C[i * ldc + col];
      }
    }
    __syncthreads();
    if (FILL && leaf) f = (f + sc < n) ? f + sc : n;
  }
}

template <typename T, typename TI, int RT, int VAR>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(VAR == 2 ? 2 : 1, VAR == 2 ? 2 : 1)))
void k_stacked_qr(QrArgs<T, TI> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  stacked_qr_task<T, TI, RT, VAR>(a, blockIdx.x, blockIdx.y, smem);
}

// ---------------------------------------------------------------------------
// wavefront panel QR (column-blocked panels of 2 to 4 sub-panels)
// ---------------------------------------------------------------------------
// Sub-panel p of chunk c needs the reflectors of sub-panels 0 .. p-1 of the
// same chunk (they update its columns) and sub-panel p of chunk c-1 (the
// head rows of the state that chunk left), nothing else.  Wave w owns the 16-column stripe w of every
// chunk and, at step tau, works on chunk tau - w: it applies the reflectors
// of panels 0 .. w-1 of that chunk, read back from the tails and T factors
// their waves stored in global memory at earlier steps, and factors its own
// panel.  The factorisations of the panels thus run concurrently on the
// four waves, and a step is bounded by wave 3 (three tile updates and one
// panel) instead of the four panels in sequence.
// LDS: stripe w keeps w + 1 chunk slots (the chunks committed to it but not
// yet factored), 64 x 17 each; per wave a staging tile for the V and T
// read back, and its panel scratch.  The head rows of the state stay in the
// owning wave's registers for the whole leaf.  The next chunk is prefetched
// into registers one step ahead and committed after the step's barrier.
// Outputs are those of the stacked QR's column-blocked mode: reflector
// tails in place of the chunk rows, one T factor per 64-row chunk and
// sub-panel, and the panel's state rows.
constexpr int kWfS = 64;  // chunk rows (the trailing update applies per 64-row chunk)

template <typename T>
__device__ __forceinline__ T* wf_stripe(T* lds, int s, int64_t c) {
  // stripe s owns slots s(s+1)/2 .. s(s+1)/2 + s
  return lds + (size_t)((s * (s + 1)) / 2 + (int)(c % (s + 1))) * (kWfS * VPLD);
}

static size_t wf_lds_bytes(int esize) {
  return (size_t)(10 * kWfS * VPLD + 4 * (kWfS * VPLD + 3 * NB * NB + kWfS)) * esize;
}

// Prefetched chunk (element e = tid + 256 t: row e / n, column e % n) into
// the stripe slots of chunk c.
template <typename T, int N>
__device__ __forceinline__ void wf_commit(const T (&pfv)[N], T* lds, int64_t c, int n, int tid) {
  int i = tid / n, col = tid - (tid / n) * n;
  const int di = 256 / n, dj = 256 - (256 / n) * n;
#pragma unroll
  for (int t = 0; t < N; ++t) {
    if (tid + t * 256 < kWfS * n) wf_stripe(lds, col >> 4, c)[i * VPLD + (col & 15)] = pfv[t];
    col += dj;
    i += di;
    if (col >= n) {
      col -= n;
      ++i;
    }
  }
}

template <typename T, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void k_panel_wf(QrArgs<T, T> a) {
  constexpr int S = kWfS, RT = S / 4, SL = S * VPLD, PF = S * 64 / 256;
  extern __shared__ __align__(16) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int n = a.n, npan = a.npanels;
  const int64_t jl = blockIdx.x;
  const int64_t row0 = jl * a.b;
  int64_t rows = (jl == a.P - 1) ? (a.m - row0) : a.b;
  if (a.rows_lim > 0 && rows > a.rows_lim) rows = a.rows_lim;
  const T* src = a.D + row0 * a.ldd;
  const int64_t ldv = a.ldv > 0 ? a.ldv : n;
  T* vout = a.V + row0 * ldv;
  T* state = a.Rbuf + jl * (int64_t)n * n;
  T* tout = a.Tleaf + jl * a.nch_leaf * npan * (NB * NB);
  const int nch = (int)((rows + S - 1) / S);
  T* Vst = lds + 10 * SL + (size_t)w * (SL + 3 * NB * NB + S);
  T* Tst = Vst + SL;
  T* Gm = Tst + NB * NB;
  T* Yw = Gm + NB * NB;
  T* vb = Yw + NB * NB;
  const bool act = w < npan;
  const int k0 = NB * w;
  const int kw = act ? ((n - k0 < NB) ? n - k0 : NB) : 0;
  T rd4[4] = {T(0), T(0), T(0), T(0)};  // diagonal block of stripe w (factor layout)
  T hd[3][4];                           // head rows of panels 0 .. w-1 in stripe w (MFMA layout)
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) hd[p][q] = T(0);
  if (a.state_mode == 1) {
    for (int idx = tid; idx < n * n; idx += 256) state[idx] = T(0);
  } else if (act) {
    load_diag4<T>(rd4, state, n, k0, lane);
#pragma unroll
    for (int p = 0; p < 3; ++p)
      if (p < w) load_head4<T>(hd[p], state, n, NB * p, NB, k0, lane);
  }
  T pf[PF];
  chunk_prefetch<T, PF>(pf, src, a.ldd, 0, rows, S, n, tid, 256);
  wf_commit<T, PF>(pf, lds, 0, n, tid);
  if (nch > 1) chunk_prefetch<T, PF>(pf, src, a.ldd, 1, rows, S, n, tid, 256);
  __syncthreads();
  const int nsteps = nch + npan - 1;
  for (int tau = 0; tau < nsteps; ++tau) {
    const int c = tau - w;
    if (act && c >= 0 && c < nch) {
      const int64_t r0 = (int64_t)c * S;
      const int sc = (int)((rows - r0) < S ? (rows - r0) : S);
      T* st = wf_stripe(lds, w, c);
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        if (p < w) {
          // V and T of panel p of this chunk (stored by wave p at step c + p):
          // every load is issued before the first is stored to LDS
          const T* vs = vout + r0 * ldv + NB * p;
          const T* ts = tout + ((int64_t)c * npan + p) * (NB * NB);
          T vv[S * NB / 64], tt[4];
#pragma unroll
          for (int e = 0; e < S * NB / 64; ++e) {
            const int idx = lane + 64 * e, r = idx >> 4;
            vv[e] = (r < sc) ? vs[r * ldv + (idx & 15)] : T(0);
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) tt[e] = ts[lane + 64 * e];
#pragma unroll
          for (int e = 0; e < S * NB / 64; ++e) {
            const int idx = lane + 64 * e;
            Vst[(idx >> 4) * VPLD + (idx & 15)] = vv[e];
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) Tst[lane + 64 * e] = tt[e];
          wave_lds_sync();
          tile_update<T, RT, true>(st, VPLD, Vst, Tst, Yw, nullptr, n - k0, 0, NB, false, 0,
                                   hd[p], lane);
        }
      }
      T pv[RT];
#pragma unroll
      for (int t = 0; t < RT; ++t) pv[t] = (j < kw) ? st[(g + 4 * t) * VPLD + j] : T(0);
      T mysc, myscal;
      factor_core<T, RT>(pv, mysc, myscal, rd4, Tst, kw, lane, Gm, vb);
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int r = g + 4 * t;
        if (j < kw && r < sc) vout[(r0 + r) * ldv + k0 + j] = (pv[t] * mysc) * myscal;
      }
      wave_lds_sync();
      T* tp = tout + ((int64_t)c * npan + w) * (NB * NB);
#pragma unroll
      for (int e = 0; e < 4; ++e) tp[lane + 64 * e] = Tst[lane + 64 * e];
    }
    __syncthreads();
    if (tau + 1 < nch) {
      wf_commit<T, PF>(pf, lds, tau + 1, n, tid);
      if (tau + 2 < nch) chunk_prefetch<T, PF>(pf, src, a.ldd, tau + 2, rows, S, n, tid, 256);
    }
    __syncthreads();
  }
  if (act) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = 4 * g + u;
      if (kk <= j && j < kw) state[(int64_t)(k0 + kk) * n + k0 + j] = rd4[u];
    }
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      if (p < w) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = Mfma<T>::drow(g, q);
          if (k0 + j < n) state[(int64_t)(NB * p + i) * n + k0 + j] = hd[p][q];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// work-queue form: every leaf and every combine of a batch in one launch
// ---------------------------------------------------------------------------
// Tasks are numbered level by level (level 0: the leaves of every problem,
// level l >= 1: the combines at h = 2^(l-1)), and each workgroup takes the
// next number from a device counter until none is left.  A combine waits
// until both of its nodes are complete through the levels below it: node j
// counts one completion for its leaf and one for each combine into it, so
// before level h it needs 1 + #{h' < h : j + h' < P}.  Every task depends
// only on tasks with smaller numbers, which workgroups already hold, so the
// queue always drains; the waits are bounded all the same (about 2^22 polls:
// a timeout sets err, which ends every later wait, and the task proceeds).
__device__ __forceinline__ unsigned int qr_need(int64_t j, int64_t h, int64_t P) {
  unsigned int need = 1;
  for (int64_t hp = 1; hp < h; hp *= 2)
    if (j + hp < P) ++need;
  return need;
}

// The poll is a relaxed device-scope load (it reads the coherent copy
// without invalidating this XCD's L2, which an acquire load does on every
// iteration and which would starve the producers the waiter depends on); the
// acquire fence follows once, after the count is reached.
__device__ __forceinline__ void queue_wait(const unsigned int* c, unsigned int need, int* err) {
  unsigned long long spins = 0;
  while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
    __builtin_amdgcn_s_sleep(8);
    if ((++spins & 255ull) == 0 &&
        (spins > (1ull << 22) || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
      atomicExch(err, 1);
      break;
    }
  }
}

// Next task number for the whole workgroup (slot: one LDS word).
__device__ __forceinline__ int64_t queue_next(unsigned long long* next, int64_t* slot) {
  if (threadIdx.x == 0) *slot = (int64_t)atomicAdd(next, 1ull);
  __syncthreads();
  const int64_t t = *slot;
  __syncthreads();
  return t;
}

template <typename T, typename TI, int RT, int VAR>
__global__ __launch_bounds__(256) void k_qr_queue(QrArgs<T, TI> a, QrQueue q) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int64_t slot;
  for (;;) {
    const int64_t t = queue_next(q.next, &slot);
    if (t >= q.lvl_off[q.nlev + 1]) break;
    int l = 0;
    while (t >= q.lvl_off[l + 1]) ++l;
    const int64_t i = t - q.lvl_off[l];
    const int64_t h = l ? ((int64_t)1 << (l - 1)) : 0;
    const int64_t per = l ? (q.P - h + 2 * h - 1) / (2 * h) : q.P;
    const int64_t prob = i / per, idx = i - prob * per;
    unsigned int* cnt = q.cnt + prob * q.P;
    int64_t node = idx;
    if (l) {
      node = 2 * h * idx;
      if (threadIdx.x == 0) {
        queue_wait(cnt + node, qr_need(node, h, q.P), q.err);
        queue_wait(cnt + node + h, qr_need(node + h, h, q.P), q.err);
        __threadfence();
      }
      __syncthreads();
    }
    QrArgs<T, TI> b = a;
    b.mode = l ? 1 : 0;
    b.h = h;
    stacked_qr_task<T, TI, RT, VAR>(b, idx, prob, smem);
    // the workgroup barrier completes every thread's stores to this XCD's
    // L2; the release by thread 0 writes them back device-wide before the
    // count
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      __hip_atomic_fetch_add(cnt + node, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
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
  // batch strides (elements), problem = blockIdx.y
  int64_t bsV, bsTleaf, bsR, bsTtree, bsW, bsU;
};

// Column tile `tile` (16 columns of W) of leaf or pair `prob` (a.mode 0 / 1)
// of problem by, by the whole workgroup.
template <typename T, typename TO>
__device__ __forceinline__ void stacked_apply_task(ApplyArgs<T, TO> a, int64_t prob, int tile,
                                                   int64_t by, unsigned char* smem) {
  typedef typename Mfma<T>::v4 v4;
  if (by) {
    const int64_t pb = by;
    if (a.V) a.V += pb * a.bsV;
    if (a.Tleaf) a.Tleaf += pb * a.bsTleaf;
    if (a.Rbuf) a.Rbuf += pb * a.bsR;
    if (a.Ttree) a.Ttree += pb * a.bsTtree;
    if (a.U) a.U += pb * a.bsU;
    a.W += pb * a.bsW;
  }
  const int n = a.n, s = a.s, npan = a.npanels;
  const int64_t ncols = a.nr ? *a.nr : a.ncols;
  if ((int64_t)tile * 16 >= ncols) return;
  const int c0 = tile * 16;
  const bool leaf = (a.mode == 0);

  T* X = reinterpret_cast<T*>(smem);  // n x 17
  T* Z = X + (size_t)n * 17;          // s x 17
  T* Vp = Z + (size_t)s * 17;         // s x 17
  T* Tm = Vp + (size_t)s * 17;        // 16 x 17
  T* Yp = Tm + NB * TLD;              // 4 x 16 x 17 partials
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, g4 = lane >> 4;

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
  // panel range of chunk c (same rule as the factorisation)
  auto prange = [&](int64_t c, int& plo, int& phi, int& fc, int& scc) {
    const int64_t r0 = c * s;
    scc = (int)((rows - r0) < s ? (rows - r0) : s);
    fc = leaf ? (int)((r0 < n) ? r0 : n) : n;
    if (leaf) {
      const int lim = (fc + scc < n) ? fc + scc : n;
      plo = 0;
      phi = (lim + NB - 1) / NB;
    } else {
      plo = (int)(r0 / NB);
      phi = npan;
    }
  };
  // register prefetch of one panel's raw reflector values (s x 16) and T
  constexpr int VPT = 4;  // values per thread for s <= 64
  T vreg[VPT];
  T treg;
  auto fetch = [&](int64_t c, int p) {
    int plo, phi, fc, scc;
    prange(c, plo, phi, fc, scc);
    const int k0 = p * NB, kw = (n - k0 < NB) ? n - k0 : NB;
    const int64_t r0 = c * s;
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int idx = tid + 256 * u;
      const int r = idx >> 4, kk = idx & 15;
      vreg[u] = (r < scc && kk < kw) ? Vsrc[(r0 + r) * n + k0 + kk] : T(0);
    }
    treg = Tsrc[(c * npan + p) * (NB * NB) + tid];
  };
  {
    int plo, phi, fc, scc;
    prange(nch - 1, plo, phi, fc, scc);
    fetch(nch - 1, phi - 1);
  }
  for (int64_t c = nch - 1; c >= 0; --c) {
    const int64_t r0 = c * s;
    int p_lo, p_hi, f, sc;
    prange(c, p_lo, p_hi, f, sc);
    const int nf = (leaf && f < n) ? ((sc < n - f) ? sc : n - f) : 0;
    for (int idx = tid; idx < s * 16; idx += 256) {
      const int r = idx >> 4, cc = idx & 15;
      Z[r * 17 + cc] = (r < nf) ? X[(f + r) * 17 + cc] : T(0);
    }
    for (int p = p_hi - 1; p >= p_lo; --p) {
      const int k0 = p * NB;
      const int kw = (n - k0 < NB) ? n - k0 : NB;
      const bool internal = leaf && (k0 >= f);
      // stage the prefetched panel as exact reflectors (0 / 1 / tail)
#pragma unroll
      for (int u = 0; u < VPT; ++u) {
        const int idx = tid + 256 * u;
        const int r = idx >> 4, kk = idx & 15;
        if (r < s) {
          T vx = vreg[u];
          if (internal && r < sc && kk < kw) {
            const int hk = k0 + kk - f;
            vx = (r < hk) ? T(0) : ((r == hk) ? T(1) : vreg[u]);
          }
          Vp[r * 17 + kk] = vx;
        }
      }
      Tm[(tid >> 4) * TLD + (tid & 15)] = treg;
      // prefetch the next panel in processing order
      if (p > p_lo) {
        fetch(c, p - 1);
      } else if (c > 0) {
        int plo2, phi2, f2, sc2;
        prange(c - 1, plo2, phi2, f2, sc2);
        fetch(c - 1, phi2 - 1);
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
      // In the FP64 16x16x4 layout, accumulator q of lane (i16, g4) holds row
      // 4q + g4, column i16, which is exactly the B operand that lane
      // supplies at step kb = q: Y and T Y feed the next products from
      // registers.
      static_assert(sizeof(T) == 8, "register operands assume the FP64 MFMA layout");
      v4 ty = vzero4<T>();
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const int k = 4 * kb + g4;
        ty = Mfma<T>::op(Tm[i16 * TLD + k], yf[kb], ty);  // (T Y)
      }
      for (int mt = wave; mt < ntr; mt += 4) {
        v4 u = vzero4<T>();
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
          const int k = 4 * kb + g4;
          u = Mfma<T>::op(Vp[(16 * mt + i16) * 17 + k], ty[kb], u);
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

template <typename T, typename TO>
__global__ __launch_bounds__(256) void k_stacked_apply(ApplyArgs<T, TO> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  // tile-major block order: the active (tile < N_r / 16) blocks are the first
  // ones and spread over all XCDs
  const int64_t nprob = a.mode == 0 ? a.P : (a.P - a.h + 2 * a.h - 1) / (2 * a.h);
  stacked_apply_task<T, TO>(a, blockIdx.x % nprob, (int)(blockIdx.x / nprob), blockIdx.y, smem);
}

// Work-queue form of the broadcast phase: the down-tree propagation of every
// level, top level first, then the leaf applies, for every problem and
// column tile, in one launch.  Node j's tile counts one completion for every
// propagation step that writes W_j; a step at level h reads W_j for its
// receiver j, which must first hold every write from the levels above h
// (apply_need), and a leaf needs every write of all levels.  Tiles at or
// beyond the device-side column count are skipped by the task and by every
// task that would wait on it.
__device__ __forceinline__ unsigned int apply_need(int64_t j, int64_t h, int64_t P) {
  unsigned int need = 0;
  for (int64_t hp = 1; hp < P; hp *= 2) {
    if (hp <= h) continue;
    const int64_t r = j % (2 * hp);
    if (r == 0) {
      if (j + hp < P) ++need;  // receiver of the pair (j, j + hp)
    } else if (r == hp) {
      ++need;                  // sender of the pair (j - hp, j)
    }
  }
  return need;
}

template <typename T, typename TO>
__global__ __launch_bounds__(256) void k_apply_queue(ApplyArgs<T, TO> tree, ApplyArgs<T, TO> leaf,
                                                     ApplyQueue q) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int64_t slot;
  for (;;) {
    const int64_t t = queue_next(q.next, &slot);
    if (t >= q.lvl_off[q.nlev + 1]) break;
    int k = 0;  // position in top-down order: k < nlev are tree levels, k = nlev the leaves
    while (t >= q.lvl_off[k + 1]) ++k;
    const int64_t i = t - q.lvl_off[k];
    const bool is_leaf = k == q.nlev;
    const int64_t h = is_leaf ? 0 : ((int64_t)1 << (q.nlev - 1 - k));
    const int64_t per = (is_leaf ? q.P : (q.P - h + 2 * h - 1) / (2 * h)) * q.ntiles;
    const int64_t prob = i / per, rem = i - prob * per;
    const int tile = (int)(rem % q.ntiles);
    const int64_t idx = rem / q.ntiles;
    const int64_t ncols = q.nr ? q.nr[prob * q.nr_stride] : q.ncols;
    if ((int64_t)tile * 16 >= ncols) continue;
    unsigned int* cnt = q.cnt + prob * q.P * q.ntiles;
    const int64_t j = is_leaf ? idx : 2 * h * idx;
    if (threadIdx.x == 0) {
      queue_wait(cnt + j * q.ntiles + tile, apply_need(j, h, q.P), q.err);
      __threadfence();
    }
    __syncthreads();
    ApplyArgs<T, TO> b = is_leaf ? leaf : tree;
    if (!is_leaf) b.h = h;
    if (q.nr) b.nr = q.nr + prob * q.nr_stride;
    stacked_apply_task<T, TO>(b, idx, tile, prob, smem);
    __syncthreads();
    if (threadIdx.x == 0 && !is_leaf) {
      __threadfence();
      __hip_atomic_fetch_add(cnt + j * q.ntiles + tile, 1u, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(cnt + (j + h) * q.ntiles + tile, 1u, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Problems of at most two panels use single-wave workgroups: their trailing
// work per step is one tile, so three of four waves would idle, while several
// single-wave leaves share a CU and overlap their panel latencies.  A plan
// may ask for single-wave workgroups on wider problems too (QrGeom::nthr).
template <typename T, typename TI, int RT, int VAR>
static hipError_t launch_qr_t(const QrArgs<T, TI>& a, int grid, int gy, size_t lds,
                              hipStream_t st) {
  hipError_t e = hipFuncSetAttribute((const void*)k_stacked_qr<T, TI, RT, VAR>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int threads = a.nthr ? a.nthr : ((a.npanels <= 2) ? 64 : 256);
  hipLaunchKernelGGL((k_stacked_qr<T, TI, RT, VAR>), dim3(grid, gy), dim3(threads), lds, st, a);
  return hipGetLastError();
}

template <typename T, typename TI, int VAR>
static hipError_t launch_qr_var(const QrArgs<T, TI>& a, int grid, size_t lds, hipStream_t st,
                                int64_t gy) {
  switch (a.s) {
    case 16: return launch_qr_t<T, TI, 4, VAR>(a, grid, (int)gy, lds, st);
    case 32: return launch_qr_t<T, TI, 8, VAR>(a, grid, (int)gy, lds, st);
    case 48: return launch_qr_t<T, TI, 12, VAR>(a, grid, (int)gy, lds, st);
    case 64: return launch_qr_t<T, TI, 16, VAR>(a, grid, (int)gy, lds, st);
    default: return hipErrorInvalidValue;
  }
}

// Compute units of the current device (cached per device).
static int device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return 256;
  }
  if (cus[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        v < 1) {
      (void)hipGetLastError();
      v = 256;
    }
    cus[dev] = v;
  }
  return cus[dev];
}

// Leaves of the stacked path fill their state from the first chunks (VAR 0,
// or VAR 3 with the small-chunk prefetch); tree combines never do (VAR 1);
// column-blocked panels run two workgroups per CU (VAR 2) unless the grid
// has at most one per CU (VAR 4).
template <typename T, typename TI>
static hipError_t launch_qr_any(const QrArgs<T, TI>& a, int grid, size_t lds, hipStream_t st,
                                int64_t gy = 1) {
  if (grid <= 0 || gy <= 0) return hipSuccess;
  if (gy > 65535) return hipErrorInvalidValue;
  if (a.mode == 0 && a.state_mode == 0) {
    const int nthr = a.nthr ? a.nthr : ((a.npanels <= 2) ? 64 : 256);
    if (!a.remove_mean && a.s * a.n <= kPfn * nthr)
      return launch_qr_var<T, TI, 3>(a, grid, lds, st, gy);
    return launch_qr_var<T, TI, 0>(a, grid, lds, st, gy);
  }
  if (a.mode == 1) return launch_qr_var<T, TI, 1>(a, grid, lds, st, gy);
  if constexpr (std::is_same<T, TI>::value) {
    if ((int64_t)grid * gy <= device_cus()) return launch_qr_var<T, TI, 4>(a, grid, lds, st, gy);
  }
  return launch_qr_var<T, TI, 2>(a, grid, lds, st, gy);
}

template <typename QA>
static void set_qr_batch(QA& a, const Batch& bt) {
  a.bsD = bt.sD; a.bsMean = bt.sMean; a.bsV = bt.sV; a.bsTleaf = bt.sTleaf; a.bsR = bt.sR;
  a.bsTtree = bt.sTtree;
}

template <typename AA>
static void set_apply_batch(AA& a, const Batch& bt) {
  a.bsV = bt.sV; a.bsTleaf = bt.sTleaf; a.bsR = bt.sR; a.bsTtree = bt.sTtree; a.bsW = bt.sW;
  a.bsU = bt.sU;
}

hipError_t launch_leaf_qr_f64(const QrGeom& g, const void* D, int in_f64, int64_t ldd, int64_t m,
                              int64_t b, int64_t P, int remove_mean, double* mean_ws, double* V,
                              double* Tleaf, int64_t nch_leaf, double* Rbuf, hipStream_t st,
                              const Batch& bt) {
  const size_t lds = qr_lds_bytes(g, 8);
  if (in_f64) {
    QrArgs<double, double> a{};
    a.n = g.n; a.s = g.s; a.ldc = g.ldc; a.npanels = g.npanels; a.nthr = g.nthr; a.mode = 0;
    a.store_q = V != nullptr;
    a.D = (const double*)D; a.ldd = ldd; a.m = m; a.b = b; a.P = P;
    a.remove_mean = remove_mean; a.mean_ws = mean_ws; a.V = V; a.Tleaf = Tleaf;
    a.nch_leaf = nch_leaf; a.Rbuf = Rbuf;
    set_qr_batch(a, bt);
    return launch_qr_any(a, (int)P, lds, st, bt.count);
  }
  QrArgs<double, float> a{};
  a.n = g.n; a.s = g.s; a.ldc = g.ldc; a.npanels = g.npanels; a.nthr = g.nthr; a.mode = 0;
  a.store_q = V != nullptr;
  a.D = (const float*)D; a.ldd = ldd; a.m = m; a.b = b; a.P = P;
  a.remove_mean = remove_mean; a.mean_ws = mean_ws; a.V = V; a.Tleaf = Tleaf;
  a.nch_leaf = nch_leaf; a.Rbuf = Rbuf;
  set_qr_batch(a, bt);
  return launch_qr_any(a, (int)P, lds, st, bt.count);
}

hipError_t launch_leaf_qr_f32(const QrGeom& g, const float* D, int64_t ldd, int64_t m, int64_t b,
                              int64_t P, int remove_mean, double* mean_ws, float* Rbuf32,
                              hipStream_t st, const Batch& bt) {
  QrArgs<float, float> a{};
  a.n = g.n; a.s = g.s; a.ldc = g.ldc; a.npanels = g.npanels; a.nthr = g.nthr; a.mode = 0; a.store_q = 0;
  a.D = D; a.ldd = ldd; a.m = m; a.b = b; a.P = P;
  a.remove_mean = remove_mean; a.mean_ws = mean_ws; a.Rbuf = Rbuf32;
  set_qr_batch(a, bt);
  return launch_qr_any(a, (int)P, qr_lds_bytes(g, 4), st, bt.count);
}

hipError_t launch_tree_combine_f64(const QrGeom& g, int64_t h, int64_t P, double* Rbuf,
                                   double* Ttree, int64_t nch_tree, int store_q, hipStream_t st,
                                   const Batch& bt) {
  QrArgs<double, double> a{};
  a.n = g.n; a.s = g.s; a.ldc = g.ldc; a.npanels = g.npanels; a.nthr = g.nthr; a.mode = 1;
  a.store_q = store_q; a.h = h; a.Ttree = Ttree; a.nch_tree = nch_tree; a.Rbuf = Rbuf;
  // combines at this level: j = 0, 2h, 4h, ... with j + h < P
  const int64_t ncomb = (P - h + 2 * h - 1) / (2 * h);
  set_qr_batch(a, bt);
  return launch_qr_any(a, (int)ncomb, qr_lds_bytes(g, 8), st, bt.count);
}

template <typename T>
hipError_t launch_panel_qr(const QrGeom& g, T* Wk, int64_t ldw, int64_t m, int64_t b, int64_t P,
                           int64_t rows_lim, T* Tf, int64_t nch, T* Rstate, int state_mode,
                           hipStream_t st) {
  QrArgs<T, T> a{};
  a.n = g.n; a.s = g.s; a.ldc = g.ldc; a.npanels = g.npanels; a.nthr = g.nthr; a.mode = 0; a.store_q = 1;
  a.D = Wk; a.ldd = ldw; a.m = m; a.b = b; a.P = P; a.remove_mean = 0; a.mean_ws = nullptr;
  a.V = Wk; a.Tleaf = Tf; a.nch_leaf = nch; a.Rbuf = Rstate;
  a.state_mode = state_mode; a.ldv = ldw; a.rows_lim = rows_lim;
  if (state_mode != 1 && state_mode != 2) return hipErrorInvalidValue;
  if (P > 0x7fffffff) return hipErrorInvalidValue;
  if (P > 0 && g.s == kWfS && g.n <= 4 * NB && g.npanels >= 2 && (g.nthr == 0 || g.nthr == 256)) {
    // wavefront form; FP32 fits two workgroups per CU in LDS and registers
    const size_t lds = wf_lds_bytes((int)sizeof(T));
    const bool two = sizeof(T) == 4 && P > device_cus();
    const void* fn = two ? (const void*)k_panel_wf<T, 2> : (const void*)k_panel_wf<T, 1>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (two)
      hipLaunchKernelGGL((k_panel_wf<T, 2>), dim3((unsigned)P), dim3(256), lds, st, a);
    else
      hipLaunchKernelGGL((k_panel_wf<T, 1>), dim3((unsigned)P), dim3(256), lds, st, a);
    return hipGetLastError();
  }
  return launch_qr_any(a, (int)P, qr_lds_bytes(g, (int)sizeof(T)), st);
}
template hipError_t launch_panel_qr<double>(const QrGeom&, double*, int64_t, int64_t, int64_t,
                                            int64_t, int64_t, double*, int64_t, double*, int,
                                            hipStream_t);
template hipError_t launch_panel_qr<float>(const QrGeom&, float*, int64_t, int64_t, int64_t,
                                           int64_t, int64_t, float*, int64_t, float*, int,
                                           hipStream_t);

template <typename TO>
static hipError_t launch_apply_t(const ApplyArgs<double, TO>& a, int grid, size_t lds,
                                 hipStream_t st, int64_t gy = 1) {
  if (grid <= 0 || gy <= 0) return hipSuccess;
  if (gy > 65535) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void*)k_stacked_apply<double, TO>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_stacked_apply<double, TO>), dim3(grid, (unsigned)gy), dim3(256), lds, st,
                     a);
  return hipGetLastError();
}

hipError_t launch_apply_leaf_f64(const QrGeom& g, int64_t m, int64_t b, int64_t P,
                                 const double* V, const double* Tleaf, int64_t nch_leaf,
                                 const double* W, int64_t ldw, const int64_t* nr, int64_t ncols,
                                 void* U, int out_f64, int64_t ldu, hipStream_t st,
                                 const Batch& bt) {
  const int ntiles = (int)((ncols + 15) / 16);
  const size_t lds = apply_lds_bytes(g, 8);
  if (P < 1) return hipErrorInvalidValue;
  if (out_f64) {
    ApplyArgs<double, double> a{};
    a.n = g.n; a.s = g.s; a.npanels = g.npanels; a.mode = 0; a.nr = nr; a.ncols = ncols;
    a.m = m; a.b = b; a.P = P; a.V = V; a.Tleaf = Tleaf; a.nch_leaf = nch_leaf;
    a.U = (double*)U; a.ldu = ldu; a.W = const_cast<double*>(W); a.ldw = ldw;
    set_apply_batch(a, bt);
    return launch_apply_t(a, (int)(P * ntiles), lds, st, bt.count);
  }
  ApplyArgs<double, float> a{};
  a.n = g.n; a.s = g.s; a.npanels = g.npanels; a.mode = 0; a.nr = nr; a.ncols = ncols;
  a.m = m; a.b = b; a.P = P; a.V = V; a.Tleaf = Tleaf; a.nch_leaf = nch_leaf;
  a.U = (float*)U; a.ldu = ldu; a.W = const_cast<double*>(W); a.ldw = ldw;
  set_apply_batch(a, bt);
  return launch_apply_t(a, (int)(P * ntiles), lds, st, bt.count);
}

hipError_t launch_apply_tree_f64(const QrGeom& g, int64_t h, int64_t P, const double* Rbuf,
                                 const double* Ttree, int64_t nch_tree, double* W, int64_t ldw,
                                 const int64_t* nr, int64_t ncols, hipStream_t st,
                                 const Batch& bt) {
  const int ntiles = (int)((ncols + 15) / 16);
  const int64_t ncomb = (P - h + 2 * h - 1) / (2 * h);
  if (P < 2 || h < 1 || ncomb < 1) return hipErrorInvalidValue;
  ApplyArgs<double, double> a{};
  a.n = g.n; a.s = g.s; a.npanels = g.npanels; a.mode = 1; a.nr = nr; a.ncols = ncols;
  a.P = P; a.h = h; a.Rbuf = Rbuf; a.Ttree = Ttree; a.nch_tree = nch_tree; a.W = W; a.ldw = ldw;
  set_apply_batch(a, bt);
  return launch_apply_t(a, (int)(ncomb * ntiles), apply_lds_bytes(g, 8), st, bt.count);
}

// ---- work queues -----------------------------------------------------------
__global__ void k_queue_reset(unsigned int* p, int64_t nwords) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nwords;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// counters: the task counter (first 256 bytes), then the node counters
size_t queue_counter_bytes(int64_t count, int64_t P, int64_t ntiles) {
  const size_t words = (size_t)count * (size_t)P * (size_t)(ntiles > 1 ? ntiles : 1);
  return (256 + 4 * words + 255) & ~(size_t)255;
}

hipError_t launch_queue_reset(void* counters, size_t bytes, hipStream_t st) {
  const int64_t nwords = (int64_t)(bytes / 4);
  int64_t g = (nwords + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_queue_reset, dim3((unsigned)g), dim3(256), 0, st, (unsigned int*)counters,
                     nwords);
  return hipGetLastError();
}

__global__ void k_queue_err_merge(const int* e1, const int* e2, int* flag) {
  if (threadIdx.x == 0 && (*e1 || (e2 && *e2))) *flag = 1;
}

hipError_t launch_queue_err_merge(const void* counters1, const void* counters2, int* flag,
                                  hipStream_t st) {
  hipLaunchKernelGGL(k_queue_err_merge, dim3(1), dim3(64), 0, st,
                     (const int*)((const char*)counters1 + 64),
                     counters2 ? (const int*)((const char*)counters2 + 64) : nullptr, flag);
  return hipGetLastError();
}

// Grid of a work-queue launch: every workgroup that can be resident at once
// (more would only wait for a free slot), at most one per task.
static int64_t queue_grid(const void* fn, int threads, size_t lds, int64_t ntasks) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess ||
      per_cu < 1) {
    (void)hipGetLastError();
    per_cu = 1;
  }
  const int64_t slots = (int64_t)per_cu * device_cus();
  return ntasks < slots ? ntasks : slots;
}

template <typename T, typename TI, int RT, int VAR>
static hipError_t launch_qrq_t(const QrArgs<T, TI>& a, const QrQueue& q, size_t lds,
                               hipStream_t st) {
  const void* fn = (const void*)k_qr_queue<T, TI, RT, VAR>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int threads = a.nthr ? a.nthr : ((a.npanels <= 2) ? 64 : 256);
  const int64_t ntasks = q.lvl_off[q.nlev + 1];
  const int64_t grid = queue_grid(fn, threads, lds, ntasks);
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL((k_qr_queue<T, TI, RT, VAR>), dim3((unsigned)grid), dim3(threads), lds, st,
                     a, q);
  return hipGetLastError();
}

template <typename T, typename TI, int VAR>
static hipError_t launch_qrq_var(const QrArgs<T, TI>& a, const QrQueue& q, size_t lds,
                                 hipStream_t st) {
  switch (a.s) {
    case 16: return launch_qrq_t<T, TI, 4, VAR>(a, q, lds, st);
    case 32: return launch_qrq_t<T, TI, 8, VAR>(a, q, lds, st);
    case 48: return launch_qrq_t<T, TI, 12, VAR>(a, q, lds, st);
    case 64: return launch_qrq_t<T, TI, 16, VAR>(a, q, lds, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename TI>
static hipError_t launch_qrq(const QrGeom& g, const TI* D, int64_t ldd, int64_t m, int64_t b,
                             int64_t P, int remove_mean, double* mean_ws, double* V,
                             double* Tleaf, int64_t nch_leaf, double* Rbuf, double* Ttree,
                             int64_t nch_tree, int store_q, void* counters, hipStream_t st,
                             const Batch& bt) {
  QrArgs<double, TI> a{};
  a.n = g.n; a.s = g.s; a.ldc = g.ldc; a.npanels = g.npanels; a.nthr = g.nthr; a.mode = 0;
  a.store_q = store_q;
  a.D = D; a.ldd = ldd; a.m = m; a.b = b; a.P = P; a.remove_mean = remove_mean;
  a.mean_ws = mean_ws;
  a.V = V; a.Tleaf = Tleaf; a.nch_leaf = nch_leaf; a.Rbuf = Rbuf;
  a.Ttree = Ttree; a.nch_tree = nch_tree;
  set_qr_batch(a, bt);
  QrQueue q{};
  q.P = P;
  int nlev = 0;
  for (int64_t h = 1; h < P; h *= 2) ++nlev;
  if (nlev > kMaxQueueLevels) return hipErrorNotSupported;
  q.nlev = nlev;
  q.lvl_off[0] = 0;
  q.lvl_off[1] = bt.count * P;
  for (int l = 1; l <= nlev; ++l) {
    const int64_t h = (int64_t)1 << (l - 1);
    q.lvl_off[l + 1] = q.lvl_off[l] + bt.count * ((P - h + 2 * h - 1) / (2 * h));
  }
  q.next = (unsigned long long*)counters;
  q.cnt = (unsigned int*)((char*)counters + 256);
  q.err = (int*)((char*)counters + 64);
  const size_t lds = qr_lds_bytes(g, 8);
  if (lds + 64 > kQrLdsBudget) return hipErrorNotSupported;
  const int nthr = a.nthr ? a.nthr : ((a.npanels <= 2) ? 64 : 256);
  if (!remove_mean && a.s * a.n <= kPfn * nthr) return launch_qrq_var<double, TI, 3>(a, q, lds, st);
  return launch_qrq_var<double, TI, 0>(a, q, lds, st);
}

hipError_t launch_qr_queue_f64(const QrGeom& g, const void* D, int in_f64, int64_t ldd, int64_t m,
                               int64_t b, int64_t P, int remove_mean, double* mean_ws, double* V,
                               double* Tleaf, int64_t nch_leaf, double* Rbuf, double* Ttree,
                               int64_t nch_tree, int store_q, void* counters, hipStream_t st,
                               const Batch& bt) {
  if (P < 1 || bt.count < 1) return hipErrorInvalidValue;
  if (in_f64)
    return launch_qrq<double>(g, (const double*)D, ldd, m, b, P, remove_mean, mean_ws, V, Tleaf,
                              nch_leaf, Rbuf, Ttree, nch_tree, store_q, counters, st, bt);
  return launch_qrq<float>(g, (const float*)D, ldd, m, b, P, remove_mean, mean_ws, V, Tleaf,
                           nch_leaf, Rbuf, Ttree, nch_tree, store_q, counters, st, bt);
}

template <typename TO>
static hipError_t launch_applyq_t(const ApplyArgs<double, TO>& tree,
                                  const ApplyArgs<double, TO>& leaf, const ApplyQueue& q,
                                  size_t lds, hipStream_t st) {
  const void* fn = (const void*)k_apply_queue<double, TO>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int64_t ntasks = q.lvl_off[q.nlev + 1];
  const int64_t grid = queue_grid(fn, 256, lds, ntasks);
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL((k_apply_queue<double, TO>), dim3((unsigned)grid), dim3(256), lds, st, tree,
                     leaf, q);
  return hipGetLastError();
}

hipError_t launch_apply_queue_f64(const QrGeom& g, int64_t m, int64_t b, int64_t P,
                                  const double* V, const double* Tleaf, int64_t nch_leaf,
                                  const double* Rbuf, const double* Ttree, int64_t nch_tree,
                                  double* W, int64_t ldw, const int64_t* nr, int64_t nr_stride,
                                  int64_t ncols, void* U, int out_f64, int64_t ldu, void* counters,
                                  hipStream_t st, const Batch& bt) {
  if (P < 1 || bt.count < 1) return hipErrorInvalidValue;
  ApplyQueue q{};
  q.P = P;
  int nlev = 0;
  for (int64_t h = 1; h < P; h *= 2) ++nlev;
  if (nlev > kMaxQueueLevels) return hipErrorNotSupported;
  q.nlev = nlev;
  q.ntiles = (ncols + 15) / 16;
  q.ncols = ncols;
  q.nr = nr;
  q.nr_stride = nr_stride;
  q.lvl_off[0] = 0;
  for (int k = 0; k < nlev; ++k) {
    const int64_t h = (int64_t)1 << (nlev - 1 - k);
    q.lvl_off[k + 1] = q.lvl_off[k] + bt.count * ((P - h + 2 * h - 1) / (2 * h)) * q.ntiles;
  }
  q.lvl_off[nlev + 1] = q.lvl_off[nlev] + bt.count * P * q.ntiles;
  q.next = (unsigned long long*)counters;
  q.cnt = (unsigned int*)((char*)counters + 256);
  q.err = (int*)((char*)counters + 64);
  const size_t lds = apply_lds_bytes(g, 8);
  if (lds + 64 > kQrLdsBudget) return hipErrorNotSupported;
  if (out_f64) {
    ApplyArgs<double, double> t{}, l{};
    t.n = l.n = g.n; t.s = l.s = g.s; t.npanels = l.npanels = g.npanels;
    t.mode = 1; l.mode = 0; t.nr = l.nr = nullptr; t.ncols = l.ncols = ncols;
    t.P = l.P = P; t.Rbuf = Rbuf; t.Ttree = Ttree; t.nch_tree = nch_tree;
    t.W = l.W = W; t.ldw = l.ldw = ldw;
    l.m = m; l.b = b; l.V = V; l.Tleaf = Tleaf; l.nch_leaf = nch_leaf; l.U = (double*)U;
    l.ldu = ldu;
    set_apply_batch(t, bt);
    set_apply_batch(l, bt);
    return launch_applyq_t<double>(t, l, q, lds, st);
  }
  ApplyArgs<double, float> t{}, l{};
  t.n = l.n = g.n; t.s = l.s = g.s; t.npanels = l.npanels = g.npanels;
  t.mode = 1; l.mode = 0; t.nr = l.nr = nullptr; t.ncols = l.ncols = ncols;
  t.P = l.P = P; t.Rbuf = Rbuf; t.Ttree = Ttree; t.nch_tree = nch_tree;
  t.W = l.W = W; t.ldw = l.ldw = ldw;
  l.m = m; l.b = b; l.V = V; l.Tleaf = Tleaf; l.nch_leaf = nch_leaf; l.U = (float*)U;
  l.ldu = ldu;
  set_apply_batch(t, bt);
  set_apply_batch(l, bt);
  return launch_applyq_t<float>(t, l, q, lds, st);
}

}  // namespace pylom
