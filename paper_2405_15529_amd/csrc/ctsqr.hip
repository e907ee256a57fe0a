// ctsqr.hip -- complex tall-skinny QR of the SPOD spectral matrices and the
// application of its Q (Alg. 1 on each frequency's Q_f of Alg. 6; Sec. 2.3
// and Sec. 3.3 with Eqs. svdqr1-3), all arithmetic in FP64.
//
// Spectra E: the column of block k of frequency f holds m complex values
// starting at complex element (f * nb + k) * ldm (T pairs re, im).
//
// Leaves are 128-row slabs, one wave each: lane l keeps rows l and 64 + l of
// its slab in registers (nb complex values per row).  Column j of the
// Householder sweep needs one wave-wide sum, g_k = sum_{r > j} conj(a_rj)
// a_rk for k >= j, done as an in-row DPP reduce-scatter, two row-pair swaps
// and an LDS all-gather; the diagonal row j is broadcast through LDS.
//
// Householder convention (LAPACK zlarfg): H = I - tau v v^H, v_j = 1,
// H^H [alpha; x] = [beta; 0] with beta real, Q = H_0 H_1 ... H_{nb-1}.
//
// Tree nodes: Rn[f][node] is a 16 x 16 complex block (row-major, the leading
// nb x nb used, exact zeros below the diagonal).  A combine of nodes j and
// j + h (level h of the binary tree of Alg. 1) runs on one 16-lane DPP row:
// lane l keeps row l of R_{j+h} in registers, row l of R_j is the diagonal row
// of step l.  The reflectors of that combine go to Vn[f][j + h] (rows 0..15
// the lower parts, row 16 the tau values).  After the root SVD the Rn blocks
// are reused for the down-tree factors C: [C_j; C_{j+h}] = Q_node [C_j; 0].
//
// The factor pass also accumulates the compact WY factor T of each leaf
// (LAPACK zlarft, forward columnwise, Q_leaf = I - V T V^H), stores the
// reflectors V in the spectra precision and W = T V_top^H (V_top the leaf's
// first nb rows of V); the apply pass then writes
//   U_leaf = Q_leaf [C; 0] = [C; 0] - V (W C)
// straight into the modes array.
#include "common.hpp"
#include "kernels.hpp"


namespace pylom {

namespace {

constexpr int kLeafRows = 128;
constexpr int kNodeZ = 256;        // complex entries per tree node block
constexpr int kVnZ = 17 * 16;      // reflector block + tau row
constexpr int kLd = 17;            // LDS row stride of the 16 x 16 complex tiles

struct zd {
  double re, im;
};

__device__ __forceinline__ zd zmul(zd a, zd b) {
  return zd{fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)};
}
// acc + conj(a) b
__device__ __forceinline__ zd zcjmac(zd a, zd b, zd acc) {
  return zd{fma(a.re, b.re, fma(a.im, b.im, acc.re)), fma(a.re, b.im, fma(-a.im, b.re, acc.im))};
}
// acc + a b
__device__ __forceinline__ zd zmac(zd a, zd b, zd acc) {
  return zd{fma(a.re, b.re, fma(-a.im, b.im, acc.re)), fma(a.re, b.im, fma(a.im, b.re, acc.im))};
}
// y - s x
__device__ __forceinline__ zd zsubmul(zd y, zd s, zd x) {
  return zd{fma(-s.re, x.re, fma(s.im, x.im, y.re)), fma(-s.re, x.im, fma(-s.im, x.re, y.im))};
}
__device__ __forceinline__ zd zconj(zd a) { return zd{a.re, -a.im}; }

constexpr int pow2ceil(int v) {
  int p = 2;
  while (p < v) p *= 2;
  return p;
}

// One halving step of a reduce-scatter over the involutive DPP pairing CTRL:
// lanes with `up` keep the upper half of x[0..2H), the others the lower half,
// and add the partner's copy of the kept half.
template <int CTRL, int H>
__device__ __forceinline__ void halve(double (&x)[32], bool up) {
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double keep = up ? x[i + H] : x[i];
    const double send = up ? x[i] : x[i + H];
    x[i] = keep + dpp<CTRL>(send);
  }
}
template <int CTRL, int H>
__device__ __forceinline__ void halve16(double (&x)[16], bool up) {
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double keep = up ? x[i + H] : x[i];
    const double send = up ? x[i] : x[i + H];
    x[i] = keep + dpp<CTRL>(send);
  }
}
template <int CTRL>
__device__ __forceinline__ double pairsum(double v) {
  return v + dpp<CTRL>(v);
}

// In-row reduce-scatter over the 16 lanes of each DPP row (pairings mirror,
// half mirror, quad 3210, quad 1032) of V doubles per lane, V a power of two
// in 2..32: the V/2 complex values part(kk) (re at 2kk, im at 2kk + 1; zero for
// kk >= cnt).  The first halving pairs value i with i + V/2 and consumes the
// partial values as they are produced.  On return x[u], u < max(1, V/16),
// holds the row total of value base + u (base returned); lanes with equal
// base hold equal bits.
template <int V, typename F>
__device__ __forceinline__ int row_rs(F&& part, double (&x)[32], int i) {
  const bool b3 = i >= 8, b2 = (i & 7) >= 4, b1 = (i & 3) >= 2, b0 = (i & 1) != 0;
  int base = b3 ? V / 2 : 0;
  if constexpr (V >= 4) {
#pragma unroll
    for (int kk = 0; kk < V / 4; ++kk) {
      const zd lo = part(kk), hi = part(kk + V / 4);
      x[2 * kk] = (b3 ? hi.re : lo.re) + dpp<0x140>(b3 ? lo.re : hi.re);
      x[2 * kk + 1] = (b3 ? hi.im : lo.im) + dpp<0x140>(b3 ? lo.im : hi.im);
    }
    halve<0x141, V / 4>(x, b2);
    base += b2 ? V / 4 : 0;
  } else {
    const zd lo = part(0);
    x[0] = lo.re;
    x[1] = lo.im;
    halve<0x140, 1>(x, b3);
    x[0] = pairsum<0x141>(x[0]);
  }
  if constexpr (V >= 8) {
    halve<0x1B, V / 8>(x, b1);
    base += b1 ? V / 8 : 0;
  } else {
    x[0] = pairsum<0x1B>(x[0]);
  }
  if constexpr (V >= 16) {
    halve<0xB1, V / 16>(x, b0);
    base += b0 ? V / 16 : 0;
  } else {
    x[0] = pairsum<0xB1>(x[0]);
  }
  return base;
}

// Halving across row pairs with one swap per 32-bit half: the swap of (lo, hi)
// leaves {own lo, partner lo} in the rows that keep the lower half and
// {partner hi, own hi} in the others, so the sum of the two outputs is the
// pair total of the kept half.  keep_hi (which half this lane's row keeps) is
// read once from a swap of constants.
template <int W>
__device__ __forceinline__ double swap_sum(double lo, double hi) {
  const long long a = __double_as_longlong(lo), b = __double_as_longlong(hi);
  const int alo = (int)(a & 0xffffffffll), ahi = (int)(a >> 32);
  const int blo = (int)(b & 0xffffffffll), bhi = (int)(b >> 32);
  if constexpr (W == 16) {
    const auto l = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    return __longlong_as_double(((long long)h[0] << 32) | (unsigned int)l[0]) +
           __longlong_as_double(((long long)h[1] << 32) | (unsigned int)l[1]);
  } else {
    const auto l = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    return __longlong_as_double(((long long)h[0] << 32) | (unsigned int)l[0]) +
           __longlong_as_double(((long long)h[1] << 32) | (unsigned int)l[1]);
  }
}
template <int W>
__device__ __forceinline__ bool swap_keeps_hi() {
  if constexpr (W == 16) return __builtin_amdgcn_permlane16_swap(0, 1, false, false)[0] != 0;
  else return __builtin_amdgcn_permlane32_swap(0, 1, false, false)[0] != 0;
}

// Totals over all 64 lanes of the V/2 complex values part(kk) (V a power of
// two, 2..32), gathered in red[0..V) (re, im interleaved): halvings across
// the 32-lane halves and across row pairs (swaps), then inside each row
// (mirror, half mirror, quad 3210), pair sums for what is left.
template <int V, typename F>
__device__ __forceinline__ void wave_allreduce(F&& part, int lane, double* red) {
  const int i = lane & 15;
  const bool h32 = swap_keeps_hi<32>(), h16 = swap_keeps_hi<16>();
  double x[16];
  int idx = h32 ? V / 2 : 0;
  if constexpr (V >= 4) {
#pragma unroll
    for (int kk = 0; kk < V / 4; ++kk) {
      const zd lo = part(kk), hi = part(kk + V / 4);
      x[2 * kk] = swap_sum<32>(lo.re, hi.re);
      x[2 * kk + 1] = swap_sum<32>(lo.im, hi.im);
    }
    // V/2 values left: halve across row pairs
#pragma unroll
    for (int u = 0; u < V / 4; ++u) x[u] = swap_sum<16>(x[u], x[u + V / 4]);
    idx += h16 ? V / 4 : 0;
  } else {
    const zd lo = part(0);
    x[0] = perm16_pairsum(swap_sum<32>(lo.re, lo.im));
  }
  if constexpr (V >= 8) {
    halve16<0x140, V / 8>(x, i >= 8);
    idx += i >= 8 ? V / 8 : 0;
  } else {
    x[0] = pairsum<0x140>(x[0]);
  }
  if constexpr (V >= 16) {
    halve16<0x141, V / 16>(x, (i & 7) >= 4);
    idx += (i & 7) >= 4 ? V / 16 : 0;
  } else {
    x[0] = pairsum<0x141>(x[0]);
  }
  if constexpr (V >= 32) {
    halve16<0x1B, V / 32>(x, (i & 3) >= 2);
    idx += (i & 3) >= 2 ? V / 32 : 0;
  } else {
    x[0] = pairsum<0x1B>(x[0]);
  }
  x[0] = pairsum<0xB1>(x[0]);
  red[idx] = x[0];
  wave_lds_sync();
}

// Totals over each 16-lane row, gathered in the row's own red[0..V).
template <int V, typename F>
__device__ __forceinline__ void row_allreduce(F&& part, int lt, double* red) {
  double x[32];
  const int base = row_rs<V>(part, x, lt);
  constexpr int U = V >= 16 ? V / 16 : 1;
#pragma unroll
  for (int u = 0; u < U; ++u) red[base + u] = x[u];
  wave_lds_sync();
}

// zlarfg on [alpha; x] with |x|^2 = xn2: beta, tau and gam = 1 / (alpha - beta)
// (v = gam x); tau = 0 (H = I) when x = 0 and alpha is real.
__device__ __forceinline__ void zlarfg(zd alpha, double xn2, double& beta, zd& tau, zd& gam) {
  if (xn2 == 0.0 && alpha.im == 0.0) {
    beta = alpha.re;
    tau = zd{0.0, 0.0};
    gam = zd{0.0, 0.0};
  } else {
    const double nrm = sqrt(fma(alpha.re, alpha.re, fma(alpha.im, alpha.im, xn2)));
    beta = alpha.re >= 0.0 ? -nrm : nrm;
    const double rb = 1.0 / beta;
    tau = zd{(beta - alpha.re) * rb, -alpha.im * rb};
    const double dr = alpha.re - beta, di = alpha.im;
    const double rden = 1.0 / fma(dr, dr, di * di);
    gam = zd{dr * rden, -di * rden};
  }
}

template <typename T>
struct T2;
template <>
struct T2<float> {
  typedef float2 type;
};
template <>
struct T2<double> {
  typedef double2 type;
};

// ---- leaf sweep -------------------------------------------------------------
// Column J of the leaf factorisation with column J of the compact WY factor T
// (LAPACK zlarft, forward columnwise).  One wave-wide sum per column gives
//   g_k = sum_{r > J} conj(x_r) a_rk   (k >= J; x = column J, g_J = |x|^2)
//   s_i = sum_{r > J} conj(v_ri) x_r   (i < J; the stored reflectors)
// and then y_i = (V^H v_J)_i = conj(v_Ji) + gam s_i,
//   T[i][J] = -tau sum_{l >= i} T[i][l] y_l,  T[J][J] = tau.
template <int NB, int J>
__device__ __forceinline__ void leaf_cols(zd (&a)[2][NB], int lane, double* red, zd* drow,
                                          zd* tbuf, zd* ybuf, zd* Tm) {
  if constexpr (J < NB) {
    constexpr int CG = NB - J;
    constexpr int V = pow2ceil(2 * NB);
    const bool below = lane > J;
    const zd c0 = below ? a[0][J] : zd{0.0, 0.0};
    const zd c1 = a[1][J];
    if (lane == J) {
#pragma unroll
      for (int k = 0; k < NB; ++k) drow[k] = a[0][k];
    }
    wave_allreduce<V>(
        [&](int kk) -> zd {
          if (kk < CG) {
            const zd p = zcjmac(c0, a[0][J + kk], zd{0.0, 0.0});
            return zcjmac(c1, a[1][J + kk], p);
          }
          if (kk < NB) {
            const int i = kk - CG;
            const zd p = zcjmac(a[0][i], c0, zd{0.0, 0.0});
            return zcjmac(a[1][i], c1, p);
          }
          return zd{0.0, 0.0};
        },
        lane, red);
    double beta;
    zd tau, gam;
    zlarfg(drow[J], red[0], beta, tau, gam);
    // lane k > J: t_k = conj(tau) (d_k + conj(gam) g_k);  lane i < J: y_i
    if (lane < NB && lane != J) {
      const zd dk = drow[lane];
      if (lane > J) {
        const int o = 2 * (lane - J);
        const zd q = zmul(zconj(gam), zd{red[o], red[o + 1]});
        tbuf[lane] = zmul(zconj(tau), zd{dk.re + q.re, dk.im + q.im});
      } else {
        const int o = 2 * (CG + lane);
        const zd q = zmul(gam, zd{red[o], red[o + 1]});
        ybuf[lane] = zd{dk.re + q.re, -dk.im + q.im};
      }
    }
    wave_lds_sync();
    const zd v0 = below ? zmul(gam, a[0][J]) : zd{lane == J ? 1.0 : 0.0, 0.0};
    const zd v1 = zmul(gam, a[1][J]);
#pragma unroll
    for (int k = J + 1; k < NB; ++k) {
      const zd tk = tbuf[k];
      a[0][k] = zsubmul(a[0][k], tk, v0);
      a[1][k] = zsubmul(a[1][k], tk, v1);
    }
    a[0][J] = below ? v0 : (lane == J ? zd{beta, 0.0} : a[0][J]);
    a[1][J] = v1;
    if (lane < J) {
      zd acc{0.0, 0.0};
#pragma unroll
      for (int l = 0; l < J; ++l)
        if (l >= lane) acc = zmac(Tm[lane * kLd + l], ybuf[l], acc);
      const zd r = zmul(tau, acc);
      Tm[lane * kLd + J] = zd{-r.re, -r.im};
    }
    if (lane == J) Tm[J * kLd + J] = tau;
    leaf_cols<NB, J + 1>(a, lane, red, drow, tbuf, ybuf, Tm);
  }
}

// Factor pass, one wave per 128-row leaf of every frequency (blockIdx.y):
// R of the leaf into Rn; the leaf's rows after the sweep (R above, the
// reflectors below the diagonal) into Vl (column-major per leaf, complex T);
// W = T V_top^H (V_top = rows 0..nb-1 of V, unit lower triangular) into Wl.
template <typename T, int NB>
__global__ __launch_bounds__(64, 2) void k_cleaf_factor(int64_t m, int64_t ldm, int64_t P,
                                                        const T* __restrict__ E,
                                                        zd* __restrict__ Rn, T* __restrict__ Vl,
                                                        zd* __restrict__ Wl) {
  __shared__ double red[32];
  __shared__ zd drow[16], tbuf[16], ybuf[16];
  __shared__ zd Tm[16 * kLd], Vt[16 * kLd];
  typedef typename T2<T>::type TT;
  const int lane = threadIdx.x;
  const int64_t leaf = blockIdx.x, f = blockIdx.y;
  const int64_t r0 = leaf * kLeafRows;
  zd a[2][NB];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int64_t row = r0 + 64 * s + lane;
    const bool ok = row < m;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      if (ok) {
        const TT v = reinterpret_cast<const TT*>(E)[(f * NB + k) * ldm + row];
        a[s][k] = zd{(double)v.x, (double)v.y};
      } else {
        a[s][k] = zd{0.0, 0.0};
      }
    }
  }
  leaf_cols<NB, 0>(a, lane, red, drow, tbuf, ybuf, Tm);
  const int64_t node = f * P + leaf;
  if (lane < NB) {
    zd* R = Rn + node * kNodeZ + lane * 16;
#pragma unroll
    for (int k = 0; k < NB; ++k) R[k] = k < lane ? zd{0.0, 0.0} : a[0][k];
#pragma unroll
    for (int k = 0; k < NB; ++k)
      Vt[lane * kLd + k] = k < lane ? a[0][k] : zd{k == lane ? 1.0 : 0.0, 0.0};
  }
  TT* V = reinterpret_cast<TT*>(Vl) + node * NB * kLeafRows;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      TT v;
      v.x = (T)a[s][k].re;
      v.y = (T)a[s][k].im;
      V[k * kLeafRows + 64 * s + lane] = v;
    }
  }
  wave_lds_sync();
  // W[i][r] = sum_{i <= l <= r} T[i][l] conj(V_top[r][l]), lane (ii, q) for r = q + 4 kk
  const int ii = lane & 15, q = lane >> 4;
  zd w[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) w[kk] = zd{0.0, 0.0};
#pragma unroll
  for (int l = 0; l < NB; ++l) {
    if (l >= ii) {
      const zd tl = Tm[ii * kLd + l];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        if (q + 4 * kk < NB) w[kk] = zmac(tl, zconj(Vt[(q + 4 * kk) * kLd + l]), w[kk]);
    }
  }
  if (ii < NB) {
    zd* W = Wl + node * kNodeZ + ii * 16;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      if (q + 4 * kk < NB) W[q + 4 * kk] = w[kk];
  }
}

// Apply pass: U rows of the leaf = [C; 0] - V (W C) into modes (complex T,
// [f][p][c]), C the leaf's block of Cn.
template <typename T, int NB>
__global__ __launch_bounds__(64, 2) void k_cleaf_apply(int64_t m, int64_t P,
                                                       const T* __restrict__ Vl,
                                                       const zd* __restrict__ Wl,
                                                       const zd* __restrict__ Cn,
                                                       T* __restrict__ modes) {
  __shared__ zd Cl[16 * kLd], Zl[16 * kLd], Wm[16 * kLd];
  typedef typename T2<T>::type TT;
  const int lane = threadIdx.x;
  const int64_t leaf = blockIdx.x, f = blockIdx.y;
  const int64_t r0 = leaf * kLeafRows;
  const int64_t node = f * P + leaf;
  const zd* C = Cn + node * kNodeZ;
  const zd* W = Wl + node * kNodeZ;
  {
    // every load issued before the first store
    constexpr int NE = (NB * NB + 63) / 64;
    zd cv[NE], wv[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = lane + 64 * i;
      const bool ok = e < NB * NB;
      cv[i] = ok ? C[(e / NB) * 16 + e % NB] : zd{0.0, 0.0};
      wv[i] = ok ? W[(e / NB) * 16 + e % NB] : zd{0.0, 0.0};
    }
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = lane + 64 * i;
      if (e < NB * NB) {
        Cl[(e / NB) * kLd + e % NB] = cv[i];
        Wm[(e / NB) * kLd + e % NB] = wv[i];
      }
    }
  }
  const TT* V = reinterpret_cast<const TT*>(Vl) + node * NB * kLeafRows;
  TT a[2][NB];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int k = 0; k < NB; ++k) a[s][k] = V[k * kLeafRows + 64 * s + lane];
  wave_lds_sync();
  // Z = W C, lane (ii, q) computes Z[ii][q + 4 kk]
  const int ii = lane & 15, q = lane >> 4;
  zd z[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) z[kk] = zd{0.0, 0.0};
#pragma unroll
  for (int r = 0; r < NB; ++r) {
    const zd wr = Wm[ii * kLd + r];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      if (q + 4 * kk < NB) z[kk] = zmac(wr, Cl[r * kLd + q + 4 * kk], z[kk]);
  }
  if (ii < NB) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      if (q + 4 * kk < NB) Zl[ii * kLd + q + 4 * kk] = z[kk];
  }
  wave_lds_sync();
  const int lc = lane < NB ? lane : 0;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    // re-read Z for each slot rather than keeping all of it in registers
    wave_lds_sync();
    zd acc[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const zd cv = Cl[lc * kLd + c];
      acc[c] = (s == 0 && lane < NB) ? cv : zd{0.0, 0.0};
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const zd ak = zd{(double)a[s][k].x, (double)a[s][k].y};
      const zd vk = s == 1 ? ak : (k < lane ? ak : zd{k == lane ? 1.0 : 0.0, 0.0});
#pragma unroll
      for (int c = 0; c < NB; ++c) acc[c] = zsubmul(acc[c], vk, Zl[k * kLd + c]);
    }
    const int64_t row = r0 + 64 * s + lane;
    if (row < m) {
      TT* out = reinterpret_cast<TT*>(modes) + (f * m + row) * NB;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        TT v;
        v.x = (T)acc[c].re;
        v.y = (T)acc[c].im;
        out[c] = v;
      }
    }
  }
}

// ---- tree combine -------------------------------------------------------------
// Column J of a combine: the lane's row of the lower block in b, the upper
// block in LDS (ra, row J is the diagonal row of the step).
template <int NB, int J>
__device__ __forceinline__ void comb_cols(zd (&b)[NB], zd* ra, int lt, double* red, zd* taus,
                                          zd* tbuf) {
  if constexpr (J < NB) {
    constexpr int CG = NB - J;
    constexpr int VG = pow2ceil(2 * CG);
    const zd cj = b[J];
    row_allreduce<VG>(
        [&](int kk) -> zd {
          if (kk >= CG) return zd{0.0, 0.0};
          return zcjmac(cj, b[J + kk], zd{0.0, 0.0});
        },
        lt, red);
    double beta;
    zd tau, gam;
    zlarfg(ra[J * kLd + J], red[0], beta, tau, gam);
    // t_k = conj(tau) (d_k + conj(gam) g_k), lane k - J of the row computes it
    // and also updates the diagonal row's entry k
    if constexpr (CG > 1) {
      if (lt >= 1 && lt < CG) {
        const zd dk = ra[J * kLd + J + lt];
        const zd q = zmul(zconj(gam), zd{red[2 * lt], red[2 * lt + 1]});
        const zd tk = zmul(zconj(tau), zd{dk.re + q.re, dk.im + q.im});
        tbuf[J + lt] = tk;
        ra[J * kLd + J + lt] = zd{dk.re - tk.re, dk.im - tk.im};
      }
      wave_lds_sync();
    }
    const zd v = zmul(gam, cj);
#pragma unroll
    for (int k = J + 1; k < NB; ++k) b[k] = zsubmul(b[k], tbuf[k], v);
    b[J] = v;
    if (lt == J) {
      ra[J * kLd + J] = zd{beta, 0.0};
      taus[J] = tau;
    }
    comb_cols<NB, J + 1>(b, ra, lt, red, taus, tbuf);
  }
}

// Level h of the tree: combine c = blockIdx.x*4 + (lane / 16) of frequency
// blockIdx.y merges nodes j = 2hc (upper) and j + h (lower).
template <int NB>
__global__ __launch_bounds__(64, 3) void k_ctree_combine(int64_t P, int64_t h, int64_t ncomb,
                                                         zd* __restrict__ Rn,
                                                         zd* __restrict__ Vn) {
  __shared__ double red[4][32];
  __shared__ zd ra[4][16 * kLd];
  __shared__ zd taus[4][16];
  __shared__ zd tbuf[4][16];
  const int lane = threadIdx.x, g = lane >> 4, lt = lane & 15;
  const int64_t c = (int64_t)blockIdx.x * 4 + g, f = blockIdx.y;
  const bool active = c < ncomb;
  const int64_t j = c * 2 * h, s = j + h;
  zd* Ra = Rn + (f * P + j) * kNodeZ + lt * 16;
  const zd* Rb = Rn + (f * P + s) * kNodeZ + lt * 16;
  const bool io = active && lt < NB;
  zd b[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    b[k] = zd{0.0, 0.0};
    ra[g][lt * kLd + k] = zd{0.0, 0.0};
  }
  taus[g][lt] = zd{0.0, 0.0};
  if (io) {
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      b[k] = Rb[k];
      ra[g][lt * kLd + k] = Ra[k];
    }
  }
  wave_lds_sync();
  comb_cols<NB, 0>(b, ra[g], lt, red[g], taus[g], tbuf[g]);
  wave_lds_sync();
  if (io) {
#pragma unroll
    for (int k = 0; k < NB; ++k) Ra[k] = ra[g][lt * kLd + k];
    zd* V = Vn + (f * P + s) * kVnZ;
#pragma unroll
    for (int k = 0; k < NB; ++k) V[lt * 16 + k] = b[k];
    V[16 * 16 + lt] = taus[g][lt];
  }
}

// ---- tree apply (down the tree) ---------------------------------------------------
template <int NB, int J>
__device__ __forceinline__ void tapply_cols(zd (&yb)[NB], const zd (&v)[NB], int lt, double* red,
                                            zd* ya, const zd* tau) {
  if constexpr (J >= 0) {
    constexpr int VG = pow2ceil(2 * NB);
    const zd vj = v[J];
    const bool diag = lt == J;
    // w = Y_a[J] + sum_l conj(v_lJ) Y_b[l]
    row_allreduce<VG>(
        [&](int c) -> zd {
          if (c >= NB) return zd{0.0, 0.0};
          const zd p = zcjmac(vj, yb[c], zd{0.0, 0.0});
          const zd yac = ya[J * kLd + c];
          return diag ? zd{p.re + yac.re, p.im + yac.im} : p;
        },
        lt, red);
    const zd tj = tau[J];
    const zd tv = zmul(tj, vj);
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const zd wc = zd{red[2 * c], red[2 * c + 1]};
      yb[c] = zsubmul(yb[c], tv, wc);
      if (diag) ya[J * kLd + c] = zsubmul(ya[J * kLd + c], tj, wc);
    }
    tapply_cols<NB, J - 1>(yb, v, lt, red, ya, tau);
  }
}

template <int NB>
__global__ __launch_bounds__(64, 2) void k_ctree_apply(int64_t P, int64_t h, int64_t ncomb,
                                                    zd* __restrict__ Cn,
                                                    const zd* __restrict__ Vn) {
  __shared__ double red[4][32];
  __shared__ zd ya[4][16 * kLd];
  __shared__ zd tau[4][16];
  const int lane = threadIdx.x, g = lane >> 4, lt = lane & 15;
  const int64_t c = (int64_t)blockIdx.x * 4 + g, f = blockIdx.y;
  const bool active = c < ncomb;
  const int64_t j = c * 2 * h, s = j + h;
  const bool io = active && lt < NB;
  zd* Cj = Cn + (f * P + j) * kNodeZ + lt * 16;
  zd* Cs = Cn + (f * P + s) * kNodeZ + lt * 16;
  const zd* V = Vn + (f * P + s) * kVnZ;
  zd v[NB], yb[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    v[k] = zd{0.0, 0.0};
    yb[k] = zd{0.0, 0.0};
    ya[g][lt * kLd + k] = zd{0.0, 0.0};
  }
  tau[g][lt] = zd{0.0, 0.0};
  if (io) {
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      v[k] = V[lt * 16 + k];
      ya[g][lt * kLd + k] = Cj[k];
    }
    tau[g][lt] = V[16 * 16 + lt];
  }
  wave_lds_sync();
  tapply_cols<NB, NB - 1>(yb, v, lt, red[g], ya[g], tau[g]);
  wave_lds_sync();
  if (io) {
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      Cj[k] = ya[g][lt * kLd + k];
      Cs[k] = yb[k];
    }
  }
}

int64_t combines_at(int64_t P, int64_t h) { return P > h ? (P - h - 1) / (2 * h) + 1 : 0; }

template <typename T>
hipError_t leaf_dispatch(int apply, int nb, dim3 grid, hipStream_t st, int64_t m, int64_t ldm,
                         int64_t P, const T* E, zd* Rn, T* Vl, zd* Wl, const zd* Cn, T* modes) {
  switch (nb) {
#define PYLOM_CLEAF(K)                                                                         \
  case K:                                                                                      \
    if (apply)                                                                                 \
      hipLaunchKernelGGL((k_cleaf_apply<T, K>), grid, dim3(64), 0, st, m, P, Vl, Wl, Cn,       \
                         modes);                                                               \
    else                                                                                       \
      hipLaunchKernelGGL((k_cleaf_factor<T, K>), grid, dim3(64), 0, st, m, ldm, P, E, Rn, Vl, \
                         Wl);                                                                  \
    break;
    PYLOM_CLEAF(1) PYLOM_CLEAF(2) PYLOM_CLEAF(3) PYLOM_CLEAF(4) PYLOM_CLEAF(5) PYLOM_CLEAF(6)
    PYLOM_CLEAF(7) PYLOM_CLEAF(8) PYLOM_CLEAF(9) PYLOM_CLEAF(10) PYLOM_CLEAF(11)
    PYLOM_CLEAF(12) PYLOM_CLEAF(13) PYLOM_CLEAF(14) PYLOM_CLEAF(15) PYLOM_CLEAF(16)
#undef PYLOM_CLEAF
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

int64_t ctsqr_leaves(int64_t m) { return (m + kLeafRows - 1) / kLeafRows; }
size_t ctsqr_node_bytes() { return sizeof(zd) * kNodeZ; }
size_t ctsqr_vnode_bytes() { return sizeof(zd) * kVnZ; }

size_t ctsqr_leaf_v_bytes(int nb, int t_f64) {
  return (size_t)nb * kLeafRows * 2 * (t_f64 ? 8 : 4);
}

hipError_t launch_cleaf(int t_f64, int apply, int nb, int64_t m, int64_t ldm, int64_t P,
                        int64_t nf, const void* E, double* Rn, void* Vl, double* Wl,
                        const double* Cn, void* modes, hipStream_t st) {
  if (nb < 1 || nb > 16 || P != ctsqr_leaves(m) || ldm < m || nf < 1 || nf > 65535 ||
      P > 0x7fffffff || !Vl || !Wl)
    return hipErrorInvalidValue;
  if (apply ? (!Cn || !modes) : (!Rn || !E)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)P, (unsigned)nf);
  zd* R = reinterpret_cast<zd*>(Rn);
  zd* W = reinterpret_cast<zd*>(Wl);
  const zd* C = reinterpret_cast<const zd*>(Cn);
  if (t_f64)
    return leaf_dispatch<double>(apply, nb, grid, st, m, ldm, P, (const double*)E, R,
                                 (double*)Vl, W, C, (double*)modes);
  return leaf_dispatch<float>(apply, nb, grid, st, m, ldm, P, (const float*)E, R, (float*)Vl, W,
                              C, (float*)modes);
}

hipError_t launch_ctree_combine(int nb, int64_t P, int64_t h, int64_t nf, double* Rn,
                                double* Vn, hipStream_t st) {
  const int64_t nc = combines_at(P, h);
  if (nc == 0) return hipSuccess;
  if (nb < 1 || nb > 16 || nf < 1 || nf > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((nc + 3) / 4), (unsigned)nf);
  zd* R = reinterpret_cast<zd*>(Rn);
  zd* V = reinterpret_cast<zd*>(Vn);
  switch (nb) {
#define PYLOM_CCOMB(K)                                                                  \
  case K:                                                                               \
    hipLaunchKernelGGL(k_ctree_combine<K>, grid, dim3(64), 0, st, P, h, nc, R, V);     \
    break;
    PYLOM_CCOMB(1) PYLOM_CCOMB(2) PYLOM_CCOMB(3) PYLOM_CCOMB(4) PYLOM_CCOMB(5) PYLOM_CCOMB(6)
    PYLOM_CCOMB(7) PYLOM_CCOMB(8) PYLOM_CCOMB(9) PYLOM_CCOMB(10) PYLOM_CCOMB(11)
    PYLOM_CCOMB(12) PYLOM_CCOMB(13) PYLOM_CCOMB(14) PYLOM_CCOMB(15) PYLOM_CCOMB(16)
#undef PYLOM_CCOMB
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ctree_apply(int nb, int64_t P, int64_t h, int64_t nf, double* Cn,
                              const double* Vn, hipStream_t st) {
  const int64_t nc = combines_at(P, h);
  if (nc == 0) return hipSuccess;
  if (nb < 1 || nb > 16 || nf < 1 || nf > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((nc + 3) / 4), (unsigned)nf);
  zd* C = reinterpret_cast<zd*>(Cn);
  const zd* V = reinterpret_cast<const zd*>(Vn);
  switch (nb) {
#define PYLOM_CAPPLY(K)                                                                \
  case K:                                                                              \
    hipLaunchKernelGGL(k_ctree_apply<K>, grid, dim3(64), 0, st, P, h, nc, C, V);      \
    break;
    PYLOM_CAPPLY(1) PYLOM_CAPPLY(2) PYLOM_CAPPLY(3) PYLOM_CAPPLY(4) PYLOM_CAPPLY(5)
    PYLOM_CAPPLY(6) PYLOM_CAPPLY(7) PYLOM_CAPPLY(8) PYLOM_CAPPLY(9) PYLOM_CAPPLY(10)
    PYLOM_CAPPLY(11) PYLOM_CAPPLY(12) PYLOM_CAPPLY(13) PYLOM_CAPPLY(14) PYLOM_CAPPLY(15)
    PYLOM_CAPPLY(16)
#undef PYLOM_CAPPLY
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pylom
