// spod.hip -- SPOD front end and root stage (Alg. 6 with the SVD of the
// spectral matrices, Sec. 2.3 and Eq. csdimp).
//
// Front end (k_spod_fft): for every point p the temporal mean is removed
// (optional), the series is cut into nBlks Welch blocks of npwin samples
// starting every npwin - nolap samples, each block is windowed, and the
// one-sided spectrum q_f = c_f DFT_f(w x) / sum(w) / sqrt(nBlks)
// (c_f = 2 for 0 < f < npwin/2, else 1) is kept for f = 0..npwin/2.
//
// The real block of N = npwin samples is transformed as one complex sequence
// of N2 = N/2 values z_n = y_{2n} + i y_{2n+1} (y = w x, the window carrying
// the scale 1/(sum(w) sqrt(nBlks))), Z = DFT_N2(z), and split:
// Y_k = (Z_k + conj Z_{N2-k})/2 + W_N^k (Z_k - conj Z_{N2-k})/(2i).
// The N2-point DFT runs in registers on a group of G lanes per point (C = N2/G
// values per lane, n = C q + n2 for lane q of the group): a radix-2
// decimation-in-frequency exchange across the G lanes, the twiddles
// W_N2^(n2 k1), then a C-point radix-2 DFT inside each lane, so lane q ends
// with Z_(k1 + G k2), k1 the bit reversal of q.  A wave holds 64/G points;
// for one frequency and block its 64/G consecutive points are written as one
// contiguous run of the column-major spectral matrix (column (f, blk) of ld
// ldm complex values).
//
// Root stage: the nb x nb complex root factor R of a frequency's TSQR is
// embedded as the real 2nb x 2nb matrix [[Re R, -Im R], [Im R, Re R]] (it maps
// [Re z; Im z] to [Re Rz; Im Rz]), whose singular values are those of R, each
// twice; a singular pair at index 2c de-embeds to a complex pair
// (e^{i theta} u_c, e^{i theta} v_c) of R.  k_spod_root_modes fixes the phase
// so that the largest-|.| entry of v_c (lowest index on ties) is real
// positive, writes the phase-fixed U_R as the root factor of the down-tree
// apply, and L[f][c] = S[2c]^2.  k_spod_order fills the frequency axis and the
// frequency order by leading energy L[f][0] (descending, ties by ascending
// frequency).
#include "common.hpp"
#include "kernels.hpp"

namespace pylom {

namespace {

template <typename T>
struct Cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return Cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

constexpr int bitrev_c(int i, int n) {
  int r = 0;
  for (int b = 1, rb = n >> 1; b < n; b <<= 1, rb >>= 1)
    if (i & b) r |= rb;
  return r;
}

template <typename T>
struct T2v;
template <>
struct T2v<float> {
  typedef float2 type;
};
template <>
struct T2v<double> {
  typedef double2 type;
};

// cos and sin of 2 pi e / L at compile time: reduction to a quadrant and to
// an angle in [0, pi/4] (complement otherwise), then the Taylor series (the
// 15th term is below 1e-20 there).
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double taylor_sin(double x) {
  double t = x, s = x;
  for (int k = 1; k < 15; ++k) {
    t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    s += t;
  }
  return s;
}
constexpr double taylor_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int k = 1; k < 15; ++k) {
    t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    s += t;
  }
  return s;
}
constexpr void cossin_2pi(int e, int L, double& c, double& s) {
  e %= L;
  const int qd = (4 * e) / L, r = 4 * e - qd * L;  // angle = (pi/2)(qd + r/L)
  double c0, s0;
  if (2 * r <= L) {
    const double th = 0.5 * kPi * (double)r / (double)L;
    c0 = taylor_cos(th);
    s0 = taylor_sin(th);
  } else {
    const double ph = 0.5 * kPi * (double)(L - r) / (double)L;
    c0 = taylor_sin(ph);
    s0 = taylor_cos(ph);
  }
  switch (qd) {
    case 0: c = c0; s = s0; break;
    case 1: c = -s0; s = c0; break;
    case 2: c = -c0; s = -s0; break;
    default: c = s0; s = -c0; break;
  }
}
// W_C^e = exp(-2 pi i e / C), e < C/2
template <int C>
struct InlaneTwiddles {
  double re[C / 2 + 1], im[C / 2 + 1];
  constexpr InlaneTwiddles() : re(), im() {
    for (int e = 0; e < C / 2; ++e) {
      double c = 0.0, sn = 0.0;
      cossin_2pi(e, C, c, sn);
      re[e] = c;
      im[e] = -sn;
    }
  }
};

// C-point radix-2 DFT of z inside one lane (decimation in time, natural-order
// output) with compile-time twiddles.
template <typename T, int C>
__device__ __forceinline__ void fft_inlane(Cx<T> (&z)[C]) {
  constexpr InlaneTwiddles<C> tw{};
  Cx<T> y[C];
#pragma unroll
  for (int i = 0; i < C; ++i) y[bitrev_c(i, C)] = z[i];
#pragma unroll
  for (int L = 2; L <= C; L <<= 1) {
#pragma unroll
    for (int s0 = 0; s0 < C; s0 += L) {
#pragma unroll
      for (int e = 0; e < L / 2; ++e) {
        Cx<T> bb = y[s0 + e + L / 2];
        if (e != 0) bb = cmul(bb, Cx<T>{(T)tw.re[e * (C / L)], (T)tw.im[e * (C / L)]});
        const Cx<T> aa = y[s0 + e];
        y[s0 + e] = Cx<T>{aa.re + bb.re, aa.im + bb.im};
        y[s0 + e + L / 2] = Cx<T>{aa.re - bb.re, aa.im - bb.im};
      }
    }
  }
#pragma unroll
  for (int i = 0; i < C; ++i) z[i] = y[i];
}

// Value of lane ^ H inside the group (DPP quad permutations for H = 1, 2).
template <int H, typename T>
__device__ __forceinline__ T lane_xor(T v) {
  if constexpr (H == 1) return dpp<0xB1>(v);
  else if constexpr (H == 2) return dpp<0x4E>(v);
  else return __shfl_xor(v, H, 64);
}

// Radix-2 decimation-in-frequency stages across the G lanes of a group,
// exchange distance HALF down to 1: the lower lane keeps a + b, the upper
// (b - a) W_(2 HALF)^(q mod HALF).
template <typename T, int C, int N, int HALF>
__device__ __forceinline__ void dif_lanes(Cx<T> (&z)[C], int q, const Cx<T>* tws) {
  if constexpr (HALF >= 1) {
    // d = s z + o with s = -1 on the upper lanes; their twiddle is 1 on the
    // lower lanes and at the last stage (W_2^0), where no product is taken
    const bool up = (q & HALF) != 0;
    const T sg = up ? T(-1) : T(1);
    const Cx<T> w = up ? tws[(q & (HALF - 1)) * (N / (2 * HALF))] : Cx<T>{T(1), T(0)};
#pragma unroll
    for (int n2 = 0; n2 < C; ++n2) {
      const T ore = lane_xor<HALF>(z[n2].re);
      const T oim = lane_xor<HALF>(z[n2].im);
      const Cx<T> d = {fma(sg, z[n2].re, ore), fma(sg, z[n2].im, oim)};
      if constexpr (HALF == 1) z[n2] = d;
      else z[n2] = cmul(d, w);
    }
    dif_lanes<T, C, N, HALF / 2>(z, q, tws);
  }
}

// tab: W_N^t (re, im) for t < N, then the window w_j, j < N; copied to LDS.
// VEC: D rows and block starts are 16-byte aligned (float4 loads).
template <typename T, int G, int C, bool VEC>
__global__ __launch_bounds__(256, 3) void k_spod_fft(int64_t m, int64_t nt, const float* __restrict__ D,
                                                  int64_t ldd, int step, int nb, int remove_mean,
                                                  const T* __restrict__ tab,
                                                  const double* __restrict__ scl,
                                                  T* __restrict__ E, int64_t ldm) {
  constexpr int N2 = G * C, N = 2 * N2, PW = 64 / G;
  typedef typename T2v<T>::type TT;
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* tws = reinterpret_cast<Cx<T>*>(smem);
  T* win = reinterpret_cast<T*>(tws + N);
  for (int t = threadIdx.x; t < 3 * N; t += 256) reinterpret_cast<T*>(smem)[t] = tab[t];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane % G;
  const int64_t p = ((int64_t)blockIdx.x * 4 + wave) * PW + lane / G;
  const bool valid = p < m;
  const float* row = D + (valid ? p : 0) * ldd;
  double mu = 0.0;
  if (remove_mean) {
    double acc = 0.0;
    int64_t t0 = 0;
    if constexpr (VEC) {
      const float4* r4 = reinterpret_cast<const float4*>(row);
      const int64_t nt4 = nt / 4;
      // unrolled so that several loads are in flight; the sum order is the
      // loop order either way
#pragma unroll 4
      for (int64_t t = q; t < nt4; t += G) {
        const float4 v = r4[t];
        acc += ((double)v.x + (double)v.y) + ((double)v.z + (double)v.w);
      }
      t0 = 4 * nt4;
    }
    for (int64_t t = t0 + q; t < nt; t += G) acc += (double)row[t];
    mu = group_sum<G>(acc) / (double)nt;
  }
  // x - mu: in FP64 for T = double; for T = float as (x - mu_hi) - mu_lo with
  // mu = mu_hi + mu_lo split into floats (error below one float rounding of
  // the exact difference)
  const float mu_hi = (float)mu, mu_lo = (float)(mu - (double)mu_hi);
  auto centred = [&](float v) -> T {
    if constexpr (sizeof(T) == 8) return (double)v - mu;
    else return (v - mu_hi) - mu_lo;
  };
  const int64_t fstride = (int64_t)G * nb * ldm;  // elements between k and k + G
  for (int b = 0; b < nb; ++b) {
    // lane-dependent addresses and the window and twiddle values are rebuilt
    // every block (an opaque copy of the lane index) instead of being held in
    // registers across the loop
    asm volatile("" ::: "memory");
    int qv = q;
    asm volatile("" : "+v"(qv));
    const int k1 = bitrev_c(qv, G);
    const float* x = row + (int64_t)b * step + 2 * C * qv;
    const T* wq = win + 2 * C * qv;
    TT* out = reinterpret_cast<TT*>(E) + ((int64_t)k1 * nb + b) * ldm + p;
    Cx<T> z[C];
    if constexpr (VEC) {
#pragma unroll
      for (int i = 0; i < C / 2; ++i) {
        const float4 v = reinterpret_cast<const float4*>(x)[i];
        z[2 * i].re = centred(v.x) * wq[4 * i];
        z[2 * i].im = centred(v.y) * wq[4 * i + 1];
        z[2 * i + 1].re = centred(v.z) * wq[4 * i + 2];
        z[2 * i + 1].im = centred(v.w) * wq[4 * i + 3];
      }
    } else {
#pragma unroll
      for (int n2 = 0; n2 < C; ++n2) {
        z[n2].re = centred(x[2 * n2]) * wq[2 * n2];
        z[n2].im = centred(x[2 * n2 + 1]) * wq[2 * n2 + 1];
      }
    }
    if constexpr (G > 1) {
      dif_lanes<T, C, N, G / 2>(z, qv, tws);
#pragma unroll
      for (int n2 = 1; n2 < C; ++n2) {
        asm volatile("" ::: "memory");  // load each twiddle next to its use
        z[n2] = cmul(z[n2], tws[2 * ((n2 * k1) & (N2 - 1))]);
      }
    }
    fft_inlane<T, C>(z);
    // real-input split: Z_(N2-k) is z[(C - k2) mod C] of this lane when
    // k1 = 0, else z[C - 1 - k2] of the lane holding k1' = G - k1
#pragma unroll
    for (int k2 = 0; k2 < C; ++k2) {
      asm volatile("" ::: "memory");
      Cx<T> pz = z[(C - k2) & (C - 1)];
      if constexpr (G == 4) {
        // lanes (0, 1, 2, 3) hold k1 = (0, 2, 1, 3); partners (0, 1, 3, 2)
        const T rre = dpp<0xB4>(z[C - 1 - k2].re);
        const T rim = dpp<0xB4>(z[C - 1 - k2].im);
        if (qv != 0) pz = Cx<T>{rre, rim};
      } else if constexpr (G == 2) {
        if (qv != 0) pz = z[C - 1 - k2];
      } else if constexpr (G > 4) {
        const int src = lane - qv + bitrev_c((G - k1) & (G - 1), G);
        const T rre = __shfl(z[C - 1 - k2].re, src, 64);
        const T rim = __shfl(z[C - 1 - k2].im, src, 64);
        if (qv != 0) pz = Cx<T>{rre, rim};
      }
      // 2 Ev = Z_k + conj Z_(N2-k), 2 O = (Z_k - conj Z_(N2-k)) / i; the
      // one-sided factor c_k = 2 (1 at k = 0) cancels the halves, and the
      // scale 1 / (sum(w) sqrt(nBlks)) is in the window
      const Cx<T> A = z[k2];
      const Cx<T> E2 = {A.re + pz.re, A.im - pz.im};
      const Cx<T> O2 = {A.im + pz.im, pz.re - A.re};
      const int k = k1 + G * k2;
      const Cx<T> wo = cmul(tws[k], O2);
      const T h = k == 0 ? T(0.5) : T(1);
      if (valid) {
        TT v;
        v.x = (E2.re + wo.re) * h;
        v.y = (E2.im + wo.im) * h;
        *out = v;
      }
      out += fstride;
    }
    if (valid && qv == 0) {
      TT v;
      v.x = z[0].re - z[0].im;
      v.y = T(0);
      reinterpret_cast<TT*>(E)[((int64_t)N2 * nb + b) * ldm + p] = v;
    }
  }
}

// Twiddles W_N^t in FP64, rounded to T, and the window w_j / (sum(w)
// sqrt(nb)) (the spectral scale folded in; sums and products in FP64, then
// rounded to T); scl[0] = 1 / (sum(w) sqrt(nb)).
template <typename T>
__global__ __launch_bounds__(256) void k_spod_tables(int N, int window, int nb, T* __restrict__ tab,
                                                     double* __restrict__ scl) {
  __shared__ double part[4];
  const double a0 = window == 1 ? 0.54 : 0.5, a1 = window == 1 ? 0.46 : 0.5;
  double acc = 0.0;
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    double sv, cv;
    sincospi(-2.0 * (double)t / (double)N, &sv, &cv);
    tab[2 * t] = (T)cv;
    tab[2 * t + 1] = (T)sv;
    acc += a0 - a1 * cospi(2.0 * (double)t / (double)(N - 1));
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  const double scale = 1.0 / ((part[0] + part[1] + part[2] + part[3]) * sqrt((double)nb));
  for (int t = threadIdx.x; t < N; t += blockDim.x)
    tab[2 * N + t] = (T)((a0 - a1 * cospi(2.0 * (double)t / (double)(N - 1))) * scale);
  if (threadIdx.x == 0) scl[0] = scale;
}

// values per lane: at most 32 (FP32) or 16 (FP64; 32 at N2 = 2048, where 64
// lanes per point is the limit), at least two lanes per point from N2 = 32
// (FP32) or 16 (FP64) on, which keeps the register count of a lane down
constexpr int fft_c(bool f64, int N2) {
  return f64 ? (N2 <= 8 ? N2 : (N2 == 16 ? 8 : (N2 >= 2048 ? 32 : 16)))
             : (N2 <= 16 ? N2 : (N2 == 32 ? 16 : 32));
}

template <typename T, int N2>
hipError_t fft_launch(int64_t m, int64_t nt, const float* D, int64_t ldd, int step, int nb,
                      int remove_mean, const T* tab, const double* scl, T* E, int64_t ldm,
                      hipStream_t st) {
  constexpr int C = fft_c(sizeof(T) == 8, N2), G = N2 / C, PW = 64 / G;
  const int64_t blocks = (m + 4 * PW - 1) / (4 * PW);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = (size_t)3 * 2 * N2 * sizeof(T);
  const bool vec = ((uintptr_t)D % 16 == 0) && ldd % 4 == 0 && step % 4 == 0;
  const void* fn = vec ? (const void*)k_spod_fft<T, G, C, true> : (const void*)k_spod_fft<T, G, C, false>;
  if (lds > 64 * 1024) {
    const hipError_t e =
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (vec)
    hipLaunchKernelGGL((k_spod_fft<T, G, C, true>), dim3((unsigned)blocks), dim3(256), lds, st, m,
                       nt, D, ldd, step, nb, remove_mean, tab, scl, E, ldm);
  else
    hipLaunchKernelGGL((k_spod_fft<T, G, C, false>), dim3((unsigned)blocks), dim3(256), lds, st, m,
                       nt, D, ldd, step, nb, remove_mean, tab, scl, E, ldm);
  return hipGetLastError();
}

template <typename T>
hipError_t fft_dispatch(int npwin, int64_t m, int64_t nt, const float* D, int64_t ldd, int step,
                        int nb, int remove_mean, const T* tab, const double* scl, T* E,
                        int64_t ldm, hipStream_t st) {
  switch (npwin / 2) {
#define PYLOM_FFT(K) \
  case K:            \
    return fft_launch<T, K>(m, nt, D, ldd, step, nb, remove_mean, tab, scl, E, ldm, st);
    PYLOM_FFT(2) PYLOM_FFT(4) PYLOM_FFT(8) PYLOM_FFT(16) PYLOM_FFT(32) PYLOM_FFT(64)
    PYLOM_FFT(128) PYLOM_FFT(256) PYLOM_FFT(512) PYLOM_FFT(1024) PYLOM_FFT(2048)
#undef PYLOM_FFT
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

size_t spod_table_bytes(int npwin, int t_f64) { return (size_t)3 * npwin * (t_f64 ? 8 : 4); }

hipError_t launch_spod_front(int t_f64, int64_t m, int64_t nt, const float* D, int64_t ldd,
                             int npwin, int nolap, int nb, int window, int remove_mean, void* tab,
                             double* scl, void* E, int64_t ldm, hipStream_t st) {
  if (npwin < 4 || npwin > 4096 || (npwin & (npwin - 1)) || nolap < 0 || nolap >= npwin ||
      nb < 1 || ldm < m || (int64_t)(nb - 1) * (npwin - nolap) + npwin > nt)
    return hipErrorInvalidValue;
  const int step = npwin - nolap;
  if (t_f64) {
    hipLaunchKernelGGL(k_spod_tables<double>, dim3(1), dim3(256), 0, st, npwin, window, nb,
                       (double*)tab, scl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return fft_dispatch<double>(npwin, m, nt, D, ldd, step, nb, remove_mean, (const double*)tab,
                                scl, (double*)E, ldm, st);
  }
  hipLaunchKernelGGL(k_spod_tables<float>, dim3(1), dim3(256), 0, st, npwin, window, nb,
                     (float*)tab, scl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return fft_dispatch<float>(npwin, m, nt, D, ldd, step, nb, remove_mean, (const float*)tab, scl,
                             (float*)E, ldm, st);
}

// Rr[f] (2nb x 2nb, row-major) = [[X, -Y], [Y, X]] for R = X + iY, the root
// block Rn[f * P] (16 x 16 complex, row-major).
__global__ void k_spod_root_realify(int nb, int64_t P, const double* __restrict__ Rn,
                                    double* __restrict__ Rr) {
  const int64_t f = blockIdx.x;
  const int n = 2 * nb;
  const double* R = Rn + f * P * 512;
  double* A = Rr + f * n * n;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, t = idx % n;
    const int ii = i % nb, tt = t % nb;
    const double re = R[2 * (ii * 16 + tt)], im = R[2 * (ii * 16 + tt) + 1];
    const bool top = i < nb, left = t < nb;
    A[idx] = top == left ? re : (top ? -im : im);
  }
}

hipError_t launch_spod_root_realify(int nb, int64_t P, int64_t nf, const double* Rn, double* Rr,
                                    hipStream_t st) {
  hipLaunchKernelGGL(k_spod_root_realify, dim3((unsigned)nf), dim3(256), 0, st, nb, P, Rn, Rr);
  return hipGetLastError();
}

// From the SVD of frequency f's embedded root (S, VT, UR; n = 2 nb): the
// phase-fixed complex U_R into the root block of Cn (16 x 16 complex), and L.
__global__ void k_spod_root_modes(int nb, int64_t P, const double* __restrict__ S,
                                  const double* __restrict__ VT, const double* __restrict__ UR,
                                  double* __restrict__ Cn, double* __restrict__ L) {
  __shared__ double ph_re[16], ph_im[16];
  const int64_t f = blockIdx.x;
  const int n = 2 * nb;
  const double* vt = VT + f * n * n;
  const double* ur = UR + f * n * n;
  if (threadIdx.x < nb) {
    const int c = threadIdx.x;
    const double* v = vt + (int64_t)(2 * c) * n;
    double best = -1.0;
    int bi = 0;
    for (int t = 0; t < nb; ++t) {
      const double a = hypot(v[t], v[nb + t]);
      if (a > best) {
        best = a;
        bi = t;
      }
    }
    double cr = 1.0, ci = 0.0;  // conj(phase)
    if (best > 0.0) {
      cr = v[bi] / best;
      ci = -v[nb + bi] / best;
    }
    ph_re[c] = cr;
    ph_im[c] = ci;
    const double sc = S[f * n + 2 * c];
    L[f * nb + c] = sc * sc;
  }
  __syncthreads();
  double* C = Cn + f * P * 512;
  for (int idx = threadIdx.x; idx < nb * nb; idx += blockDim.x) {
    const int i = idx / nb, c = idx % nb;
    const double ure = ur[(int64_t)i * n + 2 * c], uim = ur[(int64_t)(nb + i) * n + 2 * c];
    const double cr = ph_re[c], ci = ph_im[c];
    C[2 * (i * 16 + c)] = ure * cr - uim * ci;
    C[2 * (i * 16 + c) + 1] = ure * ci + uim * cr;
  }
}

hipError_t launch_spod_root_modes(int nb, int64_t P, int64_t nf, const double* S, const double* VT,
                                  const double* UR, double* Cn, double* L, hipStream_t st) {
  if (nb < 1 || nb > 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_spod_root_modes, dim3((unsigned)nf), dim3(64), 0, st, nb, P, S, VT, UR, Cn,
                     L);
  return hipGetLastError();
}

// freqs[f] = f / (dt npwin); order = frequencies by L[f][0] descending, ties
// by ascending f.  One workgroup.
__global__ void k_spod_order(int nf, int nb, double dt, int npwin, const double* __restrict__ L,
                             double* __restrict__ freqs, int64_t* __restrict__ order) {
  for (int f = threadIdx.x; f < nf; f += blockDim.x) {
    if (freqs) freqs[f] = (double)f / (dt * (double)npwin);
    const double e = L[(int64_t)f * nb];
    int r = 0;
    for (int g = 0; g < nf; ++g) {
      const double eg = L[(int64_t)g * nb];
      r += (eg > e) || (eg == e && g < f);
    }
    if (order) order[r] = f;
  }
}

hipError_t launch_spod_order(int nf, int nb, double dt, int npwin, const double* L, double* freqs,
                             int64_t* order, hipStream_t st) {
  hipLaunchKernelGGL(k_spod_order, dim3(1), dim3(256), 0, st, nf, nb, dt, npwin, L, freqs, order);
  return hipGetLastError();
}

}  // namespace pylom
