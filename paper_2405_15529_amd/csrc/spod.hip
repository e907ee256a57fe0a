// spod.hip -- SPOD front end and back end (Alg. 6 with the SVD of the
// spectral matrices, Sec. 2.3 and Eq. csdimp).
//
// Front end (k_spod_fft): for every point p the temporal mean is removed
// (optional), the series is cut into nBlks Welch blocks of npwin samples
// starting every npwin - nolap samples, each block is windowed and
// transformed with a radix-2 Stockham FFT in LDS (one wave per point), and
// the one-sided spectrum q_f = c_f DFT_f(w x) / sum(w) / sqrt(nBlks)
// (c_f = 2 for 0 < f < npwin/2, else 1) is kept for f = 0..npwin/2.
//
// The complex tall-skinny SVD of each frequency's m x nBlks matrix
// Q_f = X + iY is computed as the real SVD of its realification: the
// 2m x 2nBlks matrix whose rows 2p and 2p+1 are [X_p, -Y_p] and [Y_p, X_p].
// It maps [Re z; Im z] to the interleaved (Re, Im) parts of Q_f z, so every
// singular value of Q_f appears twice, and a left/right singular pair of the
// realification at index 2c de-embeds to a complex pair (e^{i theta} u_c,
// e^{i theta} v_c) of Q_f.  The front end writes each frequency's
// realification row-contiguously (the per-point staging in LDS turns the
// frequency-major scatter into 4 nBlks contiguous values per frequency).
//
// Back end: k_spod_modes de-embeds mode c from column c of the realified U
// (built from the even columns of U_R) and column 2c of V, fixes the phase so
// that the largest-|.| entry of v_c (lowest index on ties) is real positive,
// and writes L[f][c] = S_f[2c]^2; k_spod_order fills the frequency axis and
// the frequency order by leading energy L[f][0] (descending, ties by
// ascending frequency).
#include "common.hpp"
#include "kernels.hpp"

namespace pylom {

namespace {
constexpr int SW = 4;  // waves (points) per front-end workgroup
}

template <typename T>
struct Cplx {
  T re, im;
};

// LDS carve per workgroup: twiddles (npwin/2), window (npwin), then per wave
// two FFT buffers (2 * npwin) and the spectra staging (nf * nb).
size_t spod_fft_lds_bytes(int npwin, int nb, int esize) {
  const int nf = npwin / 2 + 1;
  const size_t c = (size_t)2 * esize;  // one complex value
  return c * (npwin / 2) + (size_t)esize * npwin + SW * c * ((size_t)2 * npwin + (size_t)nf * nb);
}

template <typename T>
__global__ __launch_bounds__(64 * SW) void k_spod_fft(int64_t m, int64_t nt, const float* __restrict__ D,
                                                      int64_t ldd, int npwin, int logn, int step,
                                                      int nb, int window, int remove_mean,
                                                      T* __restrict__ E, int64_t ldE,
                                                      int64_t sE) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nf = npwin / 2 + 1;
  Cplx<T>* tw = reinterpret_cast<Cplx<T>*>(smem);
  T* win = reinterpret_cast<T*>(tw + npwin / 2);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  Cplx<T>* buf0 = reinterpret_cast<Cplx<T>*>(win + npwin) + (size_t)wave * (2 * npwin + nf * nb);
  Cplx<T>* buf1 = buf0 + npwin;
  Cplx<T>* stage = buf1 + npwin;  // [f][blk]

  // twiddles exp(-2 pi i k / npwin) and the window (FP64 evaluation)
  for (int k = tid; k < npwin / 2; k += 64 * SW) {
    double sv, cv;
    sincospi(-2.0 * (double)k / (double)npwin, &sv, &cv);
    tw[k].re = (T)cv;
    tw[k].im = (T)sv;
  }
  const double a0 = window == 1 ? 0.54 : 0.5, a1 = window == 1 ? 0.46 : 0.5;
  for (int j = tid; j < npwin; j += 64 * SW)
    win[j] = (T)(a0 - a1 * cospi(2.0 * (double)j / (double)(npwin - 1)));
  __syncthreads();
  // sum of the window (every wave computes it; FP64)
  double wsum = 0.0;
  for (int j = lane; j < npwin; j += 64) wsum += (double)win[j];
  wsum = wave_sum(wsum);
  const double base_scale = 1.0 / (wsum * sqrt((double)nb));

  const int64_t p = (int64_t)blockIdx.x * SW + wave;
  if (p >= m) return;  // no block-wide barrier below this point
  const float* row = D + p * ldd;
  double mu = 0.0;
  if (remove_mean) {
    double acc = 0.0;
    for (int64_t t = lane; t < nt; t += 64) acc += (double)row[t];
    mu = wave_sum(acc) / (double)nt;
  }
  for (int b = 0; b < nb; ++b) {
    const int64_t i0 = (int64_t)b * step;
    for (int j = lane; j < npwin; j += 64) {
      buf0[j].re = (T)(((double)row[i0 + j] - mu) * (double)win[j]);
      buf0[j].im = T(0);
    }
    wave_lds_sync();
    Cplx<T>* src = buf0;
    Cplx<T>* dst = buf1;
    for (int ls = 0; ls < logn; ++ls) {
      const int Ns = 1 << ls;
      for (int jj = lane; jj < npwin / 2; jj += 64) {
        const Cplx<T> x0 = src[jj];
        const Cplx<T> x1 = src[jj + npwin / 2];
        const int k = jj & (Ns - 1);
        const Cplx<T> w = tw[k << (logn - 1 - ls)];
        const T yr = x1.re * w.re - x1.im * w.im;
        const T yi = x1.re * w.im + x1.im * w.re;
        const int d = ((jj - k) << 1) + k;
        dst[d].re = x0.re + yr;
        dst[d].im = x0.im + yi;
        dst[d + Ns].re = x0.re - yr;
        dst[d + Ns].im = x0.im - yi;
      }
      wave_lds_sync();
      Cplx<T>* t = src;
      src = dst;
      dst = t;
    }
    for (int f = lane; f < nf; f += 64) {
      const T sc = (T)(((f > 0 && f < npwin / 2) ? 2.0 : 1.0) * base_scale);
      stage[f * nb + b].re = src[f].re * sc;
      stage[f * nb + b].im = src[f].im * sc;
    }
    wave_lds_sync();
  }
  // rows 2p and 2p+1 of every frequency's realification: 4 nb contiguous values
  const int ncol = 2 * nb;
  for (int f = 0; f < nf; ++f) {
    T* dstE = E + (int64_t)f * sE + 2 * p * ldE;
    for (int t = lane; t < 2 * ncol; t += 64) {
      const int r = t / ncol, c = t % ncol;
      const int blk = c < nb ? c : c - nb;
      const Cplx<T> q = stage[f * nb + blk];
      T v;
      if (r == 0) v = c < nb ? q.re : -q.im;
      else v = c < nb ? q.im : q.re;
      dstE[(int64_t)r * ldE + c] = v;
    }
  }
}

hipError_t launch_spod_fft(int e_f64, int64_t m, int64_t nt, const float* D, int64_t ldd,
                           int npwin, int nolap, int nb, int window, int remove_mean, void* E,
                           int64_t ldE, int64_t sE, hipStream_t st) {
  int logn = 0;
  while ((1 << logn) < npwin) ++logn;
  if ((1 << logn) != npwin || npwin < 4) return hipErrorInvalidValue;
  const size_t lds = spod_fft_lds_bytes(npwin, nb, e_f64 ? 8 : 4);
  const dim3 grid((unsigned)((m + SW - 1) / SW)), block(64 * SW);
  const int step = npwin - nolap;
  if (e_f64) {
    hipError_t e = hipFuncSetAttribute((const void*)k_spod_fft<double>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_spod_fft<double>, grid, block, lds, st, m, nt, D, ldd, npwin, logn, step,
                       nb, window, remove_mean, (double*)E, ldE, sE);
  } else {
    hipError_t e = hipFuncSetAttribute((const void*)k_spod_fft<float>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_spod_fft<float>, grid, block, lds, st, m, nt, D, ldd, npwin, logn, step,
                       nb, window, remove_mean, (float*)E, ldE, sE);
  }
  return hipGetLastError();
}

// W of every problem's tree root: the even columns of U_R (one per complex
// mode): W[i][c] = UR[i][2c], i < n, c < nb.
__global__ void k_select_even(int n, int nb, const double* __restrict__ UR, int64_t sUR,
                              double* __restrict__ W, int64_t ldw, int64_t sW) {
  const int64_t f = blockIdx.y;
  const double* u = UR + f * sUR;
  double* w = W + f * sW;
  for (int idx = threadIdx.x; idx < n * nb; idx += blockDim.x) {
    const int i = idx / nb, c = idx % nb;
    w[(int64_t)i * ldw + c] = u[(int64_t)i * n + 2 * c];
  }
}

hipError_t launch_select_even(int n, int nb, int64_t count, const double* UR, int64_t sUR,
                              double* W, int64_t ldw, int64_t sW, hipStream_t st) {
  hipLaunchKernelGGL(k_select_even, dim3(1, (unsigned)count), dim3(256), 0, st, n, nb, UR, sUR, W,
                     ldw, sW);
  return hipGetLastError();
}

// Modes and energies of frequency f = blockIdx.y, points blockIdx.x*256 + ..
// Ue: 2m x nb realified U (row 2p: Re, row 2p+1: Im), VT: n x n (row 2c holds
// [Re v_c, Im v_c]), S: n.  modes[f][p][c] complex (TO re, im interleaved).
template <typename TO>
__global__ __launch_bounds__(256) void k_spod_modes(int64_t m, int nb, const double* __restrict__ Ue,
                                                    int64_t sUe, const double* __restrict__ VT,
                                                    int64_t sVT, const double* __restrict__ S,
                                                    int64_t sS, TO* __restrict__ modes,
                                                    double* __restrict__ L) {
  __shared__ double ph_re[64], ph_im[64];
  const int64_t f = blockIdx.y;
  const int n = 2 * nb;
  const double* vt = VT + f * sVT;
  const double* s = S + f * sS;
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
    if (blockIdx.x == 0) {
      const double sc = s[2 * c];
      L[f * nb + c] = sc * sc;
    }
  }
  __syncthreads();
  const double* ue = Ue + f * sUe;
  TO* out = modes + 2 * f * m * nb;
  const int64_t base = (int64_t)blockIdx.x * 256;
  for (int idx = threadIdx.x; idx < 256 * nb; idx += 256) {
    const int64_t p = base + idx / nb;
    const int c = idx % nb;
    if (p >= m) break;
    const double ur = ue[(2 * p) * nb + c], ui = ue[(2 * p + 1) * nb + c];
    const double cr = ph_re[c], ci = ph_im[c];
    out[2 * (p * nb + c)] = (TO)(ur * cr - ui * ci);
    out[2 * (p * nb + c) + 1] = (TO)(ur * ci + ui * cr);
  }
}

hipError_t launch_spod_modes(int out_f64, int64_t m, int nb, int64_t nf, const double* Ue,
                             int64_t sUe, const double* VT, int64_t sVT, const double* S,
                             int64_t sS, void* modes, double* L, hipStream_t st) {
  if (nb > 64) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((m + 255) / 256), (unsigned)nf);
  if (out_f64)
    hipLaunchKernelGGL(k_spod_modes<double>, grid, dim3(256), 0, st, m, nb, Ue, sUe, VT, sVT, S,
                       sS, (double*)modes, L);
  else
    hipLaunchKernelGGL(k_spod_modes<float>, grid, dim3(256), 0, st, m, nb, Ue, sUe, VT, sVT, S, sS,
                       (float*)modes, L);
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
