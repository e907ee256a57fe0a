// Mixed-precision POD: refinement of the FP32-QR spectrum against the input.
//
// The leaf QR of the mixed path runs in FP32, so R (and the SVD of R) carries
// errors of order u32 * sigma_1.  The spectrum is won back by a Rayleigh-Ritz
// step on the leading right singular vectors V_k of that SVD, computed against
// the input itself in FP64:
//
//   Z  = (A - mu 1^T) V_k          (m x k, FP64 accumulation, A read once)
//   G  = Z^T Z = W diag(lambda) W^T (k x k Gram, its Jacobi eigen-decomposition)
//   sigma_c = sqrt(lambda_c),  v_c = V_k w_c,  u_c = Z w_c / sigma_c.
//
// Because the u_c are formed from A V_k, their orthogonality and the Ritz
// values carry FP64 rounding of the Gram (relative error about
// u64 (sigma_1 / sigma_c)^2) plus the quadratic Ritz error in the angle
// between span(V_k) and the exact singular subspace; neither depends on the
// FP32 backward error except through that angle.  This replaces the
// reflector apply of Eq. svdqr3 in the mixed path (the Q of the FP32 QR is
// never formed).
#include <type_traits>
#include "common.hpp"
#include "kernels.hpp"

namespace pylom {

namespace {
constexpr int GR = 64;   // rows per workgroup
constexpr int GK = 8;    // K slab staged in LDS (9-13 KB per workgroup: registers bound the occupancy)
constexpr int ALD = GK + 1;
}  // namespace

__global__ void k_cast_f32_f64(const float* __restrict__ src, double* __restrict__ dst,
                               int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (double)src[i];
}

// C (m x nc) = (A - mu 1^T) (m x K) * B (K x nc), FP64 MFMA on promoted tiles.
// B(t, j) = Bs[j * ldb + t] when BT (B given by rows of its transpose), else
// Bs[t * ldb + j].  nc = min(nc_host, *nc_dev) when nc_dev is given.
// Grid: (ceil(m / 64), ceil(nc_host / GC)); 256 threads, wave w owns rows
// 16w..16w+15 of the tile and all GC / 16 column tiles.  GC = 128 lets up to
// 128 output columns read A once.
template <typename TI, typename TO, bool BT, int GC = 64>
__global__ __launch_bounds__(256) void k_tall_gemm(int64_t m, int K, int nc_host,
                                                   const int64_t* __restrict__ nc_dev,
                                                   const TI* __restrict__ A, int64_t lda,
                                                   const double* __restrict__ mu,
                                                   const double* __restrict__ Bs, int64_t ldb,
                                                   TO* __restrict__ C, int64_t ldc) {
  constexpr int BLD = GC + 1;
  constexpr int NT = GC / 16;
  __shared__ double As[GR * ALD];
  __shared__ double Bsh[GK * BLD];
  int nc = nc_host;
  if (nc_dev) {
    const int64_t d = *nc_dev;
    nc = (int)(d < nc ? d : nc);
  }
  const int64_t r0 = (int64_t)blockIdx.x * GR;
  const int j0 = blockIdx.y * GC;
  if (j0 >= nc) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, g4 = lane >> 4;
  typedef Mfma<double>::v4 v4;
  v4 acc[NT];
#pragma unroll
  for (int c = 0; c < NT; ++c) acc[c] = vzero4<double>();
  for (int k0 = 0; k0 < K; k0 += GK) {
    // stage A slab (64 x 32): consecutive threads walk a row
#pragma unroll
    for (int e = 0; e < (GR * GK) / 256; ++e) {
      const int idx = tid + 256 * e;
      const int r = idx / GK, c = idx % GK;
      const int64_t gr = r0 + r;
      const int gc = k0 + c;
      double v = 0.0;
      if (gr < m && gc < K) {
        v = (double)A[gr * lda + gc];
        if (mu) v -= mu[gr];
      }
      As[r * ALD + c] = v;
    }
    // stage B slab (32 x 64)
#pragma unroll
    for (int e = 0; e < (GK * GC) / 256; ++e) {
      const int idx = tid + 256 * e;
      int t, j;
      if (BT) {
        j = idx / GK;
        t = idx % GK;
      } else {
        t = idx / GC;
        j = idx % GC;
      }
      const int gt = k0 + t, gj = j0 + j;
      double v = 0.0;
      if (gt < K && gj < nc) v = BT ? Bs[(int64_t)gj * ldb + gt] : Bs[(int64_t)gt * ldb + gj];
      Bsh[t * BLD + j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kb = 0; kb < GK; kb += 4) {
      const double av = As[(wave * 16 + i16) * ALD + kb + g4];
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        const double bv = Bsh[(kb + g4) * BLD + c * 16 + i16];
        acc[c] = Mfma<double>::op(av, bv, acc[c]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    const int col = j0 + c * 16 + i16;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = r0 + wave * 16 + Mfma<double>::drow(g4, q);
      if (row < m && col < nc) C[row * ldc + col] = (TO)acc[c][q];
    }
  }
}

// The same product for long K: 128 rows per workgroup (each wave two 16-row
// tiles, so every B value read from LDS feeds two MFMAs), NT 16-column tiles
// (the output width rounded up to 16, not to 64 or 128), K staged in slabs
// of 16 with the next slab's A and B loaded into registers while the current
// one is multiplied (one barrier pair per slab).  A is read once per 16 NT
// columns; B once per 128 rows.
namespace {
constexpr int TR = 128;       // rows per workgroup
constexpr int TK = 16;        // K slab
constexpr int TALD = TK + 1;
}  // namespace
// VA (FP32 A with lda and K multiples of 4 and A 16-byte aligned): A is
// read as 16-byte vectors, four consecutive values of a row per thread, and
// the mean of each of the thread's two rows is read once per workgroup.
template <typename TI, typename TO, bool BT, int NT, bool VA>
__global__ __launch_bounds__(256) void k_tall_gemm_k(int64_t m, int K, int nc_host,
                                                     const int64_t* __restrict__ nc_dev,
                                                     const TI* __restrict__ A, int64_t lda,
                                                     const double* __restrict__ mu,
                                                     const double* __restrict__ Bs, int64_t ldb,
                                                     TO* __restrict__ C, int64_t ldc) {
  constexpr int GC = 16 * NT;
  constexpr int BLD = GC + 1;
  constexpr int AE = (TR * TK) / 256;          // A values staged per thread
  constexpr int BE = (TK * GC + 255) / 256;    // B values staged per thread
  __shared__ double As[TR * TALD];
  __shared__ double Bsh[TK * BLD];
  int nc = nc_host;
  if (nc_dev) {
    const int64_t d = *nc_dev;
    nc = (int)(d < nc ? d : nc);
  }
  const int64_t r0 = (int64_t)blockIdx.x * TR;
  const int j0 = blockIdx.y * GC;
  if (j0 >= nc) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, g4 = lane >> 4;
  typedef Mfma<double>::v4 v4;
  v4 acc[2][NT];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[r][c] = vzero4<double>();
  double pa[AE], pb[BE];
  // VA: vector e of a slab is row (tid + 256 e) / 4, columns 4 ((tid + 256 e)
  // % 4) + 0..3, the same two rows in every slab
  constexpr int AV = VA ? AE / 4 : 1;
  double mrow[AV];
  if constexpr (VA) {
#pragma unroll
    for (int e = 0; e < AV; ++e) {
      const int64_t gr = r0 + ((tid + 256 * e) >> 2);
      mrow[e] = (mu && gr < m) ? mu[gr] : 0.0;
    }
  }
  // A element e of a slab: row idx / TK, column idx % TK (a row's 16 values
  // are read by 16 consecutive threads); B element: BT walks t fastest
  auto fetch = [&](int k0) {
    if constexpr (VA) {
#pragma unroll
      for (int e = 0; e < AV; ++e) {
        const int idx = tid + 256 * e;
        const int64_t gr = r0 + (idx >> 2);
        const int gc = k0 + 4 * (idx & 3);
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gr < m && gc < K) v = *reinterpret_cast<const float4*>(A + gr * lda + gc);
        const bool live = gr < m && gc < K;
        pa[4 * e + 0] = live ? (double)v.x - mrow[e] : 0.0;
        pa[4 * e + 1] = live ? (double)v.y - mrow[e] : 0.0;
        pa[4 * e + 2] = live ? (double)v.z - mrow[e] : 0.0;
        pa[4 * e + 3] = live ? (double)v.w - mrow[e] : 0.0;
      }
    } else {
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        const int idx = tid + 256 * e;
        const int r = idx / TK, c = idx % TK;
        const int64_t gr = r0 + r;
        const int gc = k0 + c;
        double v = 0.0;
        if (gr < m && gc < K) {
          v = (double)A[gr * lda + gc];
          if (mu) v -= mu[gr];
        }
        pa[e] = v;
      }
    }
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int idx = tid + 256 * e;
      int t, j;
      if (BT) {
        j = idx / TK;
        t = idx % TK;
      } else {
        t = idx / GC;
        j = idx % GC;
      }
      const int gt = k0 + t, gj = j0 + j;
      double v = 0.0;
      if (idx < TK * GC && gt < K && gj < nc)
        v = BT ? Bs[(int64_t)gj * ldb + gt] : Bs[(int64_t)gt * ldb + gj];
      pb[e] = v;
    }
  };
  auto commit = [&]() {
    if constexpr (VA) {
#pragma unroll
      for (int e = 0; e < AV; ++e) {
        const int idx = tid + 256 * e;
        double* dst = As + (idx >> 2) * TALD + 4 * (idx & 3);
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = pa[4 * e + q];
      }
    } else {
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        const int idx = tid + 256 * e;
        As[(idx / TK) * TALD + idx % TK] = pa[e];
      }
    }
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int idx = tid + 256 * e;
      if (idx < TK * GC) {
        int t, j;
        if (BT) {
          j = idx / TK;
          t = idx % TK;
        } else {
          t = idx / GC;
          j = idx % GC;
        }
        Bsh[t * BLD + j] = pb[e];
      }
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += TK) {
    commit();
    __syncthreads();
    if (k0 + TK < K) fetch(k0 + TK);
#pragma unroll
    for (int kb = 0; kb < TK; kb += 4) {
      double bv[NT];
#pragma unroll
      for (int c = 0; c < NT; ++c) bv[c] = Bsh[(kb + g4) * BLD + c * 16 + i16];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const double av = As[(wave * 32 + r * 16 + i16) * TALD + kb + g4];
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[r][c] = Mfma<double>::op(av, bv[c], acc[r][c]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < NT; ++c) {
      const int col = j0 + c * 16 + i16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t row = r0 + wave * 32 + r * 16 + Mfma<double>::drow(g4, q);
        if (row < m && col < nc) C[row * ldc + col] = (TO)acc[r][c][q];
      }
    }
}

// Refined spectrum: S[c] = sqrt(lambda_c) for c < k, the unrefined S0[c] for
// c >= k; N_r from the residual-energy rule on S (tail sums from the smallest
// value upward), capped at k.  One workgroup.
__global__ __launch_bounds__(256) void k_rr_spectrum(int n, int k, const double* __restrict__ S0,
                                                     const double* __restrict__ lam,
                                                     double residual, double* __restrict__ S,
                                                     int64_t* __restrict__ nr) {
  __shared__ double tail[2049];
  const int tid = threadIdx.x;
  for (int c = tid; c < n; c += 256) {
    double s = S0[c];
    if (c < k) {
      const double l = lam[c];
      s = l > 0.0 ? sqrt(l) : 0.0;
    }
    S[c] = s;
  }
  __syncthreads();
  if (tid == 0) {
    tail[n] = 0.0;
    for (int c = n - 1; c >= 0; --c) tail[c] = tail[c + 1] + S[c] * S[c];
    const double total = tail[0];
    int64_t keep = n;
    if (!(residual > 0.0)) {
      keep = n;
    } else if (total == 0.0) {
      keep = 0;
    } else {
      for (int c = 1; c <= n; ++c)
        if (tail[c] <= residual * total) {
          keep = c;
          break;
        }
    }
    if (keep > k) keep = k;
    *nr = keep;
  }
}

// Refined right vectors and the mode-forming matrix, one workgroup per mode c
// (c < N_r): v = V_k w_c (VT row c), signed so that its largest-|.| entry
// (lowest index on ties) is positive; M[:, c] = sign * w_c / sigma_c.
// WT holds w_c as row c (k x k, ld k); VT0 holds V^T of the first SVD (ld n).
__global__ __launch_bounds__(256) void k_rr_vectors(int n, int k, const double* __restrict__ WT,
                                                    const double* __restrict__ VT0,
                                                    const double* __restrict__ S,
                                                    const int64_t* __restrict__ nr,
                                                    double* __restrict__ VT, int64_t ldvt,
                                                    double* __restrict__ M) {
  __shared__ double v[2048];
  __shared__ double best_v[256];
  __shared__ int best_i[256];
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  if (c >= *nr) return;
  const double* w = WT + (int64_t)c * k;
  double bv = -1.0;
  int bi = n;
  for (int t = tid; t < n; t += 256) {
    double x = 0.0;
    for (int j = 0; j < k; ++j) x += w[j] * VT0[(int64_t)j * n + t];
    v[t] = x;
    const double ax = fabs(x);
    if (ax > bv) {  // t increases along this thread's walk: first max kept
      bv = ax;
      bi = t;
    }
  }
  best_v[tid] = bv;
  best_i[tid] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      const double ov = best_v[tid + s];
      const int oi = best_i[tid + s];
      if (ov > best_v[tid] || (ov == best_v[tid] && oi < best_i[tid])) {
        best_v[tid] = ov;
        best_i[tid] = oi;
      }
    }
    __syncthreads();
  }
  const double sgn = (v[best_i[0]] < 0.0) ? -1.0 : 1.0;
  for (int t = tid; t < n; t += 256) VT[(int64_t)c * ldvt + t] = sgn * v[t];
  const double sc = S[c];
  for (int j = tid; j < k; j += 256) M[(int64_t)j * k + c] = (sc > 0.0) ? sgn * w[j] / sc : 0.0;
}

hipError_t launch_cast_f32_f64(const float* src, double* dst, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  int64_t g = (count + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_cast_f32_f64, dim3((unsigned)g), dim3(256), 0, st, src, dst, count);
  return hipGetLastError();
}

// The same product for a small K (<= 64) and at most 128 output columns, as
// in the DMD modes.  Every workgroup stages B once in LDS, sized to the call
// (4 ceil(K/4) rows of 16 ceil(nc/16) + 1 doubles); after that one barrier
// each wave walks 16-row strips on its own (grid-stride over strips, no
// further barriers).  The contraction index is split in four contiguous
// quarters of kq = ceil(K/4): lane (i, g) holds row i of its strip at
// columns g kq .. g kq + kq - 1, so MFMA step t takes column g kq + t of A
// and the matching row of B from LDS (the sum over k is the same, its order
// differs).  The next strip's A (and its mean) is loaded into registers
// before the current strip is multiplied, and the mean is subtracted when a
// value is used, so nothing waits on the prefetch until the strip is done.
// B(t, j) = Bs[j * ldb + t] when BT (the mixed refinement's projection onto
// the rows of V^T), else Bs[t * ldb + j] (the DMD modes).
constexpr int PK = 64;    // largest K kept whole in LDS
constexpr int PGC = 128;  // output columns
constexpr int PKQ = PK / 4;
constexpr int PNT = PGC / 16;

template <typename TI>
__device__ __forceinline__ void pb_load(int64_t strip, int64_t m, int K, int kq, int i16, int g4,
                                        const TI* __restrict__ A, int64_t lda,
                                        const double* __restrict__ mu, TI (&x)[PKQ],
                                        double& mr) {
  const int64_t row = strip * 16 + i16;
  const bool in = row < m;
  const TI* ar = A + (in ? row : 0) * lda + g4 * kq;
#pragma unroll
  for (int t = 0; t < PKQ; ++t) x[t] = (in && t < kq && g4 * kq + t < K) ? ar[t] : TI(0);
  mr = (in && mu) ? mu[row] : 0.0;
}

template <typename TI, typename TO, bool BT>
__global__ __launch_bounds__(256) void k_tall_gemm_pb(int64_t m, int K, int nc,
                                                      const int64_t* __restrict__ nc_dev,
                                                      const TI* __restrict__ A, int64_t lda,
                                                      const double* __restrict__ mu,
                                                      const double* __restrict__ Bs, int64_t ldb,
                                                      TO* __restrict__ C, int64_t ldc) {
  extern __shared__ double Bsh[];
  if (nc_dev && *nc_dev < nc) nc = (int)*nc_dev;  // the same value in every thread
  if (nc <= 0) return;
  const int kq = (K + 3) >> 2, nct = (nc + 15) >> 4;
  const int bw = 16 * nct, bld = bw + 1;
  for (int idx = threadIdx.x; idx < 4 * kq * bw; idx += 256) {
    const int t = idx / bw, j = idx % bw;
    double v = 0.0;
    if (t < K && j < nc) v = BT ? Bs[(int64_t)j * ldb + t] : Bs[(int64_t)t * ldb + j];
    Bsh[t * bld + j] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i16 = lane & 15, g4 = lane >> 4;
  const int64_t nstrips = (m + 15) >> 4;
  const int64_t stride = (int64_t)gridDim.x * 4;
  int64_t s = (int64_t)blockIdx.x * 4 + wave;
  if (s >= nstrips) return;
  typedef Mfma<double>::v4 v4;
  TI a[PKQ], an[PKQ];
  double mr, mrn;
  pb_load(s, m, K, kq, i16, g4, A, lda, mu, a, mr);
  const double* brow = Bsh + (g4 * kq) * bld + i16;
  for (; s < nstrips; s += stride) {
    const int64_t sn = s + stride;
    if (sn < nstrips) pb_load(sn, m, K, kq, i16, g4, A, lda, mu, an, mrn);
    v4 acc[PNT];
#pragma unroll
    for (int c = 0; c < PNT; ++c) acc[c] = vzero4<double>();
#pragma unroll
    for (int t = 0; t < PKQ; ++t) {
      if (t < kq) {
        const double av = (double)a[t] - mr;
#pragma unroll
        for (int c = 0; c < PNT; ++c)
          if (c < nct) acc[c] = Mfma<double>::op(av, brow[t * bld + c * 16], acc[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < PNT; ++c) {
      const int col = c * 16 + i16;
      if (c < nct && col < nc) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t row = s * 16 + Mfma<double>::drow(g4, q);
          if (row < m) C[row * ldc + col] = (TO)acc[c][q];
        }
      }
    }
#pragma unroll
    for (int t = 0; t < PKQ; ++t) a[t] = an[t];
    mr = mrn;
  }
}

// K in 1..PK, nc in 1..PGC (with nc_dev: nc = min(nc, *nc_dev), LDS sized
// for nc).
template <typename TI, typename TO, bool BT>
static hipError_t launch_pb(int64_t m, int K, int nc, const int64_t* nc_dev, const TI* A,
                            int64_t lda, const double* mu, const double* B, int64_t ldb, TO* C,
                            int64_t ldc, hipStream_t st) {
  if (K < 1 || K > PK || nc < 1 || nc > PGC) return hipErrorInvalidValue;
  const int kq = (K + 3) / 4, nct = (nc + 15) / 16;
  const size_t lds = (size_t)4 * kq * (16 * nct + 1) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_tall_gemm_pb<TI, TO, BT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int dev = 0, ncu = 0, per = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
           &per, (const void*)k_tall_gemm_pb<TI, TO, BT>, 256, lds)) != hipSuccess)
    return e;
  // one workgroup per resident slot (each wave walks its strips), no more
  // than there are groups of four strips
  const int64_t groups = ((m + 15) / 16 + 3) / 4;
  int64_t g = (int64_t)(ncu > 0 ? ncu : 1) * (per > 0 ? per : 1);
  if (g > groups) g = groups;
  hipLaunchKernelGGL((k_tall_gemm_pb<TI, TO, BT>), dim3((unsigned)g), dim3(256), lds, st, m, K,
                     nc, nc_dev, A, lda, mu, B, ldb, C, ldc);
  return hipGetLastError();
}

// One launch of the tall GEMM: 128-column workgroups when more than 64
// output columns are asked for (A is then read once per 128 columns).
template <typename TI, typename TO, bool BT, int NT>
static void launch_tgk(int64_t m, int K, int nc, const int64_t* nc_dev, const TI* A, int64_t lda,
                       const double* mu, const double* B, int64_t ldb, TO* C, int64_t ldc,
                       hipStream_t st) {
  const dim3 grid((unsigned)((m + TR - 1) / TR), (unsigned)((nc + 16 * NT - 1) / (16 * NT)));
  if constexpr (std::is_same<TI, float>::value) {
    if (lda % 4 == 0 && K % 4 == 0 && ((uintptr_t)A & 15) == 0) {
      hipLaunchKernelGGL((k_tall_gemm_k<TI, TO, BT, NT, true>), grid, dim3(256), 0, st, m, K, nc,
                         nc_dev, A, lda, mu, B, ldb, C, ldc);
      return;
    }
  }
  hipLaunchKernelGGL((k_tall_gemm_k<TI, TO, BT, NT, false>), grid, dim3(256), 0, st, m, K, nc,
                     nc_dev, A, lda, mu, B, ldb, C, ldc);
}

template <typename TI, typename TO, bool BT>
static hipError_t launch_tg(int64_t m, int K, int nc, const int64_t* nc_dev, const TI* A,
                            int64_t lda, const double* mu, const double* B, int64_t ldb, TO* C,
                            int64_t ldc, hipStream_t st) {
  if (m <= 0 || nc <= 0) return hipSuccess;
  if (K >= 512) {
    // long contractions (the refinement's projection of wide inputs): the
    // output width rounded up to 16 columns, 128-row tiles
    const int nt = (nc + 15) / 16;
    switch (nt > 8 ? 8 : nt) {
      case 1: launch_tgk<TI, TO, BT, 1>(m, K, nc, nc_dev, A, lda, mu, B, ldb, C, ldc, st); break;
      case 2: launch_tgk<TI, TO, BT, 2>(m, K, nc, nc_dev, A, lda, mu, B, ldb, C, ldc, st); break;
      case 3: launch_tgk<TI, TO, BT, 3>(m, K, nc, nc_dev, A, lda, mu, B, ldb, C, ldc, st); break;
      case 4: launch_tgk<TI, TO, BT, 4>(m, K, nc, nc_dev, A, lda, mu, B, ldb, C, ldc, st); break;
      case 5: launch_tgk<TI, TO, BT, 5>(m, K, nc, nc_dev, A, lda, mu, B, ldb, C, ldc, st); break;
      case 6: launch_tgk<TI, TO, BT, 6>(m, K, nc, nc_dev, A, lda, mu, B, ldb, C, ldc, st); break;
      case 7: launch_tgk<TI, TO, BT, 7>(m, K, nc, nc_dev, A, lda, mu, B, ldb, C, ldc, st); break;
      default: launch_tgk<TI, TO, BT, 8>(m, K, nc, nc_dev, A, lda, mu, B, ldb, C, ldc, st); break;
    }
    return hipGetLastError();
  }
  if (nc > 64) {
    const dim3 grid((unsigned)((m + GR - 1) / GR), (unsigned)((nc + 127) / 128));
    hipLaunchKernelGGL((k_tall_gemm<TI, TO, BT, 128>), grid, dim3(256), 0, st, m, K, nc, nc_dev,
                       A, lda, mu, B, ldb, C, ldc);
  } else {
    const dim3 grid((unsigned)((m + GR - 1) / GR), 1u);
    hipLaunchKernelGGL((k_tall_gemm<TI, TO, BT, 64>), grid, dim3(256), 0, st, m, K, nc, nc_dev,
                       A, lda, mu, B, ldb, C, ldc);
  }
  return hipGetLastError();
}

hipError_t launch_rr_project(int in_f64, int64_t m, int n, int k, const void* A, int64_t lda,
                             const double* mu, const double* VT0, double* Z, hipStream_t st) {
  // narrow inputs (n <= 64): B = V_k^T stays in LDS, A is read once in
  // register strips
  if (!in_f64 && m > 0 && n > 0 && n <= PK && k > 0 && k <= PGC)
    return launch_pb<float, double, true>(m, n, k, nullptr, (const float*)A, lda, mu, VT0,
                                          (int64_t)n, Z, (int64_t)k, st);
  if (in_f64)
    return launch_tg<double, double, true>(m, n, k, nullptr, (const double*)A, lda, mu, VT0,
                                           (int64_t)n, Z, (int64_t)k, st);
  return launch_tg<float, double, true>(m, n, k, nullptr, (const float*)A, lda, mu, VT0,
                                        (int64_t)n, Z, (int64_t)k, st);
}

hipError_t launch_rr_finish(int n, int k, const double* S0, const double* lam, double residual,
                            double* S, int64_t* nr, const double* WT, const double* VT0,
                            double* VT, int64_t ldvt, double* M, hipStream_t st) {
  hipLaunchKernelGGL(k_rr_spectrum, dim3(1), dim3(256), 0, st, n, k, S0, lam, residual, S, nr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rr_vectors, dim3((unsigned)k), dim3(256), 0, st, n, k, WT, VT0, S,
                     (const int64_t*)nr, VT, ldvt, M);
  return hipGetLastError();
}

hipError_t launch_rr_form_u(int out_f64, int64_t m, int k, const double* Z, const double* M,
                            const int64_t* nr, void* U, int64_t ldu, hipStream_t st) {
  // a narrow subspace (k <= 64): M in LDS, Z in register strips
  if (m > 0 && k > 0 && k <= PK) {
    if (out_f64)
      return launch_pb<double, double, false>(m, k, k, nr, Z, (int64_t)k, nullptr, M, (int64_t)k,
                                              (double*)U, ldu, st);
    return launch_pb<double, float, false>(m, k, k, nr, Z, (int64_t)k, nullptr, M, (int64_t)k,
                                           (float*)U, ldu, st);
  }
  if (out_f64)
    return launch_tg<double, double, false>(m, k, k, nr, Z, (int64_t)k, nullptr, M, (int64_t)k,
                                            (double*)U, ldu, st);
  return launch_tg<double, float, false>(m, k, k, nr, Z, (int64_t)k, nullptr, M, (int64_t)k,
                                         (float*)U, ldu, st);
}

hipError_t launch_tall_gemm_mu(int in_f64, int64_t m, int K, int nc, const void* A, int64_t lda,
                               const double* mu, const double* B, int64_t ldb, double* C,
                               int64_t ldc, hipStream_t st) {
  if (m > 0 && K > 0 && K <= PK && nc > 0 && nc <= PGC) {
    if (in_f64)
      return launch_pb<double, double, false>(m, K, nc, nullptr, (const double*)A, lda, mu, B, ldb,
                                              C, ldc, st);
    return launch_pb<float, double, false>(m, K, nc, nullptr, (const float*)A, lda, mu, B, ldb, C,
                                           ldc, st);
  }
  if (in_f64)
    return launch_tg<double, double, false>(m, K, nc, nullptr, (const double*)A, lda, mu, B, ldb,
                                            C, ldc, st);
  return launch_tg<float, double, false>(m, K, nc, nullptr, (const float*)A, lda, mu, B, ldb, C,
                                         ldc, st);
}

}  // namespace pylom
