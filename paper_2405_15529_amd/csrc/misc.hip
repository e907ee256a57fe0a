// misc.hip -- small helper kernels and the matmul of Alg. 4 on one GPU.
#include "common.hpp"
#include "kernels.hpp"

namespace pylom {

static inline int grid_for(int64_t work, int per_block = 256, int cap = 4096) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

template <typename TO>
__global__ void k_cast(const double* __restrict__ src, TO* __restrict__ dst, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (TO)src[i];
}

hipError_t launch_cast_out(const double* src, void* dst, int dst_f64, int64_t count,
                           hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (dst_f64)
    hipLaunchKernelGGL(k_cast<double>, dim3(grid_for(count)), dim3(256), 0, st, src, (double*)dst,
                       count);
  else
    hipLaunchKernelGGL(k_cast<float>, dim3(grid_for(count)), dim3(256), 0, st, src, (float*)dst,
                       count);
  return hipGetLastError();
}

__global__ void k_eye(double* W, int64_t n, int64_t ldw) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n * n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / n, j = idx % n;
    W[i * ldw + j] = (i == j) ? 1.0 : 0.0;
  }
}

hipError_t launch_eye(double* W, int64_t n, int64_t ldw, hipStream_t st) {
  hipLaunchKernelGGL(k_eye, dim3(grid_for(n * n)), dim3(256), 0, st, W, n, ldw);
  return hipGetLastError();
}

// R output with diag(R) >= 0: row i is negated when R[i][i] < 0; signs[i]
// records the flip so that the matching column of Q can follow.
__global__ void k_r_out(const double* __restrict__ Rr, int64_t n, double* R, int64_t ldr,
                        double* signs) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n * n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / n, j = idx % n;
    const double sg = (Rr[i * n + i] < 0.0) ? -1.0 : 1.0;
    R[i * ldr + j] = (j >= i) ? sg * Rr[i * n + j] : 0.0;
    if (j == 0 && signs) signs[i] = sg;
  }
}

hipError_t launch_r_out(const double* Rroot, int64_t n, double* R, int64_t ldr, double* signs,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_r_out, dim3(grid_for(n * n)), dim3(256), 0, st, Rroot, n, R, ldr, signs);
  return hipGetLastError();
}

template <typename TQ>
__global__ void k_q_signs(TQ* Q, int64_t m, int64_t n, int64_t ldq, const double* signs) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < m * n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / n, j = idx % n;
    if (signs[j] < 0.0) Q[i * ldq + j] = -Q[i * ldq + j];
  }
}

hipError_t launch_q_signs(void* Q, int q_f64, int64_t m, int64_t n, int64_t ldq,
                          const double* signs, hipStream_t st) {
  if (q_f64)
    hipLaunchKernelGGL(k_q_signs<double>, dim3(grid_for(m * n)), dim3(256), 0, st, (double*)Q, m,
                       n, ldq, signs);
  else
    hipLaunchKernelGGL(k_q_signs<float>, dim3(grid_for(m * n)), dim3(256), 0, st, (float*)Q, m, n,
                       ldq, signs);
  return hipGetLastError();
}

__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }

hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, st, p, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Alg. 4: C = sum over row blocks of A_i^T B_i.  Each workgroup owns one
// 64x64 tile of C and one slice of rows (split-K): it stages 32-row slabs of
// A (transposed) and B in LDS, promotes them to FP64 and accumulates with the
// FP64 MFMA (wave w owns rows 16w..16w+15 of the tile); its partial goes to
// an FP64 buffer, and a second kernel sums the slices in a fixed order (the
// device stand-in for the all_reduce, deterministic).
// ---------------------------------------------------------------------------
namespace {
constexpr int MT = 64;       // tile edge
constexpr int MK = 32;       // rows per slab
constexpr int MALD = MK + 1;
constexpr int MBLD = MT + 1;
}  // namespace

template <typename T>
__global__ __launch_bounds__(256) void k_matmul_tn_partial(int64_t m, int64_t p, int64_t q,
                                                           const T* __restrict__ A, int64_t lda,
                                                           const T* __restrict__ B, int64_t ldb,
                                                           double* __restrict__ part,
                                                           int64_t nsplit) {
  __shared__ double As[MT * MALD];  // As[i * MALD + r] = A[r][i0 + i]
  __shared__ double Bs[MK * MBLD];  // Bs[r * MBLD + j] = B[r][j0 + j]
  typedef Mfma<double>::v4 v4;
  const int64_t tp = (p + MT - 1) / MT, tq = (q + MT - 1) / MT;
  const int64_t tile = blockIdx.x % (tp * tq);
  const int64_t split = blockIdx.x / (tp * tq);
  const int64_t i0 = (tile / tq) * MT, j0 = (tile % tq) * MT;
  const int64_t rows_per = (m + nsplit - 1) / nsplit;
  const int64_t k0 = split * rows_per;
  const int64_t k1 = (k0 + rows_per < m) ? k0 + rows_per : m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, g4 = lane >> 4;
  v4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = vzero4<double>();
  for (int64_t kk = k0; kk < k1; kk += MK) {
#pragma unroll
    for (int e = 0; e < (MK * MT) / 256; ++e) {
      const int idx = tid + 256 * e;
      const int r = idx / MT, c = idx % MT;
      const int64_t gr = kk + r;
      const bool rok = gr < k1;
      As[c * MALD + r] = (rok && i0 + c < p) ? (double)A[gr * lda + i0 + c] : 0.0;
      Bs[r * MBLD + c] = (rok && j0 + c < q) ? (double)B[gr * ldb + j0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kb = 0; kb < MK; kb += 4) {
      const double av = As[(wave * 16 + i16) * MALD + kb + g4];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        acc[c] = Mfma<double>::op(av, Bs[(kb + g4) * MBLD + c * 16 + i16], acc[c]);
    }
    __syncthreads();
  }
  double* out = part + split * p * q;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int64_t j = j0 + c * 16 + i16;
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
      const int64_t i = i0 + wave * 16 + Mfma<double>::drow(g4, qq);
      if (i < p && j < q) out[i * q + j] = acc[c][qq];
    }
  }
}

// Symmetric products C = A^T A with p <= 128 columns (the Gram matrix of the
// mixed refinement, Z^T Z): each workgroup reads its slice of rows once, in
// 32-row slabs staged in LDS, and its four waves share the NB (NB + 1) / 2
// upper 16 x 16 blocks (wave w takes blocks w, w + 4, ...); each block is
// written with its mirror.  Slices, slabs and the 4-row MFMA steps follow the
// same row order as k_matmul_tn_partial, and the same reduce sums the slices.
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_gram_partial(int64_t m, int64_t p,
                                                      const T* __restrict__ A, int64_t lda,
                                                      double* __restrict__ part, int64_t nsplit) {
  constexpr int W = 16 * NB;
  constexpr int LD = W + 1;
  constexpr int NBLK = NB * (NB + 1) / 2;
  constexpr int MB = (NBLK + 3) / 4;          // blocks per wave
  constexpr int EL = (MK * W + 255) / 256;    // slab values per thread
  __shared__ double Zs[MK * LD];
  typedef Mfma<double>::v4 v4;
  const int64_t split = blockIdx.x;
  const int64_t rows_per = (m + nsplit - 1) / nsplit;
  const int64_t k0 = split * rows_per;
  const int64_t k1 = (k0 + rows_per < m) ? k0 + rows_per : m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, g4 = lane >> 4;
  // this wave's blocks (bi <= bj), in the order b = wave, wave + 4, ...
  int bi[MB], bj[MB];
#pragma unroll
  for (int u = 0; u < MB; ++u) {
    int b = wave + 4 * u, r = 0;
    while (r < NB && b >= NB - r) {
      b -= NB - r;
      ++r;
    }
    bi[u] = r;
    bj[u] = r + b;  // r == NB when the wave has no block u
  }
  v4 acc[MB];
#pragma unroll
  for (int u = 0; u < MB; ++u) acc[u] = vzero4<double>();
  const int pw = (int)p;
  double pv[EL];
  auto fetch = [&](int64_t kk) {
#pragma unroll
    for (int e = 0; e < EL; ++e) {
      const int idx = tid + 256 * e;
      const int r = idx / W, c = idx - (idx / W) * W;
      const int64_t gr = kk + r;
      pv[e] = (idx < MK * W && gr < k1 && c < pw) ? (double)A[gr * lda + c] : 0.0;
    }
  };
  if (k0 < k1) fetch(k0);
  for (int64_t kk = k0; kk < k1; kk += MK) {
#pragma unroll
    for (int e = 0; e < EL; ++e) {
      const int idx = tid + 256 * e;
      if (idx < MK * W) Zs[(idx / W) * LD + idx % W] = pv[e];
    }
    __syncthreads();
    if (kk + MK < k1) fetch(kk + MK);
#pragma unroll
    for (int kb = 0; kb < MK; kb += 4) {
      const double* zr = Zs + (kb + g4) * LD + i16;
#pragma unroll
      for (int u = 0; u < MB; ++u)
        if (bi[u] < NB) acc[u] = Mfma<double>::op(zr[16 * bi[u]], zr[16 * bj[u]], acc[u]);
    }
    __syncthreads();
  }
  double* out = part + split * p * p;
#pragma unroll
  for (int u = 0; u < MB; ++u) {
    if (bi[u] >= NB) continue;
    const int64_t j = 16 * bj[u] + i16;
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
      const int64_t i = 16 * bi[u] + Mfma<double>::drow(g4, qq);
      if (i < p && j < p) {
        out[i * p + j] = acc[u][qq];
        out[j * p + i] = acc[u][qq];
      }
    }
  }
}

// Small products (p, q <= 32): one wave per 16x16 tile of C and slice of
// rows, operands read straight from memory (a 64x64 tile would idle most of
// its MFMA work and staging on such shapes).
template <typename T>
__global__ __launch_bounds__(64) void k_matmul_tn_small(int64_t m, int64_t p, int64_t q,
                                                        const T* __restrict__ A, int64_t lda,
                                                        const T* __restrict__ B, int64_t ldb,
                                                        double* __restrict__ part,
                                                        int64_t nsplit) {
  typedef Mfma<double>::v4 v4;
  const int64_t tp = (p + 15) / 16, tq = (q + 15) / 16;
  const int64_t tile = blockIdx.x % (tp * tq);
  const int64_t split = blockIdx.x / (tp * tq);
  const int64_t i0 = (tile / tq) * 16, j0 = (tile % tq) * 16;
  const int64_t rows_per = (m + nsplit - 1) / nsplit;
  const int64_t k0 = split * rows_per;
  const int64_t k1 = (k0 + rows_per < m) ? k0 + rows_per : m;
  const int lane = threadIdx.x, i16 = lane & 15, g4 = lane >> 4;
  const bool iok = i0 + i16 < p, jok = j0 + i16 < q;
  v4 acc = vzero4<double>();
  for (int64_t k = k0; k < k1; k += 4) {
    const int64_t r = k + g4;
    const double av = (r < k1 && iok) ? (double)A[r * lda + i0 + i16] : 0.0;
    const double bv = (r < k1 && jok) ? (double)B[r * ldb + j0 + i16] : 0.0;
    acc = Mfma<double>::op(av, bv, acc);
  }
  double* out = part + split * p * q;
#pragma unroll
  for (int qq = 0; qq < 4; ++qq) {
    const int64_t i = i0 + Mfma<double>::drow(g4, qq), j = j0 + i16;
    if (i < p && j < q) out[i * q + j] = acc[qq];
  }
}

static bool matmul_small(int64_t p, int64_t q) { return p <= 32 && q <= 32; }

template <typename TO>
__global__ void k_matmul_reduce(int64_t p, int64_t q, const double* __restrict__ part,
                                int64_t nsplit, TO* C, int64_t ldc) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < p * q;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t k = 0; k < nsplit; ++k) s += part[k * p * q + idx];
    C[(idx / q) * ldc + (idx % q)] = (TO)s;
  }
}

int64_t matmul_tn_splits(int64_t m, int64_t p, int64_t q) {
  // small shapes: ~4096 one-wave tiles; otherwise ~1024 workgroups of 64x64
  // (four per CU); each slice at least 256 rows
  const bool sm = matmul_small(p, q);
  const int64_t e = sm ? 16 : 64;
  const int64_t tiles = ((p + e - 1) / e) * ((q + e - 1) / e);
  const int64_t target = sm ? 4096 : 1024;
  int64_t s = (target + tiles - 1) / tiles;
  const int64_t maxs = (m + 255) / 256;
  if (s > maxs) s = maxs;
  if (s < 1) s = 1;
  return s;
}

template <typename T>
static void launch_gram(int nb, int64_t m, int64_t p, const T* A, int64_t lda, double* partial,
                        int64_t nsplit, hipStream_t st) {
  const dim3 grid((unsigned)nsplit), block(256);
  switch (nb) {
    case 3:
      hipLaunchKernelGGL((k_gram_partial<T, 3>), grid, block, 0, st, m, p, A, lda, partial, nsplit);
      break;
    case 4:
      hipLaunchKernelGGL((k_gram_partial<T, 4>), grid, block, 0, st, m, p, A, lda, partial, nsplit);
      break;
    case 5:
      hipLaunchKernelGGL((k_gram_partial<T, 5>), grid, block, 0, st, m, p, A, lda, partial, nsplit);
      break;
    case 6:
      hipLaunchKernelGGL((k_gram_partial<T, 6>), grid, block, 0, st, m, p, A, lda, partial, nsplit);
      break;
    case 7:
      hipLaunchKernelGGL((k_gram_partial<T, 7>), grid, block, 0, st, m, p, A, lda, partial, nsplit);
      break;
    default:
      hipLaunchKernelGGL((k_gram_partial<T, 8>), grid, block, 0, st, m, p, A, lda, partial, nsplit);
      break;
  }
}

hipError_t launch_matmul_tn(int f64, int64_t m, int64_t p, int64_t q, const void* A, int64_t lda,
                            const void* B, int64_t ldb, void* C, int64_t ldc, double* partial,
                            int64_t nsplit, hipStream_t st) {
  if (A == B && lda == ldb && p == q && p > 32 && p <= 128) {
    // A^T A: the symmetric kernel, on the slices the caller planned for the
    // tiled kernel
    const int nb = (int)((p + 15) / 16);
    if (f64)
      launch_gram<double>(nb, m, p, (const double*)A, lda, partial, nsplit, st);
    else
      launch_gram<float>(nb, m, p, (const float*)A, lda, partial, nsplit, st);
  } else if (matmul_small(p, q)) {
    const int64_t tiles = ((p + 15) / 16) * ((q + 15) / 16);
    const dim3 grid((unsigned)(tiles * nsplit));
    if (f64)
      hipLaunchKernelGGL(k_matmul_tn_small<double>, grid, dim3(64), 0, st, m, p, q,
                         (const double*)A, lda, (const double*)B, ldb, partial, nsplit);
    else
      hipLaunchKernelGGL(k_matmul_tn_small<float>, grid, dim3(64), 0, st, m, p, q,
                         (const float*)A, lda, (const float*)B, ldb, partial, nsplit);
  } else {
    const int64_t tiles = ((p + 63) / 64) * ((q + 63) / 64);
    const dim3 grid((unsigned)(tiles * nsplit));
    if (f64)
      hipLaunchKernelGGL(k_matmul_tn_partial<double>, grid, dim3(256), 0, st, m, p, q,
                         (const double*)A, lda, (const double*)B, ldb, partial, nsplit);
    else
      hipLaunchKernelGGL(k_matmul_tn_partial<float>, grid, dim3(256), 0, st, m, p, q,
                         (const float*)A, lda, (const float*)B, ldb, partial, nsplit);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (f64)
    hipLaunchKernelGGL(k_matmul_reduce<double>, dim3(grid_for(p * q)), dim3(256), 0, st, p, q,
                       partial, nsplit, (double*)C, ldc);
  else
    hipLaunchKernelGGL(k_matmul_reduce<float>, dim3(grid_for(p * q)), dim3(256), 0, st, p, q,
                       partial, nsplit, (float*)C, ldc);
  return hipGetLastError();
}

// C (m x q) = A (m x p) B (p x q): one wave per 16x16 tile of C.
template <typename T>
__global__ __launch_bounds__(64) void k_matmul_nn(int64_t m, int64_t p, int64_t q,
                                                  const T* __restrict__ A, int64_t lda,
                                                  const T* __restrict__ B, int64_t ldb,
                                                  T* __restrict__ C, int64_t ldc) {
  typedef typename Mfma<T>::v4 v4;
  const int64_t tq = (q + 15) / 16;
  const int64_t i0 = (blockIdx.x / tq) * 16, j0 = (blockIdx.x % tq) * 16;
  const int lane = threadIdx.x, i16 = lane & 15, g4 = lane >> 4;
  const bool iok = i0 + i16 < m, jok = j0 + i16 < q;
  v4 acc = vzero4<T>();
  for (int64_t k = 0; k < p; k += 4) {
    const int64_t kk = k + g4;
    const T av = (kk < p && iok) ? A[(i0 + i16) * lda + kk] : T(0);
    const T bv = (kk < p && jok) ? B[kk * ldb + j0 + i16] : T(0);
    acc = Mfma<T>::op(av, bv, acc);
  }
#pragma unroll
  for (int qq = 0; qq < 4; ++qq) {
    const int64_t i = i0 + Mfma<T>::drow(g4, qq), j = j0 + i16;
    if (i < m && j < q) C[i * ldc + j] = acc[qq];
  }
}

hipError_t launch_matmul_nn(int f64, int64_t m, int64_t p, int64_t q, const void* A, int64_t lda,
                            const void* B, int64_t ldb, void* C, int64_t ldc, hipStream_t st) {
  const int64_t tiles = ((m + 15) / 16) * ((q + 15) / 16);
  if (tiles <= 0) return hipSuccess;
  if (f64)
    hipLaunchKernelGGL(k_matmul_nn<double>, dim3((unsigned)tiles), dim3(64), 0, st, m, p, q,
                       (const double*)A, lda, (const double*)B, ldb, (double*)C, ldc);
  else
    hipLaunchKernelGGL(k_matmul_nn<float>, dim3((unsigned)tiles), dim3(64), 0, st, m, p, q,
                       (const float*)A, lda, (const float*)B, ldb, (float*)C, ldc);
  return hipGetLastError();
}

}  // namespace pylom
