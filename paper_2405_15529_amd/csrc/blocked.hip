// blocked.hip -- column-blocked TSQR for wide snapshot matrices (n > 1024).
//
// The stacked QR keeps a chunk of s rows by all n columns in LDS, which stops
// fitting once n passes about a thousand FP64 columns.  Wide problems are
// factored one panel of PW = 64 columns at a time instead, the blocked
// Householder QR that LAPACK runs for the local QR of each rank in Alg. 1:
//
//   for each panel k (columns c0 = 64 k, width kw):
//     [0; Y(:, panel)] = Q_k [R_k; 0]          stacked QR with a zero state:
//                                              every chunk is a structured
//                                              [state; chunk] step
//     [0; Y(:, trail)] <- Q_k^T [0; Y(:, trail)] = [S_k; Y']
//                                              k_panel_apply (Q^T mode)
//
// The kw state rows [R_k S_k] are rows c0..c0+kw of the leaf's R; Y' (same
// rows as Y) carries on into the next panel.  Adding kw zero rows does not
// change R, so R^T R = Y^T Y holds panel by panel.  The thin Q of the leaf
// follows from the same recursion read backwards: with W split into row
// blocks W_k,
//
//   X <- 0;  for k = K-1 .. 0:  [*; X] <- Q_k [W_k; X]
//
// leaves X = Q_thin W (k_panel_apply in Q mode: the state starts at W_k and
// is dropped at the end).  A combine of the reduction tree runs the same
// blocked QR on the 2n x n pair [R_a; R_b]; its rows are stored interleaved
// in blocks of 64 (A_0, B_0, A_1, B_1, ...) so that the rows panel k touches
// (the first (k+1) 64 rows of each triangle; the rest are still zero in
// those columns) form a prefix.
#include "common.hpp"
#include "kernels.hpp"

namespace pylom {

namespace {
constexpr int PS = 64;        // chunk rows (the stacked QR's s for panels of <= 64 columns)
constexpr int PW = 64;        // panel width
constexpr int CT = 64;        // columns per workgroup: 4 waves x 16
constexpr int CLD = CT + 1;   // LDS row stride of the chunk tile and of the state tile
constexpr int PLD = PW + 1;   // LDS row stride of the reflector block
}  // namespace

size_t panel_apply_lds_bytes(int esize) {
  return (size_t)esize * ((size_t)PS * CLD + (size_t)PS * PLD + (size_t)PW * CLD +
                          4 * (size_t)NB * NB + 4 * (size_t)NB * YLD);
}

// Applies the panel reflectors of every leaf to a 64-column tile of X.
// Leaf l owns rows [l b, l b + rows_l) of X and V (rows_l = b, the last leaf
// m - l b, both capped at rows_lim); its reflector tails for chunk c are V
// rows c*64.., its T factors Tf[((l nch + c) npan + p) 256].  The state tile
// (kw rows) is S + l s_leaf (row stride s_ld): zero at the start and written
// at the end (Q^T), or read at the start and dropped (Q, FWD).
// Grid: (ceil(ncols / 64), leaves); 256 threads, wave w owns 16 columns.
template <typename T, bool FWD>
__global__ __launch_bounds__(256) void k_panel_apply(PanelApplyArgs<T> a) {
  typedef typename Mfma<T>::v4 v4;
  extern __shared__ __align__(16) unsigned char smem[];
  T* Cs = reinterpret_cast<T*>(smem);
  T* Vs = Cs + PS * CLD;
  T* St = Vs + PS * PLD;
  T* Ts = St + PW * CLD;
  T* Yb = Ts + 4 * NB * NB;
  int64_t nc = a.ncols;
  if (a.nc_dev) {
    const int64_t d = *a.nc_dev - a.nc_off;
    if (d < nc) nc = d;
  }
  const int64_t c0 = (int64_t)blockIdx.x * CT;
  if (c0 >= nc) return;
  const int64_t l = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, g4 = lane >> 4;
  const int kw = a.kw, npan = a.npan;
  int64_t rows = (l == a.nlv - 1) ? a.m - l * a.b : a.b;
  if (a.rows_lim > 0 && rows > a.rows_lim) rows = a.rows_lim;
  const int nch = (int)((rows + PS - 1) / PS);
  const int64_t row0 = l * a.b;
  T* Sl = a.S + l * a.s_leaf;
  for (int idx = tid; idx < PW * CT; idx += 256) {
    const int i = idx / CT, j = idx - (idx / CT) * CT;
    T v = T(0);
    if (FWD && i < kw && c0 + j < nc) v = Sl[(int64_t)i * a.s_ld + c0 + j];
    St[i * CLD + j] = v;
  }
  T* Yw = Yb + wave * NB * YLD;
  const int cw = 16 * wave + i16;  // this lane's column of the tile
  for (int cc = 0; cc < nch; ++cc) {
    const int c = FWD ? nch - 1 - cc : cc;
    const int64_t r0 = (int64_t)c * PS;
    const int sc = (int)((rows - r0) < PS ? (rows - r0) : PS);
    // stage the chunk rows of the tile, the reflector tails and the T factors
    for (int idx = tid; idx < PS * CT; idx += 256) {
      const int r = idx / CT, j = idx - (idx / CT) * CT;
      T v = T(0);
      if (!a.x_zero && r < sc && c0 + j < nc) v = a.X[(row0 + r0 + r) * a.ldx + c0 + j];
      Cs[r * CLD + j] = v;
    }
    for (int idx = tid; idx < PS * PW; idx += 256) {
      const int r = idx / PW, j = idx - (idx / PW) * PW;
      T v = T(0);
      if (r < sc && j < kw) v = a.V[(row0 + r0 + r) * a.ldv + j];
      Vs[r * PLD + j] = v;
    }
    const T* tsrc = a.Tf + ((l * a.nch + c) * npan) * (NB * NB);
    for (int idx = tid; idx < npan * NB * NB; idx += 256) Ts[idx] = tsrc[idx];
    __syncthreads();
    for (int pp = 0; pp < npan; ++pp) {
      const int p = FWD ? npan - 1 - pp : pp;
      const int k0 = NB * p;
      // Y = V_p^T C + (state rows k0..k0+15): the reflector heads are the
      // unit vectors of those state rows
      v4 y0 = vzero4<T>(), y1 = vzero4<T>();
#pragma unroll
      for (int kb0 = 0; kb0 < PS / 4; kb0 += 4) {
        T av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = 4 * (kb0 + u) + g4;
          av[u] = Vs[r * PLD + k0 + i16];
          bv[u] = Cs[r * CLD + cw];
        }
        y0 = Mfma<T>::op(av[0], bv[0], y0);
        y1 = Mfma<T>::op(av[1], bv[1], y1);
        y0 = Mfma<T>::op(av[2], bv[2], y0);
        y1 = Mfma<T>::op(av[3], bv[3], y1);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = Mfma<T>::drow(g4, q);
        Yw[i * YLD + i16] = y0[q] + y1[q] + St[(k0 + i) * CLD + cw];
      }
      wave_lds_sync();
      // Z = T^T Y for Q^T, T Y for Q (T row-major, upper triangular)
      const T* Tp = Ts + p * NB * NB;
      v4 z = vzero4<T>();
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const int k = 4 * kb + g4;
        const T ta = FWD ? Tp[i16 * NB + k] : Tp[k * NB + i16];
        z = Mfma<T>::op(ta, Yw[k * YLD + i16], z);
      }
      wave_lds_sync();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = Mfma<T>::drow(g4, q);
        Yw[i * YLD + i16] = z[q];
        St[(k0 + i) * CLD + cw] -= z[q];
      }
      wave_lds_sync();
      // C -= V_p Z, one 16-row tile at a time
      T zb[4];
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) zb[kb] = Yw[(4 * kb + g4) * YLD + i16];
#pragma unroll
      for (int mt = 0; mt < PS / 16; ++mt) {
        v4 u = vzero4<T>();
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
          u = Mfma<T>::op(Vs[(16 * mt + i16) * PLD + k0 + 4 * kb + g4], zb[kb], u);
#pragma unroll
        for (int q = 0; q < 4; ++q) Cs[(16 * mt + Mfma<T>::drow(g4, q)) * CLD + cw] -= u[q];
      }
      wave_lds_sync();
    }
    __syncthreads();
    for (int idx = tid; idx < PS * CT; idx += 256) {
      const int r = idx / CT, j = idx - (idx / CT) * CT;
      if (r < sc && c0 + j < nc) a.X[(row0 + r0 + r) * a.ldx + c0 + j] = Cs[r * CLD + j];
    }
    __syncthreads();
  }
  if (!FWD) {
    for (int idx = tid; idx < PW * CT; idx += 256) {
      const int i = idx / CT, j = idx - (idx / CT) * CT;
      if (i < kw && c0 + j < nc) Sl[(int64_t)i * a.s_ld + c0 + j] = St[i * CLD + j];
    }
  }
}

// Working copy of the snapshot matrix: W = D - mu 1^T in the compute type
// (mu accumulated in FP64 per row, written to mean_out), row stride n.
// One wave per row.
template <typename TI, typename T>
__global__ __launch_bounds__(256) void k_make_work(int64_t m, int n, const TI* __restrict__ D,
                                                   int64_t ldd, int remove_mean,
                                                   double* __restrict__ mean_out,
                                                   T* __restrict__ W) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= m) return;
  const TI* row = D + r * ldd;
  double mu = 0.0;
  if (remove_mean) {
    double acc = 0.0;
    for (int col = lane; col < n; col += 64) acc += (double)row[col];
    acc = wave_sum(acc);
    mu = acc / (double)n;
    if (lane == 0 && mean_out) mean_out[r] = mu;
  }
  T* out = W + r * (int64_t)n;
  for (int col = lane; col < n; col += 64) out[col] = (T)((double)row[col] - mu);
}

// Row map of the interleaved pair layout: pair row pr -> (triangle, row).
__device__ __forceinline__ void pair_row(int pr, int n, int& isB, int& srow) {
  const int nblk = (n + PW - 1) / PW;
  int i = pr / (2 * PW);
  if (i > nblk - 1) i = nblk - 1;
  const int base = 2 * i * PW;
  const int sz = (n - i * PW < PW) ? n - i * PW : PW;
  const int within = pr - base;
  isB = within >= sz;
  srow = i * PW + (isB ? within - sz : within);
}

// Pairs of tree level h: pair q packs R_j (j = 2hq) and R_{j+h} (n x n,
// upper triangular, row stride n) into Pb + q 2n n, interleaved.
// Grid: (2n, pairs).
__global__ __launch_bounds__(256) void k_pair_pack(int n, int64_t h, const double* __restrict__ R,
                                                   double* __restrict__ Pb) {
  const int pr = blockIdx.x;
  const int64_t q = blockIdx.y;
  int isB, srow;
  pair_row(pr, n, isB, srow);
  const int64_t j = 2 * h * q + (isB ? h : 0);
  const double* src = R + j * (int64_t)n * n + (int64_t)srow * n;
  double* dst = Pb + q * 2 * (int64_t)n * n + (int64_t)pr * n;
  for (int col = threadIdx.x; col < n; col += 256) dst[col] = src[col];
}

// The inverse map for the propagation: X rows of pair q go to the W blocks
// of nodes j and j + h (columns < min(ncols, *nc_dev)).  Grid: (2n, pairs).
__global__ __launch_bounds__(256) void k_pair_unpack(int n, int64_t h, const double* __restrict__ Xp,
                                                     int64_t ldx, double* __restrict__ W,
                                                     int64_t ldw, int64_t ncols,
                                                     const int64_t* __restrict__ nc_dev) {
  int64_t nc = ncols;
  if (nc_dev && *nc_dev < nc) nc = *nc_dev;
  const int pr = blockIdx.x;
  const int64_t q = blockIdx.y;
  int isB, srow;
  pair_row(pr, n, isB, srow);
  const int64_t j = 2 * h * q + (isB ? h : 0);
  const double* src = Xp + (q * 2 * (int64_t)n + pr) * ldx;
  double* dst = W + j * (int64_t)n * ldw + (int64_t)srow * ldw;
  for (int64_t col = threadIdx.x; col < nc; col += 256) dst[col] = src[col];
}

// Completes the R of each problem from the per-panel states: row r of panel
// k = r / 64 gets zeros left of the panel and the panel's upper-triangular
// state block (kw_k x kw_k, row stride kw_k, at PSt + k pstride + l kw_k^2);
// the part right of the panel was written by the trailing apply.
// Grid: (n, problems).
template <typename T>
__global__ __launch_bounds__(256) void k_assemble_r(int n, const T* __restrict__ PSt,
                                                    int64_t pstride, T* __restrict__ R,
                                                    int64_t rstride) {
  const int r = blockIdx.x;
  const int64_t l = blockIdx.y;
  const int k = r / PW, i = r - k * PW;
  const int c0 = k * PW;
  const int kw = (n - c0 < PW) ? n - c0 : PW;
  const T* blk = PSt + (int64_t)k * pstride + l * (int64_t)kw * kw;
  T* row = R + l * rstride + (int64_t)r * n;
  for (int col = threadIdx.x; col < c0 + kw; col += 256) {
    T v = T(0);
    if (col >= c0 + i) v = blk[i * kw + (col - c0)];
    row[col] = v;
  }
}

// U[:, col0 + j] = X[:, j] for col0 + j < min(ncols_total, *nc_dev) and j < ncg.
template <typename TO>
__global__ __launch_bounds__(256) void k_copy_cols(int64_t m, int64_t col0, int64_t ncg,
                                                   int64_t ncols, const int64_t* __restrict__ nc_dev,
                                                   const double* __restrict__ X, int64_t ldx,
                                                   TO* __restrict__ U, int64_t ldu) {
  int64_t nc = ncols;
  if (nc_dev && *nc_dev < nc) nc = *nc_dev;
  int64_t w = nc - col0;
  if (w > ncg) w = ncg;
  if (w <= 0) return;
  const int64_t total = m * w;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * 256) {
    const int64_t r = idx / w, j = idx - (idx / w) * w;
    U[r * ldu + col0 + j] = (TO)X[r * ldx + j];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_panel_apply(const PanelApplyArgs<T>& a, bool fwd, hipStream_t st) {
  if (a.nlv <= 0 || a.ncols <= 0) return hipSuccess;
  if (a.kw < 1 || a.kw > PW || a.npan != (a.kw + NB - 1) / NB) return hipErrorInvalidValue;
  if (a.nlv > 65535) return hipErrorInvalidValue;
  const size_t lds = panel_apply_lds_bytes((int)sizeof(T));
  const dim3 grid((unsigned)((a.ncols + CT - 1) / CT), (unsigned)a.nlv);
  hipError_t e;
  if (fwd) {
    e = hipFuncSetAttribute((const void*)k_panel_apply<T, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_panel_apply<T, true>), grid, dim3(256), lds, st, a);
  } else {
    e = hipFuncSetAttribute((const void*)k_panel_apply<T, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_panel_apply<T, false>), grid, dim3(256), lds, st, a);
  }
  return hipGetLastError();
}
template hipError_t launch_panel_apply<double>(const PanelApplyArgs<double>&, bool, hipStream_t);
template hipError_t launch_panel_apply<float>(const PanelApplyArgs<float>&, bool, hipStream_t);

hipError_t launch_make_work(int in_f64, int out_f64, int64_t m, int n, const void* D, int64_t ldd,
                            int remove_mean, double* mean_out, void* W, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  const dim3 grid((unsigned)((m + 3) / 4));
  if (in_f64 && out_f64)
    hipLaunchKernelGGL((k_make_work<double, double>), grid, dim3(256), 0, st, m, n,
                       (const double*)D, ldd, remove_mean, mean_out, (double*)W);
  else if (!in_f64 && out_f64)
    hipLaunchKernelGGL((k_make_work<float, double>), grid, dim3(256), 0, st, m, n,
                       (const float*)D, ldd, remove_mean, mean_out, (double*)W);
  else if (!in_f64 && !out_f64)
    hipLaunchKernelGGL((k_make_work<float, float>), grid, dim3(256), 0, st, m, n,
                       (const float*)D, ldd, remove_mean, mean_out, (float*)W);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_pair_pack(int n, int64_t h, int64_t npairs, const double* R, double* Pb,
                            hipStream_t st) {
  if (npairs <= 0) return hipSuccess;
  if (npairs > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pair_pack, dim3((unsigned)(2 * n), (unsigned)npairs), dim3(256), 0, st, n,
                     h, R, Pb);
  return hipGetLastError();
}

hipError_t launch_pair_unpack(int n, int64_t h, int64_t npairs, const double* Xp, int64_t ldx,
                              double* W, int64_t ldw, int64_t ncols, const int64_t* nc_dev,
                              hipStream_t st) {
  if (npairs <= 0) return hipSuccess;
  if (npairs > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pair_unpack, dim3((unsigned)(2 * n), (unsigned)npairs), dim3(256), 0, st,
                     n, h, Xp, ldx, W, ldw, ncols, nc_dev);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_assemble_r(int n, int64_t nprob, const T* PSt, int64_t pstride, T* R,
                             int64_t rstride, hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  if (nprob > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_assemble_r<T>), dim3((unsigned)n, (unsigned)nprob), dim3(256), 0, st, n,
                     PSt, pstride, R, rstride);
  return hipGetLastError();
}
template hipError_t launch_assemble_r<double>(int, int64_t, const double*, int64_t, double*,
                                              int64_t, hipStream_t);
template hipError_t launch_assemble_r<float>(int, int64_t, const float*, int64_t, float*, int64_t,
                                             hipStream_t);

hipError_t launch_copy_cols(int out_f64, int64_t m, int64_t col0, int64_t ncg, int64_t ncols,
                            const int64_t* nc_dev, const double* X, int64_t ldx, void* U,
                            int64_t ldu, hipStream_t st) {
  if (m <= 0 || ncg <= 0) return hipSuccess;
  int64_t g = (m * ncg + 255) / 256;
  if (g > 16384) g = 16384;
  if (out_f64)
    hipLaunchKernelGGL((k_copy_cols<double>), dim3((unsigned)g), dim3(256), 0, st, m, col0, ncg,
                       ncols, nc_dev, X, ldx, (double*)U, ldu);
  else
    hipLaunchKernelGGL((k_copy_cols<float>), dim3((unsigned)g), dim3(256), 0, st, m, col0, ncg,
                       ncols, nc_dev, X, ldx, (float*)U, ldu);
  return hipGetLastError();
}

}  // namespace pylom
