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
// is dropped at the end).
//
// A combine of the reduction tree, [R_a; R_b] = Q [R; 0], is the blocked QR
// of the two triangles with the rows of R_a as the state: panel k starts from
// the diagonal block of R_a's rows c0.. (untouched by earlier panels, whose
// reflectors do not reach those rows) and streams R_b's rows 0..c0+kw (the
// rest are still zero in those columns), in place: the reflector tails
// overwrite R_b, R_a's rows become R's.  The Q of the pair then maps
// [W; 0] to [W_a; W_b] by the Q-mode apply with the state read from and
// written back to W's rows c0.., panels from the last to the first.
#include "common.hpp"
#include "kernels.hpp"

namespace pylom {

namespace {
constexpr int PS = 64;        // chunk rows (the stacked QR's s for panels of <= 64 columns)
constexpr int PW = 64;        // panel width
constexpr int PLD = PW + 1;   // LDS row stride of the reflector block
}  // namespace

// LDS of k_panel_apply: the reflector block, the T factors, one Y tile per
// wave (the chunk tile itself stays in registers).
size_t panel_apply_lds_bytes(int esize) {
  return (size_t)esize * ((size_t)PS * PLD + 4 * (size_t)NB * NB + 4 * (size_t)NB * YLD);
}

// Row of a 16-row MFMA tile that lane slot i16 of the A operand loads so
// that the product lands, register q of lane (i16, g4), on tile row
// 4 q + g4: the rows the same lane holds as a B operand.  The FP64 output
// layout is already 4 q + g4; the FP32 one (4 g4 + q) needs the 4 x 4
// transpose of the slot index.
template <typename T>
__device__ __forceinline__ int a_row_for_b_layout(int i16);
template <>
__device__ __forceinline__ int a_row_for_b_layout<double>(int i16) { return i16; }
template <>
__device__ __forceinline__ int a_row_for_b_layout<float>(int i16) {
  return 4 * (i16 & 3) + (i16 >> 2);
}

// Applies the panel reflectors of every leaf to a 64-column tile of X.
// Leaf l owns rows [l b, l b + rows_l) of X and V (rows_l = b, the last leaf
// m - l b, both capped at rows_lim); its reflector tails for chunk c are V
// rows c*64.., its T factors Tf[((l nch + c) npan + p) 256].  The state tile
// (kw rows) is S + l s_leaf (row stride s_ld): read at the start if
// load_state (else zero), written at the end if store_state.
// Grid: (column tiles, leaves), or (leaves, column tiles) when leaf_major
// (launches where only the first tiles are live, so that the live
// workgroups spread over all XCDs); 256 threads, wave w owns columns
// 16 w .. 16 w + 15 of the tile.
//
// Every lane keeps, for its column, the 16 chunk rows 4 k + g4 (k < 16) and
// the state rows 16 p + 4 q + g4 in registers: the B operand of V^T C, the
// output of V Z (A rows permuted, see a_row_for_b_layout) and the state
// slots of Y and Z all use that row set, so the chunk tile never goes
// through LDS.  Only the reflector block and T factors are staged in LDS,
// through registers; the next chunk's loads (C, V, T) are issued before the
// products of the current one, so their HBM latency overlaps the MFMA work.
// Two workgroups share a CU.
template <typename T, bool FWD>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(2, 2)))
void k_panel_apply(PanelApplyArgs<T> a) {
  typedef typename Mfma<T>::v4 v4;
  extern __shared__ __align__(16) unsigned char smem[];
  T* Vs = reinterpret_cast<T*>(smem);
  T* Ts = Vs + PS * PLD;
  T* Yb = Ts + 4 * NB * NB;
  int64_t nc = a.ncols;
  if (a.nc_dev) {
    const int64_t d = *a.nc_dev - a.nc_off;
    if (d < nc) nc = d;
  }
  int64_t tile = a.leaf_major ? blockIdx.y : blockIdx.x;
  int64_t l = a.leaf_major ? blockIdx.x : blockIdx.y;
  if (!a.leaf_major && (a.nlv & 7) == 0) {
    // workgroup ids go to the eight XCDs round-robin: give each XCD whole
    // leaves, so that the tiles of a leaf share one L2 for its V and T
    const int64_t id = blockIdx.x + (int64_t)gridDim.x * blockIdx.y;
    const int64_t xcd = id & 7, k = id >> 3;
    l = xcd + 8 * (k / gridDim.x);
    tile = k % gridDim.x;
  }
  const int64_t c0 = tile * 64;
  if (c0 >= nc) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, g4 = lane >> 4;
  const int kw = a.kw, npan = a.npan;
  int64_t rows = (l == a.nlv - 1) ? a.m - l * a.b : a.b;
  if (a.rows_lim > 0 && rows > a.rows_lim) rows = a.rows_lim;
  const int nch = (int)((rows + PS - 1) / PS);
  const int64_t row0 = l * a.b;
  T* Sl = a.S + l * a.s_leaf;
  const int cw = 16 * wave + i16;  // this lane's column of the tile
  const bool cw_ok = c0 + cw < nc;
  T st[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = NB * p + Mfma<T>::drow(g4, q);
      T v = T(0);
      if (a.load_state && i < kw && cw_ok) v = Sl[(int64_t)i * a.s_ld + c0 + cw];
      st[p][q] = v;
    }
  T* Yw = Yb + wave * NB * YLD;
  const int arow = a_row_for_b_layout<T>(i16);
  // reflector block staging: thread (rw, jw) holds rows rw + 4 e of column jw
  constexpr int EPV = PS / 4;
  const int jw = tid & 63, rw = tid >> 6;
  // the FP64 trailing update has no registers left for a second chunk tile:
  // it loads the tile after the barrier and leaves the latency to the
  // second workgroup on the CU
  constexpr bool PREF_C = FWD || sizeof(T) == 4;
  T cc_[16], cn[PREF_C ? 16 : 1], rv[EPV], rt[4];
  auto load_c = [&](int c, T* dst) {
    const int64_t r0 = (int64_t)c * PS;
    const int sc = (int)((rows - r0) < PS ? (rows - r0) : PS);
    const T* xs = a.X + (row0 + r0 + g4) * a.ldx + c0 + cw;
    const int64_t xstep = 4 * a.ldx;
    const bool xon = !a.x_zero && cw_ok;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      dst[k] = (xon && 4 * k + g4 < sc) ? *xs : T(0);
      xs += xstep;
    }
  };
  auto fetch = [&](int c) {
    const int64_t r0 = (int64_t)c * PS;
    const int sc = (int)((rows - r0) < PS ? (rows - r0) : PS);
    if (PREF_C) load_c(c, cn);
    const T* vs = a.V + (row0 + r0 + rw) * a.ldv + jw;
    const int64_t vstep = 4 * a.ldv;
    const bool von = jw < kw;
#pragma unroll
    for (int e = 0; e < EPV; ++e) {
      rv[e] = (von && rw + 4 * e < sc) ? *vs : T(0);
      vs += vstep;
    }
    const T* tsrc = a.Tf + ((l * a.nch + c) * npan) * (NB * NB);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + 256 * e;
      rt[e] = (idx < npan * NB * NB) ? tsrc[idx] : T(0);
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int e = 0; e < EPV; ++e) Vs[(rw + 4 * e) * PLD + jw] = rv[e];
#pragma unroll
    for (int e = 0; e < 4; ++e) Ts[tid + 256 * e] = rt[e];
    if (PREF_C) {
#pragma unroll
      for (int k = 0; k < 16; ++k) cc_[k] = cn[PREF_C ? k : 0];
    }
  };
  fetch(FWD ? nch - 1 : 0);
  commit();
  if (!PREF_C) load_c(FWD ? nch - 1 : 0, cc_);
  __syncthreads();
  for (int ci = 0; ci < nch; ++ci) {
    const int c = FWD ? nch - 1 - ci : ci;
    if (ci + 1 < nch) fetch(FWD ? c - 1 : c + 1);
#pragma unroll
    for (int pp = 0; pp < 4; ++pp) {
      const int p = FWD ? 3 - pp : pp;  // sub-panels >= npan are empty
      if (p < npan) {
        const int k0 = NB * p;
        // Y = V_p^T C + (state rows k0..k0+15): the reflector heads are the
        // unit vectors of those state rows
        v4 y0 = vzero4<T>(), y1 = vzero4<T>();
#pragma unroll
        for (int k = 0; k < 16; k += 2) {
          y0 = Mfma<T>::op(Vs[(4 * k + g4) * PLD + k0 + i16], cc_[k], y0);
          y1 = Mfma<T>::op(Vs[(4 * (k + 1) + g4) * PLD + k0 + i16], cc_[k + 1], y1);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
          Yw[Mfma<T>::drow(g4, q) * YLD + i16] = y0[q] + y1[q] + st[p][q];
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
          Yw[Mfma<T>::drow(g4, q) * YLD + i16] = z[q];
          st[p][q] -= z[q];
        }
        wave_lds_sync();
        // C -= V_p Z: 16-row tile mt lands on the lane's rows 16 mt + 4 q + g4
        T zb[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) zb[kb] = Yw[(4 * kb + g4) * YLD + i16];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          v4 u = vzero4<T>();
#pragma unroll
          for (int kb = 0; kb < 4; ++kb)
            u = Mfma<T>::op(Vs[(16 * mt + arow) * PLD + k0 + 4 * kb + g4], zb[kb], u);
#pragma unroll
          for (int q = 0; q < 4; ++q) cc_[4 * mt + q] -= u[q];
        }
        wave_lds_sync();
      }
    }
    // write back the chunk rows of this lane's column
    {
      const int64_t r0 = (int64_t)c * PS;
      const int sc = (int)((rows - r0) < PS ? (rows - r0) : PS);
      T* xd = a.X + (row0 + r0 + g4) * a.ldx + c0 + cw;
      const int64_t xstep = 4 * a.ldx;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if (cw_ok && 4 * k + g4 < sc) *xd = cc_[k];
        xd += xstep;
      }
    }
    if (ci + 1 < nch) {
      __syncthreads();  // every wave is done with this chunk's V and T
      commit();
      if (!PREF_C) load_c(FWD ? c - 1 : c + 1, cc_);
      __syncthreads();
    }
  }
  if (a.store_state) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = NB * p + Mfma<T>::drow(g4, q);
        if (i < kw && cw_ok) Sl[(int64_t)i * a.s_ld + c0 + cw] = st[p][q];
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

// The same pass with 16-byte accesses, for rows of n % VL == 0 elements
// starting on 16-byte boundaries: each lane loads its NV vectors of the row
// once, keeps them in registers across the mean, and stores the shifted
// values (one HBM read and one write per element).
template <typename TI>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float4 type;
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  typedef double2 type;
  static constexpr int n = 2;
};

template <typename TI, typename T>
__device__ __forceinline__ void store_shifted(T* __restrict__ out, int64_t e0, float4 x, double mu) {
  if constexpr (sizeof(T) == 4) {
    float4 y;
    y.x = (float)((double)x.x - mu);
    y.y = (float)((double)x.y - mu);
    y.z = (float)((double)x.z - mu);
    y.w = (float)((double)x.w - mu);
    *reinterpret_cast<float4*>(out + e0) = y;
  } else {
    double2 y0, y1;
    y0.x = (double)x.x - mu;
    y0.y = (double)x.y - mu;
    y1.x = (double)x.z - mu;
    y1.y = (double)x.w - mu;
    *reinterpret_cast<double2*>(out + e0) = y0;
    *reinterpret_cast<double2*>(out + e0 + 2) = y1;
  }
}
template <typename TI, typename T>
__device__ __forceinline__ void store_shifted(T* __restrict__ out, int64_t e0, double2 x,
                                              double mu) {
  double2 y;
  y.x = x.x - mu;
  y.y = x.y - mu;
  *reinterpret_cast<double2*>(out + e0) = y;
}
__device__ __forceinline__ double vsum(float4 x) {
  return ((double)x.x + (double)x.y) + ((double)x.z + (double)x.w);
}
__device__ __forceinline__ double vsum(double2 x) { return x.x + x.y; }

template <typename TI, typename T, int NV>
__global__ __launch_bounds__(256) void k_make_work_v(int64_t m, int n, const TI* __restrict__ D,
                                                     int64_t ldd, int remove_mean,
                                                     double* __restrict__ mean_out,
                                                     T* __restrict__ W) {
  typedef typename Vec16<TI>::type V;
  constexpr int VL = Vec16<TI>::n;
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= m) return;
  const V* row = reinterpret_cast<const V*>(D + r * ldd);
  const int nv = n / VL;
  V x[NV];
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < NV; ++t) {
    const int idx = lane + 64 * t;
    if (idx < nv) {
      x[t] = row[idx];
      acc += vsum(x[t]);
    }
  }
  double mu = 0.0;
  if (remove_mean) {
    mu = wave_sum(acc) / (double)n;
    if (lane == 0 && mean_out) mean_out[r] = mu;
  }
  T* out = W + r * (int64_t)n;
#pragma unroll
  for (int t = 0; t < NV; ++t) {
    const int idx = lane + 64 * t;
    if (idx < nv) store_shifted<TI, T>(out, (int64_t)idx * VL, x[t], mu);
  }
}

// Diagonal block (c0, c0) of R_j, j = 2 h q (R_j at R + q rstride), into
// the panel state slot of pair q (kw x kw, zeros below the diagonal).
template <typename T>
__global__ __launch_bounds__(256) void k_diag_load(int n, int64_t c0, int kw,
                                                   const T* __restrict__ R, int64_t rstride,
                                                   T* __restrict__ PS) {
  const int64_t q = blockIdx.x;
  const T* src = R + q * rstride + c0 * n + c0;
  T* dst = PS + q * (int64_t)kw * kw;
  for (int idx = threadIdx.x; idx < kw * kw; idx += 256) {
    const int i = idx / kw, j = idx - (idx / kw) * kw;
    dst[idx] = (j >= i) ? src[(int64_t)i * n + j] : T(0);
  }
}

// Completes the R of each problem from the per-panel states: row r of panel
// k = r / 64 gets zeros left of the panel and the panel's upper-triangular
// state block (kw_k x kw_k, row stride kw_k, at PSt + k pstride + l kw_k^2);
// the part right of the panel was written by the trailing apply.
// Grid: (rows, problems), rows r0 .. r0 + rows - 1.
template <typename T>
__global__ __launch_bounds__(256) void k_assemble_r(int n, int r0, const T* __restrict__ PSt,
                                                    int64_t pstride, T* __restrict__ R,
                                                    int64_t rstride) {
  const int r = r0 + blockIdx.x;
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
template <typename T, bool FWD>
static hipError_t launch_panel_apply_t(const PanelApplyArgs<T>& a, hipStream_t st) {
  const int64_t tiles = (a.ncols + 63) / 64;
  if ((a.leaf_major ? tiles : a.nlv) > 65535) return hipErrorInvalidValue;
  const size_t lds = panel_apply_lds_bytes((int)sizeof(T));
  const dim3 grid = a.leaf_major ? dim3((unsigned)a.nlv, (unsigned)tiles)
                                 : dim3((unsigned)tiles, (unsigned)a.nlv);
  hipError_t e = hipFuncSetAttribute((const void*)k_panel_apply<T, FWD>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_panel_apply<T, FWD>), grid, dim3(256), lds, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_panel_apply(const PanelApplyArgs<T>& a, bool fwd, hipStream_t st) {
  if (a.nlv <= 0 || a.ncols <= 0) return hipSuccess;
  if (a.kw < 1 || a.kw > PW || a.npan != (a.kw + NB - 1) / NB) return hipErrorInvalidValue;
  return fwd ? launch_panel_apply_t<T, true>(a, st) : launch_panel_apply_t<T, false>(a, st);
}
template hipError_t launch_panel_apply<double>(const PanelApplyArgs<double>&, bool, hipStream_t);
template hipError_t launch_panel_apply<float>(const PanelApplyArgs<float>&, bool, hipStream_t);

hipError_t launch_make_work(int in_f64, int out_f64, int64_t m, int n, const void* D, int64_t ldd,
                            int remove_mean, double* mean_out, void* W, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  const dim3 grid((unsigned)((m + 3) / 4));
  const int vl = in_f64 ? 2 : 4;
  const bool vec = n % vl == 0 && ldd % vl == 0 && ((uintptr_t)D & 15) == 0 &&
                   ((uintptr_t)W & 15) == 0 && n <= 2048;
  if (vec) {
    // 16-byte accesses, the row held in registers (up to 2048 elements)
    if (in_f64 && out_f64)
      hipLaunchKernelGGL((k_make_work_v<double, double, 16>), grid, dim3(256), 0, st, m, n,
                         (const double*)D, ldd, remove_mean, mean_out, (double*)W);
    else if (!in_f64 && out_f64)
      hipLaunchKernelGGL((k_make_work_v<float, double, 8>), grid, dim3(256), 0, st, m, n,
                         (const float*)D, ldd, remove_mean, mean_out, (double*)W);
    else if (!in_f64 && !out_f64)
      hipLaunchKernelGGL((k_make_work_v<float, float, 8>), grid, dim3(256), 0, st, m, n,
                         (const float*)D, ldd, remove_mean, mean_out, (float*)W);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
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

template <typename T>
hipError_t launch_diag_load(int n, int64_t c0, int kw, int64_t npairs, const T* R,
                            int64_t rstride, T* PS, hipStream_t st) {
  if (npairs <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_diag_load<T>), dim3((unsigned)npairs), dim3(256), 0, st, n, c0, kw, R,
                     rstride, PS);
  return hipGetLastError();
}
template hipError_t launch_diag_load<double>(int, int64_t, int, int64_t, const double*, int64_t,
                                             double*, hipStream_t);
template hipError_t launch_diag_load<float>(int, int64_t, int, int64_t, const float*, int64_t,
                                            float*, hipStream_t);

template <typename T>
hipError_t launch_assemble_r(int n, int64_t nprob, const T* PSt, int64_t pstride, T* R,
                             int64_t rstride, hipStream_t st, int r0, int rows) {
  if (rows < 0) rows = n - r0;
  if (nprob <= 0 || rows <= 0) return hipSuccess;
  if (nprob > 65535 || r0 < 0 || r0 + rows > n) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_assemble_r<T>), dim3((unsigned)rows, (unsigned)nprob), dim3(256), 0, st,
                     n, r0, PSt, pstride, R, rstride);
  return hipGetLastError();
}
template hipError_t launch_assemble_r<double>(int, int64_t, const double*, int64_t, double*,
                                              int64_t, hipStream_t, int, int);
template hipError_t launch_assemble_r<float>(int, int64_t, const float*, int64_t, float*, int64_t,
                                             hipStream_t, int, int);

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
