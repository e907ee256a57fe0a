// Exact DMD on top of the TS-SVD (Sec. 3.2; Alg. 3 with the product of
// Alg. 4 and the amplitudes of Alg. 5).
//
// After the TS-SVD of Y1 = Y[:, :N-1] (U, S, W = the first N_r rows of VT
// taken as columns), every step below runs on the device:
//
//   A   = (U^T Y2) W S^-1                     k_dmd_linear_map   (N_r x N_r)
//         (U^T Y2 arrives as U_R^T R_f[:N-1, 1:], from the R-only TSQR of all
//         N snapshots; k_dmd_r1 extracts the R1 whose SVD is that of Y1)
//   A   = Q H Q^T, H upper Hessenberg           k_dmd_hess         (Householder)
//   mu  = eig(H)                                k_dmd_hqr          (Francis double-shift QR)
//   w_i = Q x_i, (H - mu_i I) x_i = 0           k_dmd_invit        (complex inverse iteration)
//   P, q of the amplitude fit (Alg. 5)          k_dmd_amp_matrix
//   b   = P^-1 q by Cholesky                    k_dmd_cholsolve
//   order by |b|, frequencies, growth rates     k_dmd_order
//   B   = W S^-1 w / mu (interleaved complex)   k_dmd_mode_rhs
//   phi = (D2 - mean 1^T) B                     the tall FP64 MFMA GEMM of refine.hip
//
// The eigen-solver is LAPACK's dgeev recast for one workgroup: the linear map
// is at most kDmdMax = 128 wide, so H (ld = N_r | 1) sits in LDS, the QR
// sweeps update the active window only (eigenvalues), and each eigenvector
// comes from two steps of inverse iteration on the Hessenberg matrix with the
// computed eigenvalue as shift (LU with adjacent-row pivoting), one workgroup
// per eigenvalue.  Eigenvectors are scaled to unit 2-norm with their
// largest-magnitude entry (lowest index on ties) real and positive.
#include "common.hpp"
#include "kernels.hpp"

namespace pylom {

namespace {

__device__ __forceinline__ double2 cmk(double re, double im) { return make_double2(re, im); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return cmk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return cmk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return cmk(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return cmk(a.x * s, a.y * s); }
__device__ __forceinline__ double cabs2(double2 a) { return hypot(a.x, a.y); }
// a / b by Smith's scaling (no overflow of |b|^2)
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + r * b.y;
    return cmk((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  const double r = b.x / b.y, d = b.y + r * b.x;
  return cmk((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}

// Sum over the 256 threads of a workgroup; every thread gets the total.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

__device__ __forceinline__ double block_max(double v, double* red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

constexpr double kEps = 1.1102230246251565e-16;  // 2^-53

}  // namespace

// A[i][j] = (sum_t aux[i][t] VT[j][t]) / S[j]: row i per workgroup.
__global__ __launch_bounds__(256) void k_dmd_linear_map(int k, int n1,
                                                        const double* __restrict__ aux,
                                                        const double* __restrict__ VT,
                                                        int64_t ldvt,
                                                        const double* __restrict__ S,
                                                        double* __restrict__ A) {
  const int i = blockIdx.x;
  const double* ar = aux + (int64_t)i * n1;
  for (int j = threadIdx.x; j < k; j += 256) {
    const double* vr = VT + (int64_t)j * ldvt;
    double acc = 0.0;
    for (int t = 0; t < n1; ++t) acc += ar[t] * vr[t];
    A[(int64_t)i * k + j] = acc / S[j];
  }
}

// Householder reduction to upper Hessenberg form, A = Q H Q^T with
// Q = H_0 H_1 ... H_{k-3}, H_j = I - tau_j v_j v_j^T acting on rows j+1..k-1
// (v_j[j+1] = 1, v_j[r] = 0 for r <= j).  One workgroup; A in LDS.
__global__ __launch_bounds__(256) void k_dmd_hess(int k, const double* __restrict__ A,
                                                  double* __restrict__ H0,
                                                  double* __restrict__ Qv,
                                                  double* __restrict__ Qtau) {
  extern __shared__ __align__(16) double sm[];
  const int ld = k | 1;
  double* Hs = sm;
  double* vb = Hs + (size_t)k * ld;
  double* red = vb + k;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < k * k; idx += 256) Hs[(idx / k) * ld + idx % k] = A[idx];
  __syncthreads();
  for (int j = 0; j + 2 < k; ++j) {
    double part = 0.0;
    for (int i = j + 2 + tid; i < k; i += 256) part += Hs[i * ld + j] * Hs[i * ld + j];
    const double sigma = block_sum(part, red);
    const double alpha = Hs[(j + 1) * ld + j];
    double tau = 0.0, beta = alpha, scal = 0.0;
    if (sigma > 0.0) {
      const double nrm = sqrt(alpha * alpha + sigma);
      beta = (alpha >= 0.0) ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    for (int i = tid; i < k; i += 256)
      vb[i] = (i <= j) ? 0.0 : ((i == j + 1) ? 1.0 : Hs[i * ld + j] * scal);
    __syncthreads();
    if (tau != 0.0) {
      // left: rows j+1..k-1, columns j..k-1
      for (int c = j + tid; c < k; c += 256) {
        double d = 0.0;
        for (int i = j + 1; i < k; ++i) d += vb[i] * Hs[i * ld + c];
        d *= tau;
        for (int i = j + 1; i < k; ++i) Hs[i * ld + c] -= d * vb[i];
      }
      __syncthreads();
      // right: rows 0..k-1, columns j+1..k-1
      for (int r = tid; r < k; r += 256) {
        double d = 0.0;
        for (int i = j + 1; i < k; ++i) d += Hs[r * ld + i] * vb[i];
        d *= tau;
        for (int i = j + 1; i < k; ++i) Hs[r * ld + i] -= d * vb[i];
      }
      __syncthreads();
      for (int i = j + 2 + tid; i < k; i += 256) Hs[i * ld + j] = 0.0;
      if (tid == 0) Hs[(j + 1) * ld + j] = beta;
    }
    if (tid == 0) Qtau[j] = tau;
    for (int i = tid; i < k; i += 256) Qv[(int64_t)j * k + i] = vb[i];
    __syncthreads();
  }
  for (int idx = tid; idx < k * k; idx += 256) H0[idx] = Hs[(idx / k) * ld + idx % k];
}

// Eigenvalues of the Hessenberg H0 by the implicit double-shift (Francis) QR
// algorithm with deflation at negligible subdiagonals (Golub & Van Loan,
// Alg. 7.5.1-7.5.2); exceptional shifts at the 10th and 20th sweep of a block
// (LAPACK dlahqr's); at most 30 max(10, k) sweeps.  status[0] = sweeps, or -1
// when the limit is hit; hnorm = max |H0| for the inverse iteration.
__global__ __launch_bounds__(256) void k_dmd_hqr(int k, const double* __restrict__ H0,
                                                 double* __restrict__ wr, double* __restrict__ wi,
                                                 double* __restrict__ hnorm_out,
                                                 int* __restrict__ status) {
  extern __shared__ __align__(16) double sm[];
  const int ld = k | 1;
  double* H = sm;
  double* red = H + (size_t)k * ld;
  const int tid = threadIdx.x;
  double amax = 0.0;
  for (int idx = tid; idx < k * k; idx += 256) {
    const double v = H0[idx];
    H[(idx / k) * ld + idx % k] = v;
    amax = fmax(amax, fabs(v));
  }
  const double hnorm = block_max(amax, red);
  if (tid == 0) *hnorm_out = hnorm;
#define HH(r, c) H[(r) * ld + (c)]
  int nn = k - 1, its = 0, total = 0;
  const int limit = 30 * (k > 10 ? k : 10);
  bool failed = false;
  while (nn >= 0) {
    // largest l <= nn with a negligible H[l][l-1] (l = 0 if none)
    int l = nn;
    while (l > 0) {
      double s = fabs(HH(l - 1, l - 1)) + fabs(HH(l, l));
      if (s == 0.0) s = hnorm;
      if (fabs(HH(l, l - 1)) <= kEps * s) break;
      --l;
    }
    __syncthreads();
    if (l > 0 && tid == 0) HH(l, l - 1) = 0.0;
    if (l == nn) {
      if (tid == 0) {
        wr[nn] = HH(nn, nn);
        wi[nn] = 0.0;
      }
      --nn;
      its = 0;
      __syncthreads();
      continue;
    }
    if (l == nn - 1) {
      const double a = HH(nn - 1, nn - 1), b = HH(nn - 1, nn), c = HH(nn, nn - 1),
                   d = HH(nn, nn);
      const double p = 0.5 * (a - d), q = p * p + b * c;
      if (tid == 0) {
        if (q >= 0.0) {
          const double z = p + copysign(sqrt(q), p);
          wr[nn - 1] = d + z;
          wr[nn] = (z != 0.0) ? d - b * c / z : d + z;
          wi[nn - 1] = 0.0;
          wi[nn] = 0.0;
        } else {
          const double im = sqrt(-q);
          wr[nn - 1] = d + p;
          wr[nn] = d + p;
          wi[nn - 1] = im;
          wi[nn] = -im;
        }
      }
      nn -= 2;
      its = 0;
      __syncthreads();
      continue;
    }
    if (total >= limit) {
      failed = true;
      break;
    }
    ++its;
    ++total;
    double s, t;
    if (its == 10 || its == 20) {
      const double ss = fabs(HH(nn, nn - 1)) + fabs(HH(nn - 1, nn - 2));
      const double h11 = 0.75 * ss + HH(nn, nn), h12 = -0.4375 * ss, h21 = ss;
      s = 2.0 * h11;
      t = h11 * h11 - h12 * h21;
    } else {
      s = HH(nn - 1, nn - 1) + HH(nn, nn);
      t = HH(nn - 1, nn - 1) * HH(nn, nn) - HH(nn - 1, nn) * HH(nn, nn - 1);
    }
    // first column of (H - s1 I)(H - s2 I) on rows l..l+2
    double x = HH(l, l) * HH(l, l) + HH(l, l + 1) * HH(l + 1, l) - s * HH(l, l) + t;
    double y = HH(l + 1, l) * (HH(l, l) + HH(l + 1, l + 1) - s);
    double z = HH(l + 1, l) * HH(l + 2, l + 1);
    for (int kk = l; kk <= nn - 2; ++kk) {
      if (kk > l) {
        x = HH(kk, kk - 1);
        y = HH(kk + 1, kk - 1);
        z = HH(kk + 2, kk - 1);
      }
      const double sigma = y * y + z * z;
      double tau = 0.0, v1 = 0.0, v2 = 0.0, beta = x;
      if (sigma > 0.0) {
        const double nrm = sqrt(x * x + sigma);
        beta = (x >= 0.0) ? -nrm : nrm;
        tau = (beta - x) / beta;
        const double sc = 1.0 / (x - beta);
        v1 = y * sc;
        v2 = z * sc;
      }
      __syncthreads();
      if (tau != 0.0) {
        const int c0 = (kk > l) ? kk - 1 : l;
        for (int c = c0 + tid; c <= nn; c += 256) {
          const double d = tau * (HH(kk, c) + v1 * HH(kk + 1, c) + v2 * HH(kk + 2, c));
          HH(kk, c) -= d;
          HH(kk + 1, c) -= d * v1;
          HH(kk + 2, c) -= d * v2;
        }
        __syncthreads();
        const int r1 = (kk + 3 < nn) ? kk + 3 : nn;
        for (int r = l + tid; r <= r1; r += 256) {
          const double d = tau * (HH(r, kk) + v1 * HH(r, kk + 1) + v2 * HH(r, kk + 2));
          HH(r, kk) -= d;
          HH(r, kk + 1) -= d * v1;
          HH(r, kk + 2) -= d * v2;
        }
        __syncthreads();
        if (kk > l && tid == 0) {
          HH(kk, kk - 1) = beta;
          HH(kk + 1, kk - 1) = 0.0;
          HH(kk + 2, kk - 1) = 0.0;
        }
      }
      __syncthreads();
    }
    // last step: a 2-row reflector on rows nn-1, nn
    {
      x = HH(nn - 1, nn - 2);
      y = HH(nn, nn - 2);
      const double sigma = y * y;
      double tau = 0.0, v1 = 0.0, beta = x;
      if (sigma > 0.0) {
        const double nrm = sqrt(x * x + sigma);
        beta = (x >= 0.0) ? -nrm : nrm;
        tau = (beta - x) / beta;
        v1 = y / (x - beta);
      }
      __syncthreads();
      if (tau != 0.0) {
        for (int c = nn - 2 + tid; c <= nn; c += 256) {
          const double d = tau * (HH(nn - 1, c) + v1 * HH(nn, c));
          HH(nn - 1, c) -= d;
          HH(nn, c) -= d * v1;
        }
        __syncthreads();
        for (int r = l + tid; r <= nn; r += 256) {
          const double d = tau * (HH(r, nn - 1) + v1 * HH(r, nn));
          HH(r, nn - 1) -= d;
          HH(r, nn) -= d * v1;
        }
        __syncthreads();
        if (tid == 0) {
          HH(nn - 1, nn - 2) = beta;
          HH(nn, nn - 2) = 0.0;
        }
      }
      __syncthreads();
    }
  }
#undef HH
  if (tid == 0) {
    status[0] = failed ? -1 : total;
    status[1] = 0;
    if (failed)
      for (int i = 0; i <= nn; ++i) {
        wr[i] = 0.0;
        wi[i] = 0.0;
      }
  }
}

// Eigenvector of eigenvalue i (one workgroup each): two steps of inverse
// iteration, (H0 - mu I) x_{s+1} = x_s / |x_s| from x_0 = 1, with the LU
// factors of the shifted Hessenberg matrix (adjacent-row partial pivoting; a
// zero pivot becomes eps max|H0|), then w = Q x and the scaling convention.
// Ub: k x k complex scratch per eigenvalue.
__global__ __launch_bounds__(256) void k_dmd_invit(int k, const double* __restrict__ H0,
                                                   const double* __restrict__ wr,
                                                   const double* __restrict__ wi,
                                                   const double* __restrict__ hnorm_in,
                                                   const double* __restrict__ Qv,
                                                   const double* __restrict__ Qtau,
                                                   double2* __restrict__ Ubuf,
                                                   double2* __restrict__ Wout) {
  __shared__ double2 cur[kDmdMax];
  __shared__ double2 rhs[kDmdMax];
  __shared__ double2 xs[kDmdMax];
  __shared__ double2 lmul[kDmdMax];
  __shared__ int swp[kDmdMax];
  __shared__ double red[8];
  const int i = blockIdx.x, tid = threadIdx.x;
  const double2 lam = cmk(wr[i], wi[i]);
  const double hn = *hnorm_in;
  const double small = (hn > 0.0) ? kEps * hn : 1e-300;
  double2* Ub = Ubuf + (int64_t)i * k * k;
  for (int c = tid; c < k; c += 256) cur[c] = cmk(H0[c] - (c == 0 ? lam.x : 0.0), c == 0 ? -lam.y : 0.0);
  __syncthreads();
  for (int j = 0; j + 1 < k; ++j) {
    const double2 piv = cur[j];
    const double2 nxt = cmk(H0[(int64_t)(j + 1) * k + j], 0.0);
    const bool sw = cabs2(nxt) > cabs2(piv);
    double2 pj = sw ? nxt : piv;
    if (pj.x == 0.0 && pj.y == 0.0) pj = cmk(small, 0.0);
    const double2 lj = cdiv(sw ? piv : nxt, pj);
    for (int c = j + tid; c < k; c += 256) {
      const double2 mrow =
          cmk(H0[(int64_t)(j + 1) * k + c] - (c == j + 1 ? lam.x : 0.0), c == j + 1 ? -lam.y : 0.0);
      double2 pc = sw ? mrow : cur[c];
      const double2 oc = sw ? cur[c] : mrow;
      if (c == j) pc = pj;
      Ub[(int64_t)j * k + c] = pc;
      if (c > j) cur[c] = csub(oc, cmul(lj, pc));
    }
    if (tid == 0) {
      lmul[j] = lj;
      swp[j] = sw ? 1 : 0;
    }
    __syncthreads();
  }
  if (tid == 0) {
    double2 last = cur[k - 1];
    if (last.x == 0.0 && last.y == 0.0) last = cmk(small, 0.0);
    Ub[(int64_t)(k - 1) * k + (k - 1)] = last;
  }
  __threadfence_block();
  __syncthreads();
  for (int it = 0; it < 2; ++it) {
    if (it == 0) {
      for (int c = tid; c < k; c += 256) rhs[c] = cmk(1.0, 0.0);
    } else {
      double part = 0.0;
      for (int c = tid; c < k; c += 256) part += xs[c].x * xs[c].x + xs[c].y * xs[c].y;
      const double nrm = sqrt(block_sum(part, red));
      const double inv = (nrm > 0.0) ? 1.0 / nrm : 1.0;
      for (int c = tid; c < k; c += 256) rhs[c] = cscale(xs[c], inv);
    }
    __syncthreads();
    if (tid == 0) {
      for (int j = 0; j + 1 < k; ++j) {
        if (swp[j]) {
          const double2 tmp = rhs[j];
          rhs[j] = rhs[j + 1];
          rhs[j + 1] = tmp;
        }
        rhs[j + 1] = csub(rhs[j + 1], cmul(lmul[j], rhs[j]));
      }
    }
    __syncthreads();
    for (int j = k - 1; j >= 0; --j) {
      const double2 xj = cdiv(rhs[j], Ub[(int64_t)j * k + j]);
      __syncthreads();
      if (tid == 0) xs[j] = xj;
      for (int r = tid; r < j; r += 256) rhs[r] = csub(rhs[r], cmul(Ub[(int64_t)r * k + j], xj));
      __syncthreads();
    }
  }
  // rescale once more before applying Q (the second solve grows by 1/eps)
  {
    double part = 0.0;
    for (int c = tid; c < k; c += 256) part += xs[c].x * xs[c].x + xs[c].y * xs[c].y;
    const double nrm = sqrt(block_sum(part, red));
    const double inv = (nrm > 0.0) ? 1.0 / nrm : 1.0;
    for (int c = tid; c < k; c += 256) xs[c] = cscale(xs[c], inv);
    __syncthreads();
  }
  // w = H_0 H_1 ... H_{k-3} x
  for (int j = k - 3; j >= 0; --j) {
    const double tau = Qtau[j];
    if (tau == 0.0) continue;
    const double* v = Qv + (int64_t)j * k;
    double pr = 0.0, pi = 0.0;
    for (int r = j + 1 + tid; r < k; r += 256) {
      pr += v[r] * xs[r].x;
      pi += v[r] * xs[r].y;
    }
    const double dr = block_sum(pr, red) * tau;
    const double di = block_sum(pi, red) * tau;
    for (int r = j + 1 + tid; r < k; r += 256) xs[r] = cmk(xs[r].x - dr * v[r], xs[r].y - di * v[r]);
    __syncthreads();
  }
  // unit 2-norm, largest-magnitude entry (lowest index on ties) real positive
  double part = 0.0;
  for (int c = tid; c < k; c += 256) part += xs[c].x * xs[c].x + xs[c].y * xs[c].y;
  const double nrm = sqrt(block_sum(part, red));
  __shared__ int jmax;
  if (tid == 0) {
    int jm = 0;
    double best = -1.0;
    for (int c = 0; c < k; ++c) {
      const double a = cabs2(xs[c]);
      if (a > best) {
        best = a;
        jm = c;
      }
    }
    jmax = jm;
  }
  __syncthreads();
  const double2 xm = xs[jmax];
  const double am = cabs2(xm);
  const double2 ph = (am > 0.0 && nrm > 0.0) ? cscale(cconj(xm), 1.0 / (am * nrm)) : cmk(1.0, 0.0);
  for (int c = tid; c < k; c += 256) {
    double2 v = cmul(xs[c], ph);
    if (c == jmax) v = cmk(nrm > 0.0 ? am / nrm : 0.0, 0.0);
    Wout[(int64_t)c * k + i] = v;
  }
}

// Alg. 5, row i of P and entry i of q (one workgroup per i):
//   P[i][j] = (sum_r conj(w_ri) w_rj) * sum_t (conj(mu_i) mu_j)^t,
//   q[i]    = conj(sum_j s_j w_ji sum_t VT[j][t] mu_i^t),   t = 0..n1-1.
__global__ __launch_bounds__(256) void k_dmd_amp_matrix(int k, int n1,
                                                        const double* __restrict__ wr,
                                                        const double* __restrict__ wi,
                                                        const double2* __restrict__ W,
                                                        const double* __restrict__ VT,
                                                        int64_t ldvt,
                                                        const double* __restrict__ S,
                                                        double2* __restrict__ P,
                                                        double2* __restrict__ q) {
  extern __shared__ __align__(16) double2 pw[];  // mu_i^t, t < n1
  __shared__ double2 gq[kDmdMax];
  const int i = blockIdx.x, tid = threadIdx.x;
  const double2 mi = cmk(wr[i], wi[i]);
  for (int t = tid; t < n1; t += 256) {
    // mu_i^t by repeated squaring
    double2 acc = cmk(1.0, 0.0), base = mi;
    for (int e = t; e > 0; e >>= 1) {
      if (e & 1) acc = cmul(acc, base);
      base = cmul(base, base);
    }
    pw[t] = acc;
  }
  __syncthreads();
  for (int j = tid; j < k; j += 256) {
    double2 g = cmk(0.0, 0.0);
    for (int r = 0; r < k; ++r) g = cadd(g, cmul(cconj(W[(int64_t)r * k + i]), W[(int64_t)r * k + j]));
    const double2 zz = cmul(cconj(mi), cmk(wr[j], wi[j]));
    double2 sum = cmk(0.0, 0.0), pz = cmk(1.0, 0.0);
    for (int t = 0; t < n1; ++t) {
      sum = cadd(sum, pz);
      pz = cmul(pz, zz);
    }
    P[(int64_t)i * k + j] = cmul(g, sum);
    const double* vr = VT + (int64_t)j * ldvt;
    double2 gj = cmk(0.0, 0.0);
    for (int t = 0; t < n1; ++t) gj = cadd(gj, cscale(pw[t], vr[t]));
    gq[j] = cscale(cmul(W[(int64_t)j * k + i], gj), S[j]);
  }
  __syncthreads();
  if (tid == 0) {
    double2 acc = cmk(0.0, 0.0);
    for (int j = 0; j < k; ++j) acc = cadd(acc, gq[j]);
    q[i] = cconj(acc);
  }
}

// b = P^-1 q with P = L L^H (P Hermitian positive definite; its lower
// triangle is overwritten by L).  One workgroup.  status[0] = -1 when a
// pivot is not positive.
__global__ __launch_bounds__(256) void k_dmd_cholsolve(int k, double2* __restrict__ P,
                                                       const double2* __restrict__ q,
                                                       double2* __restrict__ b,
                                                       int* __restrict__ status) {
  __shared__ double2 y[kDmdMax];
  const int tid = threadIdx.x;
  bool ok = true;
  for (int j = 0; j < k; ++j) {
    const double d = P[(int64_t)j * k + j].x;
    if (!(d > 0.0)) {
      ok = false;
      break;
    }
    const double ljj = sqrt(d);
    __syncthreads();
    if (tid == 0) P[(int64_t)j * k + j] = cmk(ljj, 0.0);
    for (int r = j + 1 + tid; r < k; r += 256)
      P[(int64_t)r * k + j] = cscale(P[(int64_t)r * k + j], 1.0 / ljj);
    __threadfence_block();
    __syncthreads();
    const int w = k - j - 1;
    for (int idx = tid; idx < w * w; idx += 256) {
      const int r = j + 1 + idx / w, c = j + 1 + idx % w;
      if (c <= r)
        P[(int64_t)r * k + c] =
            csub(P[(int64_t)r * k + c], cmul(P[(int64_t)r * k + j], cconj(P[(int64_t)c * k + j])));
    }
    __threadfence_block();
    __syncthreads();
  }
  if (!ok) {
    if (tid == 0) status[0] = -1;
    for (int j = tid; j < k; j += 256) b[j] = cmk(0.0, 0.0);
    return;
  }
  for (int j = tid; j < k; j += 256) y[j] = q[j];
  __syncthreads();
  // L y = q
  for (int j = 0; j < k; ++j) {
    const double2 yj = cscale(y[j], 1.0 / P[(int64_t)j * k + j].x);
    __syncthreads();
    if (tid == 0) y[j] = yj;
    for (int r = j + 1 + tid; r < k; r += 256) y[r] = csub(y[r], cmul(P[(int64_t)r * k + j], yj));
    __syncthreads();
  }
  // L^H b = y
  for (int j = k - 1; j >= 0; --j) {
    const double2 bj = cscale(y[j], 1.0 / P[(int64_t)j * k + j].x);
    __syncthreads();
    if (tid == 0) y[j] = bj;
    for (int r = tid; r < j; r += 256) y[r] = csub(y[r], cmul(cconj(P[(int64_t)j * k + r]), bj));
    __syncthreads();
  }
  for (int j = tid; j < k; j += 256) b[j] = y[j];
}

// Order by |b| descending (ties: Im(mu) descending, then index); write mu, b,
// f = arg(mu) / (2 pi dt) and log|mu| / dt in that order, and perm (output
// position -> eigenvalue index).  One workgroup.
__global__ __launch_bounds__(256) void k_dmd_order(int k, double dt, const double* __restrict__ wr,
                                                   const double* __restrict__ wi,
                                                   const double2* __restrict__ bv,
                                                   double2* __restrict__ mu_out,
                                                   double2* __restrict__ b_out,
                                                   double* __restrict__ freq,
                                                   double* __restrict__ growth,
                                                   int* __restrict__ perm) {
  for (int i = threadIdx.x; i < k; i += 256) {
    const double ai = cabs2(bv[i]);
    int rank = 0;
    for (int j = 0; j < k; ++j) {
      const double aj = cabs2(bv[j]);
      if (aj > ai || (aj == ai && (wi[j] > wi[i] || (wi[j] == wi[i] && j < i)))) ++rank;
    }
    mu_out[rank] = cmk(wr[i], wi[i]);
    b_out[rank] = bv[i];
    if (freq) freq[rank] = atan2(wi[i], wr[i]) / (2.0 * 3.14159265358979323846 * dt);
    if (growth) growth[rank] = log(hypot(wr[i], wi[i])) / dt;
    perm[rank] = i;
  }
}

// B[t][2c], B[t][2c+1] = Re, Im of (sum_j VT[j][t] / s_j w[j][perm[c]]) / mu_perm[c]
// for t < n1, c < k: the right factor of phi = Y2 W S^-1 w / mu (Eq. dmdmodes).
__global__ __launch_bounds__(128) void k_dmd_mode_rhs(int k, int n1, const double* __restrict__ VT,
                                                      int64_t ldvt, const double* __restrict__ S,
                                                      const double2* __restrict__ W,
                                                      const double* __restrict__ wr,
                                                      const double* __restrict__ wi,
                                                      const int* __restrict__ perm,
                                                      double* __restrict__ B) {
  __shared__ double vs[kDmdMax];
  const int t = blockIdx.x;
  for (int j = threadIdx.x; j < k; j += 128) vs[j] = VT[(int64_t)j * ldvt + t] / S[j];
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += 128) {
    const int e = perm[c];
    double2 acc = cmk(0.0, 0.0);
    for (int j = 0; j < k; ++j) acc = cadd(acc, cscale(W[(int64_t)j * k + e], vs[j]));
    const double2 v = cdiv(acc, cmk(wr[e], wi[e]));
    B[(int64_t)t * 2 * k + 2 * c] = v.x;
    B[(int64_t)t * 2 * k + 2 * c + 1] = v.y;
  }
}

__global__ void k_dmd_r1(int64_t n1, int64_t n, const double* __restrict__ R,
                         double* __restrict__ R1) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n1 * n1;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / n1, j = idx % n1;
    R1[idx] = R[i * n + j];
  }
}

hipError_t launch_dmd_r1(int64_t n1, int64_t n, const double* R, double* R1, hipStream_t st) {
  int64_t g = (n1 * n1 + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_dmd_r1, dim3((unsigned)g), dim3(256), 0, st, n1, n, R, R1);
  return hipGetLastError();
}

size_t dmd_eig_lds_bytes(int k) {
  return sizeof(double) * ((size_t)k * (size_t)(k | 1) + (size_t)k + 8);
}

hipError_t launch_dmd_small(const DmdSmallArgs& a, hipStream_t st) {
  const int k = a.k, n1 = a.n1;
  if (k < 1 || k > kDmdMax || n1 < k) return hipErrorInvalidValue;
  const size_t lds = dmd_eig_lds_bytes(k);
  hipError_t e;
  hipLaunchKernelGGL(k_dmd_linear_map, dim3(k), dim3(256), 0, st, k, n1, a.aux, a.VT, a.ldvt, a.S,
                     a.A);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_dmd_hess, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dmd_hess, dim3(1), dim3(256), lds, st, k, a.A, a.H0, a.Qv, a.Qtau);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_dmd_hqr, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dmd_hqr, dim3(1), dim3(256), lds, st, k, a.H0, a.wr, a.wi, a.hnorm,
                     a.status);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_dmd_invit, dim3(k), dim3(256), 0, st, k, a.H0, a.wr, a.wi, a.hnorm, a.Qv,
                     a.Qtau, a.Ubuf, a.W);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t lds_pw = sizeof(double2) * (size_t)n1;
  e = hipFuncSetAttribute((const void*)k_dmd_amp_matrix,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_pw);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dmd_amp_matrix, dim3(k), dim3(256), lds_pw, st, k, n1, a.wr, a.wi, a.W,
                     a.VT, a.ldvt, a.S, a.P, a.q);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_dmd_cholsolve, dim3(1), dim3(256), 0, st, k, a.P, a.q, a.b, a.status);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_dmd_order, dim3(1), dim3(256), 0, st, k, a.dt, a.wr, a.wi, a.b, a.mu_out,
                     a.b_out, a.freq, a.growth, a.perm);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_dmd_mode_rhs, dim3(n1), dim3(128), 0, st, k, n1, a.VT, a.ldvt, a.S, a.W,
                     a.wr, a.wi, a.perm, a.B);
  return hipGetLastError();
}

}  // namespace pylom
