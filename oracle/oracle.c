/*
 * oracle.c -- plain, slow, obviously-correct CPU oracle for the POD
 * tall-skinny SVD path of pyLOM (arXiv 2405.15529).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or helper with the
 * HIP implementation.
 *
 * Everything is FP64 (complex128 for SPOD), unblocked, single-threaded, and
 * follows the plain mathematical definition of each step:
 *
 *   mean removal      Alg. 2 (POD algorithm, appendix B): row mean over the n
 *                     snapshots, subtracted from every snapshot.
 *   QR                Eq. svdqr1: D = Q [R; 0], computed by unblocked
 *                     Householder reflections on the WHOLE matrix (no tree:
 *                     the TSQR tree of Alg. 1 reaches the same R up to row
 *                     signs, so the definition is a plain QR).
 *   SVD of R          Eq. svdqr2, by one-sided (Hestenes) Jacobi rotations
 *                     with Rutishauser's formula, cyclic-by-rows ordering.
 *   U = Q U_R         Eq. svdqr3, by applying the reflectors to [U_R; 0].
 *   energy            Sec. 3.1 cumulative-energy ratio; truncation residual r
 *                     of Alg. 3 read as: N_r = min{k>=1 : sum_{i>k} s_i^2 <=
 *                     r * sum_i s_i^2}.
 *   matmul            Alg. 4: C = sum over row blocks of A_i^T B_i, i.e. a
 *                     plain triple loop.
 *   SPOD              Alg. 6 + Sec. 3.3 (Frame-Towne): Welch blocks, window,
 *                     a DIRECT DFT (the definition, not an FFT), one-sided
 *                     doubling, then the complex SVD of Q_f / sqrt(nBlks).
 *
 * All matrices at this interface are ROW-MAJOR with an explicit leading
 * dimension, like the product's C-ABI; internally the oracle works on
 * column-major copies.
 */
#define _DEFAULT_SOURCE 1
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex zdouble;

static const double ORC_PI = 3.14159265358979323846264338327950288;

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOCONV 1

/* ------------------------------------------------------------------ */
/* mean removal (Alg. 2)                                               */
/* ------------------------------------------------------------------ */

/* mean[j] = (1/n) * sum_{t=0}^{n-1} D[j, t]  (D row-major, m x n). */
int orc_mean(int64_t m, int64_t n, const double* D, int64_t ldd, double* mean) {
  if (m < 0 || n < 1 || ldd < n) return ORC_EINVAL;
  for (int64_t j = 0; j < m; ++j) {
    double s = 0.0;
    for (int64_t t = 0; t < n; ++t) s += D[j * ldd + t];
    mean[j] = s / (double)n;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* real Householder QR (Eq. svdqr1), column-major A (m x n, lda)       */
/* ------------------------------------------------------------------ */

/* On exit the upper triangle of A holds R, the strict lower part holds the
 * reflector tails v (v_k[k] = 1 implicit), tau[k] the scalar factors, so that
 * Q = H_0 H_1 ... H_{n-1},  H_k = I - tau_k v_k v_k^T.  Requires m >= n. */
static void householder_qr_cm(int64_t m, int64_t n, double* A, int64_t lda, double* tau) {
  for (int64_t k = 0; k < n; ++k) {
    double* x = A + k * lda;
    double alpha = x[k];
    double sig = 0.0;
    for (int64_t i = k + 1; i < m; ++i) sig += x[i] * x[i];
    if (sig == 0.0) {
      tau[k] = 0.0;
      continue;
    }
    double beta = sqrt(alpha * alpha + sig);
    if (alpha >= 0.0) beta = -beta;
    tau[k] = (beta - alpha) / beta;
    double scal = 1.0 / (alpha - beta);
    for (int64_t i = k + 1; i < m; ++i) x[i] *= scal;
    x[k] = beta;
    /* apply H_k to the trailing columns: a_j -= tau * v * (v^T a_j) */
    for (int64_t j = k + 1; j < n; ++j) {
      double* a = A + j * lda;
      double w = a[k];
      for (int64_t i = k + 1; i < m; ++i) w += x[i] * a[i];
      w *= tau[k];
      a[k] -= w;
      for (int64_t i = k + 1; i < m; ++i) a[i] -= w * x[i];
    }
  }
}

/* X (m x k, column-major, ldx) <- Q X, Q = H_0 ... H_{n-1}. */
static void apply_q_cm(int64_t m, int64_t n, const double* A, int64_t lda, const double* tau,
                       int64_t k, double* X, int64_t ldx) {
  for (int64_t r = n - 1; r >= 0; --r) {
    if (tau[r] == 0.0) continue;
    const double* v = A + r * lda;
    for (int64_t c = 0; c < k; ++c) {
      double* x = X + c * ldx;
      double w = x[r];
      for (int64_t i = r + 1; i < m; ++i) w += v[i] * x[i];
      w *= tau[r];
      x[r] -= w;
      for (int64_t i = r + 1; i < m; ++i) x[i] -= w * v[i];
    }
  }
}

/* ------------------------------------------------------------------ */
/* one-sided Jacobi SVD of a square matrix (Eq. svdqr2)                */
/* ------------------------------------------------------------------ */

static double dot_cm(int64_t n, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* Complete a set of orthonormal columns: column `col` of U (n x n, col-major)
 * gets the unit vector most orthogonal to columns [0, col), built from the
 * standard basis by two Gram-Schmidt passes. */
static void complete_basis_cm(int64_t n, double* U, int64_t col) {
  double* best = (double*)malloc(sizeof(double) * n);
  double* tmp = (double*)malloc(sizeof(double) * n);
  double bestn = -1.0;
  for (int64_t e = 0; e < n; ++e) {
    for (int64_t i = 0; i < n; ++i) tmp[i] = (i == e) ? 1.0 : 0.0;
    for (int pass = 0; pass < 2; ++pass)
      for (int64_t c = 0; c < col; ++c) {
        double p = dot_cm(n, U + c * n, tmp);
        for (int64_t i = 0; i < n; ++i) tmp[i] -= p * U[c * n + i];
      }
    double nn = sqrt(dot_cm(n, tmp, tmp));
    if (nn > bestn) {
      bestn = nn;
      memcpy(best, tmp, sizeof(double) * n);
    }
  }
  for (int64_t i = 0; i < n; ++i) U[col * n + i] = best[i] / bestn;
  free(best);
  free(tmp);
}

/* SVD of R (n x n, column-major, ldr):  R = U_R diag(S) V^T.
 * W <- R; V <- I; cyclic sweeps over pairs (p<q): if the pair is not yet
 * orthogonal to the tolerance n*eps, rotate columns p,q of W and V by the
 * Jacobi rotation that makes them orthogonal (Rutishauser's formula).
 * Then S = column norms sorted descending (stable), U_R = W / S.
 * Returns sweeps used, or -1 if max_sweeps was reached without convergence. */
static int jacobi_svd_cm(int64_t n, const double* R, int64_t ldr, double* S, double* UR,
                         double* V, int max_sweeps) {
  double* W = (double*)malloc(sizeof(double) * n * n);
  double* Vt = (double*)malloc(sizeof(double) * n * n);
  double* nrm = (double*)malloc(sizeof(double) * n);
  int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * n);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i) {
      W[j * n + i] = R[j * ldr + i];
      Vt[j * n + i] = (i == j) ? 1.0 : 0.0;
    }
  const double tol = (double)n * 0x1p-53;
  int sweeps = -1;
  for (int sw = 1; sw <= max_sweeps; ++sw) {
    int rotated = 0;
    for (int64_t p = 0; p < n - 1; ++p)
      for (int64_t q = p + 1; q < n; ++q) {
        double* wp = W + p * n;
        double* wq = W + q * n;
        double a = dot_cm(n, wp, wp);
        double b = dot_cm(n, wq, wq);
        double g = dot_cm(n, wp, wq);
        if (a == 0.0 || b == 0.0) continue;
        if (fabs(g) <= tol * sqrt(a) * sqrt(b)) continue;
        rotated = 1;
        double zeta = (b - a) / (2.0 * g);
        double t = 1.0 / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        if (zeta < 0.0) t = -t;
        double c = 1.0 / sqrt(1.0 + t * t);
        double s = c * t;
        for (int64_t i = 0; i < n; ++i) {
          double x = wp[i], y = wq[i];
          wp[i] = c * x - s * y;
          wq[i] = s * x + c * y;
        }
        double* vp = Vt + p * n;
        double* vq = Vt + q * n;
        for (int64_t i = 0; i < n; ++i) {
          double x = vp[i], y = vq[i];
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
      }
    if (!rotated) {
      sweeps = sw;
      break;
    }
  }
  for (int64_t j = 0; j < n; ++j) {
    nrm[j] = sqrt(dot_cm(n, W + j * n, W + j * n));
    idx[j] = j;
  }
  /* stable insertion sort, descending */
  for (int64_t i = 1; i < n; ++i) {
    int64_t k = idx[i];
    int64_t j = i - 1;
    while (j >= 0 && nrm[idx[j]] < nrm[k]) {
      idx[j + 1] = idx[j];
      --j;
    }
    idx[j + 1] = k;
  }
  for (int64_t c = 0; c < n; ++c) {
    int64_t src = idx[c];
    S[c] = nrm[src];
    for (int64_t i = 0; i < n; ++i) V[c * n + i] = Vt[src * n + i];
  }
  for (int64_t c = 0; c < n; ++c) {
    int64_t src = idx[c];
    if (S[c] > 0.0) {
      for (int64_t i = 0; i < n; ++i) UR[c * n + i] = W[src * n + i] / S[c];
    }
  }
  for (int64_t c = 0; c < n; ++c)
    if (!(S[c] > 0.0)) complete_basis_cm(n, UR, c);
  free(W);
  free(Vt);
  free(nrm);
  free(idx);
  return sweeps;
}

/* Sign convention for the (u_i, v_i) pairs: the entry of v_i with the largest
 * magnitude (lowest index on ties) is made positive; u_i follows. */
static void sign_normalize_cm(int64_t n, int64_t k, double* UR, int64_t ldu, double* V,
                              int64_t ldv) {
  for (int64_t c = 0; c < k; ++c) {
    int64_t arg = 0;
    double best = -1.0;
    for (int64_t i = 0; i < n; ++i) {
      double a = fabs(V[c * ldv + i]);
      if (a > best) {
        best = a;
        arg = i;
      }
    }
    if (V[c * ldv + arg] < 0.0) {
      for (int64_t i = 0; i < n; ++i) V[c * ldv + i] = -V[c * ldv + i];
      for (int64_t i = 0; i < n; ++i) UR[c * ldu + i] = -UR[c * ldu + i];
    }
  }
}

/* ------------------------------------------------------------------ */
/* energy truncation                                                   */
/* ------------------------------------------------------------------ */

/* N_r = min{k >= 1 : sum_{i>k} S_i^2 <= r * sum_i S_i^2}, S descending.
 * Tail sums are accumulated from the smallest value upward.  r <= 0 keeps
 * all n modes; an all-zero spectrum keeps none. */
int64_t orc_truncate(int64_t n, const double* S, double r) {
  if (n <= 0) return 0;
  if (!(r > 0.0)) return n;
  double* tail = (double*)malloc(sizeof(double) * (n + 1));
  tail[n] = 0.0;
  for (int64_t k = n - 1; k >= 0; --k) tail[k] = tail[k + 1] + S[k] * S[k];
  double total = tail[0];
  int64_t nr = n;
  if (total == 0.0) {
    nr = 0;
  } else {
    for (int64_t k = 1; k <= n; ++k)
      if (tail[k] <= r * total) {
        nr = k;
        break;
      }
  }
  free(tail);
  return nr;
}

/* ------------------------------------------------------------------ */
/* public real entry points                                            */
/* ------------------------------------------------------------------ */

/* Householder QR of a row-major m x n matrix; outputs (both row-major):
 *   R  n x n upper triangular with diag(R) >= 0,
 *   Q  m x n with orthonormal columns (may be NULL).
 * A = Q R. */
int orc_qr(int64_t m, int64_t n, const double* A, int64_t lda, double* Q, int64_t ldq, double* R,
           int64_t ldr) {
  if (n < 1 || m < n || lda < n || ldr < n || (Q && ldq < n)) return ORC_EINVAL;
  double* Ac = (double*)malloc(sizeof(double) * m * n);
  double* tau = (double*)malloc(sizeof(double) * n);
  if (!Ac || !tau) return ORC_ENOMEM;
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) Ac[j * m + i] = A[i * lda + j];
  householder_qr_cm(m, n, Ac, m, tau);
  double* sgn = (double*)malloc(sizeof(double) * n);
  for (int64_t k = 0; k < n; ++k) sgn[k] = (Ac[k * m + k] < 0.0) ? -1.0 : 1.0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) R[i * ldr + j] = (j >= i) ? sgn[i] * Ac[j * m + i] : 0.0;
  if (Q) {
    double* X = (double*)calloc((size_t)(m * n), sizeof(double));
    for (int64_t k = 0; k < n; ++k) X[k * m + k] = 1.0;
    apply_q_cm(m, n, Ac, m, tau, n, X, m);
    for (int64_t i = 0; i < m; ++i)
      for (int64_t j = 0; j < n; ++j) Q[i * ldq + j] = sgn[j] * X[j * m + i];
    free(X);
  }
  free(sgn);
  free(Ac);
  free(tau);
  return ORC_OK;
}

/* SVD of a square row-major n x n matrix by one-sided Jacobi, with the sign
 * convention applied.  Outputs row-major: U (n x n, columns = u_i),
 * S (n, descending), VT (n x n, rows = v_i^T).  Returns sweeps or -1. */
int orc_svd_square(int64_t n, const double* R, int64_t ldr, double* U, int64_t ldu, double* S,
                   double* VT, int64_t ldvt, int max_sweeps) {
  double* Rc = (double*)malloc(sizeof(double) * n * n);
  double* UR = (double*)malloc(sizeof(double) * n * n);
  double* V = (double*)malloc(sizeof(double) * n * n);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) Rc[j * n + i] = R[i * ldr + j];
  int sw = jacobi_svd_cm(n, Rc, n, S, UR, V, max_sweeps);
  sign_normalize_cm(n, n, UR, n, V, n);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      U[i * ldu + j] = UR[j * n + i];
      VT[i * ldvt + j] = V[i * n + j];
    }
  free(Rc);
  free(UR);
  free(V);
  return sw;
}

/* POD (Alg. 2 -> Alg. 1 -> Eqs. svdqr1-3 -> truncation).
 * D: row-major m x n snapshot matrix (rows = points, columns = snapshots).
 * Outputs (row-major): mean (m, may be NULL), U (m x n: all n modes),
 * S (n), VT (n x n: all n rows), *n_r (truncation count for residual r).
 * Returns the Jacobi sweep count (>0), or -1 on non-convergence, <-1 error. */
int orc_pod(int64_t m, int64_t n, const double* D, int64_t ldd, int remove_mean, double r,
            double* mean, double* U, int64_t ldu, double* S, double* VT, int64_t ldvt,
            int64_t* n_r, int max_sweeps) {
  if (n < 1 || m < n || ldd < n || ldu < n || ldvt < n) return -100;
  double* mu = (double*)calloc((size_t)m, sizeof(double));
  if (remove_mean) orc_mean(m, n, D, ldd, mu);
  if (mean)
    for (int64_t j = 0; j < m; ++j) mean[j] = mu[j];
  double* Y = (double*)malloc(sizeof(double) * m * n);
  double* tau = (double*)malloc(sizeof(double) * n);
  if (!Y || !tau) return -101;
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) Y[j * m + i] = D[i * ldd + j] - mu[i];
  householder_qr_cm(m, n, Y, m, tau);
  double* Rc = (double*)calloc((size_t)(n * n), sizeof(double));
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i <= j; ++i) Rc[j * n + i] = Y[j * m + i];
  double* UR = (double*)malloc(sizeof(double) * n * n);
  double* V = (double*)malloc(sizeof(double) * n * n);
  int sw = jacobi_svd_cm(n, Rc, n, S, UR, V, max_sweeps);
  sign_normalize_cm(n, n, UR, n, V, n);
  *n_r = orc_truncate(n, S, r);
  double* X = (double*)calloc((size_t)(m * n), sizeof(double));
  for (int64_t c = 0; c < n; ++c)
    for (int64_t i = 0; i < n; ++i) X[c * m + i] = UR[c * n + i];
  apply_q_cm(m, n, Y, m, tau, n, X, m);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t c = 0; c < n; ++c) U[i * ldu + c] = X[c * m + i];
  for (int64_t c = 0; c < n; ++c)
    for (int64_t j = 0; j < n; ++j) VT[c * ldvt + j] = V[c * n + j];
  free(mu);
  free(Y);
  free(tau);
  free(Rc);
  free(UR);
  free(V);
  free(X);
  return sw;
}

/* Alg. 4 on one address space: C = A^T B (trans_a = 1; A m x p, B m x q,
 * C p x q) or C = A B (trans_a = 0; A m x p, B p x q, C m x q).  All
 * row-major, FP64 accumulation in natural order. */
int orc_matmul(int trans_a, int64_t m, int64_t p, int64_t q, const double* A, int64_t lda,
               const double* B, int64_t ldb, double* C, int64_t ldc) {
  if (trans_a) {
    for (int64_t i = 0; i < p; ++i)
      for (int64_t j = 0; j < q; ++j) {
        double s = 0.0;
        for (int64_t k = 0; k < m; ++k) s += A[k * lda + i] * B[k * ldb + j];
        C[i * ldc + j] = s;
      }
  } else {
    for (int64_t i = 0; i < m; ++i)
      for (int64_t j = 0; j < q; ++j) {
        double s = 0.0;
        for (int64_t k = 0; k < p; ++k) s += A[i * lda + k] * B[k * ldb + j];
        C[i * ldc + j] = s;
      }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* complex128 versions (SPOD per-frequency SVD, Sec. 3.3 / Alg. 6)     */
/* ------------------------------------------------------------------ */

/* Householder QR, column-major complex A. Reflector k: H_k = I - tau_k v v^H
 * with H_k^H [alpha; x] = [beta; 0], beta real.  Q = H_0 ... H_{n-1}. */
static void zhouseholder_qr_cm(int64_t m, int64_t n, zdouble* A, int64_t lda, zdouble* tau) {
  for (int64_t k = 0; k < n; ++k) {
    zdouble* x = A + k * lda;
    zdouble alpha = x[k];
    double sig = 0.0;
    for (int64_t i = k + 1; i < m; ++i) sig += creal(x[i] * conj(x[i]));
    if (sig == 0.0 && cimag(alpha) == 0.0) {
      tau[k] = 0.0;
      continue;
    }
    double beta = sqrt(creal(alpha * conj(alpha)) + sig);
    if (creal(alpha) >= 0.0) beta = -beta;
    tau[k] = (beta - alpha) / beta;
    zdouble scal = 1.0 / (alpha - beta);
    for (int64_t i = k + 1; i < m; ++i) x[i] *= scal;
    x[k] = beta;
    /* apply H_k^H = I - conj(tau) v v^H to the trailing columns */
    zdouble tc = conj(tau[k]);
    for (int64_t j = k + 1; j < n; ++j) {
      zdouble* a = A + j * lda;
      zdouble w = a[k];
      for (int64_t i = k + 1; i < m; ++i) w += conj(x[i]) * a[i];
      w *= tc;
      a[k] -= w;
      for (int64_t i = k + 1; i < m; ++i) a[i] -= w * x[i];
    }
  }
}

/* X <- Q X with Q = H_0 ... H_{n-1}, H = I - tau v v^H. */
static void zapply_q_cm(int64_t m, int64_t n, const zdouble* A, int64_t lda, const zdouble* tau,
                        int64_t k, zdouble* X, int64_t ldx) {
  for (int64_t r = n - 1; r >= 0; --r) {
    if (tau[r] == 0.0) continue;
    const zdouble* v = A + r * lda;
    for (int64_t c = 0; c < k; ++c) {
      zdouble* x = X + c * ldx;
      zdouble w = x[r];
      for (int64_t i = r + 1; i < m; ++i) w += conj(v[i]) * x[i];
      w *= tau[r];
      x[r] -= w;
      for (int64_t i = r + 1; i < m; ++i) x[i] -= w * v[i];
    }
  }
}

static zdouble zdotc_cm(int64_t n, const zdouble* a, const zdouble* b) {
  zdouble s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += conj(a[i]) * b[i];
  return s;
}

static void zcomplete_basis_cm(int64_t n, zdouble* U, int64_t col) {
  zdouble* best = (zdouble*)malloc(sizeof(zdouble) * n);
  zdouble* tmp = (zdouble*)malloc(sizeof(zdouble) * n);
  double bestn = -1.0;
  for (int64_t e = 0; e < n; ++e) {
    for (int64_t i = 0; i < n; ++i) tmp[i] = (i == e) ? 1.0 : 0.0;
    for (int pass = 0; pass < 2; ++pass)
      for (int64_t c = 0; c < col; ++c) {
        zdouble p = zdotc_cm(n, U + c * n, tmp);
        for (int64_t i = 0; i < n; ++i) tmp[i] -= p * U[c * n + i];
      }
    double nn = sqrt(creal(zdotc_cm(n, tmp, tmp)));
    if (nn > bestn) {
      bestn = nn;
      memcpy(best, tmp, sizeof(zdouble) * n);
    }
  }
  for (int64_t i = 0; i < n; ++i) U[col * n + i] = best[i] / bestn;
  free(best);
  free(tmp);
}

/* Complex one-sided Jacobi: for a non-orthogonal pair with g = w_p^H w_q =
 * |g| e^{i phi}, the unitary J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] acting
 * on columns (p, q) makes them orthogonal (real rotation of w_p against
 * e^{-i phi} w_q).  R = U_R S V^H on exit. */
static int zjacobi_svd_cm(int64_t n, const zdouble* R, int64_t ldr, double* S, zdouble* UR,
                          zdouble* V, int max_sweeps) {
  zdouble* W = (zdouble*)malloc(sizeof(zdouble) * n * n);
  zdouble* Vt = (zdouble*)malloc(sizeof(zdouble) * n * n);
  double* nrm = (double*)malloc(sizeof(double) * n);
  int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * n);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i) {
      W[j * n + i] = R[j * ldr + i];
      Vt[j * n + i] = (i == j) ? 1.0 : 0.0;
    }
  const double tol = (double)n * 0x1p-53;
  int sweeps = -1;
  for (int sw = 1; sw <= max_sweeps; ++sw) {
    int rotated = 0;
    for (int64_t p = 0; p < n - 1; ++p)
      for (int64_t q = p + 1; q < n; ++q) {
        zdouble* wp = W + p * n;
        zdouble* wq = W + q * n;
        double a = creal(zdotc_cm(n, wp, wp));
        double b = creal(zdotc_cm(n, wq, wq));
        zdouble g = zdotc_cm(n, wp, wq);
        double ga = cabs(g);
        if (a == 0.0 || b == 0.0) continue;
        if (ga <= tol * sqrt(a) * sqrt(b)) continue;
        rotated = 1;
        zdouble ph = conj(g) / ga; /* e^{-i phi} */
        double zeta = (b - a) / (2.0 * ga);
        double t = 1.0 / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        if (zeta < 0.0) t = -t;
        double c = 1.0 / sqrt(1.0 + t * t);
        double s = c * t;
        for (int64_t i = 0; i < n; ++i) {
          zdouble x = wp[i], y = ph * wq[i];
          wp[i] = c * x - s * y;
          wq[i] = s * x + c * y;
        }
        zdouble* vp = Vt + p * n;
        zdouble* vq = Vt + q * n;
        for (int64_t i = 0; i < n; ++i) {
          zdouble x = vp[i], y = ph * vq[i];
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
      }
    if (!rotated) {
      sweeps = sw;
      break;
    }
  }
  for (int64_t j = 0; j < n; ++j) {
    nrm[j] = sqrt(creal(zdotc_cm(n, W + j * n, W + j * n)));
    idx[j] = j;
  }
  for (int64_t i = 1; i < n; ++i) {
    int64_t k = idx[i];
    int64_t j = i - 1;
    while (j >= 0 && nrm[idx[j]] < nrm[k]) {
      idx[j + 1] = idx[j];
      --j;
    }
    idx[j + 1] = k;
  }
  for (int64_t c = 0; c < n; ++c) {
    int64_t src = idx[c];
    S[c] = nrm[src];
    for (int64_t i = 0; i < n; ++i) V[c * n + i] = Vt[src * n + i];
    if (S[c] > 0.0)
      for (int64_t i = 0; i < n; ++i) UR[c * n + i] = W[src * n + i] / S[c];
  }
  for (int64_t c = 0; c < n; ++c)
    if (!(S[c] > 0.0)) zcomplete_basis_cm(n, UR, c);
  free(W);
  free(Vt);
  free(nrm);
  free(idx);
  return sweeps;
}

/* Phase convention: (u_i, v_i) are multiplied by e^{-i theta}, theta the
 * argument of the largest-magnitude entry of v_i (lowest index on ties). */
static void zphase_normalize_cm(int64_t n, int64_t k, zdouble* UR, zdouble* V) {
  for (int64_t c = 0; c < k; ++c) {
    int64_t arg = 0;
    double best = -1.0;
    for (int64_t i = 0; i < n; ++i) {
      double a = cabs(V[c * n + i]);
      if (a > best) {
        best = a;
        arg = i;
      }
    }
    if (best > 0.0) {
      zdouble ph = conj(V[c * n + arg]) / best;
      for (int64_t i = 0; i < n; ++i) V[c * n + i] *= ph;
      for (int64_t i = 0; i < n; ++i) UR[c * n + i] *= ph;
      V[c * n + arg] = best; /* exactly real */
    }
  }
}

/* Complex tall-skinny SVD of a row-major m x n complex matrix (interleaved
 * re/im doubles).  Outputs: U (m x n row-major complex), S (n),
 * VH (n x n row-major complex, rows = v_i^H).  Returns sweeps or -1. */
int orc_zsvd_tall(int64_t m, int64_t n, const double* Ain, int64_t lda, double* Uout,
                  int64_t ldu, double* S, double* VHout, int64_t ldvh, int max_sweeps) {
  if (n < 1 || m < n) return -100;
  const zdouble* A = (const zdouble*)Ain;
  zdouble* U = (zdouble*)Uout;
  zdouble* VH = (zdouble*)VHout;
  zdouble* Y = (zdouble*)malloc(sizeof(zdouble) * m * n);
  zdouble* tau = (zdouble*)malloc(sizeof(zdouble) * n);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) Y[j * m + i] = A[i * lda + j];
  zhouseholder_qr_cm(m, n, Y, m, tau);
  zdouble* Rc = (zdouble*)calloc((size_t)(n * n), sizeof(zdouble));
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i <= j; ++i) Rc[j * n + i] = Y[j * m + i];
  zdouble* UR = (zdouble*)malloc(sizeof(zdouble) * n * n);
  zdouble* V = (zdouble*)malloc(sizeof(zdouble) * n * n);
  int sw = zjacobi_svd_cm(n, Rc, n, S, UR, V, max_sweeps);
  zphase_normalize_cm(n, n, UR, V);
  zdouble* X = (zdouble*)calloc((size_t)(m * n), sizeof(zdouble));
  for (int64_t c = 0; c < n; ++c)
    for (int64_t i = 0; i < n; ++i) X[c * m + i] = UR[c * n + i];
  zapply_q_cm(m, n, Y, m, tau, n, X, m);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t c = 0; c < n; ++c) U[i * ldu + c] = X[c * m + i];
  for (int64_t c = 0; c < n; ++c)
    for (int64_t j = 0; j < n; ++j) VH[c * ldvh + j] = conj(V[c * n + j]);
  free(Y);
  free(tau);
  free(Rc);
  free(UR);
  free(V);
  free(X);
  return sw;
}

/* ------------------------------------------------------------------ */
/* SPOD front end (Alg. 6): Welch blocks, window, direct DFT           */
/* ------------------------------------------------------------------ */

/* Number of Welch blocks (Alg. 6): floor((N - nolap) / (npwin - nolap)). */
int64_t orc_spod_nblocks(int64_t nt, int64_t npwin, int64_t nolap) {
  if (npwin <= nolap || nt < npwin) return 0;
  return (nt - nolap) / (npwin - nolap);
}

/* Window over j = 0..npwin-1 with an (npwin - 1) denominator:
 * kind 0 = Hann 0.5 - 0.5 cos(2 pi j/(npwin-1)),
 * kind 1 = Hamming 0.54 - 0.46 cos(2 pi j/(npwin-1)) (the paper's choice). */
void orc_window(int64_t npwin, int kind, double* w) {
  const double a0 = kind == 1 ? 0.54 : 0.5;
  const double a1 = kind == 1 ? 0.46 : 0.5;
  for (int64_t j = 0; j < npwin; ++j)
    w[j] = a0 - a1 * cos(2.0 * ORC_PI * (double)j / (double)(npwin - 1));
}

/* Spectral array of Alg. 6 for an even npwin:
 * Q[f][p][blk] = c_f * DFT_f(Y[p, i0:i0+npwin] * w) / sum(w) / sqrt(nBlks),
 * i0 = blk*(npwin - nolap), f = 0..npwin/2, c_f = 2 for 0 < f < npwin/2 and 1
 * otherwise.  DFT_f(x) = sum_j x_j exp(-2 pi i j f / npwin).
 * D row-major m x nt real; Q complex (interleaved) of size nfreq*m*nblk. */
int orc_spod_spectra(int64_t m, int64_t nt, const double* D, int64_t ldd, int64_t npwin,
                     int64_t nolap, int window_kind, int remove_mean, double* Qout) {
  if (npwin < 2 || (npwin & 1)) return ORC_EINVAL;
  int64_t nblk = orc_spod_nblocks(nt, npwin, nolap);
  if (nblk < 1) return ORC_EINVAL;
  int64_t nfreq = npwin / 2 + 1;
  zdouble* Q = (zdouble*)Qout;
  double* w = (double*)malloc(sizeof(double) * npwin);
  orc_window(npwin, window_kind, w);
  double wsum = 0.0;
  for (int64_t j = 0; j < npwin; ++j) wsum += w[j];
  double* x = (double*)malloc(sizeof(double) * npwin);
  double inv_sqrt_nblk = 1.0 / sqrt((double)nblk);
  for (int64_t p = 0; p < m; ++p) {
    double mu = 0.0;
    if (remove_mean) {
      for (int64_t t = 0; t < nt; ++t) mu += D[p * ldd + t];
      mu /= (double)nt;
    }
    for (int64_t b = 0; b < nblk; ++b) {
      int64_t i0 = b * (npwin - nolap);
      for (int64_t j = 0; j < npwin; ++j) x[j] = (D[p * ldd + i0 + j] - mu) * w[j];
      for (int64_t f = 0; f < nfreq; ++f) {
        zdouble s = 0.0;
        for (int64_t j = 0; j < npwin; ++j) {
          double ang = -2.0 * ORC_PI * (double)((j * f) % npwin) / (double)npwin;
          s += x[j] * (cos(ang) + I * sin(ang));
        }
        double cf = (f > 0 && f < npwin / 2) ? 2.0 : 1.0;
        Q[(f * m + p) * nblk + b] = s * (cf / wsum) * inv_sqrt_nblk;
      }
    }
  }
  free(w);
  free(x);
  return ORC_OK;
}
