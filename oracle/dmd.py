"""CPU oracle for exact DMD on top of the TS-SVD (pyLOM, arXiv 2405.15529).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/`` may
import it.  The product never imports or calls it.

Plain FP64 / complex128 numpy, following Sec. 3.2 (exact DMD of Tu et al.),
Alg. 3 (DMD), Alg. 4 (the product U^T Y2 on one address space) and Alg. 5
(amplitudes of Jovanovic et al.).  Library primitives used as steps: the
oracle's own TS-SVD (``oracle.pod``), numpy matmul, ``numpy.linalg.eig``
(the non-symmetric eigendecomposition Alg. 3 takes from LAPACK) and
``numpy.linalg.cholesky`` / ``solve`` (the Cholesky solve of Alg. 5).

Readings (where the printed text is garbled or terse):

* V in the linear map A = U^T Y2 V S^-1 is the matrix of right singular
  vectors as columns, W = VT[:N_r].T; the listing's A = aux (S^-1 V)^T is the
  same matrix with V the rows of VT.
* The mean of the remove-mean option is taken over all N snapshots (the
  listing removes it from D before splitting off Y1 and Y2).
* In Alg. 5, q = conj(diag(V_and W S w)) (the listing's product G w lacks
  the transpose of G = S V that makes the shapes agree), and
  P = (w^H w) o conj(V_and V_and^H) with o the elementwise product.
* Each eigenvector is scaled to unit 2-norm with its largest-magnitude
  entry (lowest index on ties) real and positive, as LAPACK's dgeev does.
* Modes are ordered by |b| descending; ties by Im(mu) descending, then by
  the eigenvalue's index.
* Frequencies f = arg(mu) / (2 pi dt) (Eq. freq); growth rates
  log|mu| / dt.
"""
from __future__ import annotations

import numpy as np

from . import pod as _tsvd_pod


def normalise_eigvecs(w):
    """Unit 2-norm columns, the largest-|.| entry (lowest index on ties) real
    and positive."""
    w = np.array(w, dtype=np.complex128)
    for i in range(w.shape[1]):
        c = w[:, i] / np.linalg.norm(w[:, i])
        j = int(np.argmax(np.abs(c)))
        c = c * (np.conj(c[j]) / abs(c[j]))
        c[j] = abs(c[j])  # exactly real
        w[:, i] = c
    return w


def dmd(D, remove_mean: bool = False, r: float = 0.0, dt: float = 1.0):
    """Exact DMD of the m x N snapshot matrix D (Alg. 3).

    Returns dict(nr, mu, b, phi (m x nr), freq, growth, w (nr x nr), A, S, U,
    VT, mean) with every modal quantity in the |b|-descending order."""
    D = np.asarray(D, dtype=np.float64)
    m, N = D.shape
    if N < 2:
        raise ValueError("DMD needs at least two snapshots")
    mean = D.mean(axis=1) if remove_mean else np.zeros(m)
    Y = D - mean[:, None]
    Y1, Y2 = Y[:, :-1], Y[:, 1:]
    # TS-SVD of Y1 and truncation (Alg. 1, residual r)
    s = _tsvd_pod(Y1, remove_mean=False, r=r)
    k = s["nr"]
    if k == 0:
        return dict(nr=0, mu=np.zeros(0, complex), b=np.zeros(0, complex),
                    phi=np.zeros((m, 0), complex), freq=np.zeros(0), growth=np.zeros(0),
                    w=np.zeros((0, 0), complex), A=np.zeros((0, 0)), S=s["S"], U=s["U"],
                    VT=s["VT"], mean=mean)
    U = s["U"][:, :k]
    S = s["S"][:k]
    W = s["VT"][:k].T                                  # (N - 1) x k
    # linear map A = U^T Y2 W S^-1 (Alg. 4 gives U^T Y2)
    aux = U.T @ Y2
    A = (aux @ W) / S[None, :]
    mu, w = np.linalg.eig(A)
    mu = mu.astype(np.complex128)
    w = normalise_eigvecs(w)
    # amplitudes (Alg. 5): least squares fit of S W^T by w diag(b) V_and
    t = np.arange(N - 1)
    Vand = mu[:, None] ** t[None, :]                  # k x (N - 1)
    P = (w.conj().T @ w) * np.conj(Vand @ Vand.conj().T)
    q = np.conj(np.diag(Vand @ (W * S[None, :]) @ w))
    L = np.linalg.cholesky(P)
    y = np.linalg.solve(L, q)
    b = np.linalg.solve(L.conj().T, y)
    # order by |b| descending, ties by Im(mu) descending, then index
    order = sorted(range(k), key=lambda i: (-abs(b[i]), -mu[i].imag, i))
    order = np.array(order, dtype=np.int64)
    mu, b, w = mu[order], b[order], w[:, order]
    # exact DMD modes (Eq. dmdmodes): phi = Y2 W S^-1 w / mu
    phi = (Y2 @ (W / S[None, :]) @ w) / mu[None, :]
    freq = np.angle(mu) / (2.0 * np.pi * dt)
    growth = np.log(np.abs(mu)) / dt
    return dict(nr=k, mu=mu, b=b, phi=phi, freq=freq, growth=growth, w=w, A=A, S=s["S"],
                U=s["U"], VT=s["VT"], mean=mean)
