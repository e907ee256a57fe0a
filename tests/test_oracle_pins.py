"""Pins of the CPU oracle to facts outside itself (closed forms, exact
arithmetic, independent library routines, invariants).

Each test names the passage of the paper the checked function follows.  A
plausible slip in the oracle (a dropped term, a wrong sign or index, a
transposed operand) breaks at least one of these.
"""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle
from paper_2405_15529_amd import synth

EPS = 2.0 ** -52


# ---------------------------------------------------------------- mean (Alg. 2)

def test_mean_exact_rational():
    rng = np.random.default_rng(11)
    D = rng.integers(-50, 50, size=(37, 13)).astype(np.float64) / 8.0  # exact binary fractions
    mu = oracle.mean(D)
    for j in range(D.shape[0]):
        exact = sum(Fraction(x) for x in D[j]) / D.shape[1]
        assert abs(Fraction(mu[j]) - exact) <= Fraction(1, 2 ** 48) * (1 + abs(exact))


def test_mean_constant_field_gives_empty_pod():
    # D = c 1^T: removing the temporal mean leaves Y = 0, every sigma is 0 and
    # the energy-truncated basis is empty.
    c = np.arange(-25, 25) / 8.0  # binary fractions: the row sums are exact
    D = np.repeat(c[:, None], 8, axis=1)
    out = oracle.pod(D, remove_mean=True, r=0.01)
    assert np.array_equal(out["mean"], c)
    assert np.all(out["S"] == 0.0)
    assert out["nr"] == 0


def test_mean_is_subtracted_not_ignored():
    # A rank-one field plus an offset: with the mean removed the offset is gone.
    rng = np.random.default_rng(5)
    phi = rng.standard_normal(200)
    a = np.sin(np.arange(12) * 0.7)
    a -= a.mean()
    D = np.outer(phi, a) + 5.0
    out = oracle.pod(D, remove_mean=True, r=0.0)
    assert out["S"][0] == pytest.approx(np.linalg.norm(phi) * np.linalg.norm(a), rel=1e-13)
    assert np.all(out["S"][1:] < 1e-12)


# ------------------------------------------------------------- QR (Eq. svdqr1)

def test_qr_worked_2x2():
    # A = [[3,0],[4,5]]: first column norm 5, R = [[5,4],[0,3]] (diag >= 0).
    Q, R = oracle.qr(np.array([[3.0, 0.0], [4.0, 5.0]]))
    np.testing.assert_allclose(R, [[5.0, 4.0], [0.0, 3.0]], atol=1e-15)
    np.testing.assert_allclose(Q, [[0.6, -0.8], [0.8, 0.6]], atol=1e-15)


def test_qr_exact_gram_integer_inputs():
    # R^T R = A^T A exactly (uniqueness of the Cholesky factor with diag > 0).
    rng = np.random.default_rng(3)
    for trial in range(5):
        m, n = 9 + trial, 4 + (trial % 3)
        A = rng.integers(-9, 10, size=(m, n)).astype(np.float64)
        Q, R = oracle.qr(A)
        G = [[sum(Fraction(int(A[k, i])) * int(A[k, j]) for k in range(m)) for j in range(n)]
             for i in range(n)]
        RtR = R.T @ R
        for i in range(n):
            for j in range(n):
                assert abs(RtR[i, j] - float(G[i][j])) <= 1e-12 * (1 + abs(float(G[i][j])))
        assert np.all(np.diag(R) >= 0)
        assert np.allclose(np.tril(R, -1), 0)
        np.testing.assert_allclose(Q @ R, A, atol=1e-12)
        np.testing.assert_allclose(Q.T @ Q, np.eye(n), atol=1e-14)


def test_qr_single_column():
    a = np.array([[3.0], [0.0], [4.0], [12.0]])
    Q, R = oracle.qr(a)
    assert R[0, 0] == pytest.approx(13.0, rel=1e-15)
    np.testing.assert_allclose(Q[:, 0], a[:, 0] / 13.0, atol=1e-16)


def test_qr_orthogonal_invariance():
    # R(H A) = R(A) for orthogonal H (R unique with positive diagonal).
    rng = np.random.default_rng(8)
    A = rng.standard_normal((40, 7))
    H, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    _, R1 = oracle.qr(A, want_q=False)
    _, R2 = oracle.qr(H @ A, want_q=False)
    np.testing.assert_allclose(R1, R2, atol=1e-12)


# ------------------------------------------------- SVD of R (Eq. svdqr2)

def test_svd_worked_2x2():
    # [[3,0],[4,5]]: A^T A = [[25,20],[20,25]] -> sigma^2 = 45, 5.
    U, S, VT, sw = oracle.svd_square(np.array([[3.0, 0.0], [4.0, 5.0]]))
    assert S[0] == pytest.approx(3.0 * math.sqrt(5.0), rel=1e-15)
    assert S[1] == pytest.approx(math.sqrt(5.0), rel=1e-15)
    assert sw > 0


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_svd_brute_force_small_integer(n):
    # sigma^2 are the eigenvalues of the exact integer Gram matrix; compared
    # with numpy's symmetric eigensolver on that Gram (independent routine).
    rng = np.random.default_rng(100 + n)
    for _ in range(6):
        A = rng.integers(-6, 7, size=(n, n)).astype(np.float64)
        _, S, _, _ = oracle.svd_square(A)
        G = A.T @ A  # exact: small integers
        lam = np.sort(np.linalg.eigvalsh(G))[::-1]
        ref = np.sqrt(np.maximum(lam, 0.0))
        np.testing.assert_allclose(S, ref, rtol=1e-12, atol=1e-12 * max(1.0, ref[0]))


def test_svd_known_spectrum_and_vectors():
    # A = Q1 diag(s) Q2^T: sigma = s, u_i = +-Q1[:, i], v_i = +-Q2[:, i].
    n = 24
    s = synth.graded_spectrum(n, per_decade=8.0)
    A, Q1, Q2 = synth.known_spectrum(n, n, s, seed=21)
    U, S, VT, _ = oracle.svd_square(A)
    np.testing.assert_allclose(S, s, rtol=1e-12, atol=1e-14)
    for i in range(n):
        su = np.sign(U[:, i] @ Q1[:, i])
        sv = np.sign(VT[i] @ Q2[:, i])
        assert su == sv  # same sign flip on u and v
        np.testing.assert_allclose(U[:, i], su * Q1[:, i], atol=1e-11 * s[0] / s[i])
        np.testing.assert_allclose(VT[i], sv * Q2[:, i], atol=1e-11 * s[0] / s[i])


def test_svd_identities_and_library():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((30, 30))
    U, S, VT, _ = oracle.svd_square(A)
    assert np.sum(S ** 2) == pytest.approx(np.sum(A ** 2), rel=1e-13)
    assert np.prod(S) == pytest.approx(abs(np.linalg.det(A)), rel=1e-10)
    np.testing.assert_allclose(S, np.linalg.svd(A, compute_uv=False), rtol=1e-12)
    np.testing.assert_allclose(U @ np.diag(S) @ VT, A, atol=1e-12)
    np.testing.assert_allclose(U.T @ U, np.eye(30), atol=1e-13)
    np.testing.assert_allclose(VT @ VT.T, np.eye(30), atol=1e-13)
    # sign convention: largest |v_i| entry positive
    for i in range(30):
        j = int(np.argmax(np.abs(VT[i])))
        assert VT[i, j] > 0


def test_svd_rank_deficient_completes_basis():
    rng = np.random.default_rng(12)
    B = rng.standard_normal((6, 3))
    A = B @ rng.standard_normal((3, 6))  # rank 3
    A[:, 5] = 0.0
    U, S, VT, _ = oracle.svd_square(A)
    np.testing.assert_allclose(U.T @ U, np.eye(6), atol=1e-12)
    assert np.all(S[3:] < 1e-13 * S[0])


# -------------------------------------------- truncation (Sec. 3.1, Alg. 3)

def test_truncation_hand_cases():
    assert oracle.truncate([2.0, 1.0], 0.2) == 1   # tail 1 <= 0.2 * 5
    assert oracle.truncate([2.0, 1.0], 0.19) == 2
    assert oracle.truncate([0.0, 0.0, 0.0], 0.01) == 0
    assert oracle.truncate([3.0, 2.0, 1.0], 0.0) == 3
    assert oracle.truncate([1.0, 0.0, 0.0], 0.01) == 1
    assert oracle.truncate([1.0, 1.0, 1.0, 1.0], 0.5) == 2  # tail(2) = 2 <= 0.5*4


def test_truncation_graded_closed_form():
    # s_i = 10^(-i/32): kept energy after k modes is (1 - 10^(-k/16)) / (1 - 10^(-16))
    # (geometric series), which crosses 0.99 at k = 32 up to 1e-15: the tie rule
    # accepts k or k+1.
    s = synth.graded_spectrum(256)
    nr = oracle.truncate(s, 0.01)
    assert nr in (32, 33)
    for r, lo in [(0.1, 16), (0.5, 5), (0.001, 48)]:
        # closed form: smallest k with 10^(-k/16) - 10^(-16) <= r (1 - 10^(-16))
        k = next(k for k in range(1, 257) if 10 ** (-k / 16) - 1e-16 <= r * (1 - 1e-16))
        assert oracle.truncate(s, r) == k
        assert k >= lo


# -------------------------------------------------------- POD pipeline

def test_pod_eckart_young_and_orthogonality():
    D = synth.plain_pod_fp64(m=600, n=20, seed=4, noise=1e-3)
    out = oracle.pod(D, remove_mean=True, r=0.01)
    Y = D - D.mean(axis=1, keepdims=True)
    U, S, VT, nr = out["U"], out["S"], out["VT"], out["nr"]
    good = S > 1e-10 * S[0]
    Ug = U[:, good]
    np.testing.assert_allclose(Ug.T @ Ug, np.eye(good.sum()), atol=1e-13)
    np.testing.assert_allclose(U @ np.diag(S) @ VT, Y, atol=1e-12)
    for k in (1, 3, nr):
        err = np.linalg.norm(Y - U[:, :k] @ np.diag(S[:k]) @ VT[:k], "fro") ** 2
        assert err == pytest.approx(np.sum(S[k:] ** 2), rel=1e-9, abs=1e-24)
    np.testing.assert_allclose(S, np.linalg.svd(Y, compute_uv=False), rtol=1e-11, atol=1e-14 * S[0])


def test_pod_known_spectrum_tall():
    m, n = 3000, 16
    s = synth.graded_spectrum(n, per_decade=4.0)
    A, Q1, Q2 = synth.known_spectrum(m, n, s, seed=7)
    out = oracle.pod(A, remove_mean=False, r=0.0)
    np.testing.assert_allclose(out["S"], s, rtol=1e-11)
    for i in range(n):
        sg = np.sign(out["U"][:, i] @ Q1[:, i])
        np.testing.assert_allclose(out["U"][:, i], sg * Q1[:, i], atol=1e-10 * s[0] / s[i])
        np.testing.assert_allclose(out["VT"][i], sg * Q2[:, i], atol=1e-10 * s[0] / s[i])


# ------------------------------------------------------ matmul (Alg. 4)

def test_matmul_exact_small_integers():
    rng = np.random.default_rng(2)
    A = rng.integers(-8, 9, size=(57, 5)).astype(np.float64)
    B = rng.integers(-8, 9, size=(57, 3)).astype(np.float64)
    C = oracle.matmul(A, B, trans_a=True)
    ref = [[sum(int(A[k, i]) * int(B[k, j]) for k in range(57)) for j in range(3)] for i in range(5)]
    assert np.array_equal(C, np.array(ref, dtype=np.float64))
    B2 = rng.integers(-8, 9, size=(5, 4)).astype(np.float64)
    C2 = oracle.matmul(A, B2, trans_a=False)
    ref2 = [[sum(int(A[i, k]) * int(B2[k, j]) for k in range(5)) for j in range(4)] for i in range(57)]
    assert np.array_equal(C2, np.array(ref2, dtype=np.float64))


# ------------------------------------------------ complex SVD (SPOD step)

def test_zsvd_known_spectrum():
    m, n = 400, 9
    s = synth.graded_spectrum(n, per_decade=3.0)
    A, Q1, Q2 = synth.known_spectrum(m, n, s, seed=31, dtype=np.complex128)
    U, S, VH, sw = oracle.zsvd_tall(A)
    np.testing.assert_allclose(S, s, rtol=1e-11)
    np.testing.assert_allclose(U @ np.diag(S) @ VH, A, atol=1e-12)
    np.testing.assert_allclose(U.conj().T @ U, np.eye(n), atol=1e-13)
    for i in range(n):
        # u_i equals Q1[:, i] up to a unit phase, which is the same on v_i
        ph = np.vdot(Q1[:, i], U[:, i])
        assert abs(abs(ph) - 1.0) < 1e-9 * s[0] / s[i]
        np.testing.assert_allclose(U[:, i], ph * Q1[:, i], atol=1e-9 * s[0] / s[i])
        j = int(np.argmax(np.abs(VH[i])))
        assert abs(VH[i, j].imag) < 1e-15 and VH[i, j].real > 0
    np.testing.assert_allclose(S, np.linalg.svd(A, compute_uv=False), rtol=1e-11)


def test_zsvd_rank_deficient_completes_unitary_basis():
    # two exactly zero columns give two exactly zero singular values; their
    # left vectors come from the complex basis completion, which must make
    # the whole U unitary (U^H U = I): a completion that projects with the
    # plain transpose instead of the conjugate transpose, or skips the second
    # Gram-Schmidt pass, leaves U^H U - I of order one in the affected block
    rng = np.random.default_rng(57)
    m, n = 30, 6
    A = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    A[:, 2] = 0.0
    A[:, 4] = 0.0
    U, S, VH, _ = oracle.zsvd_tall(A)
    assert S[4] == 0.0 and S[5] == 0.0 and S[3] > 0.1
    np.testing.assert_allclose(U.conj().T @ U, np.eye(n), atol=1e-13)
    np.testing.assert_allclose(U @ np.diag(S) @ VH, A, atol=1e-12)
    # the completed columns are orthogonal to the range of A as well
    assert np.max(np.abs(A.conj().T @ U[:, 4:])) < 1e-12
    np.testing.assert_allclose(S[:4], np.linalg.svd(A, compute_uv=False)[:4], rtol=1e-12)


# ------------------------------------------------ SPOD front end (Alg. 6)

def test_spod_block_count_closed_form():
    assert oracle.spod_nblocks(2048, 256, 128) == 15
    assert oracle.spod_nblocks(151, 60, 30) == 4  # floor((151-30)/30)
    assert oracle.spod_nblocks(256, 256, 128) == 1


def test_window_closed_form():
    w = oracle.window(256, "hann")
    assert w[0] == 0.0 and abs(w[-1]) < 1e-16
    np.testing.assert_allclose(w, w[::-1], atol=1e-15)
    j = np.arange(256)
    np.testing.assert_allclose(w, 0.5 - 0.5 * np.cos(2 * np.pi * j / 255), atol=1e-15)
    h = oracle.window(60, "hamming")
    np.testing.assert_allclose(h, 0.54 - 0.46 * np.cos(2 * np.pi * np.arange(60) / 59), atol=1e-15)


def test_spod_spectra_against_library_fft():
    rng = np.random.default_rng(44)
    D = rng.standard_normal((7, 96))
    npwin, nolap = 32, 16
    Q = oracle.spod_spectra(D, npwin, nolap, "hann", remove_mean=True)
    nblk = oracle.spod_nblocks(96, npwin, nolap)
    w = 0.5 - 0.5 * np.cos(2 * np.pi * np.arange(npwin) / (npwin - 1))
    Y = D - D.mean(axis=1, keepdims=True)
    for b in range(nblk):
        seg = Y[:, b * (npwin - nolap): b * (npwin - nolap) + npwin] * w
        F = np.fft.rfft(seg, axis=1) / w.sum()
        F[:, 1:-1] *= 2.0
        np.testing.assert_allclose(Q[:, :, b].T, F / np.sqrt(nblk), atol=1e-13)


@pytest.mark.parametrize("npwin,nolap,kind", [(32, 16, "hann"), (16, 4, "hamming")])
def test_spod_one_sided_doubling_parseval(npwin, nolap, kind):
    # Parseval per block, written without any FFT: for a real block y = w x
    # with DFT Y, sum_f |Y_f|^2 = npwin sum_j y_j^2 and Y_{npwin-f} = conj(Y_f),
    # so with q_f = c_f Y_f / sum(w) / sqrt(nBlks) (c_f = 2 for the interior
    # bins, 1 at f = 0 and npwin/2):
    #   |q_0|^2 + |q_{N/2}|^2 + (1/2) sum_{0<f<N/2} |q_f|^2
    #       = npwin sum_j y_j^2 / (sum w)^2 / nBlks.
    # Holds with amplitude doubling; fails without it (factor 1/2 on the
    # interior) and with power doubling (sqrt 2).
    rng = np.random.default_rng(npwin + nolap)
    nt = 3 * npwin
    D = rng.standard_normal((5, nt))
    Q = oracle.spod_spectra(D, npwin, nolap, kind, remove_mean=True)
    nblk = oracle.spod_nblocks(nt, npwin, nolap)
    j = np.arange(npwin)
    a0, a1 = (0.5, 0.5) if kind == "hann" else (0.54, 0.46)
    w = a0 - a1 * np.cos(2 * np.pi * j / (npwin - 1))
    Y = D - D.mean(axis=1, keepdims=True)
    for b in range(nblk):
        y = Y[:, b * (npwin - nolap): b * (npwin - nolap) + npwin] * w
        rhs = npwin * np.sum(y * y, axis=1) / w.sum() ** 2 / nblk
        q2 = np.abs(Q[:, :, b]) ** 2           # nfreq x points
        lhs = q2[0] + q2[npwin // 2] + 0.5 * q2[1:npwin // 2].sum(axis=0)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


def test_spod_dc_closed_form():
    # A field constant in time, phi(x) * c, with the mean kept: at f = 0 the
    # spectra are c phi / sqrt(nBlks) in every block, so Lambda_0 has the single
    # nonzero value c^2 |phi|^2.
    rng = np.random.default_rng(45)
    phi = rng.standard_normal(40)
    c = 1.7
    D = np.repeat((c * phi)[:, None], 64, axis=1)
    out = oracle.spod(D, dt=1.0, npwin=16, nolap=8, remove_mean=False)
    L0 = out["L"][0]
    assert L0[0] == pytest.approx(c * c * phi @ phi, rel=1e-12)
    assert np.all(L0[1:] < 1e-20 * L0[0])
    # energy identity: sum_j Lambda_f,j = |Q_f|_F^2 (Q_f already carries 1/sqrt(nBlks))
    Q = oracle.spod_spectra(D, 16, 8, remove_mean=False)
    for f in range(Q.shape[0]):
        assert out["L"][f].sum() == pytest.approx(np.sum(np.abs(Q[f]) ** 2), rel=1e-12, abs=1e-25)
    assert out["f"][1] == pytest.approx(1.0 / 16.0)
    # frequencies ordered by their leading energy, descending (Alg. 6, last step)
    lead = out["L"][out["order"], 0]
    assert np.all(np.diff(lead) <= 0)
    assert sorted(out["order"].tolist()) == list(range(Q.shape[0]))
