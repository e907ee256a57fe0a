"""Seeded synthetic snapshot matrices (host, numpy).

This module only draws inputs; it holds none of the decomposition's
arithmetic and is shared by the tests (oracle side and device side) and by
the benchmark.  The paper's workloads are CFD fields (Table "test cases":
2-D cylinder 1.78e5 x 151, Stanford diffuser 1.14e8 x 1808, ...) that are not
available here; these generators stand in for them with the same structure
(tall-skinny, smooth decaying spectrum plus noise, or a known spectrum).

Haar-distributed orthogonal factors are drawn as the Q factor of a Gaussian
matrix with the column signs fixed by sign(diag R) (Mezzadri, 2007), using
numpy's LAPACK QR as a library primitive.
"""
from __future__ import annotations

import numpy as np


def haar(rng: np.random.Generator, m: int, n: int, dtype=np.float64) -> np.ndarray:
    """m x n matrix with Haar-distributed orthonormal columns (m >= n)."""
    if np.issubdtype(dtype, np.complexfloating):
        G = (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) / np.sqrt(2.0)
    else:
        G = rng.standard_normal((m, n))
    Q, R = np.linalg.qr(G)
    d = np.diagonal(R)
    ph = d / np.abs(d)
    return np.ascontiguousarray(Q * ph[None, :])


def known_spectrum(m: int, n: int, s, seed: int, dtype=np.float64):
    """A = Q1 diag(s) Q2^T with Haar Q1 (m x n), Q2 (n x n).  Returns (A, Q1, Q2)."""
    rng = np.random.default_rng(seed)
    cplx = np.issubdtype(dtype, np.complexfloating)
    Q1 = haar(rng, m, n, np.complex128 if cplx else np.float64)
    Q2 = haar(rng, n, n, np.complex128 if cplx else np.float64)
    s = np.asarray(s, dtype=np.float64)
    A = (Q1 * s[None, :]) @ (Q2.conj().T if cplx else Q2.T)
    return np.ascontiguousarray(A.astype(dtype)), Q1, Q2


def graded_spectrum(n: int, per_decade: float = 32.0) -> np.ndarray:
    """s_i = 10^(-i/per_decade), i = 0..n-1 (sigma_1 = 1)."""
    return 10.0 ** (-np.arange(n) / per_decade)


def plain_pod_fp64(m: int = 20_000, n: int = 100, seed: int = 0, nmodes: int = 10,
                   noise: float = 1e-3) -> np.ndarray:
    """Sum of nmodes standing waves phi_k(x) sin(w_k t + th_k) with random unit
    phi_k, amplitudes 10^(-k/3) (k = 1..nmodes), w_k ~ U[0.1, 5],
    th_k ~ U[0, 2 pi), t_j = j, plus noise * N(0, 1).  Draw order: phi, w, th,
    noise.  Row-major m x n FP64 (rows = points, columns = snapshots)."""
    rng = np.random.default_rng(seed)
    phi = rng.standard_normal((nmodes, m))
    phi /= np.linalg.norm(phi, axis=1, keepdims=True)
    w = rng.uniform(0.1, 5.0, nmodes)
    th = rng.uniform(0.0, 2.0 * np.pi, nmodes)
    t = np.arange(n, dtype=np.float64)
    a = 10.0 ** (-np.arange(1, nmodes + 1) / 3.0)
    temporal = a[:, None] * np.sin(w[:, None] * t[None, :] + th[:, None])  # nmodes x n
    D = phi.T @ temporal
    D += noise * rng.standard_normal((m, n))
    return np.ascontiguousarray(D)


def graded_fp64(m: int = 1_048_576, n: int = 256, seed: int = 1, per_decade: float = 32.0):
    """A = Q1 diag(s) Q2^T, Haar Q1 (m x n), Q2 (n x n), s_i = 10^(-i/32).
    Returns (A, s)."""
    s = graded_spectrum(n, per_decade)
    A, _, _ = known_spectrum(m, n, s, seed)
    return A, s


def travelling_waves(m: int, n: int, seed: int = 2, nwaves: int = 64, noise: float = 1e-4,
                     dtype=np.float32) -> np.ndarray:
    """Sum of nwaves travelling waves a_k cos(kappa_k x - w_k t + th_k) on a
    periodic grid x_j = 2 pi j / m, t = 0..n-1, distinct integer wavenumbers
    kappa_k ~ U{1..min(2048, m/2-1)}, w_k ~ U[0.1, 5], th_k ~ U[0, 2 pi),
    a_k = 2^(-k/8), plus noise * N(0,1).  Row-major m x n."""
    rng = np.random.default_rng(seed)
    kmax = max(2, min(2048, m // 2 - 1))
    kap = rng.choice(np.arange(1, kmax + 1), size=nwaves, replace=False).astype(np.float64)
    w = rng.uniform(0.1, 5.0, nwaves)
    th = rng.uniform(0.0, 2.0 * np.pi, nwaves)
    a = 2.0 ** (-np.arange(nwaves) / 8.0)
    x = 2.0 * np.pi * np.arange(m) / m
    t = np.arange(n, dtype=np.float64)
    # cos(kx - wt + th) = cos(kx) cos(wt - th) + sin(kx) sin(wt - th)
    spatial_c = np.cos(np.outer(x, kap))  # m x nwaves
    spatial_s = np.sin(np.outer(x, kap))
    arg = np.outer(w, t) - th[:, None]  # nwaves x n
    D = spatial_c @ (a[:, None] * np.cos(arg)) + spatial_s @ (a[:, None] * np.sin(arg))
    D += noise * rng.standard_normal((m, n))
    return np.ascontiguousarray(D.astype(dtype))


def travelling_wave_params(m: int, seed: int = 2, nwaves: int = 64):
    """The draws of ``travelling_waves_device`` in their order: distinct integer
    wavenumbers kappa, angular frequencies w ~ U[0.1, 5] (per snapshot),
    phases and amplitudes a_k = 2^(-k/8).  Each wave is two exponentials in
    time, e^{+-i w t}: the eigenvalues exact DMD recovers."""
    rng = np.random.default_rng(seed)
    kmax = max(2, min(2048, m // 2 - 1))
    kap = rng.choice(np.arange(1, kmax + 1), size=nwaves, replace=False).astype(np.float64)
    w = rng.uniform(0.1, 5.0, nwaves)
    th = rng.uniform(0.0, 2.0 * np.pi, nwaves)
    a = 2.0 ** (-np.arange(nwaves) / 8.0)
    return kap, w, th, a


def travelling_waves_rows(m: int, n: int, r0: int, r1: int, seed: int = 2, nwaves: int = 64,
                          noise: float = 1e-4, dtype=np.float32) -> np.ndarray:
    """Rows r0..r1-1 of the m-row travelling-wave field of
    ``travelling_waves_device`` (same wave parameters and grid), formed on
    the host; the noise term is drawn by numpy (seeded by seed and r0), not
    by the device generator."""
    kap, w, th, a = travelling_wave_params(m, seed, nwaves)
    x = 2.0 * np.pi * np.arange(r0, r1, dtype=np.float64) / m
    t = np.arange(n, dtype=np.float64)
    arg = np.outer(w, t) - th[:, None]
    D = (np.cos(np.outer(x, kap)) @ (a[:, None] * np.cos(arg))
         + np.sin(np.outer(x, kap)) @ (a[:, None] * np.sin(arg)))
    D += noise * np.random.default_rng([seed, r0]).standard_normal(D.shape)
    return np.ascontiguousarray(D.astype(dtype))


def travelling_waves_device(m: int, n: int, seed: int = 2, nwaves: int = 64,
                            noise: float = 1e-4, device: str = "cuda", rows_per_pass: int = 131072):
    """Device-side twin of ``travelling_waves`` for large m (FP32, m x n):
    the same wave parameters (numpy draws in the same order), the same
    cos/sin factorisation as two GEMMs in FP64, rows formed in passes of
    rows_per_pass; the N(0, noise^2) term comes from torch's seeded device
    generator, so it is not the CPU generator's noise sample."""
    import torch

    kap, w, th, a = travelling_wave_params(m, seed, nwaves)
    t = np.arange(n, dtype=np.float64)
    arg = np.outer(w, t) - th[:, None]
    temporal = np.concatenate([a[:, None] * np.cos(arg), a[:, None] * np.sin(arg)], axis=0)
    Tt = torch.from_numpy(np.ascontiguousarray(temporal)).to(device)   # 2 nwaves x n
    kap_d = torch.from_numpy(kap).to(device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    D = torch.empty((m, n), dtype=torch.float32, device=device)
    for r0 in range(0, m, rows_per_pass):
        r1 = min(m, r0 + rows_per_pass)
        x = 2.0 * np.pi * torch.arange(r0, r1, dtype=torch.float64, device=device) / m
        ph = x[:, None] * kap_d[None, :]
        S = torch.cat([torch.cos(ph), torch.sin(ph)], dim=1)               # rows x 2 nwaves
        blk = S @ Tt
        blk += noise * torch.randn((r1 - r0, n), generator=gen, dtype=torch.float64, device=device)
        D[r0:r1] = blk.to(torch.float32)
    return D


def spod_field(m: int, nt: int, seed: int = 3, nmodes: int = 32, noise: float = 1e-3,
               on_bins: int = 0, dtype=np.float32) -> np.ndarray:
    """nmodes random unit spatial modes, each oscillating at its own random
    frequency f_k ~ U(0, 0.5) cycles/sample (or, with on_bins = npwin > 0, at
    random multiples of 1/npwin), phase th_k ~ U[0, 2 pi), amplitude
    10^(-k/16), plus noise * N(0,1).  Row-major m x nt."""
    rng = np.random.default_rng(seed)
    phi = rng.standard_normal((nmodes, m))
    phi /= np.linalg.norm(phi, axis=1, keepdims=True)
    if on_bins:
        f = rng.integers(1, on_bins // 2, nmodes) / float(on_bins)
    else:
        f = rng.uniform(0.0, 0.5, nmodes)
    th = rng.uniform(0.0, 2.0 * np.pi, nmodes)
    a = 10.0 ** (-np.arange(nmodes) / 16.0)
    t = np.arange(nt, dtype=np.float64)
    temporal = a[:, None] * np.cos(2.0 * np.pi * f[:, None] * t[None, :] + th[:, None])
    D = phi.T @ temporal
    D += noise * rng.standard_normal((m, nt))
    return np.ascontiguousarray(D.astype(dtype))


def uneven_batch(count: int = 64, seed: int = 4, m_lo: float = 5e4, m_hi: float = 2e6,
                 n_lo: int = 32, n_hi: int = 512):
    """Shapes of an uneven POD batch: m_i log-uniform in [m_lo, m_hi],
    n_i uniform in [n_lo, n_hi].  Returns a list of (m_i, n_i)."""
    rng = np.random.default_rng(seed)
    ms = np.round(np.exp(rng.uniform(np.log(m_lo), np.log(m_hi), count))).astype(np.int64)
    ns = rng.integers(n_lo, n_hi + 1, count)
    return [(int(a), int(max(b, 1))) for a, b in zip(ms, ns)]


def graded_fp64_device(m: int = 1_048_576, n: int = 256, seed: int = 1, per_decade: float = 32.0,
                       device: str = "cuda", with_factors: bool = False):
    """Device-side twin of ``graded_fp64`` for large m: A = Q1 diag(s) Q2^T.

    Q1 is the Q factor of an m x n Gaussian matrix G (seeded numpy draw),
    formed as G L^{-T} with L L^T = G^T G (positive-diagonal Cholesky, so it
    is the same Haar-distributed factor as the QR with diag R > 0; G is
    well conditioned, kappa ~ 1 + 2 sqrt(n/m)).  The Gram and the products run
    as library GEMMs on the device; Q2 is drawn on the host.  Returns
    (A, s) or (A, s, Q1, Q2) as torch tensors on `device`."""
    import torch

    rng = np.random.default_rng(seed)
    G = torch.from_numpy(rng.standard_normal((m, n))).to(device)
    Q2 = haar(rng, n, n)
    gram = (G.T @ G).cpu().numpy()
    L = np.linalg.cholesky(gram)
    Linv_t = np.linalg.inv(L).T  # L^{-T}
    s = graded_spectrum(n, per_decade)
    Q1 = G @ torch.from_numpy(np.ascontiguousarray(Linv_t)).to(device)
    del G
    Q2d = torch.from_numpy(Q2).to(device)
    A = (Q1 * torch.from_numpy(s).to(device)[None, :]) @ Q2d.T.contiguous()
    A = A.contiguous()
    if with_factors:
        return A, s, Q1, Q2
    del Q1
    return A, s


def known_spectrum_device(m: int, n: int, s, seed: int, device: str = "cuda",
                          dtype=None):
    """A = Q1 diag(s) Q2^T on the device, Q1 (m x n) and Q2 (n x n) Haar: the
    Q factors of Gaussian matrices drawn with torch's seeded device generator,
    formed as G L^{-T} with L L^T = G^T G (positive-diagonal Cholesky, the
    same factor as the QR with diag R > 0).  Returns A in `dtype` (default
    float64)."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    s = torch.as_tensor(np.asarray(s, dtype=np.float64), device=device)

    def haar_dev(rows, cols):
        G = torch.randn((rows, cols), generator=gen, dtype=torch.float64, device=device)
        L = torch.linalg.cholesky(G.T @ G)
        eye = torch.eye(cols, dtype=torch.float64, device=device)
        Linv = torch.linalg.solve_triangular(L, eye, upper=False)  # n x n
        return (G @ Linv.T.contiguous()).contiguous()               # G L^{-T}

    Q2 = haar_dev(n, n)
    A = haar_dev(m, n) * s[None, :]
    A = A @ Q2.T.contiguous()
    if dtype is not None:
        A = A.to(dtype)
    return A.contiguous()


def uneven_spectrum(n: int) -> np.ndarray:
    """s_i = 10^(-6 i / n), i = 0..n-1: six decades over every instance."""
    return 10.0 ** (-6.0 * np.arange(n) / n)


def linear_dynamics(m: int, nt: int, seed: int = 6, pairs=None, real_eigs=(), noise: float = 0.0):
    """Snapshots of an exactly linear system, d_t = sum_i phi_i b_i lambda_i^t
    (t = 0..nt-1), real because the complex eigenvalues come in conjugate
    pairs with conjugate modes and amplitudes.

    pairs: (radius, angle) of each conjugate pair lambda = r e^{+-i angle};
    real_eigs: real eigenvalues (real modes and amplitudes).  Modes are
    random complex unit vectors, amplitudes random of modulus in [0.5, 2].
    Returns (D m x nt float64, lam, phi m x k complex, b) listing every
    eigenvalue (both members of each pair)."""
    rng = np.random.default_rng(seed)
    if pairs is None:
        pairs = [(0.99, 0.3), (0.97, 0.9), (0.93, 1.7)]
    lam, phi, amp = [], [], []
    for rad, ang in pairs:
        v = rng.standard_normal(m) + 1j * rng.standard_normal(m)
        v /= np.linalg.norm(v)
        a = rng.uniform(0.5, 2.0) * np.exp(1j * rng.uniform(0.0, 2.0 * np.pi))
        z = rad * np.exp(1j * ang)
        lam += [z, np.conj(z)]
        phi += [v, np.conj(v)]
        amp += [a, np.conj(a)]
    for z in real_eigs:
        v = rng.standard_normal(m).astype(np.complex128)
        v /= np.linalg.norm(v)
        lam.append(complex(z))
        phi.append(v)
        amp.append(complex(rng.uniform(0.5, 2.0) * rng.choice([-1.0, 1.0])))
    lam = np.array(lam)
    phi = np.array(phi).T
    amp = np.array(amp)
    t = np.arange(nt)
    D = np.real((phi * amp[None, :]) @ (lam[:, None] ** t[None, :]))
    if noise:
        D = D + noise * rng.standard_normal(D.shape)
    return np.ascontiguousarray(D), lam, phi, amp


def linear_dynamics_device(m: int, nt: int, seed: int = 6, npairs: int = 24,
                           real_eigs=(0.95, -0.9), device: str = "cuda",
                           rows_per_pass: int = 1 << 20):
    """Device-side exactly linear snapshots for large m (FP64, m x nt):
    d_t = sum_i phi_i b_i lambda_i^t with npairs conjugate pairs
    lambda = r e^{+-i theta} (r drawn in [0.97, 1], theta evenly spaced over
    [0.1, 3.0], so that the snapshot matrix is well conditioned) and the
    given real eigenvalues; the radii and amplitudes are numpy draws, the
    complex unit-norm modes come from torch's seeded device generator.
    Returns (D, lam, phi m x k complex128 on the device, amp)."""
    import torch

    rng = np.random.default_rng(seed)
    rad = rng.uniform(0.97, 1.0, npairs)
    ang = np.linspace(0.1, 3.0, npairs)
    a = rng.uniform(0.5, 2.0, npairs) * np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, npairs))
    z = rad * np.exp(1j * ang)
    lam = np.concatenate([np.ravel(np.column_stack([z, np.conj(z)])),
                          np.asarray(real_eigs, dtype=np.complex128)])
    amp = np.concatenate([np.ravel(np.column_stack([a, np.conj(a)])),
                          rng.uniform(0.5, 2.0, len(real_eigs)).astype(np.complex128)])
    k = len(lam)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    re = torch.randn((m, npairs), generator=gen, dtype=torch.float64, device=device)
    im = torch.randn((m, npairs), generator=gen, dtype=torch.float64, device=device)
    rl = torch.randn((m, len(real_eigs)), generator=gen, dtype=torch.float64, device=device)
    phi = torch.empty((m, k), dtype=torch.complex128, device=device)
    pc = torch.complex(re, im)
    pc /= torch.linalg.norm(pc, dim=0, keepdim=True)
    rl /= torch.linalg.norm(rl, dim=0, keepdim=True)
    phi[:, 0:2 * npairs:2] = pc
    phi[:, 1:2 * npairs:2] = pc.conj()
    phi[:, 2 * npairs:] = rl.to(torch.complex128)
    del re, im, rl, pc
    t = np.arange(nt)
    Vt = torch.from_numpy((amp[:, None] * lam[:, None] ** t[None, :]).astype(np.complex128)).to(device)
    D = torch.empty((m, nt), dtype=torch.float64, device=device)
    for r0 in range(0, m, rows_per_pass):
        r1 = min(m, r0 + rows_per_pass)
        D[r0:r1] = torch.real(phi[r0:r1] @ Vt)
    return D, lam, phi, amp
