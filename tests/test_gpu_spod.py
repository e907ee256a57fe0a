"""GPU parity of SPOD (windowed FFT front end + one batch of realified
TSQR-SVD problems) against the CPU oracle (direct DFT of Alg. 6 and a complex
Householder QR + complex one-sided Jacobi per frequency), on the same FP32
snapshot buffer.

Bars.  C128 spectra (FP64 FFT): energies L = S^2 within 1e-11 relative of
the oracle for S_i >= 1e-3 S_1(f) (normwise 1e-11 S_1(f)^2 otherwise), modes
within 1e-8 after phase alignment on well-separated modes.  C64 spectra (FP32
FFT): the spectra carry about log2(npwin) u32 relative rounding, so
|S - S_ref| <= 64 log2(npwin) u32 S_1(f) and modes are compared by the span
of the modes with S_i >= 0.1 S_1(f).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2405_15529_amd import synth

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_spod(D32, npwin, nolap, window="hann", remove_mean=True, spectra="c128", block_rows=0,
             dt=1.0):
    import torch
    from paper_2405_15529_amd import api
    ctx = api.Context(0)
    if block_rows:
        ctx.set_option("block_rows", block_rows)
    Dg = torch.from_numpy(np.ascontiguousarray(D32)).cuda()
    out = api.spod(Dg, dt=dt, npwin=npwin, nolap=nolap, window=window, remove_mean=remove_mean,
                   spectra=spectra, ctx=ctx)
    rc, sweeps = ctx.status()
    res = dict(modes=out.modes.cpu().numpy().astype(np.complex128), L=out.L.cpu().numpy(),
               f=out.f.cpu().numpy(), order=out.order.cpu().numpy(), rc=rc, sweeps=sweeps)
    ctx.close()
    return res


def phase_aligned_err(u, uref):
    z = np.vdot(uref, u)
    ph = z / abs(z) if abs(z) > 0 else 1.0
    return float(np.max(np.abs(u / ph - uref)))


def span_distance(A, B):
    """Sine of the largest principal angle between span(A) and span(B)
    (orthonormal columns): |A - B (B^H A)|_2."""
    return float(np.linalg.norm(A - B @ (B.conj().T @ A), 2))


def check_order(order, L):
    """A permutation, non-increasing in the leading energy (near-ties within
    1e-9 relative may come in either order)."""
    lead = L[:, 0]
    assert sorted(order.tolist()) == list(range(len(lead)))
    for a, b in zip(order[:-1], order[1:]):
        assert lead[a] >= lead[b] - 1e-9 * max(lead[a], 1e-300), (a, b, lead[a], lead[b])


def assert_spod_c128(g, ref):
    assert g["rc"] == 0
    L, Lr = g["L"], ref["L"]
    nf, nb = Lr.shape
    for f in range(nf):
        s1 = Lr[f, 0]
        for c in range(nb):
            if Lr[f, c] >= 1e-6 * s1:
                assert abs(L[f, c] - Lr[f, c]) <= 1e-11 * Lr[f, c], (f, c, L[f, c], Lr[f, c])
            else:
                assert abs(L[f, c] - Lr[f, c]) <= 1e-11 * s1, (f, c)
        Sr = np.sqrt(np.maximum(Lr[f], 0))
        for c in range(nb):
            gap_ok = (c == 0 or (Sr[c - 1] - Sr[c]) >= 1e-3 * Sr[c - 1]) and \
                     (c == nb - 1 or (Sr[c] - Sr[c + 1]) >= 1e-3 * Sr[c])
            if gap_ok and Sr[c] >= 1e-3 * Sr[0]:
                e = phase_aligned_err(g["modes"][f][:, c], ref["modes"][f][:, c])
                assert e <= 1e-8, (f, c, e)
    np.testing.assert_allclose(g["f"], ref["f"], rtol=1e-15, atol=0)
    check_order(g["order"], L)


SPOD_CASES = [
    # (m, nt, npwin, nolap, block_rows): several leaves with a ragged last
    # leaf, a single leaf, no overlap, a short window
    (1500, 512, 64, 32, 512),
    (700, 256, 32, 16, 0),
    (900, 480, 32, 0, 256),
]


@pytest.mark.parametrize("m,nt,npwin,nolap,b", SPOD_CASES)
def test_spod_c128_parity(m, nt, npwin, nolap, b):
    say(f"[gpu] spod c128 m={m} nt={nt} npwin={npwin} nolap={nolap} b={b}")
    D32 = synth.spod_field(m, nt, seed=m + nt, nmodes=12)
    ref = oracle.spod(D32.astype(np.float64), 1.0, npwin, nolap, "hann", True)
    g = run_spod(D32, npwin, nolap, "hann", True, "c128", b)
    assert_spod_c128(g, ref)


def test_spod_hamming_no_mean_removal():
    say("[gpu] spod c128 hamming, mean kept")
    D32 = synth.spod_field(800, 300, seed=9, nmodes=8) + np.float32(0.5)
    ref = oracle.spod(D32.astype(np.float64), 0.25, 64, 32, "hamming", False)
    g = run_spod(D32, 64, 32, "hamming", False, "c128", 0, dt=0.25)
    assert_spod_c128(g, ref)


def test_spod_c64_parity():
    say("[gpu] spod c64 m=2000 nt=1024 npwin=128 nolap=64")
    npwin = 128
    D32 = synth.spod_field(2000, 1024, seed=17, nmodes=16)
    ref = oracle.spod(D32.astype(np.float64), 1.0, npwin, 64, "hann", True)
    g = run_spod(D32, npwin, 64, "hann", True, "c64", 1024)
    assert g["rc"] == 0
    tol = 64 * np.log2(npwin) * U32
    nf, nb = ref["L"].shape
    for f in range(nf):
        S, Sr = np.sqrt(np.maximum(g["L"][f], 0)), np.sqrt(np.maximum(ref["L"][f], 0))
        assert np.max(np.abs(S - Sr)) <= tol * Sr[0], (f, np.max(np.abs(S - Sr)) / Sr[0])
        keep = [c for c in range(nb) if Sr[c] >= 0.1 * Sr[0]]
        # compare the span of the leading modes up to the first gap
        k = len(keep)
        if k and (k == nb or Sr[k - 1] - Sr[k] >= 0.05 * Sr[0]):
            d = span_distance(g["modes"][f][:, :k], ref["modes"][f][:, :k])
            assert d <= 1e-4, (f, d)


def test_spod_dc_closed_form():
    # a time-constant field c phi(x), mean kept: q_0 = c phi for every window
    # and block, so Q_0 = (c / sqrt(nBlks)) phi 1^T has L_0 = (c^2 |phi|^2, 0, ...)
    say("[gpu] spod DC closed form")
    rng = np.random.default_rng(5)
    m, nt, npwin, nolap = 1200, 320, 64, 32
    phi = rng.standard_normal(m).astype(np.float32)
    c = 0.75
    D32 = np.repeat((c * phi)[:, None], nt, axis=1).astype(np.float32)
    g = run_spod(D32, npwin, nolap, "hann", False, "c128", 512)
    assert g["rc"] == 0
    L0 = g["L"][0]
    expect = float(np.sum(D32[:, 0].astype(np.float64) ** 2))
    assert abs(L0[0] - expect) <= 1e-12 * expect, (L0[0], expect)
    assert np.all(np.abs(L0[1:]) <= 1e-24 * expect)
    # v_0 is the constant vector, so the phase rule makes u_0 = D[:, 0] / |D[:, 0]|
    u = g["modes"][0][:, 0]
    col = D32[:, 0].astype(np.float64)
    ref = col / np.linalg.norm(col)
    assert np.max(np.abs(u - ref)) <= 1e-12
