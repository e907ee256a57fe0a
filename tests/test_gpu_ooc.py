"""GPU tests of the out-of-core POD (pylom_pod_host): the snapshot matrix
stays in host memory and streams through the device in windows of whole
leaves, twice (Alg. 2 + Alg. 1 + Eqs. svdqr1-3).

Every case forces a window smaller than the matrix.  The leaves, the tree
and every reflector are those of the in-device column-blocked path at the
same leaf height, so S, V^T, U and the mean must equal pylom_pod's on that
path bit for bit; they are also compared with the CPU oracle at the FP64
bars (sigma 1e-12, |U^T U - I|_F 1e-12, vectors and span 1e-9).
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_2405_15529_amd import synth
from tests import checks

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [
    # (m, n, block_rows, window_rows, remove_mean, dtype)
    (20000, 100, 1024, 4096, True, np.float64),    # 19 leaves, 5 windows, ragged last leaf
    (30000, 300, 1000, 5000, True, np.float64),    # 5 panels of 64 columns, 6 windows
    (12000, 70, 700, 2100, False, np.float32),     # FP32 storage promoted on load
    (5000, 40, 1000, 100000, True, np.float64),    # one window holds everything
]


def in_device(D, rm, r, b):
    import torch
    from paper_2405_15529_amd import api
    ctx = api.Context(0)
    ctx.set_option("blocked_from", 2)
    ctx.set_option("block_rows", b)
    out = api.pod(torch.from_numpy(D).cuda(), remove_mean=rm, r=r, ctx=ctx)
    rc, _ = ctx.status()
    assert rc == 0
    k = out.nr
    res = dict(U=out.U_full[:, :k].cpu().numpy(), S=out.S.cpu().numpy(),
               VT=out.VT_full[:k].cpu().numpy(), nr=k,
               mean=None if out.mean is None else out.mean.cpu().numpy())
    ctx.close()
    return res


@pytest.mark.parametrize("m,n,b,wr,rm,dt", CASES)
def test_pod_host_matches_in_device_and_oracle(m, n, b, wr, rm, dt):
    from paper_2405_15529_amd import api
    say(f"[gpu] pod_host m={m} n={n} b={b} window={wr} rm={rm} {dt.__name__}")
    D = synth.plain_pod_fp64(m=m, n=n, seed=m + n).astype(dt)
    r = 0.01
    ctx = api.Context(0)
    ctx.set_option("block_rows", b)
    ctx.set_option("ooc_window_rows", wr)
    ws, rows, nwin = api.ooc_query(m, n, api.R64 if dt == np.float64 else api.R32, ctx)
    say(f"    windows {nwin} of {rows} rows, workspace {ws / 1e6:.1f} MB")
    assert (nwin > 1) == (wr < m)
    h = api.pod_host(D, remove_mean=rm, r=r, ctx=ctx)
    rc, _ = ctx.status()
    assert rc == 0
    ctx.close()
    g = in_device(D, rm, r, b)
    assert h.nr == g["nr"]
    assert np.array_equal(h.S, g["S"])
    assert np.array_equal(h.VT, g["VT"])
    assert np.array_equal(h.U, g["U"])
    if rm:
        assert np.array_equal(h.mean, g["mean"])
    ref = oracle.pod(D.astype(np.float64), remove_mean=rm, r=r)
    assert checks.nr_agrees(h.nr, ref["nr"], ref["S"], r)
    k = min(h.nr, ref["nr"])
    rel, nw = checks.sigma_errors(h.S, ref["S"], k)
    U = h.U.astype(np.float64)
    live = [i for i in range(k) if ref["S"][i] > 1e3 * n * checks.EPS64 * ref["S"][0]]
    oe = checks.orth_error(U[:, live]) if live else 0.0
    eu, ev, proj = checks.mode_errors(U, ref["U"], h.VT, ref["VT"], ref["S"], len(live))
    say(f"    N_r {h.nr} sigma rel {rel:.2e} normwise {nw:.2e} orth {oe:.2e} "
        f"u {eu:.2e} v {ev:.2e} span {proj:.2e}")
    assert rel <= 1e-12 and nw <= 1e-12
    if dt == np.float64:
        # products of orthogonal factors applied in floating point are
        # orthogonal to O(n u) per column (Higham, Sec. 19.3): above n = 256
        # the SVD of R applies its rotations as 32 x 32 orthogonal blocks
        orth = max(1e-12, 10.0 * np.sqrt(max(len(live), 1)) * n * checks.EPS64)
        assert oe <= orth and eu <= 1e-9 and ev <= 1e-9 and proj <= 1e-9
    else:
        # U is stored in FP32
        assert oe <= 1e-6 and eu <= 2e-7 and ev <= 1e-9 and proj <= 1e-6
    if rm:
        np.testing.assert_allclose(h.mean.astype(np.float64), ref["mean"], rtol=0,
                                   atol=1e-14 if dt == np.float64 else 0)


def test_pod_host_strided_rows_through_the_abi():
    # leading dimensions larger than n on the host side, through the C-ABI
    from paper_2405_15529_amd import api
    m, n, ldd, ldu = 9000, 48, 53, 50
    say(f"[gpu] pod_host ldd={ldd} ldu={ldu}")
    base = synth.plain_pod_fp64(m=m, n=n, seed=5)
    Dp = np.full((m, ldd), np.nan)
    Dp[:, :n] = base
    U = np.full((m, ldu), -7.0)
    S = np.zeros(n)
    VT = np.zeros((n, n))
    mean = np.zeros(m)
    nr = ctypes.c_int64(0)
    ctx = api.Context(0)
    ctx.set_option("block_rows", 600)
    ctx.set_option("ooc_window_rows", 2000)
    vp = ctypes.c_void_p
    rc = ctx.lib.pylom_pod_host(ctx.h, api.R64, api.FP64, m, n, vp(Dp.ctypes.data), ldd, 1, 0.01,
                                vp(mean.ctypes.data), vp(U.ctypes.data), ldu, vp(S.ctypes.data),
                                vp(VT.ctypes.data), n, ctypes.byref(nr))
    assert rc == 0
    assert ctx.status()[0] == 0
    ctx.close()
    k = nr.value
    g = in_device(np.ascontiguousarray(base), True, 0.01, 600)
    assert k == g["nr"]
    assert np.array_equal(S, g["S"])
    assert np.array_equal(U[:, :k], g["U"])
    assert np.all(U[:, k:] == -7.0)       # columns beyond N_r untouched
    assert np.array_equal(mean, g["mean"])
