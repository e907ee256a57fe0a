"""GPU parity of the column-blocked TSQR (the path of wide snapshot matrices,
n > 1024; forced on narrower shapes with the blocked_from option so that the
oracle finishes in seconds) against the CPU oracle, and a wide known-spectrum
case on the default path.

The blocked Householder QR is backward stable like the stacked one, so the
FP64 bars are those of the FP64 POD tests (sigma 1e-12 relative and
normwise, |U^T U - I|_F <= 1e-12, vectors 1e-9 on separated modes); the
mixed path keeps its 1e-6 bars.  The wide case checks what holds at any
size: sigma against the exact spectrum within 1e-12 sigma_1 (p(n) u with
n = 1100), orthogonality of U and V and the reconstruction to bars derived
from n and u in the test.
"""
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


def run_blocked(D, remove_mean, r, block_rows, precision="fp64", blocked_from=2, mixed_tree=None,
                opts=None):
    import torch
    from paper_2405_15529_amd import api
    ctx = api.Context(0)
    ctx.set_option("blocked_from", blocked_from)
    ctx.set_option("block_rows", block_rows)
    if mixed_tree is not None:
        ctx.set_option("mixed_tree", mixed_tree)
    for k, v in (opts or {}).items():
        ctx.set_option(k, v)
    Dg = torch.from_numpy(np.ascontiguousarray(D)).cuda()
    out = api.pod(Dg, remove_mean=remove_mean, r=r, precision=precision, ctx=ctx)
    rc, sweeps = ctx.status()
    res = dict(U=out.U_full[:, :out.nr].cpu().numpy().astype(np.float64), S=out.S.cpu().numpy(),
               VT=out.VT_full.cpu().numpy(), nr=out.nr, rc=rc, sweeps=sweeps,
               mean=None if out.mean is None else out.mean.cpu().numpy().astype(np.float64))
    ctx.close()
    return res


def assert_parity(g, ref, r, srel=1e-12, snorm=1e-12, orth=1e-12, vec=1e-9, tie=1e-10):
    assert g["rc"] == 0
    nr = g["nr"]
    assert checks.nr_agrees(nr, ref["nr"], ref["S"], r, tie=tie), (nr, ref["nr"])
    k = min(nr, ref["nr"])
    if k == 0:
        return
    rel, nw = checks.sigma_errors(g["S"], ref["S"], k)
    say(f"    sigma rel {rel:.2e} normwise {nw:.2e}")
    assert rel <= srel, rel
    assert nw <= snorm, nw
    live = [i for i in range(k) if ref["S"][i] > 1e3 * len(ref["S"]) * checks.EPS64 * ref["S"][0]]
    if live:
        oe = checks.orth_error(g["U"][:, live])
        say(f"    |U^T U - I|_F {oe:.2e}")
        assert oe <= orth, oe
    eu, ev, proj = checks.mode_errors(g["U"], ref["U"], g["VT"], ref["VT"], ref["S"], len(live))
    say(f"    modes u {eu:.2e} v {ev:.2e} span {proj:.2e}")
    assert eu <= vec and ev <= vec and proj <= vec, (eu, ev, proj)
    assert checks.sign_convention_holds(g["VT"], nr)


SHAPES = [
    # (m, n, block_rows, remove_mean): several panels with a ragged last panel
    # (n = 200: 3 x 64 + 8; n = 130: 2 x 64 + 2; n = 129: 2 x 64 + 1), odd leaf
    # counts (an unpaired node), ragged last leaves, leaf rows that are not a
    # multiple of the 64-row chunk, exactly one panel, a single leaf (no tree)
    (3000, 200, 700, True),
    (5000, 130, 1000, False),
    (1000, 64, 256, True),
    (2000, 300, 2000, False),
    (4100, 97, 512, True),
    (2600, 129, 300, False),
    # the Jacobi of R with 4-column blocks: n = 257 is the narrowest such
    # problem (33 workgroups), n = 500 has a 52-column last panel
    (2600, 257, 1300, True),
    (3000, 500, 1500, False),
]


@pytest.mark.parametrize("m,n,b,rm", SHAPES)
def test_blocked_pod_parity(m, n, b, rm):
    say(f"[gpu] blocked pod m={m} n={n} b={b} rm={rm}")
    rng = np.random.default_rng(m * 13 + n)
    D = rng.standard_normal((m, n)) * np.exp(-np.arange(n) / 9.0)[None, :] + 0.3
    r = 0.05
    ref = oracle.pod(D, remove_mean=rm, r=r)
    g = run_blocked(D, rm, r, b)
    assert_parity(g, ref, r)
    if rm:
        np.testing.assert_allclose(g["mean"], ref["mean"], rtol=0, atol=1e-14)


def test_blocked_pod_keep_all_modes():
    # r = 0: every mode, so U = Q U_R over the whole basis (known spectrum,
    # full rank)
    say("[gpu] blocked pod r=0 3000x150")
    s = 2.0 ** (-np.arange(150) / 16.0)
    A, _, _ = synth.known_spectrum(3000, 150, s, seed=31)
    ref = oracle.pod(A, remove_mean=False, r=0.0)
    g = run_blocked(A, False, 0.0, 640)
    assert g["nr"] == 150
    assert_parity(g, ref, 0.0)
    assert checks.orth_error(g["U"][:, :150]) <= 1e-12


def test_blocked_pod_fp32_input_promoted():
    say("[gpu] blocked pod fp32 input 4000x140")
    D = synth.plain_pod_fp64(m=4000, n=140, seed=8).astype(np.float32)
    ref = oracle.pod(D.astype(np.float64), remove_mean=True, r=0.01)
    g = run_blocked(D, True, 0.01, 1000)
    assert_parity(g, ref, 0.01, vec=2e-7, orth=1e-6)


@pytest.mark.parametrize("m,n,b", [(3000, 150, 700), (2000, 64, 512), (1500, 100, 1500)])
def test_blocked_tsqr_parity(m, n, b):
    import torch
    from paper_2405_15529_amd import api
    say(f"[gpu] blocked tsqr m={m} n={n} b={b}")
    rng = np.random.default_rng(m + 3 * n)
    A = rng.standard_normal((m, n))
    Qr, Rr = oracle.qr(A)
    ctx = api.Context(0)
    ctx.set_option("blocked_from", 2)
    ctx.set_option("block_rows", b)
    Q, R = api.tsqr(torch.from_numpy(A).cuda(), want_q=True, ctx=ctx)
    Q = Q.cpu().numpy()
    R = R.cpu().numpy()
    ctx.close()
    scale = np.abs(Rr).max()
    assert np.max(np.abs(R - Rr)) <= 1e-12 * scale
    assert np.all(np.diag(R) >= 0) and np.allclose(np.tril(R, -1), 0)
    assert np.max(np.abs(Q - Qr)) <= 1e-11
    assert checks.orth_error(Q) <= 1e-12
    assert np.max(np.abs(Q @ R - A)) <= 1e-12 * scale


@pytest.mark.parametrize("m,n,b,rm", [(6000, 200, 1500, True), (3000, 97, 700, False)])
def test_blocked_mixed_parity(m, n, b, rm):
    say(f"[gpu] blocked mixed m={m} n={n} b={b}")
    rng = np.random.default_rng(m * 5 + n)
    D = (rng.standard_normal((m, n)) * np.exp(-np.arange(n) / 8.0)[None, :] + 0.3)
    D32 = D.astype(np.float32)
    r = 0.02
    ref = oracle.pod(D32.astype(np.float64), remove_mean=rm, r=r)
    g = run_blocked(D32, rm, r, b, precision="mixed")
    assert_parity(g, ref, r, srel=1e-6, snorm=1e-6, orth=1e-6, vec=1e-5, tie=1e-5)
    if rm:
        np.testing.assert_allclose(g["mean"], ref["mean"], rtol=2.0 ** -23, atol=0)


@pytest.mark.parametrize("mixed_tree", [0, 1])
def test_blocked_mixed_tree_levels(mixed_tree):
    # 21 leaves (ragged tree, 5 levels): with mixed_tree = 1 the levels
    # h = 1..8 combine FP32 R factors and only h = 16 runs in FP64; with 0
    # every level is FP64.  Same bars as the other mixed cases.
    m, n, b = 20500, 130, 1000
    say(f"[gpu] blocked mixed tree={mixed_tree} m={m} n={n} b={b}")
    rng = np.random.default_rng(77)
    D = (rng.standard_normal((m, n)) * np.exp(-np.arange(n) / 10.0)[None, :] + 0.1)
    D32 = D.astype(np.float32)
    r = 0.02
    ref = oracle.pod(D32.astype(np.float64), remove_mean=True, r=r)
    g = run_blocked(D32, True, r, b, precision="mixed", mixed_tree=mixed_tree)
    assert_parity(g, ref, r, srel=1e-6, snorm=1e-6, orth=1e-6, vec=1e-5, tie=1e-5)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_blocked_tree_wavefront_matches_serial(precision):
    # 37 leaves (6 tree levels, ragged) of a 3-panel problem: the wavefront
    # tree over four of the library's streams (tree_pipeline = 4) runs the same
    # kernels on the same operands as the serial levels, so every output is
    # bit-identical; both are also held to the oracle.
    m, n, b = 9300, 150, 250
    say(f"[gpu] blocked tree wavefront {precision} m={m} n={n} b={b}")
    rng = np.random.default_rng(91)
    D = (rng.standard_normal((m, n)) * np.exp(-np.arange(n) / 12.0)[None, :] + 0.2)
    if precision == "mixed":
        D = D.astype(np.float32)
    r = 0.02
    ser = run_blocked(D, True, r, b, precision=precision, opts={"tree_pipeline": 0})
    pip = run_blocked(D, True, r, b, precision=precision, opts={"tree_pipeline": 4})
    assert ser["nr"] == pip["nr"]
    np.testing.assert_array_equal(pip["S"], ser["S"])
    np.testing.assert_array_equal(pip["VT"][:pip["nr"]], ser["VT"][:ser["nr"]])
    np.testing.assert_array_equal(pip["U"], ser["U"])
    ref = oracle.pod(np.asarray(D, dtype=np.float64), remove_mean=True, r=r)
    if precision == "fp64":
        assert_parity(pip, ref, r)
    else:
        assert_parity(pip, ref, r, srel=1e-6, snorm=1e-6, orth=1e-6, vec=1e-5, tie=1e-5)


def test_blocked_wide_known_spectrum():
    # n = 1100 > 1024: the default path for wide problems (two-level Jacobi
    # kernel with 32 rows per lane).  A = Q1 diag(s) Q2^T, s_i = 10^(-i/400).
    import torch
    from paper_2405_15529_amd import api
    m, n = 16384, 1100
    say(f"[gpu] blocked wide known spectrum {m}x{n}")
    s = 10.0 ** (-np.arange(n) / 400.0)
    A_np, Q1, _ = synth.known_spectrum(m, n, s, seed=41)
    A = torch.from_numpy(A_np).cuda()
    ctx = api.Context(0)
    assert ctx.get_option("blocked_from") == 0  # automatic: n >= 512 is column-blocked
    out = api.pod(A, remove_mean=False, r=0.0, ctx=ctx)
    rc, sweeps = ctx.status()
    say(f"    rc {rc} sweeps {sweeps} nr {out.nr}")
    assert rc == 0 and out.nr == n
    S = out.S.cpu().numpy()
    err = np.max(np.abs(S - s)) / s[0]
    say(f"    max |S - s| / s_1 {err:.2e}")
    assert err <= 1e-12
    U = out.U_full[:, :n]
    V = out.VT_full[:n].T
    eye = torch.eye(n, dtype=torch.float64, device=U.device)
    ou = torch.linalg.norm(U.T @ U - eye).item()
    ov = torch.linalg.norm(V.T @ V - eye).item()
    rec = (torch.linalg.norm(A - (U * out.S) @ V.T) / torch.linalg.norm(A)).item()
    say(f"    |U^T U - I|_F {ou:.2e} |V^T V - I|_F {ov:.2e} rel reconstruction {rec:.2e}")
    # bars from the arithmetic (u = 2^-53): U = Q U_R is orthogonal to
    # O(n u) in the 2-norm, so the Frobenius norm over n^2 entries is O(n^1.5 u);
    # V is orthogonal to the Jacobi stopping test n u per pair, n^2 pairs;
    # the reconstruction is backward stable, O(n u)
    u = 2.0 ** -53
    assert ou <= 10 * n ** 1.5 * u and ov <= n * n * u and rec <= 10 * n * u
    # leading modes against the exact factor (relative gaps 0.6 %)
    Uh = out.U_full[:, :8].cpu().numpy()
    for i in range(8):
        sg = np.sign(Uh[:, i] @ Q1[:, i])
        assert np.max(np.abs(sg * Uh[:, i] - Q1[:, i])) <= 1e-9
    ctx.close()


def test_blocked_wide_mixed_matches_fp64():
    import torch
    from paper_2405_15529_amd import api
    m, n = 16384, 1100
    say(f"[gpu] blocked wide mixed vs FP64 {m}x{n}")
    s = 10.0 ** (-np.arange(n) / 64.0)
    A_np, _, _ = synth.known_spectrum(m, n, s, seed=43)
    A32 = torch.from_numpy(A_np.astype(np.float32)).cuda()
    ctx = api.Context(0)
    g32 = api.pod(A32, remove_mean=False, r=0.01, precision="mixed", ctx=ctx)
    rc32, _ = ctx.status()
    g64 = api.pod(A32, remove_mean=False, r=0.01, ctx=ctx)
    rc64, _ = ctx.status()
    assert rc32 == 0 and rc64 == 0
    S32, S64 = g32.S.cpu().numpy(), g64.S.cpu().numpy()
    k = min(g32.nr, g64.nr)
    assert abs(g32.nr - g64.nr) <= 1 and k > 0
    rel = np.max(np.abs(S32[:k] - S64[:k]) / S64[:k])
    U = g32.U.double()
    oe = torch.linalg.norm(U.T @ U - torch.eye(U.shape[1], dtype=torch.float64,
                                               device=U.device)).item()
    say(f"    N_r {g32.nr}/{g64.nr} sigma rel vs FP64 {rel:.2e} |U^T U - I|_F {oe:.2e}")
    assert rel <= 1e-6 and oe <= 1e-6
    ctx.close()
