"""GPU parity of the FP64 POD / TSQR path (HIP kernels through the C-ABI)
against the CPU oracle, on seeded synthetic inputs.

Tolerances (FP64, from the arithmetic): both sides are backward-stable QR +
Jacobi, so sigma agrees to ~p(n) u sigma_1.  Bars: retained sigma relative
error <= 1e-12, normwise sigma error <= 1e-12, |U^T U - I|_F <= 1e-12,
per-mode vector error <= 1e-9 on modes whose relative gap is >= 1e-3, span of
the retained modes within 1e-9.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2405_15529_amd import synth
from tests import checks

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_pod(D, remove_mean, r, block_rows):
    torch = _torch()
    from paper_2405_15529_amd import api
    ctx = api.Context(0)
    ctx.set_option("block_rows", block_rows)
    Dg = torch.from_numpy(np.ascontiguousarray(D)).cuda()
    out = api.pod(Dg, remove_mean=remove_mean, r=r, ctx=ctx)
    rc, sweeps = ctx.status()
    res = dict(U=out.U_full[:, :out.nr].cpu().numpy().astype(np.float64), S=out.S.cpu().numpy(),
               VT=out.VT_full.cpu().numpy(), nr=out.nr, rc=rc, sweeps=sweeps,
               mean=None if out.mean is None else out.mean.cpu().numpy())
    ctx.close()
    return res


def assert_pod_parity(g, ref, r, srel=1e-12, snorm=1e-12, orth=1e-12, vec=1e-9):
    assert g["rc"] == 0
    nr = g["nr"]
    assert checks.nr_agrees(nr, ref["nr"], ref["S"], r), (nr, ref["nr"])
    k = min(nr, ref["nr"])
    rel, nw = checks.sigma_errors(g["S"], ref["S"], k)
    assert rel <= srel, rel
    assert nw <= snorm, nw
    live = [i for i in range(nr) if ref["S"][i] > 1e3 * len(ref["S"]) * checks.EPS64 * ref["S"][0]]
    if live:
        assert checks.orth_error(g["U"][:, live]) <= orth
    eu, ev, proj = checks.mode_errors(g["U"], ref["U"], g["VT"], ref["VT"], ref["S"], k)
    assert eu <= vec and ev <= vec, (eu, ev)
    assert proj <= vec, proj
    assert checks.sign_convention_holds(g["VT"], nr)


SHAPES = [
    # (m, n, block_rows, remove_mean): several chunks and panels, ragged tails,
    # non-power-of-two leaf counts, single leaf, square, single column
    (1000, 37, 200, True),
    (4099, 48, 512, False),
    (6000, 130, 600, True),
    (2048, 16, 4096, False),
    (200, 200, 200, False),
    (300, 1, 64, False),
    (777, 64, 300, True),
    (3000, 100, 400, True),
    (2500, 5, 100, True),
]


@pytest.mark.parametrize("m,n,b,rm", SHAPES)
def test_pod_small_shapes(m, n, b, rm):
    say(f"[gpu] pod small m={m} n={n} b={b} rm={rm}")
    rng = np.random.default_rng(m * 7 + n)
    D = rng.standard_normal((m, n)) * np.exp(-np.arange(n) / 7.0)[None, :] + 0.3
    r = 0.05
    ref = oracle.pod(D, remove_mean=rm, r=r)
    g = run_pod(D, rm, r, b)
    assert_pod_parity(g, ref, r)
    if rm:
        np.testing.assert_allclose(g["mean"], ref["mean"], rtol=0, atol=1e-14)


def test_pod_plain_small_case():
    # 20,000 x 100 sum of 10 standing waves + noise, 8 row blocks, 99 % energy
    say("[gpu] pod plain 20000x100 b=2500")
    D = synth.plain_pod_fp64(m=20_000, n=100, seed=0)
    ref = oracle.pod(D, remove_mean=True, r=0.01)
    g = run_pod(D, True, 0.01, 2500)
    assert_pod_parity(g, ref, 0.01)
    np.testing.assert_allclose(g["mean"], ref["mean"], rtol=0, atol=1e-15)


def test_pod_known_spectrum_mid():
    # A = Q1 diag(s) Q2^T, s_i = 10^(-i/32): sigma, U and V are known exactly
    say("[gpu] pod known spectrum 65536x256 b=4096")
    m, n = 65536, 256
    A, s = synth.graded_fp64(m=m, n=n, seed=5)
    _, Q1, Q2 = synth.known_spectrum(m, n, s, seed=5)
    g = run_pod(A, False, 0.01, 4096)
    assert g["rc"] == 0
    assert g["nr"] in (32, 33)
    rel = np.abs(g["S"] - s) / s
    assert np.max(rel[:33]) <= 1e-12, np.max(rel[:33])
    assert np.max(np.abs(g["S"] - s)) <= 1e-12
    for i in range(g["nr"]):
        sg = np.sign(g["U"][:, i] @ Q1[:, i])
        assert np.max(np.abs(sg * g["U"][:, i] - Q1[:, i])) <= 1e-10
        assert np.max(np.abs(sg * g["VT"][i] - Q2[:, i])) <= 1e-10
    assert checks.orth_error(g["U"][:, : g["nr"]]) <= 1e-12


def test_pod_constant_field_empty_basis():
    say("[gpu] pod constant field")
    c = np.arange(-40, 40) / 8.0
    D = np.repeat(c[:, None], 16, axis=1)
    g = run_pod(D, True, 0.01, 64)
    assert g["nr"] == 0
    assert np.all(g["S"] == 0.0)
    assert np.array_equal(g["mean"], c)


def test_pod_deterministic():
    say("[gpu] pod determinism")
    D = synth.plain_pod_fp64(m=5000, n=40, seed=9)
    a = run_pod(D, True, 0.01, 700)
    b = run_pod(D, True, 0.01, 700)
    assert np.array_equal(a["S"], b["S"])
    assert np.array_equal(a["U"][:, : a["nr"]], b["U"][:, : b["nr"]])
    assert np.array_equal(a["VT"], b["VT"])


def test_pod_fp32_input_promoted():
    say("[gpu] pod fp32 input")
    D = synth.plain_pod_fp64(m=4000, n=30, seed=3).astype(np.float32)
    ref = oracle.pod(D.astype(np.float64), remove_mean=True, r=0.01)
    g = run_pod(D, True, 0.01, 500)
    # FP64 compute on the promoted input; U is stored in FP32
    assert_pod_parity(g, ref, 0.01, vec=2e-7, orth=1e-6)


def test_tsqr_parity():
    torch = _torch()
    from paper_2405_15529_amd import api
    for (m, n, b) in [(3000, 50, 300), (1024, 17, 1024), (5000, 96, 256)]:
        say(f"[gpu] tsqr m={m} n={n} b={b}")
        rng = np.random.default_rng(m + n)
        A = rng.standard_normal((m, n))
        Qr, Rr = oracle.qr(A)
        ctx = api.Context(0)
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


def test_matmul_exact_integers():
    torch = _torch()
    from paper_2405_15529_amd import api
    rng = np.random.default_rng(4)
    for dt in (np.float64, np.float32):
        for (m, p, q) in [(5000, 16, 33), (777, 5, 3), (20000, 40, 40)]:
            say(f"[gpu] matmul tn {dt.__name__} {m}x{p}x{q}")
            A = rng.integers(-8, 9, size=(m, p)).astype(dt)
            B = rng.integers(-8, 9, size=(m, q)).astype(dt)
            C = api.matmul(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), trans_a=True)
            ref = oracle.matmul(A.astype(np.float64), B.astype(np.float64), trans_a=True)
            assert np.array_equal(C.cpu().numpy().astype(np.float64), ref)
            B2 = rng.integers(-8, 9, size=(p, q)).astype(dt)
            C2 = api.matmul(torch.from_numpy(A).cuda(), torch.from_numpy(B2).cuda(), trans_a=False)
            ref2 = oracle.matmul(A.astype(np.float64), B2.astype(np.float64), trans_a=False)
            assert np.array_equal(C2.cpu().numpy().astype(np.float64), ref2)


@pytest.mark.parametrize("p", [33, 67, 128])
def test_matmul_gram_exact_integers(p):
    # A^T A with the same buffer for both operands and 33 <= p <= 128 takes
    # the symmetric kernel (upper 16 x 16 blocks written with their mirror):
    # integers make every partial sum exact, so C equals the oracle's
    # product bit for bit, is exactly symmetric, and equals the tiled
    # kernel's A^T B on a copy B of A.
    torch = _torch()
    from paper_2405_15529_amd import api
    rng = np.random.default_rng(40 + p)
    for dt in (np.float64, np.float32):
        m = 30011
        say(f"[gpu] gram {dt.__name__} {m}x{p}")
        A = rng.integers(-8, 9, size=(m, p)).astype(dt)
        Ag = torch.from_numpy(A).cuda()
        C = api.matmul(Ag, Ag, trans_a=True).cpu().numpy().astype(np.float64)
        ref = oracle.matmul(A.astype(np.float64), A.astype(np.float64), trans_a=True)
        assert np.array_equal(C, ref)
        assert np.array_equal(C, C.T)
        Ct = api.matmul(Ag, Ag.clone(), trans_a=True).cpu().numpy().astype(np.float64)
        assert np.array_equal(C, Ct)


def test_max_sweeps_zero_reports_nonconvergence():
    torch = _torch()
    from paper_2405_15529_amd import api
    say("[gpu] max_sweeps=0")
    D = synth.plain_pod_fp64(m=1000, n=20, seed=2)
    ctx = api.Context(0)
    ctx.set_option("max_sweeps", 0)
    api.pod(torch.from_numpy(D).cuda(), ctx=ctx)
    rc, sweeps = ctx.status()
    assert rc == 1 and sweeps == -1
    ctx.close()


def test_pod_exactly_repeated_columns_converges():
    # columns repeated exactly make R geometrically graded (diagonal down to
    # ~1e-100): the Jacobi rotation must stay representable and converge
    say("[gpu] pod repeated columns 3000x24 r=0")
    rng = np.random.default_rng(31)
    x, y = rng.standard_normal(3000), rng.standard_normal(3000)
    D = np.column_stack([x] * 12 + [y] * 12)
    g = run_pod(D, False, 0.0, 1000)
    assert g["rc"] == 0, g["rc"]
    S = g["S"]
    ref = np.linalg.svd(np.column_stack([x, y]) * np.sqrt(12.0), compute_uv=False)
    np.testing.assert_allclose(S[:2], ref, rtol=1e-13)
    assert np.all(S[2:] <= 1e-13 * S[0])
    assert checks.orth_error(g["U"]) <= 1e-12


@pytest.mark.parametrize("precision,blocked_from,bad", [("fp64", 0, np.nan), ("fp64", 2, np.inf),
                                                        ("mixed", 0, np.nan), ("mixed", 2, -np.inf)])
def test_pod_nonfinite_input_reported(precision, blocked_from, bad):
    # a NaN or Inf in the snapshots propagates into R; the call completes
    # (every loop in the kernels is bounded) and pylom_check reports
    # PYLOM_WNONFINITE
    torch = _torch()
    from paper_2405_15529_amd import api
    say(f"[gpu] pod non-finite input {precision} blocked_from={blocked_from} {bad}")
    D = synth.plain_pod_fp64(m=3000, n=40, seed=12)
    D[1234, 7] = bad
    if precision == "mixed":
        D = D.astype(np.float32)
    ctx = api.Context(0)
    ctx.set_option("blocked_from", blocked_from)
    ctx.set_option("block_rows", 512)
    api.pod(torch.from_numpy(D).cuda(), remove_mean=True, r=0.01, precision=precision, ctx=ctx)
    rc, _ = ctx.status()
    assert rc == api.WNONFINITE, rc
    # the context stays usable: a finite input afterwards is clean
    out = api.pod(torch.from_numpy(np.nan_to_num(D, nan=0.0, posinf=0.0, neginf=0.0)).cuda(),
                  remove_mean=True, r=0.01, precision=precision, ctx=ctx)
    rc, _ = ctx.status()
    assert rc == 0 and out.nr > 0
    ctx.close()


def test_autotune_records_a_measured_height_and_stays_exact(tmp_path):
    # the measured leaf height is one of the candidates, steers later calls
    # of the same shape class, survives a JSON round trip, and the POD at
    # that height still matches the oracle
    torch = _torch()
    from paper_2405_15529_amd import api
    m, n = 60000, 48
    say(f"[gpu] autotune {m}x{n}")
    D = synth.plain_pod_fp64(m=m, n=n, seed=17)
    Dg = torch.from_numpy(D).cuda()
    ctx = api.Context(0)
    b, ms = ctx.autotune(Dg, precision="fp64", remove_mean=True, reps=2)
    say(f"    best leaf height {b} rows, {ms:.3f} ms")
    assert b >= n and ms > 0
    assert ctx.plan(m, n)["block_rows"] == b
    path = tmp_path / "tune.json"
    ctx.tune_save(str(path))
    ctx.close()
    ctx2 = api.Context(0)
    assert ctx2.tune_load(str(path)) == 1
    assert ctx2.plan(m, n)["block_rows"] == b
    out = api.pod(Dg, remove_mean=True, r=0.01, ctx=ctx2)
    assert ctx2.status()[0] == 0
    ref = oracle.pod(D, remove_mean=True, r=0.01)
    res = dict(U=out.U.cpu().numpy(), S=out.S.cpu().numpy(), VT=out.VT_full.cpu().numpy(),
               nr=out.nr, rc=0)
    assert_pod_parity(res, ref, 0.01)
    ctx2.close()
