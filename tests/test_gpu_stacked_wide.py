"""GPU parity of the stacked (flat) TSQR at the widths the benchmarks run it
(n = 256 with 16 panels of 16 columns, n = 320, n = 512), FP64 and mixed,
with and without mean removal, against the CPU oracle.

The library's automatic path choice sends these widths to the column-blocked
TSQR at test sizes, so every case here forces the stacked QR with
blocked_from = 1025 (the setting of the headline known-spectrum benchmark).
Leaf heights are chosen so that each case spans several leaves, several
chunks per leaf and a ragged last leaf.

Bars as the other parity tests (Alg. 1, Eqs. svdqr1-3): FP64 retained sigma
relative error <= 1e-12, normwise <= 1e-12, vectors and span <= 1e-9; mixed
sigma <= 1e-6 relative, |U^T U - I|_F <= 1e-6, vectors and span <= 1e-5.

FP64 orthogonality: a product of Householder reflectors applied in floating
point is orthogonal to O(n u) in the 2-norm (Higham, Accuracy and Stability
of Numerical Algorithms, Sec. 19.3), so over the N_r retained columns the
Frobenius norm is at most sqrt(N_r) times that: the bar is
max(1e-12, 10 sqrt(N_r) n u).  The fixed 1e-12 of the narrower tests does
not grow with n; at n = 512 with 32-row chunks (32 chunk steps of 512
reflectors per leaf) the first run measured 1.53e-12.
"""
import sys

import numpy as np
import pytest

import oracle
from tests import checks

pytestmark = pytest.mark.gpu

CASES = [
    # (m, n, block_rows, remove_mean)
    (16384, 256, 4096, False),   # the headline geometry: 16 panels, 64-row chunks
    (16000, 256, 3000, True),    # ragged leaves and last chunk, mean removed
    (9000, 320, 2048, True),     # 20 panels, 48-row chunks
    (5000, 512, 1024, False),    # 32 panels, 32-row chunks
]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_input(m, n, seed):
    rng = np.random.default_rng(seed)
    # graded columns plus an offset, so that mean removal changes the problem
    return rng.standard_normal((m, n)) * np.exp(-np.arange(n) / 40.0)[None, :] + 0.25


def run_stacked(D, remove_mean, r, b, precision):
    import torch
    from paper_2405_15529_amd import api
    ctx = api.Context(0)
    ctx.set_option("blocked_from", 1025)
    ctx.set_option("block_rows", b)
    m, n = D.shape
    plan = ctx.plan(m, n)
    assert plan["leaves"] >= 2 and plan["block_rows"] == b
    Dg = torch.from_numpy(np.ascontiguousarray(D)).cuda()
    out = api.pod(Dg, remove_mean=remove_mean, r=r, precision=precision, ctx=ctx)
    rc, sweeps = ctx.status()
    k = out.nr
    res = dict(U=out.U_full[:, :k].cpu().numpy().astype(np.float64), S=out.S.cpu().numpy(),
               VT=out.VT_full.cpu().numpy(), nr=k, rc=rc, sweeps=sweeps,
               mean=None if out.mean is None else out.mean.cpu().numpy().astype(np.float64))
    ctx.close()
    return res


def assert_parity(g, ref, r, mixed):
    nr = g["nr"]
    n = len(ref["S"])
    orth64 = max(1e-12, 10.0 * np.sqrt(max(nr, 1)) * n * checks.EPS64)
    srel, orth, vec = (1e-6, 1e-6, 1e-5) if mixed else (1e-12, orth64, 1e-9)
    assert g["rc"] == 0
    assert checks.nr_agrees(nr, ref["nr"], ref["S"], r, tie=1e-5 if mixed else 1e-10), \
        (nr, ref["nr"])
    k = min(nr, ref["nr"])
    rel, nw = checks.sigma_errors(g["S"], ref["S"], k)
    say(f"    N_r {nr}/{ref['nr']} sigma rel {rel:.2e} normwise {nw:.2e}")
    assert rel <= srel, rel
    if not mixed:
        assert nw <= 1e-12, nw
    live = [i for i in range(k) if ref["S"][i] > 1e3 * len(ref["S"]) * checks.EPS64 * ref["S"][0]]
    if live:
        oe = checks.orth_error(g["U"][:, live])
        say(f"    |U^T U - I|_F {oe:.2e} (oracle {checks.orth_error(ref['U'][:, live]):.2e}, "
            f"bar {orth:.2e})")
        assert oe <= orth, oe
    eu, ev, proj = checks.mode_errors(g["U"], ref["U"], g["VT"], ref["VT"], ref["S"], len(live),
                                      gap=1e-2 if mixed else 1e-3)
    say(f"    mode errors u {eu:.2e} v {ev:.2e} span {proj:.2e}")
    assert eu <= vec and ev <= vec and proj <= vec, (eu, ev, proj)
    assert checks.sign_convention_holds(g["VT"], nr)


@pytest.mark.parametrize("m,n,b,rm", CASES)
def test_stacked_fp64_parity(m, n, b, rm):
    say(f"[gpu] stacked fp64 m={m} n={n} b={b} rm={rm}")
    D = make_input(m, n, seed=m + 3 * n)
    r = 0.02
    ref = oracle.pod(D, remove_mean=rm, r=r)
    g = run_stacked(D, rm, r, b, "fp64")
    assert_parity(g, ref, r, mixed=False)
    if rm:
        np.testing.assert_allclose(g["mean"], ref["mean"], rtol=0, atol=1e-14)


@pytest.mark.parametrize("m,n,b,rm", CASES)
def test_stacked_mixed_parity(m, n, b, rm):
    say(f"[gpu] stacked mixed m={m} n={n} b={b} rm={rm}")
    D32 = make_input(m, n, seed=m + 5 * n).astype(np.float32)
    r = 0.02
    ref = oracle.pod(D32.astype(np.float64), remove_mean=rm, r=r)
    g = run_stacked(D32, rm, r, b, "mixed")
    assert_parity(g, ref, r, mixed=True)
    if rm:
        np.testing.assert_allclose(g["mean"], ref["mean"], rtol=2.0 ** -23, atol=0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_wide_instances(precision):
    # uneven instances at n = 256 and 512 inside one batched call (graph
    # captured, replayed twice), each against the oracle
    import torch
    from paper_2405_15529_amd import api
    shapes = [(6000, 256, False), (4500, 512, True), (3000, 96, False), (7000, 300, True)]
    say(f"[gpu] batched wide instances {precision} {shapes}")
    mixed = precision == "mixed"
    r = 0.02
    Ds, refs = [], []
    for i, (m, n, rm) in enumerate(shapes):
        D = make_input(m, n, seed=100 + i)
        if mixed:
            D = D.astype(np.float32)
        Ds.append(D)
        refs.append(oracle.pod(D.astype(np.float64), remove_mean=rm, r=r))
    ctx = api.Context(0)
    ctx.set_option("streams", 2)
    Dg = [torch.from_numpy(np.ascontiguousarray(D)).cuda() for D in Ds]
    batch = api.PodBatch(Dg, remove_mean=[rm for _, _, rm in shapes], r=r, precision=precision,
                         use_graph=True, ctx=ctx)
    for rep in range(2):
        for o in batch.out:
            o["S"].fill_(-1.0)
            o["nr"].fill_(-1)
        batch.run()
        rc, _ = ctx.status()
        assert rc == 0
        for i, (res, ref) in enumerate(zip(batch.results(), refs)):
            k = res.nr
            g = dict(U=res.U_full[:, :k].cpu().numpy().astype(np.float64),
                     S=res.S.cpu().numpy(), VT=res.VT_full.cpu().numpy(), nr=k, rc=rc)
            say(f"  instance {i} {shapes[i]} rep {rep}")
            assert_parity(g, ref, r, mixed)
    ctx.close()
