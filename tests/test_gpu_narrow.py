"""GPU parity of the narrow-leaf variant of the stacked TSQR (3 to 6 panels,
33 <= n <= 96, up to 8 panels for the FP32 leaves of the mixed path; at
least two leaves per CU: 32-row chunks and single-wave workgroups) against
the CPU oracle, with the variant on and off.

Leaf heights are set small so that P >= 512 leaves at sizes the oracle
finishes in seconds; the stacked path is named explicitly (blocked_from =
1025) because the automatic choice would send n = 64 at these heights to the
column-blocked TSQR.  Bars as for the other FP64 POD tests (sigma 1e-12,
|U^T U - I|_F 1e-12, vectors 1e-9 on separated modes); mixed 1e-6.
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


def run(D, remove_mean, r, b, narrow, precision="fp64"):
    import torch
    from paper_2405_15529_amd import api
    ctx = api.Context(0)
    ctx.set_option("blocked_from", 1025)
    ctx.set_option("block_rows", b)
    ctx.set_option("narrow_leaves", narrow)
    assert ctx.get_option("narrow_leaves") == narrow
    Dg = torch.from_numpy(np.ascontiguousarray(D)).cuda()
    out = api.pod(Dg, remove_mean=remove_mean, r=r, precision=precision, ctx=ctx)
    rc, sweeps = ctx.status()
    res = dict(U=out.U_full[:, :out.nr].cpu().numpy().astype(np.float64), S=out.S.cpu().numpy(),
               VT=out.VT_full.cpu().numpy(), nr=out.nr, rc=rc,
               mean=None if out.mean is None else out.mean.cpu().numpy().astype(np.float64),
               leaves=ctx.plan(D.shape[0], D.shape[1])["leaves"])
    ctx.close()
    return res


def assert_parity(g, ref, r, srel=1e-12, orth=1e-12, vec=1e-9, tie=1e-10):
    assert g["rc"] == 0
    assert checks.nr_agrees(g["nr"], ref["nr"], ref["S"], r, tie=tie), (g["nr"], ref["nr"])
    k = min(g["nr"], ref["nr"])
    rel, nw = checks.sigma_errors(g["S"], ref["S"], k)
    live = [i for i in range(k) if ref["S"][i] > 1e3 * len(ref["S"]) * checks.EPS64 * ref["S"][0]]
    oe = checks.orth_error(g["U"][:, live]) if live else 0.0
    eu, ev, proj = checks.mode_errors(g["U"], ref["U"], g["VT"], ref["VT"], ref["S"], len(live))
    say(f"    sigma rel {rel:.2e} normwise {nw:.2e} orth {oe:.2e} modes {eu:.2e} {ev:.2e} {proj:.2e}")
    assert rel <= srel and nw <= srel and oe <= orth
    assert eu <= vec and ev <= vec and proj <= vec


@pytest.mark.parametrize("m,n,b,rm", [
    (48 * 520 + 17, 48, 48, True),     # mean removal, ragged last leaf
    (64 * 600, 40, 64, False),         # no mean removal (register prefetch)
    (64 * 512 + 100, 64, 64, True),    # four full panels
    (40 * 515, 33, 40, False),         # three panels, the last one column wide
    (96 * 520, 90, 96, True),          # six panels, the last one ten columns wide
])
def test_narrow_leaves_pod(m, n, b, rm):
    rng = np.random.default_rng(m + n)
    D = rng.standard_normal((m, n)) * np.exp(-np.arange(n) / 7.0)[None, :] + 0.2
    r = 0.02
    ref = oracle.pod(D, remove_mean=rm, r=r)
    for narrow in (1, 0):
        say(f"[gpu] narrow leaves={narrow} pod m={m} n={n} b={b} rm={rm}")
        g = run(D, rm, r, b, narrow)
        assert g["leaves"] >= 512
        assert_parity(g, ref, r)
        if rm:
            np.testing.assert_allclose(g["mean"], ref["mean"], rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [56, 120])
def test_narrow_leaves_mixed(n):
    b = 128 if n > 64 else 64
    m = b * 530
    rng = np.random.default_rng(77)
    D32 = (rng.standard_normal((m, n)) * np.exp(-np.arange(n) / 8.0)[None, :] + 0.3).astype(np.float32)
    ref = oracle.pod(D32.astype(np.float64), remove_mean=True, r=0.02)
    say(f"[gpu] narrow leaves mixed m={m} n={n} b={b}")
    g = run(D32, True, 0.02, b, 1, precision="mixed")
    assert_parity(g, ref, 0.02, srel=1e-6, orth=1e-6, vec=1e-5, tie=1e-5)


def test_narrow_leaves_known_spectrum_tall():
    # a taller case: 2048 leaves of 256 rows, known spectrum
    m, n, b = 256 * 2048, 60, 256
    s = 10.0 ** (-np.arange(n) / 12.0)
    A, _, _ = synth.known_spectrum(m, n, s, seed=78)
    say(f"[gpu] narrow leaves known spectrum m={m} n={n} b={b}")
    g = run(A, False, 0.0, b, 1)
    assert g["rc"] == 0 and g["nr"] == n
    err = np.max(np.abs(g["S"] - s)) / s[0]
    say(f"    max |S - s| / s_1 {err:.2e}, orth {checks.orth_error(g['U'][:, :n]):.2e}")
    assert err <= 1e-12 and checks.orth_error(g["U"][:, :n]) <= 1e-12
