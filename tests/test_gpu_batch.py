"""GPU parity of the batched POD of uneven instances (pylom_pod_batched):
every instance against the CPU oracle, eagerly and through a captured HIP
graph replayed several times with unrelated device work in between.

Bars: as the single-instance tests (FP64: sigma 1e-12, vectors 1e-9; mixed:
sigma 1e-6 relative on retained modes, |U^T U - I|_F <= 1e-6).
"""
import sys

import numpy as np
import pytest

import oracle
from tests import checks

pytestmark = pytest.mark.gpu

SHAPES = [
    # (m, n, remove_mean): uneven heights and widths, ragged leaves
    (3000, 20, False),
    (5000, 37, True),
    (1200, 64, False),
    (20000, 100, True),
    (800, 16, False),
    (4096, 48, True),
    (9000, 130, False),
]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_inputs(seed, dtype):
    rng = np.random.default_rng(seed)
    Ds = []
    for m, n, _ in SHAPES:
        D = rng.standard_normal((m, n)) * np.exp(-np.arange(n) / 9.0)[None, :] + 0.2
        Ds.append(D.astype(dtype))
    return Ds


def check_instance(g, ref, r, mixed):
    assert checks.nr_agrees(g.nr, ref["nr"], ref["S"], r, tie=1e-5 if mixed else 1e-10)
    k = min(g.nr, ref["nr"])
    S = g.S.cpu().numpy()
    rel, nw = checks.sigma_errors(S, ref["S"], k)
    assert rel <= (1e-6 if mixed else 1e-12), rel
    U = g.U_full[:, :g.nr].cpu().numpy().astype(np.float64)
    VT = g.VT_full.cpu().numpy()
    live = [i for i in range(k) if ref["S"][i] > 1e3 * len(ref["S"]) * checks.EPS64 * ref["S"][0]]
    if live:
        assert checks.orth_error(U[:, live]) <= (1e-6 if mixed else 1e-12)
    eu, ev, proj = checks.mode_errors(U, ref["U"], VT, ref["VT"], ref["S"], len(live),
                                      gap=1e-2 if mixed else 1e-3)
    tol = 1e-5 if mixed else 1e-9
    assert eu <= tol and ev <= tol and proj <= tol, (eu, ev, proj)
    assert checks.sign_convention_holds(VT, g.nr)


@pytest.mark.parametrize("precision,use_graph", [("fp64", False), ("fp64", True),
                                                 ("mixed", False), ("mixed", True)])
def test_batched_pod_parity(precision, use_graph):
    import torch
    from paper_2405_15529_amd import api
    say(f"[gpu] batched pod {precision} graph={use_graph} ({len(SHAPES)} instances)")
    mixed = precision == "mixed"
    Ds = make_inputs(41, np.float32 if mixed else np.float64)
    r = 0.05
    refs = [oracle.pod(D.astype(np.float64), remove_mean=rm, r=r)
            for D, (_, _, rm) in zip(Ds, SHAPES)]
    ctx = api.Context(0)
    ctx.set_option("streams", 3)
    Dg = [torch.from_numpy(D).cuda() for D in Ds]
    batch = api.PodBatch(Dg, remove_mean=[rm for _, _, rm in SHAPES], r=r, precision=precision,
                         use_graph=use_graph, ctx=ctx)
    scratch = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
    for rep in range(3 if use_graph else 1):
        for o in batch.out:   # poison the outputs: every replay must rewrite them
            o["S"].fill_(-1.0)
            o["nr"].fill_(-1)
        batch.run()
        scratch.add_(1.0)     # unrelated device work between replays
        rc, sweeps = ctx.status()
        assert rc == 0
        for i, (g, ref) in enumerate(zip(batch.results(), refs)):
            check_instance(g, ref, r, mixed)
            if SHAPES[i][2]:
                np.testing.assert_allclose(g.mean.cpu().numpy().astype(np.float64), ref["mean"],
                                           rtol=2.0 ** -23 if mixed else 1e-14, atol=1e-15)
        torch.cuda.synchronize()
    assert float(scratch[0].item()) == (3.0 if use_graph else 1.0)
    ctx.close()


def test_batched_reports_nonconvergence():
    import torch
    from paper_2405_15529_amd import api
    say("[gpu] batched pod max_sweeps=0")
    Ds = [torch.from_numpy(D).cuda() for D in make_inputs(3, np.float64)[:3]]
    ctx = api.Context(0)
    ctx.set_option("max_sweeps", 0)
    api.PodBatch(Ds, r=0.05, use_graph=False, ctx=ctx).run()
    rc, sweeps = ctx.status()
    assert rc == api.WNOCONV and sweeps == -1
    ctx.close()


def test_batched_wide_jacobi_grids_are_chained():
    # three instances with n = 600, 1000, 700 on three streams: widths above
    # 256 use the block Jacobi, whose grids (n / 32 block pairs of 4
    # workgroups, one CU each: 76 + 128 + 88) sum to 292 > 256 CUs, so the
    # batch must order them one after another (never a barrier timeout);
    # checked against the exact spectra, eagerly and through the graph
    import torch
    from paper_2405_15529_amd import api, synth
    shapes = [(2400, 600), (3000, 1000), (2100, 700)]
    say(f"[gpu] batched wide Jacobi chaining {shapes}")
    Ds, specs = [], []
    for i, (m, n) in enumerate(shapes):
        s = 10.0 ** (-np.arange(n) / (n / 4.0))
        A, _, _ = synth.known_spectrum(m, n, s, seed=300 + i)
        Ds.append(torch.from_numpy(A).cuda())
        specs.append(s)
    ctx = api.Context(0)
    ctx.set_option("streams", 3)
    for use_graph in (False, True):
        batch = api.PodBatch(Ds, r=0.0, precision="fp64", use_graph=use_graph, ctx=ctx)
        for rep in range(2 if use_graph else 1):
            batch.run()
            rc, _ = ctx.status()
            assert rc == 0, rc
            assert ctx.get_option("batch_jacobi_chained") == 1
            for res, s, (m, n) in zip(batch.results(), specs, shapes):
                assert res.nr == n
                err = np.max(np.abs(res.S.cpu().numpy() - s)) / s[0]
                U = res.U_full.double()
                oe = torch.linalg.norm(U.T @ U - torch.eye(n, dtype=torch.float64,
                                                           device=U.device)).item()
                say(f"  n={n} graph={use_graph} sigma err {err:.2e} |U^T U - I|_F {oe:.2e}")
                assert err <= 1e-12
                assert oe <= 10.0 * n ** 1.5 * 2.0 ** -53
    # a batch of narrow instances needs no chaining
    small = [torch.from_numpy(D).cuda() for D in make_inputs(5, np.float64)[:3]]
    api.PodBatch(small, r=0.05, use_graph=False, ctx=ctx).run()
    assert ctx.status()[0] == 0
    assert ctx.get_option("batch_jacobi_chained") == 0
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_wide_instance_on_blocked_path(precision):
    # an instance wider than the stacked QR factors (n = 1100) beside a
    # narrow one: the wide one takes the column-blocked TSQR inside the
    # batch, eagerly and through the graph (two replays); checked against
    # the exact spectrum (mixed: FP32 data, the normwise bar of the mixed
    # tests) and for orthogonality
    import torch
    from paper_2405_15529_amd import api, synth
    shapes = [(4400, 1100), (3000, 40)]
    say(f"[gpu] batched wide instance {precision} {shapes}")
    dt = torch.float64 if precision == "fp64" else torch.float32
    Ds, specs = [], []
    for i, (m, n) in enumerate(shapes):
        s = 10.0 ** (-np.arange(n) / (n / 4.0))
        A, _, _ = synth.known_spectrum(m, n, s, seed=500 + i)
        Ds.append(torch.from_numpy(A).to(dt).cuda())
        specs.append(s)
    ctx = api.Context(0)
    for use_graph in (False, True):
        batch = api.PodBatch(Ds, r=0.01, precision=precision, use_graph=use_graph, ctx=ctx)
        for rep in range(2 if use_graph else 1):
            batch.run()
            rc, _ = ctx.status()
            assert rc == 0, rc
            for res, s, (m, n) in zip(batch.results(), specs, shapes):
                S = res.S.cpu().numpy()
                nw = np.max(np.abs(S - s)) / s[0]
                k = res.nr
                U = res.U_full[:, :k].double()
                oe = torch.linalg.norm(U.T @ U - torch.eye(k, dtype=torch.float64,
                                                           device=U.device)).item()
                say(f"  n={n} graph={use_graph} N_r={k} sigma normwise {nw:.2e} "
                    f"|U^T U - I|_F {oe:.2e}")
                if precision == "fp64":
                    assert nw <= 1e-12
                    assert oe <= 10.0 * n ** 1.5 * 2.0 ** -53
                else:
                    assert nw <= 1e-6
                    assert oe <= 1e-6
    ctx.close()
