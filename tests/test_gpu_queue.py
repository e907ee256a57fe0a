"""GPU tests of the work-queue launches (option "work_queue"): every leaf QR
and every tree combine of a TSQR (Alg. 1, reduce phase), and every
propagation step and leaf apply (broadcast phase, Eq. svdqr3), each drained
from a device task counter by one persistent launch with per-node dependency
counters.  Each task runs the same code on the same data as the per-level
launches, so the results must be identical bit for bit; the per-level form
itself is compared with the CPU oracle by the other tests.  The leaf counts
are chosen so that the trees are ragged (nodes without partners at several
levels) and deep.
"""
import sys

import numpy as np
import pytest

from paper_2405_15529_amd import synth

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="the work-queue launch did not complete on the GPU (two runs, the "
                            "second after a change to its spin loop); the path is switched off "
                            "until its cause is found"),
]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def pod_both(D, rm, r, b, precision="fp64"):
    import torch
    from paper_2405_15529_amd import api
    outs = []
    for wq in (0, 1):
        ctx = api.Context(0)
        ctx.set_option("work_queue", wq)
        ctx.set_option("blocked_from", 2049)
        ctx.set_option("block_rows", b)
        o = api.pod(torch.from_numpy(D).cuda(), remove_mean=rm, r=r, precision=precision, ctx=ctx)
        rc, _ = ctx.status()
        say(f"    work_queue={wq}: status {rc}, N_r {o.nr}")
        assert rc == 0
        outs.append(dict(S=o.S.cpu().numpy(), U=o.U.cpu().numpy(), VT=o.VT.cpu().numpy(),
                         nr=o.nr, mean=None if o.mean is None else o.mean.cpu().numpy()))
        ctx.close()
    return outs


@pytest.mark.parametrize("m,n,b,rm", [(50000, 48, 700, True), (30000, 20, 100, False),
                                      (9000, 130, 600, True), (4096, 16, 4096, False)])
def test_stacked_pod_queue_equals_per_level(m, n, b, rm):
    say(f"[gpu] work queue vs per-level launches, pod m={m} n={n} b={b} ({m // b} leaves)")
    D = synth.plain_pod_fp64(m=m, n=n, seed=m + n)
    a, q = pod_both(D, rm, 0.02, b)
    assert a["nr"] == q["nr"]
    assert np.array_equal(a["S"], q["S"])
    assert np.array_equal(a["VT"], q["VT"])
    assert np.array_equal(a["U"], q["U"])
    if rm:
        assert np.array_equal(a["mean"], q["mean"])


def test_spod_queue_equals_per_level():
    import torch
    from paper_2405_15529_amd import api
    m, nt = 1500, 512
    say(f"[gpu] work queue vs per-level launches, spod m={m} nt={nt}")
    D = torch.from_numpy(synth.spod_field(m, nt, seed=8, nmodes=6)).cuda()
    res = []
    for wq in (0, 1):
        ctx = api.Context(0)
        ctx.set_option("work_queue", wq)
        ctx.set_option("block_rows", 96)   # 2m = 3000 rows of the realification: 31 leaves
        out = api.spod(D, npwin=64, nolap=32, spectra="c128", ctx=ctx)
        assert ctx.status()[0] == 0
        res.append((out.modes.cpu().numpy(), out.L.cpu().numpy(), out.order.cpu().numpy()))
        ctx.close()
    for x, y in zip(res[0], res[1]):
        assert np.array_equal(x, y)


def test_batched_queue_equals_per_level():
    import torch
    from paper_2405_15529_amd import api
    shapes = [(7000, 40), (12000, 33), (3000, 96), (20000, 20)]
    say(f"[gpu] work queue vs per-level launches, batched graph {shapes}")
    rng = np.random.default_rng(3)
    Ds = [torch.from_numpy(rng.standard_normal((m, n)) * np.exp(-np.arange(n) / 5.0)).cuda()
          for m, n in shapes]
    res = []
    for wq in (0, 1):
        ctx = api.Context(0)
        ctx.set_option("work_queue", wq)
        ctx.set_option("block_rows", 512)
        batch = api.PodBatch(Ds, r=0.05, precision="fp64", use_graph=True, ctx=ctx)
        for _ in range(2):
            batch.run()
        assert ctx.status()[0] == 0
        res.append([(g.S.cpu().numpy(), g.U.cpu().numpy()) for g in batch.results()])
        ctx.close()
    for (s0, u0), (s1, u1) in zip(res[0], res[1]):
        assert np.array_equal(s0, s1) and np.array_equal(u0, u1)
