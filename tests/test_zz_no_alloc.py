"""GPU test of the allocation-free entry point pylom_matmul_noalloc (Alg. 4
into the caller's C, split-K partials in the library's fixed device
scratch), through the C-ABI, against pylom_matmul on the same inputs: two
calls in a row, the second smaller, so that the second runs over the
scratch contents the first left behind.

Bar: bit-exact.  Where the split count is the same as pylom_matmul's the
same kernels add the same terms in the same order; where the scratch caps
the splits, the inputs are small integers, so every product and partial sum
is exact in FP64 whatever the order.
"""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _call(ctx, name, A, B, C, trans_a):
    from paper_2405_15529_amd import api
    m, p = A.shape
    q = B.shape[1]
    vp = ctypes.c_void_p
    fn = getattr(ctx.lib, name)
    ctx.bind_stream()
    return fn(ctx.h, api.R64 if A.dtype.itemsize == 8 else api.R32, api.FP64, int(trans_a), m, p,
              q, vp(A.data_ptr()), A.stride(0), vp(B.data_ptr()), B.stride(0), vp(C.data_ptr()),
              C.stride(0))


def test_matmul_noalloc_matches_matmul():
    import torch
    from paper_2405_15529_amd import api
    ctx = api.Context(0)
    rng = np.random.default_rng(77)
    cases = [
        # (m, p, q, trans_a, dtype, integer inputs)
        (200000, 48, 40, True, np.float64, False),   # 64x64-tile path, many splits
        (30000, 20, 7, True, np.float64, False),     # smaller: one-wave tiles
        (4096, 1500, 1500, True, np.float64, True),  # splits capped to fit 32 MiB
        (5000, 30, 20, True, np.float32, False),     # FP32 inputs, FP64 partials
        (9000, 24, 16, False, np.float64, False),    # A B: no scratch involved
    ]
    for (m, p, q, ta, dt, ints) in cases:
        say(f"[gpu] matmul_noalloc m={m} p={p} q={q} trans_a={ta} {dt.__name__} ints={ints}")
        if ints:
            A = rng.integers(-8, 9, size=(m, p)).astype(dt)
            B = rng.integers(-8, 9, size=(m if ta else p, q)).astype(dt)
        else:
            A = rng.standard_normal((m, p)).astype(dt)
            B = rng.standard_normal((m if ta else p, q)).astype(dt)
        Ag, Bg = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        shape = (p, q) if ta else (m, q)
        C1 = torch.full(shape, np.nan, dtype=Ag.dtype, device="cuda")
        C2 = torch.full(shape, np.nan, dtype=Ag.dtype, device="cuda")
        assert _call(ctx, "pylom_matmul", Ag, Bg, C1, ta) == 0
        assert _call(ctx, "pylom_matmul_noalloc", Ag, Bg, C2, ta) == 0
        torch.cuda.synchronize()
        c1, c2 = C1.cpu().numpy(), C2.cpu().numpy()
        assert np.all(np.isfinite(c2))
        assert np.array_equal(c1, c2)
        # the Python binding of the same entry point
        C3 = torch.empty(shape, dtype=Ag.dtype, device="cuda")
        api.matmul_noalloc(Ag, Bg, ta, C3, ctx=ctx)
        assert np.array_equal(C3.cpu().numpy(), c2)
        del Ag, Bg, C1, C2, C3
    # p x q beyond the fixed scratch: refused before any launch
    A = torch.zeros((64, 2049), dtype=torch.float64, device="cuda")
    C = torch.zeros((2049, 2049), dtype=torch.float64, device="cuda")
    rc = _call(ctx, "pylom_matmul_noalloc", A, A, C, True)
    assert rc == -4, rc
    assert "scratch" in ctx.lib.pylom_last_error(ctx.h).decode()
    ctx.close()
