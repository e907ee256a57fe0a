"""CPU tests of the C-ABI boundary: the library loads, exports every entry
point declared in include/pylom.h, validates arguments on the host before any
device work, and plans the in-device reduction tree exactly as Alg. 1's
XOR/AND schedule (emulated here with P virtual ranks)."""
import ctypes
import os
import re

import pytest

from paper_2405_15529_amd import _lib, api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "pylom.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pylom_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), f"{n} declared in pylom.h but not exported"
    # the binding covers exactly the declared set
    assert sorted(_lib.SIGNATURES) == names


def test_strerror_names_every_code():
    lib = _lib.load()
    for code in (0, -1, -2, -3, -4, -5, -6, -7, 1, 2):
        assert lib.pylom_strerror(code).decode() not in ("", "unknown status")
    assert lib.pylom_strerror(12345).decode() == "unknown status"


@pytest.fixture
def hctx():
    c = api.Context(-1)  # host-only: validates and plans, never touches a device
    yield c
    c.close()


def _pod(ctx, dtype=api.R64, prec=api.FP64, m=100, n=10, D=1, ldd=None, r=0.01, U=1, ldu=None,
         S=1, VT=1, ldvt=None, nr=1):
    ldd = n if ldd is None else ldd
    ldu = n if ldu is None else ldu
    ldvt = n if ldvt is None else ldvt
    vp = ctypes.c_void_p
    return ctx.lib.pylom_pod(ctx.h, dtype, prec, m, n, vp(D), ldd, 1, r, vp(0), vp(U), ldu, vp(S),
                             vp(VT), ldvt, vp(nr))


def test_argument_validation_before_device(hctx):
    assert _pod(hctx) == -7                        # valid args: only the missing device
    assert _pod(hctx, m=5, n=10) == -2             # m < n
    assert _pod(hctx, n=0) == -2
    assert _pod(hctx, ldd=5) == -2                 # ld < n
    assert _pod(hctx, ldu=5) == -2
    assert _pod(hctx, ldvt=5) == -2
    assert _pod(hctx, D=0) == -1                   # null input
    assert _pod(hctx, nr=0) == -1
    assert _pod(hctx, r=1.0) == -1                 # residual outside [0, 1)
    assert _pod(hctx, r=-0.5) == -1
    assert _pod(hctx, dtype=99) == -3
    assert _pod(hctx, prec=7) == -3
    assert _pod(hctx, m=5000, n=3000) == -6        # wider than the kernels
    assert _pod(hctx, m=5000, n=2000) == -7        # column-blocked path
    assert _pod(hctx, prec=api.MIXED) == -3        # mixed precision needs FP32 storage
    assert _pod(hctx, dtype=api.R32, prec=api.MIXED) == -7
    assert _pod(hctx, dtype=api.R32, prec=api.MIXED, m=5000, n=2000) == -7
    assert _pod(hctx, dtype=api.R32, prec=api.MIXED, m=5000, n=2049) == -6
    assert hctx.lib.pylom_pod(None, 2, 0, 10, 2, None, 2, 0, 0.0, None, None, 2, None, None, 2,
                              None) == -1


def test_options_roundtrip(hctx):
    hctx.set_option("block_rows", 2500)
    assert hctx.get_option("block_rows") == 2500
    hctx.set_option("max_sweeps", 0)
    assert hctx.get_option("max_sweeps") == 0
    with pytest.raises(api.PylomError):
        hctx.set_option("no_such_option", 1)
    with pytest.raises(api.PylomError):
        hctx.set_option("max_sweeps", -1)


def test_plan_geometry(hctx):
    # the small plain-POD case: 20,000 x 100 over 8 row blocks of 2,500
    hctx.set_option("block_rows", 2500)
    p = hctx.plan(20_000, 100)
    assert p["leaves"] == 8 and p["block_rows"] == 2500 and p["levels"] == 3
    assert p["chunk_rows"] % 16 == 0 and p["chunk_rows"] > 0
    # the known-spectrum case: 1,048,576 x 256 in blocks of 4,096
    hctx.set_option("block_rows", 4096)
    p = hctx.plan(1_048_576, 256)
    assert p["leaves"] == 256 and p["levels"] == 8
    # leaves never get fewer than n rows; the last takes the remainder
    p = hctx.plan(1000, 300)
    assert p["block_rows"] >= 300 and p["leaves"] == max(1, 1000 // p["block_rows"])
    hctx.set_option("block_rows", 100)  # raised to n
    p = hctx.plan(1000, 300)
    assert p["block_rows"] == 300 and p["leaves"] == 3
    assert hctx.workspace_bytes(1_048_576, 256) > 1_048_576 * 256 * 8


def test_blocked_plan_geometry(hctx):
    # the wide mixed-precision case: 4,194,304 x 1,808, one leaf per CU
    assert hctx.get_option("blocked_from") == 0  # automatic
    ncu = 256
    m, n = 4_194_304, 1808
    p = hctx.plan(m, n)
    assert p["chunk_rows"] == 64
    b = p["block_rows"]
    assert b % 64 == 0 and b >= n and p["leaves"] == m // b
    assert api.tune_block_rows(m, n, hctx) == b
    if b == 8192:
        assert p["leaves"] == 2 * ncu and p["levels"] == 9
    # working copy + reflectors and T factors + tree pairs: a few times the
    # input, well inside 288 GB of HBM
    w64 = hctx.workspace_bytes(m, n)
    w32 = hctx.workspace_bytes(m, n, dtype=api.R32, precision="mixed")
    assert m * n * 8 < w64 < 150e9
    assert m * n * 4 < w32 < 150e9
    # forcing narrow problems through the blocked path
    hctx.set_option("blocked_from", 64)
    p = hctx.plan(10_000, 200)
    assert p["chunk_rows"] == 64 and p["block_rows"] % 64 == 0
    hctx.set_option("block_rows", 1000)
    p = hctx.plan(10_000, 200)
    assert p["block_rows"] == 1000 and p["leaves"] == 10
    with pytest.raises(api.PylomError):
        hctx.set_option("blocked_from", 1)
    with pytest.raises(api.PylomError):
        hctx.set_option("blocked_from", 4096)


def test_automatic_path_choice(hctx):
    # blocked_from = 0: column-blocked for n >= 512, or n >= 64 with
    # m <= 8,388,608; the stacked QR otherwise.  Each path has its own leaf
    # height, read here with the path forced by an explicit threshold.
    def rows(m, n, bf):
        hctx.set_option("blocked_from", bf)
        return api.tune_block_rows(m, n, hctx)

    for m, n, blocked in [(1_048_576, 256, True), (1_048_576, 63, False),
                          (8_388_608, 64, True), (8_388_609, 64, False),
                          (36_000_000, 320, False), (18_000_000, 630, True),
                          (58_300_000, 56, False), (4_194_304, 1808, True)]:
        want = rows(m, n, 2 if blocked else 2049)
        other = rows(m, n, 2049 if blocked else 2)
        assert want != other, (m, n)
        hctx.set_option("blocked_from", 0)
        assert api.tune_block_rows(m, n, hctx) == want, (m, n)
        assert hctx.plan(m, n)["block_rows"] == want, (m, n)
    assert hctx.get_option("blocked_from") == 0


def emulate_alg1(P):
    """Alg. 1 with P virtual ranks.  Reduce phase: at blevel = 1, 2, 4, ...
    (while blevel < 2^ceil(log2 P)), a rank that has not yet sent is a sender
    if rank & blevel, else a receiver; partner = rank ^ blevel, skipped if it
    does not exist.  Broadcast phase: blevel from the top down, ranks with
    rank & (blevel-1) == 0 take part; rank & blevel receives from the partner."""
    npow = 1
    while npow < P:
        npow *= 2
    sent = [False] * P
    combines = []
    level = 0
    blevel = 1
    while blevel < npow:
        for rank in range(P):
            if sent[rank] or rank & blevel:
                continue
            prank = rank ^ blevel
            if prank < P and not sent[prank]:
                combines.append((level, rank, prank))
        for rank in range(P):
            if not sent[rank] and rank & blevel and (rank ^ blevel) < P:
                sent[rank] = True
        blevel *= 2
        level += 1
    nlevels = level
    received_from = {}
    blevel = 1 << (nlevels - 1) if nlevels else 0
    while blevel >= 1:
        mask = blevel - 1
        for rank in range(P):
            if rank & mask:
                continue
            prank = rank ^ blevel
            if rank & blevel and prank < P:
                assert rank not in received_from
                received_from[rank] = prank
        blevel //= 2
    return combines, received_from


@pytest.mark.parametrize("P", list(range(1, 40)) + [6, 64, 100, 255, 256, 300])
def test_tree_plan_matches_alg1(P):
    combines, received = emulate_alg1(P)
    plan = api.tree_plan(P)
    assert sorted(plan) == sorted(combines)
    assert len(plan) == P - 1
    # every non-root leaf gets its broadcast exactly once, from its absorber
    assert sorted(received) == list(range(1, P))
    for lvl, recv, send in plan:
        assert received[send] == recv


def test_tree_plan_six_ranks_truth_table():
    # the 6-processor example: level 0 pairs (0,1),(2,3),(4,5); level 1 (0,2);
    # level 2 (0,4)
    assert api.tree_plan(6) == [(0, 0, 1), (0, 2, 3), (0, 4, 5), (1, 0, 2), (2, 0, 4)]


def test_spod_query_and_validation(hctx):
    nb, nf, ws = api.spod_query(262144, 2048, 256, 128, "c64", hctx)
    assert (nb, nf) == (15, 129)          # floor((2048 - 128) / 128) blocks, npwin/2 + 1 bins
    spectra = 129 * 15 * 262144 * 8        # compact complex64 spectra
    # spectra, leaf reflectors in complex64 (same size), and the tree blocks;
    # no realified copy
    assert 2 * spectra <= ws < 3 * spectra
    assert api.spod_query(1000, 512, 64, 32, "c128", hctx)[:2] == (15, 33)
    assert api.spod_query(1000, 100, 64, 0, "c64", hctx)[:2] == (1, 33)
    lib, h = hctx.lib, hctx.h
    nbv, nfv, wsv = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()

    def q(m=1000, nt=512, npwin=64, nolap=32, spectra=api.C64):
        return lib.pylom_spod_query(h, spectra, m, nt, npwin, nolap, ctypes.byref(nbv),
                                    ctypes.byref(nfv), ctypes.byref(wsv))
    assert q() == 0
    assert q(npwin=48) == -6               # not a power of two
    assert q(npwin=8192) == -6
    assert q(nolap=64) == -1               # overlap >= window
    assert q(nolap=-1) == -1
    assert q(nt=32) == -2                  # shorter than one window
    assert q(nt=4096) == -6                # more than 16 blocks
    assert q(m=10) == -2                   # fewer points than blocks
    assert q(spectra=api.R64) == -3
    vp = ctypes.c_void_p

    def run(prec=api.FP64, D=1, dt=1.0, window=0, modes=1, L=1, ldd=512):
        return lib.pylom_spod(h, api.C64, prec, 1000, 512, vp(D), ldd, dt, 64, 32, window, 1,
                              vp(modes), vp(L), vp(0), vp(0))
    assert run() == -7                     # valid: only the device is missing
    assert run(prec=api.MIXED) == -6
    assert run(D=0) == -1
    assert run(modes=0) == -1
    assert run(dt=0.0) == -1
    assert run(window=3) == -1
    assert run(ldd=100) == -2


def test_block_rows_tuner(hctx):
    # the stacked QR's latency model keeps the 4096-row leaves of the
    # 1048576 x 256 workload (the automatic path choice puts that shape on
    # the column-blocked TSQR, so the stacked path is named here)
    hctx.set_option("blocked_from", 1025)
    assert api.tune_block_rows(1 << 20, 256, hctx) == 4096
    for m, n in [(20000, 100), (50000, 32), (2_000_000, 512), (1000, 1000), (300, 200)]:
        b = api.tune_block_rows(m, n, hctx)
        assert b >= n and (b & (b - 1)) == 0 or b == n
    hctx.set_option("blocked_from", 0)
    assert hctx.lib.pylom_tune_block_rows(hctx.h, 10, 20) < 0   # m < n


def test_batched_validation_before_device(hctx):
    from paper_2405_15529_amd import _lib
    lib, h = hctx.lib, hctx.h
    ok = dict(m=1000, n=20, D=1, ldd=20, remove_mean=0, residual=0.01, mean=0, U=1, ldu=20, S=1,
              VT=1, ldvt=20, n_r=1)

    def run(probs, dtype=api.R64, prec=api.FP64, graph=0):
        arr = (_lib.Problem * len(probs))(*[_lib.Problem(**p) for p in probs])
        return lib.pylom_pod_batched(h, dtype, prec, len(probs), ctypes.cast(arr, ctypes.c_void_p),
                                     graph)
    assert run([ok, dict(ok, m=5000, n=64, ldd=64, ldu=64, ldvt=64)]) == -7   # valid: no device
    assert lib.pylom_pod_batched(h, api.R64, api.FP64, 0, None, 0) == 0       # empty batch
    assert lib.pylom_pod_batched(h, api.R64, api.FP64, 2, None, 0) == -1
    assert run([ok, dict(ok, D=0)]) == -1
    assert run([ok, dict(ok, m=10)]) == -2                                    # m < n
    assert run([dict(ok, ldu=5)]) == -2
    assert run([dict(ok, residual=1.5)]) == -1
    assert run([ok], prec=api.MIXED) == -3                                   # mixed needs R32
    assert run([ok], dtype=api.R32, prec=api.MIXED) == -7
    # wide instances plan on the column-blocked TSQR (valid: no device);
    # n > 2048 is not supported
    assert run([dict(ok, m=5000, n=2000, ldd=2000, ldu=2000, ldvt=2000)]) == -7
    assert run([dict(ok, m=5000, n=2100, ldd=2100, ldu=2100, ldvt=2100)]) == -6
    hctx.set_option("streams", 8)
    assert hctx.get_option("streams") == 8
    with pytest.raises(api.PylomError):
        hctx.set_option("streams", 0)


def test_dmd_validation_before_device(hctx):
    lib, h = hctx.lib, hctx.h
    vp = ctypes.c_void_p

    def call(m=1000, n=20, D=1, ldd=None, r=0.01, dt=1.0, phi=1, ldphi=None, mu=1, b=1, nr=1,
             dtype=api.R64):
        ldd = n if ldd is None else ldd
        ldphi = max(1, min(n - 1, 128)) if ldphi is None else ldphi
        return lib.pylom_dmd(h, dtype, m, n, vp(D), ldd, 0, r, dt, vp(phi), ldphi, vp(mu), vp(b),
                             None, None, vp(nr))
    assert call() == -7                       # valid: no device
    assert call(dtype=api.R32) == -7
    assert call(n=1) == -2                    # one snapshot
    assert call(m=10, n=20) == -2             # m < n
    assert call(ldd=10) == -2
    assert call(ldphi=5) == -2                # ldphi < min(n - 1, 128)
    assert call(D=0) == -1 and call(phi=0) == -1 and call(nr=0) == -1
    assert call(r=1.0) == -1 and call(dt=0.0) == -1
    assert call(dtype=api.C64) == -3
    b = ctypes.c_size_t()
    assert lib.pylom_dmd_workspace_query(h, api.R64, 58_300_000, 56, 0, ctypes.byref(b)) == 0
    # an R-only TSQR of the snapshots plus O(n^2): far below the 26 GB input
    assert 0 < b.value < 8 * 58_300_000 * 56


def test_workspace_cap_returns_enomem(hctx):
    # the cap is checked with the plan, before the device: a host-only
    # context reports PYLOM_ENOMEM for a call whose workspace exceeds it
    need = hctx.workspace_bytes(100000, 64)
    hctx.set_option("ws_cap_mb", max(1, need // (1 << 20) // 2))
    assert _pod(hctx, m=100000, n=64) == -4
    assert "ws_cap_mb" in hctx.lib.pylom_last_error(hctx.h).decode()
    assert _pod(hctx, dtype=api.R32, prec=api.MIXED, m=100000, n=64) == -4
    vp = ctypes.c_void_p
    R = ctypes.c_void_p(1)
    assert hctx.lib.pylom_tsqr(hctx.h, api.R64, api.FP64, 100000, 64, vp(1), 64, vp(1), 64, R,
                               64) == -4
    hctx.set_option("ws_cap_mb", 1 << 30)   # large enough: only the device is missing
    assert _pod(hctx, m=100000, n=64) == -7
    hctx.set_option("ws_cap_mb", 0)         # 0 = unlimited
    assert _pod(hctx, m=100000, n=64) == -7


def test_batched_workspace_cap(hctx):
    arr = (_lib.Problem * 2)()
    for i in range(2):
        arr[i] = _lib.Problem(50000, 40, 1, 40, 0, 0.01, 0, 1, 40, 1, 1, 40, 1)
    hctx.set_option("ws_cap_mb", 1)
    assert hctx.lib.pylom_pod_batched(hctx.h, api.R64, api.FP64, 2,
                                      ctypes.cast(arr, ctypes.c_void_p), 0) == -4
    hctx.set_option("ws_cap_mb", 0)
    assert hctx.lib.pylom_pod_batched(hctx.h, api.R64, api.FP64, 2,
                                      ctypes.cast(arr, ctypes.c_void_p), 0) == -7


def test_binding_rejects_host_tensors():
    # a host pointer handed to the kernels would be a GPU page fault: every
    # entry of the binding refuses CPU tensors before calling the library
    import torch
    A = torch.zeros((64, 8), dtype=torch.float64)
    B = torch.zeros((64, 4), dtype=torch.float64)
    for call in (lambda: api.pod(A), lambda: api.tsvd(A), lambda: api.tsqr(A),
                 lambda: api.matmul(A, B, trans_a=True), lambda: api.dmd(A),
                 lambda: api.spod(A.float())):
        with pytest.raises(ValueError):
            call()


def test_ooc_plan_and_failure_paths(hctx):
    # windows of whole leaves; the device holds the tree part and two windows
    hctx.set_option("block_rows", 1024)
    hctx.set_option("ooc_window_rows", 4096)
    ws, rows, nwin = api.ooc_query(20000, 100, api.R64, hctx)
    assert rows == 4096 and nwin == 5            # 19 leaves, 4 per window
    hctx.set_option("ooc_window_rows", 100)      # raised to 4 n = 400: leaves of 400 rows,
    ws2, rows2, nwin2 = api.ooc_query(20000, 100, api.R64, hctx)   # one per window
    assert rows2 == 400 and nwin2 == 50 and ws2 < ws
    vp = ctypes.c_void_p
    one = ctypes.c_int64(0)

    def call(prec=api.FP64, cap=0, m=20000, n=100):
        hctx.set_option("ws_cap_mb", cap)
        return hctx.lib.pylom_pod_host(hctx.h, api.R64, prec, m, n, vp(1), n, 1, 0.01, vp(0),
                                       vp(1), n, vp(1), vp(1), n, ctypes.byref(one))
    assert call() == -7                          # valid: only the device is missing
    assert call(cap=1) == -4                     # over the workspace cap: PYLOM_ENOMEM
    assert call(prec=api.MIXED) == -6            # FP64 compute only
    assert call(m=50, n=100) == -2
    hctx.set_option("ws_cap_mb", 0)


def test_work_queue_option_is_switched_off(hctx):
    # the work-queue launches are switched off: the option keeps its default
    # (one launch per phase and level) and refuses to be turned on
    assert hctx.get_option("work_queue") == 0
    with pytest.raises(api.PylomError) as e:
        hctx.set_option("work_queue", 1)
    assert e.value.status == -6
    hctx.set_option("work_queue", 0)


def test_tuning_file_round_trip(hctx, tmp_path):
    # a measured table read from JSON steers the leaf height of every shape
    # in its class (path, precision, floor(log2 m), n rounded up to 16)
    m, n = 10_000_000, 100        # the stacked path (more than 8,388,608 rows)
    p = tmp_path / "tune.json"
    p.write_text('{"pylom_tuning": 1, "entries": [\n'
                 '  {"path": "stacked", "precision": "fp64", "m_log2": 23, "n_bucket": 112, '
                 '"block_rows": 1536, "ms": 12.5},\n'
                 '  {"path": "blocked", "precision": "mixed", "m_log2": 22, "n_bucket": 1808, '
                 '"block_rows": 16384, "ms": 1500}\n]}\n')
    assert hctx.tune_load(str(p)) == 2
    assert api.tune_block_rows(m, n, hctx) == 1536           # 2^23 <= m < 2^24, n -> 112
    assert hctx.plan(m, n)["block_rows"] == 1536
    assert hctx.plan(m, 97)["block_rows"] == 1536            # same n bucket
    assert hctx.plan(m, 120)["block_rows"] != 1536           # another bucket
    assert hctx.plan(20_000_000, n)["block_rows"] != 1536    # another m bucket
    hctx.set_option("block_rows", 2048)                      # an explicit height wins
    assert hctx.plan(m, n)["block_rows"] == 2048
    hctx.set_option("block_rows", 0)
    q = tmp_path / "saved.json"
    hctx.tune_save(str(q))
    other = api.Context(-1)
    assert other.tune_load(str(q)) == 2
    assert other.plan(m, n)["block_rows"] == 1536
    other.close()
    bad = tmp_path / "bad.json"
    bad.write_text('{"pylom_tuning": 1, "entries": [{"path": "sideways", "precision": "fp64", '
                   '"m_log2": 3, "n_bucket": 16, "block_rows": 64}]}')
    with pytest.raises(api.PylomError):
        hctx.tune_load(str(bad))
    with pytest.raises(api.PylomError):
        hctx.tune_load(str(tmp_path / "missing.json"))


def test_mixed_tree_option(hctx):
    # 1 (default): FP32 tree levels below the final combine on the mixed
    # column-blocked path; 0: every level in FP64; nothing else is accepted
    assert hctx.get_option("mixed_tree") == 1
    hctx.set_option("mixed_tree", 0)
    assert hctx.get_option("mixed_tree") == 0
    for bad in (-1, 2):
        with pytest.raises(api.PylomError):
            hctx.set_option("mixed_tree", bad)
    hctx.set_option("mixed_tree", 1)
    assert hctx.get_option("mixed_tree") == 1


def test_mixed_svd_tol_option(hctx):
    # 1 (default): the first SVD of a mixed call stops rotating at cosines of
    # 2^-24; 0: the FP64 threshold n 2^-53
    assert hctx.get_option("mixed_svd_tol") == 1
    hctx.set_option("mixed_svd_tol", 0)
    assert hctx.get_option("mixed_svd_tol") == 0
    for bad in (-1, 2):
        with pytest.raises(api.PylomError):
            hctx.set_option("mixed_svd_tol", bad)
    hctx.set_option("mixed_svd_tol", 1)


def test_tree_pipeline_option(hctx):
    # S (default 8): the column-blocked tree levels as a wavefront over up to
    # S of the library's streams; 0 or 1: one level after another
    assert hctx.get_option("tree_pipeline") == 8
    for v in (0, 1, 8, 16):
        hctx.set_option("tree_pipeline", v)
        assert hctx.get_option("tree_pipeline") == v
    for bad in (-1, 17):
        with pytest.raises(api.PylomError):
            hctx.set_option("tree_pipeline", bad)
    hctx.set_option("tree_pipeline", 8)
