"""Benchmark of the POD TSQR-SVD hot path on one MI355X.

Headline (the metric's own comparison, mixed precision against FP64 on one
input): the travelling-wave POD of m = 4,194,304 grid points by n = 1,808
FP32 snapshots (64 travelling waves plus N(0, 1e-8) noise), mean removed,
99 % energy, on the column-blocked TSQR.  One step = one mixed-precision
pylom_pod call (FP32 leaf QR, FP64 tree and SVD of R, Rayleigh-Ritz
refinement against the input); the FP64 call on the same buffer is timed
beside it for the speed-up and the sigma agreement.

value = algorithmic TFLOP/s of the mixed step, F = 2 m n^2 + 2 m n N_r (the
TSQR leaf term of Eq. flops + U = Q U_R); gbps counts B = 2 s_in m n +
s_out m N_r.  The roofline object rates the dominant kernel of the mixed
step, timed live with an event pair around each launch inside the timed
region.  cpu_baseline times the CPU oracle on a bounded row slice of the
same field.  The known-spectrum FP64 workload (1,048,576 x 256, row blocks
4,096) runs as the "c2" sub-object, SPOD, the uneven batch and DMD after it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBPS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5,
                    help="timed mixed-precision calls of the headline workload")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=5,
                    help="timed FP64 calls beside the headline (at most --steps)")
    ap.add_argument("--c2-steps", type=int, default=10)
    ap.add_argument("--c2-warmup", type=int, default=3)
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--m", type=int, default=1_048_576)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--block-rows", type=int, default=4096)
    ap.add_argument("--blocked-from", type=int, default=1025,
                    help="the library's blocked_from option for the main workload (default "
                         "1025: the stacked QR, the faster path at 4096-row leaves; 0: the "
                         "library's automatic choice)")
    ap.add_argument("--no-default-path", action="store_true",
                    help="skip the run of the main matrix on the library's automatic path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=8192)
    ap.add_argument("--no-spod", action="store_true")
    ap.add_argument("--spod-m", type=int, default=262144)
    ap.add_argument("--spod-nt", type=int, default=2048)
    ap.add_argument("--spod-steps", type=int, default=3)
    ap.add_argument("--only-spod", action="store_true",
                    help="run only the SPOD leg (once per --spod-block-rows value)")
    ap.add_argument("--spod-block-rows", type=int, nargs="*", default=None,
                    help="leaf heights of the SPOD realification to time (0: the library's)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-ooc", action="store_true")
    ap.add_argument("--only-ooc", action="store_true",
                    help="run only the out-of-core leg and print its object")
    ap.add_argument("--ooc-m", type=int, default=8_388_608)
    ap.add_argument("--ooc-n", type=int, default=256)
    ap.add_argument("--ooc-window", type=int, default=1_048_576)
    ap.add_argument("--no-dmd", action="store_true")
    ap.add_argument("--dmd-wide", action="store_true",
                    help="also time exact DMD of the headline field (N = 1808 snapshots)")
    ap.add_argument("--dmd-m", type=int, default=58_300_000)
    ap.add_argument("--dmd-n", type=int, default=56)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--wide-m", type=int, default=4_194_304)
    ap.add_argument("--wide-n", type=int, default=1808)
    ap.add_argument("--wide-block-rows", type=int, default=0, help="0: the library's choice")
    ap.add_argument("--paper-shapes", action="store_true",
                    help="run only the shapes of the paper's performance study (the JSM "
                         "matrix and the weak scaling in N) and print their object")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed region, copy one 1 GiB FP64 buffer on the device "
                         "(a plain copy of known size, for calibrating HBM byte counters)")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=2)
    return ap.parse_args()


def timed_spod(api, m, nt, npwin, nolap, steps, warmup, block_rows=0):
    """Batched SPOD (C4 shape): one pylom_spod call per step on a resident
    FP32 snapshot matrix; complex64 spectra and modes."""
    import torch
    from paper_2405_15529_amd import synth

    D = torch.from_numpy(synth.spod_field(m, nt, seed=3, nmodes=32)).cuda()
    ctx = api.Context(0)
    ctx.set_option("timing", max(1, steps))
    if block_rows:
        ctx.set_option("block_rows", block_rows)
    nb, nf, ws = api.spod_query(m, nt, npwin, nolap, "c64", ctx)
    ctx.check(ctx.lib.pylom_reserve(ctx.h, ws))
    out = None
    for _ in range(warmup):
        out = api.spod(D, npwin=npwin, nolap=nolap, spectra="c64", ctx=ctx)
    torch.cuda.synchronize()
    if warmup:
        ctx.phase_times()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        out = api.spod(D, npwin=npwin, nolap=nolap, spectra="c64", ctx=ctx)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    ph = ctx.phase_times()
    rc, sweeps = ctx.status()
    # complex SVD flops per frequency, 4x real: 2 m nb^2 (QR) + 2 m nb nb (U)
    flops = nf * 4.0 * (2.0 * m * nb * nb + 2.0 * m * nb * nb)
    fft_bytes = 4.0 * m * nt + 8.0 * nf * m * nb
    lead = out.L[:, 0].cpu().numpy()
    res = {
        "workload": f"batched SPOD {m} points x {nt} FP32 snapshots, npwin {npwin}, "
                    f"nolap {nolap}, Hann, {nf} frequencies x {nb} blocks, complex64",
        "ms_per_step": round(ms, 3),
        "tflops": round(flops / (ms * 1e-3) / 1e12, 4),
        "front_end_gbps": round(fft_bytes / (ph["front_end"] * 1e-3) / 1e9, 1),
        "front_end_hbm_frac": round(fft_bytes / (ph["front_end"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "phase_ms": {k: round(v, 4) for k, v in ph.items()},
        "status": rc,
        "jacobi_sweeps_max": sweeps,
        "top_frequency": int(out.order[0].item()),
        "leading_energy": float(lead.max()),
    }
    ctx.close()
    del D, out
    torch.cuda.empty_cache()
    return res


def host_info():
    """nproc and the CPU model of this host (for the CPU baseline)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count() or 0, model


def cpu_baseline_c3(m: int, n: int, rows: int):
    """The oracle (plain single-threaded C, FP64) on the first `rows` rows of
    the headline field: its temporal mean (Alg. 2) and its Householder QR
    with R only (the 2 rows n^2 leaf term of Eq. flops, which dominates F).
    The Jacobi SVD of the 1808 x 1808 R is left out: its cost does not
    shrink with the row sample (several minutes of one core).  Rate in
    TFLOP/s of the same accounting, 2 rows n^2 over the timed seconds."""
    import numpy as np
    import oracle
    from paper_2405_15529_amd import synth

    D = synth.travelling_waves_rows(m, n, 0, rows, seed=2).astype(np.float64)
    oracle.build()
    t0 = time.perf_counter()
    mu = oracle.mean(D)
    Y = D - mu[:, None]
    oracle.qr(Y, want_q=False)
    dt = time.perf_counter() - t0
    nproc, model = host_info()
    return dict(value=2.0 * rows * n * n / dt / 1e12, unit="TFLOP/s", cores=1, kind="oracle",
                sample=f"rows 0..{rows - 1} of the {m} x {n} travelling-wave field (FP64): the "
                       f"oracle's temporal mean and Householder QR (R only, the 2 m n^2 term); "
                       f"{dt:.2f} s on one thread",
                seconds=dt, host_nproc=nproc, host_cpu=model, threads=1)


def cpu_baseline_c2(n: int, rows: int, r: float):
    """The oracle's whole POD (single-threaded C, FP64) on a row sample of
    the known-spectrum workload."""
    import oracle
    from paper_2405_15529_amd import synth

    A, _ = synth.graded_fp64(m=rows, n=n, seed=11)
    oracle.build()
    t0 = time.perf_counter()
    out = oracle.pod(A, remove_mean=False, r=r)
    dt = time.perf_counter() - t0
    nr = out["nr"]
    flops = 2.0 * rows * n * n + 2.0 * rows * n * nr
    return dict(value=flops / dt / 1e12, unit="TFLOP/s", cores=1, kind="oracle",
                sample=f"{rows} x {n} rows of the same known-spectrum generator, FP64, "
                       f"{dt:.2f} s, one thread", seconds=dt)


# HBM bytes per launch, from two rocprofv3 --pmc passes (FETCH_SIZE, then
# WRITE_SIZE) scaled by the same counters read on a plain 1 GiB device copy;
# each entry is valid only for the kernel sources it was taken on (their
# SHA-256) and for its shape.  The counter summaries are in profiles/.
TRAFFIC = {
    # FP64 stacked leaf QR, 1048576 x 256, row blocks 4096 (one launch)
    "stacked_leaf_fp64": {
        "sources": ("tsqr.hip", "common.hpp"),
        "sources_sha256": "0b49fd0300209348e07114a140783bae57365fd1073257084b0a0f828fcb92c1",
        "shape": (1048576, 256, 4096),
        "bytes": 13615113691,  # FETCH 6.575e+09 (x1.99992) + WRITE 7.040e+09 (x1.0)
    },
    # FP32 leaf trailing updates of the column-blocked QR, 4194304 x 1808, row
    # blocks 8192: mean over the 28 launches of one mixed call
    "blocked_trailing_fp32": {
        "sources": ("blocked.hip", "common.hpp"),
        "sources_sha256": "75e6e080d46d8080999a088c8f6fd96206012b641062f304d55639085f540e2e",
        "shape": (4194304, 1808, 8192),
        "bytes": 33617105460,  # FETCH 5.139e+11 (x1.99992) + WRITE 4.274e+11 (x1.0), / 28
    },
}


def sources_sha256(names) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2405_15529_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(key: str, shape):
    """Bytes per launch of a kernel, or None if none were taken for these
    sources and this shape."""
    t = TRAFFIC.get(key)
    if not t or tuple(t["shape"]) != tuple(shape):
        return None
    if t["sources_sha256"] != sources_sha256(t["sources"]):
        return None  # the kernel changed since the counters were taken
    return t["bytes"]


def timed_pod(api, ctx, A, m, n, r, precision, steps, warmup, remove_mean=False,
              kernel_timing=False):
    """Run pylom_pod `warmup` + `steps` times on the resident A; returns the
    mean ms per call (HIP events on the library stream), phase means, the
    outputs of the last call and, with kernel_timing, the summed duration and
    launch count of every kernel role over the timed calls (an event pair
    around each launch, on the library stream)."""
    import ctypes
    import torch

    dev = A.device
    lib = ctx.lib
    prec = api.FP64 if precision == "fp64" else api.MIXED
    dt = api.R64 if A.dtype == torch.float64 else api.R32
    ctx.check(lib.pylom_reserve(ctx.h, ctx.workspace_bytes(m, n, dt, precision)))
    U = torch.empty((m, n), dtype=A.dtype, device=dev)
    S = torch.empty(n, dtype=torch.float64, device=dev)
    VT = torch.empty((n, n), dtype=torch.float64, device=dev)
    nr_d = torch.empty(1, dtype=torch.int64, device=dev)
    mean = torch.empty(m, dtype=A.dtype, device=dev) if remove_mean else None
    vp = ctypes.c_void_p

    def step():
        rc = lib.pylom_pod(ctx.h, dt, prec, m, n, vp(A.data_ptr()), n, 1 if remove_mean else 0, r,
                           vp(mean.data_ptr() if remove_mean else 0),
                           vp(U.data_ptr()), n, vp(S.data_ptr()), vp(VT.data_ptr()), n,
                           vp(nr_d.data_ptr()))
        if rc != 0:
            raise RuntimeError(lib.pylom_last_error(ctx.h).decode())

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.status()
    if warmup:
        ctx.phase_times()  # drop warm-up samples
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    if kernel_timing:
        ctx.set_option("kernel_timing", 1)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    for _ in range(steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1) / steps
    kt = None
    if kernel_timing:
        kt = ctx.kernel_times()
        ctx.set_option("kernel_timing", 0)
    phases = ctx.phase_times()
    rc, sweeps = ctx.status()
    return dict(ms=ms, wall=wall, phases=phases, rc=rc, sweeps=sweeps, U=U, S=S, VT=VT,
                nr=int(nr_d.item()), kernels=kt)


FP32_PEAK_TFLOPS = 157.3


def blocked_trailing_flops(m: int, n: int, pw: int = 64) -> float:
    """Algorithmic flops of all leaf trailing updates of the column-blocked
    TSQR: panel k (pw columns) applies its block reflector to the
    n - (k+1) pw columns right of it over all m rows, W = V^T C then
    C -= V (T^T W): 4 m pw (n - (k+1) pw) flops per launch (the small T^T W
    product is not counted)."""
    K = (n + pw - 1) // pw
    return sum(4.0 * m * pw * (n - (k + 1) * pw) for k in range(K - 1))


def kernel_summary(kt, steps):
    """Per-call milliseconds and launches of every kernel role."""
    return {k: {"ms_per_call": round(v[0] / steps, 3), "launches_per_call": v[1] // steps}
            for k, v in kt.items() if v[1]}


def timed_c3(api, m, n, steps, warmup, block_rows=0, fp64_steps=None):
    """The headline: mixed precision against FP64 on one FP32 buffer, m x n
    travelling waves (64 waves + N(0, 1e-8)), mean removed, 99 % energy,
    through the column-blocked TSQR.  Kernel roles are timed live during the
    timed mixed and FP64 calls."""
    import numpy as np
    import torch
    from paper_2405_15529_amd import synth

    r = 0.01
    D = synth.travelling_waves_device(m, n, seed=2, device="cuda")
    torch.cuda.synchronize()
    ctx = api.Context(0)
    ctx.set_option("timing", max(1, steps))
    ctx.bind_stream()
    if block_rows:
        ctx.set_option("block_rows", block_rows)
    b = block_rows or api.tune_block_rows(m, n, ctx)
    fp64_steps = steps if fp64_steps is None else fp64_steps

    def orth_err(U, k):
        Ur = U[:, :k].double()
        return float(torch.linalg.norm(Ur.T @ Ur - torch.eye(k, dtype=torch.float64,
                                                               device=U.device)).item())

    x = timed_pod(api, ctx, D, m, n, r, "mixed", steps, warmup, remove_mean=True,
                  kernel_timing=True)
    Sx = x["S"].cpu().numpy()
    nrx = x["nr"]
    orth_x = orth_err(x["U"], nrx)
    del x["U"]
    torch.cuda.empty_cache()
    f = timed_pod(api, ctx, D, m, n, r, "fp64", fp64_steps, min(warmup, 1), remove_mean=True,
                  kernel_timing=True)
    Sf = f["S"].cpu().numpy()
    nrf = f["nr"]
    orth_f = orth_err(f["U"], nrf)
    del f["U"]
    ctx.close()
    del D
    torch.cuda.empty_cache()
    k = min(nrx, nrf)

    def rates(ms, nr, s_in, s_out):
        fl = 2.0 * m * n * n + 2.0 * m * n * nr
        by = 2.0 * s_in * m * n + s_out * m * nr
        return fl / (ms * 1e-3) / 1e12, by / (ms * 1e-3) / 1e9

    tf_f, gb_f = rates(f["ms"], nrf, 4, 4)
    tf_x, gb_x = rates(x["ms"], nrx, 4, 4)
    # roofline of the leaf trailing updates (the 2 m n^2 term on MFMA):
    # algorithmic flops of all launches over their summed live durations
    trail_fl = blocked_trailing_flops(m, n)
    kx, kf = x["kernels"], f["kernels"]
    t32_ms, t32_n = kx["leaf_trailing_update"]
    t64_ms, t64_n = kf["leaf_trailing_update"]
    ach32 = trail_fl * steps / (t32_ms * 1e-3) / 1e12
    ach64 = trail_fl * fp64_steps / (t64_ms * 1e-3) / 1e12
    return {
        "workload": f"travelling-wave POD FP32 {m}x{n} (64 waves + N(0,1e-8)), mean removed, "
                    f"99% energy, column-blocked TSQR (64-column panels), row blocks {b}",
        "m": m, "n": n, "block_rows": b,
        "mixed": {"ms_per_step": round(x["ms"], 3), "tflops": round(tf_x, 4),
                  "gbps": round(gb_x, 2), "n_r": nrx, "orth_err_U": orth_x,
                  "jacobi_sweeps_first": x["sweeps"], "status": x["rc"],
                  "wall_s": round(x["wall"], 3),
                  "phase_ms": {"working_copy": round(x["phases"]["front_end"], 3),
                               "leaf_qr_fp32": round(x["phases"]["leaf_qr"], 3),
                               "tree_combine": round(x["phases"]["tree_combine"], 3),
                               "small_svd": round(x["phases"]["small_svd"], 3),
                               "refine_project_gram_eig": round(x["phases"]["tree_propagate"], 3),
                               "form_u": round(x["phases"]["leaf_apply"], 3)},
                  "kernels": kernel_summary(kx, steps)},
        "fp64": {"ms_per_step": round(f["ms"], 3), "tflops": round(tf_f, 4),
                 "gbps": round(gb_f, 2), "n_r": nrf, "orth_err_U": orth_f,
                 "jacobi_sweeps": f["sweeps"], "status": f["rc"], "steps": fp64_steps,
                 "phase_ms": {k2: round(v, 3) for k2, v in f["phases"].items()},
                 "kernels": kernel_summary(kf, fp64_steps)},
        "speedup_mixed_vs_fp64": round(f["ms"] / x["ms"], 3),
        "sigma_rel_err_mixed_vs_fp64_run":
            float(np.max(np.abs(Sx[:k] - Sf[:k]) / Sf[:k])) if k else 0.0,
        "trailing_update": {
            "algorithmic_flops_per_call": trail_fl,
            "fp32_launches_per_call": t32_n // steps,
            "fp32_mean_launch_ms": round(t32_ms / t32_n, 4),
            "fp32_tflops": round(ach32, 3), "fp32_frac": round(ach32 / FP32_PEAK_TFLOPS, 4),
            "fp64_mean_launch_ms": round(t64_ms / t64_n, 4),
            "fp64_tflops": round(ach64, 3), "fp64_frac": round(ach64 / FP64_PEAK_TFLOPS, 4)},
        "steps": steps, "warmup": warmup,
    }


def fit_power(xs, ts):
    """Least-squares exponent x and prefactor c of t = c n^x (log-log fit)."""
    import numpy as np
    lx, lt = np.log(np.asarray(xs, dtype=np.float64)), np.log(np.asarray(ts, dtype=np.float64))
    x, lc = np.polyfit(lx, lt, 1)
    return float(x), float(np.exp(lc))


def timed_paper_shapes(api, steps, warmup, jsm_m=58_300_000, jsm_n=56, weak_m=36_000_000,
                       weak_ns=(10, 20, 40, 80, 160, 320), top_m=18_000_000, top_n=630):
    """The shapes of the paper's performance study (Sec. 5) on one GPU.

    * The JSM strong-scaling matrix, 5.83e7 x 56 (FP64, 26 GB; a known
      spectrum s_i = 10^(-i/8) stands in for the flow data): FP64 and mixed
      at the tuned leaf height, then a sweep of leaf heights that splits the
      time into leaf QR and tree levels, the one-GPU counterpart of the
      paper's QR-versus-communication breakdown.
    * The weak scaling in N: n = 10 sqrt(k) columns at M = 3.6e7 rows (FP32
      travelling waves, mean removed), FP64 and mixed, for n up to 320; the
      exponent x of t ~ n^x is fitted over that range.  n = 630 does not fit
      one GPU at M = 3.6e7 (input, U and the reflectors alone are 273 GB in
      mixed precision), so it runs at 1.8e7 rows, mixed, and stays out of
      the fit."""
    import numpy as np
    import torch
    from paper_2405_15529_amd import synth

    def log(msg):
        print(f"[paper-shapes] {msg}", file=sys.stderr, flush=True)

    def orth_err(U, k):
        if k == 0:
            return 0.0
        Ur = U[:, :k].double()
        return float(torch.linalg.norm(Ur.T @ Ur - torch.eye(k, dtype=torch.float64,
                                                               device=U.device)).item())

    def levels(P):
        lv, h = 0, 1
        while h < P:
            lv, h = lv + 1, 2 * h
        return lv

    def run(A, m, n, precision, remove_mean, b=0):
        ctx = api.Context(0)
        ctx.set_option("timing", max(1, steps))
        ctx.bind_stream()
        if b:
            ctx.set_option("block_rows", b)
        bb = b or api.tune_block_rows(m, n, ctx)
        res = timed_pod(api, ctx, A, m, n, 0.01, precision, steps, warmup, remove_mean=remove_mean)
        ctx.close()
        res["b"] = bb
        res["orth"] = orth_err(res["U"], res["nr"])
        del res["U"]
        torch.cuda.empty_cache()
        return res

    def summary(res, m, n, s_in):
        fl = 2.0 * m * n * n + 2.0 * m * n * res["nr"]
        P = max(1, m // res["b"])
        return {"ms": round(res["ms"], 3), "tflops": round(fl / (res["ms"] * 1e-3) / 1e12, 4),
                "gbps": round((2.0 * s_in * m * n + s_in * m * res["nr"]) / (res["ms"] * 1e-3) / 1e9, 2),
                "n_r": res["nr"], "orth_err_U": res["orth"], "status": res["rc"],
                "block_rows": res["b"], "leaves": P, "tree_levels": levels(P),
                "phase_ms": {k: round(v, 3) for k, v in res["phases"].items()}}

    out = {}
    # --- JSM strong-scaling matrix ---------------------------------------
    m, n = jsm_m, jsm_n
    s = 10.0 ** (-np.arange(n) / 8.0)
    log(f"JSM {m}x{n} FP64 known spectrum")
    A = synth.known_spectrum_device(m, n, s, seed=5)
    torch.cuda.synchronize()
    f = run(A, m, n, "fp64", False)
    Sf = f["S"].cpu().numpy()
    jsm = {"workload": f"JSM strong-scaling shape {m}x{n} FP64, known spectrum "
                       f"s_i=10^(-i/8), 99% energy", "fp64": summary(f, m, n, 8),
           "sigma_rel_err_retained": float(np.max(np.abs(Sf[:f["nr"]] - s[:f["nr"]]) / s[:f["nr"]]))}
    log(f"  fp64 {jsm['fp64']['ms']} ms")
    sweep = []
    for b in (2048, 8192, 32768, 131072):
        g = run(A, m, n, "fp64", False, b=b)
        row = summary(g, m, n, 8)
        sweep.append({k: row[k] for k in ("block_rows", "leaves", "tree_levels", "ms")} |
                     {"leaf_qr_ms": row["phase_ms"]["leaf_qr"],
                      "tree_ms": row["phase_ms"]["tree_combine"],
                      "tree_ms_per_level": round(row["phase_ms"]["tree_combine"] /
                                                 max(1, row["tree_levels"]), 4)})
        log(f"  b={b}: {row['ms']} ms (leaf {sweep[-1]['leaf_qr_ms']}, tree {sweep[-1]['tree_ms']})")
    jsm["leaf_height_sweep_fp64"] = sweep
    A32 = A.float()
    del A
    torch.cuda.empty_cache()
    x = run(A32, m, n, "mixed", False)
    Sx = x["S"].cpu().numpy()
    k = min(x["nr"], f["nr"])
    jsm["mixed"] = summary(x, m, n, 4)
    jsm["mixed"]["sigma_rel_err_vs_fp64_run"] = float(np.max(np.abs(Sx[:k] - Sf[:k]) / Sf[:k])) if k else 0.0
    jsm["mixed"]["speedup_vs_fp64"] = round(f["ms"] / x["ms"], 3)
    log(f"  mixed {jsm['mixed']['ms']} ms")
    del A32
    torch.cuda.empty_cache()
    out["jsm"] = jsm

    # --- weak scaling in N ------------------------------------------------
    pts = []
    for n in weak_ns:
        m = weak_m
        log(f"weak-N {m}x{n} FP32 travelling waves")
        D = synth.travelling_waves_device(m, n, seed=2)
        torch.cuda.synchronize()
        f = run(D, m, n, "fp64", True)
        x = run(D, m, n, "mixed", True)
        Sf, Sx = f["S"].cpu().numpy(), x["S"].cpu().numpy()
        k = min(f["nr"], x["nr"])
        pt = {"m": m, "n": n, "fp64": summary(f, m, n, 4), "mixed": summary(x, m, n, 4),
              "sigma_rel_err_mixed_vs_fp64": float(np.max(np.abs(Sx[:k] - Sf[:k]) / Sf[:k])) if k else 0.0}
        pts.append(pt)
        log(f"  fp64 {pt['fp64']['ms']} ms, mixed {pt['mixed']['ms']} ms")
        del D
        torch.cuda.empty_cache()
    ns = [p["n"] for p in pts]
    fits = {}
    for prec in ("fp64", "mixed"):
        xe, c = fit_power(ns, [p[prec]["ms"] for p in pts])
        xl, _ = fit_power(ns, [p[prec]["phase_ms"]["leaf_qr"] for p in pts])
        fits[prec] = {"x_total": round(xe, 4), "x_leaf_qr": round(xl, 4)}
    m, n = top_m, top_n
    log(f"weak-N top point {m}x{n} FP32, mixed")
    D = synth.travelling_waves_device(m, n, seed=2)
    torch.cuda.synchronize()
    x = run(D, m, n, "mixed", True)
    top = {"m": m, "n": n, "mixed": summary(x, m, n, 4)}
    log(f"  mixed {top['mixed']['ms']} ms")
    del D
    torch.cuda.empty_cache()
    out["weak_n"] = {"workload": f"weak scaling in N: FP32 travelling waves {weak_m} x n, "
                                 f"n = 10 sqrt(k), mean removed, 99% energy",
                     "points": pts, "fit_t_vs_n": fits, "paper_exponent": 1.387,
                     "top_point": top}
    out["steps"], out["warmup"] = steps, warmup
    return out


def timed_dmd(api, m, n, steps, warmup):
    """Exact DMD (Alg. 3-5) of exactly linear FP64 snapshots, m x n with 50
    modes (24 conjugate pairs and two real eigenvalues), residual 1e-10: one
    pylom_dmd call per step, and its first step alone (the R-only TSQR of the
    snapshots, pylom_tsqr without Q) to split the time.  TFLOP/s counts that
    TSQR (2 m n^2) and the mode GEMM (4 m (n - 1) N_r)."""
    import ctypes
    import numpy as np
    import torch
    from paper_2405_15529_amd import synth

    D, lam, phi, amp = synth.linear_dynamics_device(m, n, seed=24)
    del phi
    torch.cuda.empty_cache()
    ctx = api.Context(0)
    ctx.bind_stream()
    kc = min(n - 1, api.DMD_MAX_MODES)
    dev = D.device
    phi = torch.empty((m, kc), dtype=torch.complex128, device=dev)
    mu_d = torch.empty(kc, dtype=torch.complex128, device=dev)
    b_d = torch.empty(kc, dtype=torch.complex128, device=dev)
    fr = torch.empty(kc, dtype=torch.float64, device=dev)
    gr = torch.empty(kc, dtype=torch.float64, device=dev)
    nr_d = torch.empty(1, dtype=torch.int64, device=dev)
    vp = ctypes.c_void_p
    ctx.check(ctx.lib.pylom_reserve(ctx.h, api.dmd_workspace_bytes(m, n, api.R64, False, ctx)))

    def step():
        ctx.check(ctx.lib.pylom_dmd(ctx.h, api.R64, m, n, vp(D.data_ptr()), n, 0, 1e-10, 1.0,
                                    vp(phi.data_ptr()), kc, vp(mu_d.data_ptr()),
                                    vp(b_d.data_ptr()), vp(fr.data_ptr()), vp(gr.data_ptr()),
                                    vp(nr_d.data_ptr())))
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record()
    for _ in range(steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - wall0) / steps
    ms = t0.elapsed_time(t1) / steps
    rc, _ = ctx.status()
    k = int(nr_d.item())
    mu = mu_d[:k].cpu().numpy()
    emu = float(max(np.min(np.abs(lam - z)) for z in mu)) if k else 0.0
    del phi
    torch.cuda.empty_cache()
    # the R-only TSQR of the snapshots alone (the first step of pylom_dmd)
    R = torch.empty((n, n), dtype=torch.float64, device=D.device)

    def tsqr():
        ctx.check(ctx.lib.pylom_tsqr(ctx.h, api.R64, api.FP64, m, n, vp(D.data_ptr()), n, None, n,
                                     vp(R.data_ptr()), n))
    tsqr()
    torch.cuda.synchronize()
    t0.record()
    for _ in range(steps):
        tsqr()
    t1.record()
    torch.cuda.synchronize()
    ms_qr = t0.elapsed_time(t1) / steps
    ctx.close()
    del D, R
    torch.cuda.empty_cache()
    n1 = n - 1
    flops = 2.0 * m * n * n + 2.0 * m * n1 * 2 * k   # R-only TSQR of Y + phi = Y2 B (complex B)
    return {
        "workload": f"exact DMD of the JSM shape {m}x{n} FP64, exactly linear dynamics with "
                    f"{len(lam)} modes, residual 1e-10",
        "ms_per_step": round(ms, 3), "wall_ms_per_step": round(wall * 1e3, 3),
        "tflops": round(flops / (ms * 1e-3) / 1e12, 4),
        "r_only_tsqr_ms": round(ms_qr, 3),
        "svd_linear_map_eig_amplitudes_modes_ms": round(ms - ms_qr, 3),
        "n_r": k, "status": rc, "max_abs_mu_minus_lambda": emu,
        "steps": steps, "warmup": warmup,
    }


def timed_dmd_wide(api, m, n, steps, warmup):
    """Exact DMD of the wide FP32 travelling waves (m x n, 64 waves plus
    N(0, 1e-8) noise, mean removed, 99 % energy): N = 1808 snapshots, the
    count of the paper's diffuser data, through the column-blocked R-only
    TSQR.  Every wave is two exponentials e^{+-i w t}, so each retained
    eigenvalue is compared with the nearest true one."""
    import ctypes
    import numpy as np
    import torch
    from paper_2405_15529_amd import synth

    D = synth.travelling_waves_device(m, n, seed=2, device="cuda")
    _, w, _, _ = synth.travelling_wave_params(m, 2)
    lam = np.concatenate([np.exp(1j * w), np.exp(-1j * w)])
    torch.cuda.synchronize()
    ctx = api.Context(0)
    ctx.bind_stream()
    kc = min(n - 1, api.DMD_MAX_MODES)
    dev = D.device
    phi = torch.empty((m, kc), dtype=torch.complex128, device=dev)
    mu_d = torch.empty(kc, dtype=torch.complex128, device=dev)
    b_d = torch.empty(kc, dtype=torch.complex128, device=dev)
    gr = torch.empty(kc, dtype=torch.float64, device=dev)
    nr_d = torch.empty(1, dtype=torch.int64, device=dev)
    vp = ctypes.c_void_p
    ctx.check(ctx.lib.pylom_reserve(ctx.h, api.dmd_workspace_bytes(m, n, api.R32, True, ctx)))

    def step():
        ctx.check(ctx.lib.pylom_dmd(ctx.h, api.R32, m, n, vp(D.data_ptr()), n, 1, 0.01, 1.0,
                                    vp(phi.data_ptr()), kc, vp(mu_d.data_ptr()),
                                    vp(b_d.data_ptr()), None, vp(gr.data_ptr()),
                                    vp(nr_d.data_ptr())))
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    rc, _ = ctx.status()
    k = int(nr_d.item())
    mu = mu_d[:k].cpu().numpy()
    dist = [float(np.min(np.abs(lam - z))) for z in mu]
    ctx.close()
    del D, phi
    torch.cuda.empty_cache()
    return {
        "workload": f"exact DMD of FP32 travelling waves {m}x{n} (64 waves + N(0,1e-8)), mean "
                    f"removed, 99% energy, column-blocked R-only TSQR",
        "ms_per_step": round(ms, 3),
        "tflops": round((2.0 * m * n * n + 2.0 * m * (n - 1) * 2 * k) / (ms * 1e-3) / 1e12, 4),
        "n_r": k, "status": rc,
        "max_abs_mu_minus_nearest_true": max(dist) if dist else 0.0,
        "median_abs_mu_minus_nearest_true": float(np.median(dist)) if dist else 0.0,
        "max_abs_growth": float(torch.max(torch.abs(gr[:k])).item()) if k else 0.0,
        "steps": steps, "warmup": warmup,
    }


def timed_ooc(api, m, n, window_rows, steps):
    """Out-of-core POD (pylom_pod_host) of an m x n FP32 travelling-wave field
    held in host memory, streamed through the device in windows of
    window_rows rows (two passes), against the in-device POD of the same
    matrix on the same path and leaf height.  Rates count the host traffic
    of the two passes (2 x 4 m n read, 4 m N_r written) over the wall time
    of the call, which includes every PCIe transfer and host-side copy."""
    import numpy as np
    import torch
    from paper_2405_15529_amd import synth

    Dd = synth.travelling_waves_device(m, n, seed=2, device="cuda")
    D = Dd.cpu().numpy()
    torch.cuda.synchronize()
    # leaves of window_rows / 512 rows: two per CU within a window
    b = max(n, window_rows // 512)
    ctx = api.Context(0)
    ctx.set_option("ooc_window_rows", window_rows)
    ctx.set_option("block_rows", b)
    ws, rows, nwin = api.ooc_query(m, n, api.R32, ctx)
    U = np.empty((m, n), dtype=np.float32)
    api.pod_host(D, remove_mean=True, r=0.01, ctx=ctx, U=U)   # warm-up: workspace, staging
    times = []
    h = None
    for _ in range(steps):
        t0 = time.perf_counter()
        h = api.pod_host(D, remove_mean=True, r=0.01, ctx=ctx, U=U)
        times.append(time.perf_counter() - t0)
    rc, _ = ctx.status()
    ctx.close()
    # the same matrix resident on the device, column-blocked at the same leaf height
    ctx2 = api.Context(0)
    ctx2.set_option("blocked_from", 2)
    ctx2.set_option("block_rows", b)
    ctx2.bind_stream()
    g = api.pod(Dd, remove_mean=True, r=0.01, ctx=ctx2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = api.pod(Dd, remove_mean=True, r=0.01, ctx=ctx2)
    torch.cuda.synchronize()
    t_dev = time.perf_counter() - t0
    Sg = g.S.cpu().numpy()
    same = bool(np.array_equal(Sg, h.S))
    ctx2.close()
    del Dd, g
    torch.cuda.empty_cache()
    t = min(times)
    host_bytes = 2.0 * 4 * m * n + 4.0 * m * h.nr
    return {
        "workload": f"out-of-core POD of a {m}x{n} FP32 travelling-wave field in host memory, "
                    f"mean removed, 99% energy, windows of {rows} rows ({nwin} windows, two "
                    f"passes), leaves of {b} rows",
        "s_per_call": round(t, 4), "host_gbps": round(host_bytes / t / 1e9, 2),
        "tflops": round((2.0 * m * n * n + 2.0 * m * n * h.nr) / t / 1e12, 4),
        "in_device_s_per_call": round(t_dev, 4), "n_r": h.nr, "status": rc,
        "sigma_equal_to_in_device": same, "device_workspace_gb": round(ws / 1e9, 2),
        "steps": steps,
    }


def timed_batch(api, count, seed, steps, warmup):
    """Uneven POD batch: `count` instances, m log-uniform in [5e4, 2e6], n
    uniform in [32, 512], FP32 known spectra s_i = 10^(-6i/n), 99 % energy.
    The mixed-precision batch (one graph-captured pylom_pod_batched call) is
    timed against `count` sequential FP64 pylom_pod calls on the promoted
    instances."""
    import numpy as np
    import torch
    from paper_2405_15529_amd import synth

    shapes = synth.uneven_batch(count=count, seed=seed)
    A32 = [synth.known_spectrum_device(m, n, synth.uneven_spectrum(n), seed=1000 + i,
                                       dtype=torch.float32) for i, (m, n) in enumerate(shapes)]
    torch.cuda.synchronize()
    flops = sum(2.0 * m * n * n for m, n in shapes)
    ctx = api.Context(0)
    batch = api.PodBatch(A32, remove_mean=False, r=0.01, precision="mixed", use_graph=True, ctx=ctx)
    for _ in range(max(1, warmup)):
        batch.run()   # the first call captures the graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.run()
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / steps
    rc_mixed, _ = ctx.status()
    res = batch.results()
    # sequential FP64 solves, one pylom_pod per instance on the promoted data
    ctx64 = api.Context(0)
    t_seq = 0.0
    worst_vs64 = 0.0
    worst_exact = 0.0
    nr_diff = 0
    for i, (m, n) in enumerate(shapes):
        A64 = A32[i].double()
        api.pod(A64, remove_mean=False, r=0.01, ctx=ctx64, sync=False)  # warm workspace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g64 = api.pod(A64, remove_mean=False, r=0.01, ctx=ctx64, sync=False)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        S64 = g64.S.cpu().numpy()
        Sx = res[i].S.cpu().numpy()
        s = synth.uneven_spectrum(n)
        k = res[i].nr
        if k:
            worst_vs64 = max(worst_vs64, float(np.max(np.abs(Sx[:k] - S64[:k]) / S64[:k])))
            worst_exact = max(worst_exact, float(np.max(np.abs(Sx[:k] - s[:k]) / s[:k])))
        del A64, g64
    rc64, _ = ctx64.status()
    out = {
        "workload": f"{count} POD instances, m log-uniform [5e4, 2e6], n uniform [32, 512], "
                    f"FP32 known spectra 10^(-6i/n), 99% energy",
        "total_rows": int(sum(m for m, _ in shapes)),
        "mixed_batched_graph_s": round(t_mixed, 4),
        "fp64_sequential_s": round(t_seq, 4),
        "speedup": round(t_seq / t_mixed, 3),
        "mixed_tflops": round(flops / t_mixed / 1e12, 4),
        "fp64_seq_tflops": round(flops / t_seq / 1e12, 4),
        "sigma_rel_err_vs_fp64_max": worst_vs64,
        "sigma_rel_err_vs_exact_max": worst_exact,
        "status_mixed": rc_mixed,
        "status_fp64": rc64,
        "streams": ctx.get_option("streams"),
    }
    ctx.close()
    ctx64.close()
    del A32, batch, res
    torch.cuda.empty_cache()
    return out


def timed_c2(api, args):
    """The known-spectrum FP64 workload, A = Q1 diag(s) Q2^T, m x n with
    s_i = 10^(-i/32), fixed row blocks, 99 % energy (no mean removal): FP64
    on the stacked QR, the library's automatic path beside it, and the mixed
    path on the FP32 copy of the same matrix."""
    import numpy as np
    import torch
    from paper_2405_15529_amd import synth

    m, n, r = args.m, args.n, 0.01
    dev = torch.device("cuda:0")
    A, s = synth.graded_fp64_device(m=m, n=n, seed=1, device="cuda")
    ctx = api.Context(0)
    ctx.set_option("block_rows", args.block_rows)
    ctx.set_option("blocked_from", args.blocked_from)
    ctx.set_option("timing", max(1, args.c2_steps))
    ctx.bind_stream()

    def orth_err(U, k):
        Ur = U[:, :k].double()
        return float(torch.linalg.norm(Ur.T @ Ur - torch.eye(k, dtype=torch.float64,
                                                               device=dev)).item())

    f = timed_pod(api, ctx, A, m, n, r, "fp64", args.c2_steps, args.c2_warmup,
                  kernel_timing=True)
    nr = f["nr"]
    S_h = f["S"].cpu().numpy()
    sig_rel = float(np.max(np.abs(S_h[:nr] - s[:nr]) / s[:nr])) if nr else 0.0
    sig_norm = float(np.max(np.abs(S_h - s)) / s[0])
    orth = orth_err(f["U"], nr)
    del f["U"]
    flops = 2.0 * m * n * n + 2.0 * m * n * nr
    bytes64 = 2.0 * 8 * m * n + 8.0 * m * nr
    ms = f["ms"]
    leaf_ms, leaf_n = f["kernels"]["stacked_leaf_qr"]
    leaf_tflops = 2.0 * m * n * n * leaf_n / (leaf_ms * 1e-3) / 1e12
    auto = None
    if not args.no_default_path:
        ctx_a = api.Context(0)
        ctx_a.set_option("timing", max(1, args.c2_steps))
        ctx_a.bind_stream()
        a = timed_pod(api, ctx_a, A, m, n, r, "fp64", args.c2_steps, args.c2_warmup)
        Sa = a["S"].cpu().numpy()
        nra = a["nr"]
        b_auto = api.tune_block_rows(m, n, ctx_a)
        ctx_a.set_option("blocked_from", 2)
        b_blk = api.tune_block_rows(m, n, ctx_a)
        ctx_a.set_option("blocked_from", 0)
        auto = {"path": "column-blocked TSQR" if b_auto == b_blk else "stacked TSQR",
                "block_rows": b_auto,
                "ms_per_step": round(a["ms"], 4),
                "tflops": round((2.0 * m * n * n + 2.0 * m * n * nra) / (a["ms"] * 1e-3) / 1e12, 4),
                "n_r": nra,
                "sigma_rel_err_retained": float(np.max(np.abs(Sa[:nra] - s[:nra]) / s[:nra])) if nra else 0.0,
                "orth_err_U": orth_err(a["U"], nra),
                "phase_ms": {k: round(v, 4) for k, v in a["phases"].items()}}
        ctx_a.close()
        del a
        torch.cuda.empty_cache()
    A32 = A.float().contiguous()
    del A
    mixed = None
    if not args.no_mixed:
        x = timed_pod(api, ctx, A32, m, n, r, "mixed", args.c2_steps, args.c2_warmup)
        mixed = mixed_summary(x, ms, flops, m, n, s, S_h, nr, orth_err)
        del x["U"]
    ctx.close()
    del A32
    torch.cuda.empty_cache()
    out = {
        "workload": f"known-spectrum POD FP64 {m}x{n}, s_i=10^(-i/32), row blocks "
                    f"{args.block_rows}, 99% energy, stacked TSQR",
        "m": m, "n": n, "block_rows": args.block_rows, "blocked_from": args.blocked_from,
        "ms_per_step": round(ms, 4), "tflops": round(flops / (ms * 1e-3) / 1e12, 4),
        "gbps": round(bytes64 / (ms * 1e-3) / 1e9, 2), "n_r": nr,
        "sigma_rel_err_retained": sig_rel, "sigma_err_normwise": sig_norm, "orth_err_U": orth,
        "jacobi_sweeps": f["sweeps"],
        "phase_ms": {k: round(v, 4) for k, v in f["phases"].items()},
        "kernels": kernel_summary(f["kernels"], args.c2_steps),
        "roofline_leaf_qr": {"bound": "mfma", "kernel": "k_stacked_qr (leaf QR, FP64)",
                             "achieved": round(leaf_tflops, 3), "peak": FP64_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(leaf_tflops / FP64_PEAK_TFLOPS, 4),
                             "traffic": measured_traffic("stacked_leaf_fp64",
                                                         (m, n, args.block_rows))},
        "mixed": mixed, "library_default": auto,
        "steps": args.c2_steps, "warmup": args.c2_warmup,
    }
    return out


def copy_probe():
    """One plain 1 GiB FP64 device copy, a kernel of known traffic for
    calibrating the HBM byte counters of rocprofv3 --pmc."""
    import torch
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2405_15529_amd import api

    if args.only_spod:
        res = []
        for b in (args.spod_block_rows or [0]):
            r = timed_spod(api, args.spod_m, args.spod_nt, 256, 128, args.spod_steps,
                           1 if args.warmup else 0, b)
            r["block_rows"] = b
            res.append(r)
            print(f"[bench] spod b={b}: {r['ms_per_step']} ms {r['phase_ms']}", file=sys.stderr,
                  flush=True)
        print(json.dumps({"spod": res}), flush=True)
        return
    if args.only_ooc:
        print(json.dumps({"out_of_core": timed_ooc(api, args.ooc_m, args.ooc_n, args.ooc_window,
                                                   2)}), flush=True)
        return
    if args.paper_shapes:
        print(json.dumps({"paper_shapes": timed_paper_shapes(api, 2, 1 if args.warmup else 0)}),
              flush=True)
        return
    m, n = args.wide_m, args.wide_n
    print(f"[bench] headline {m}x{n} mixed vs fp64: {args.steps} steps, {args.warmup} warm-up",
          file=sys.stderr, flush=True)
    c3 = timed_c3(api, m, n, args.steps, args.warmup, args.wide_block_rows,
                  fp64_steps=min(args.steps, args.fp64_steps))
    x, f = c3["mixed"], c3["fp64"]
    tu = c3["trailing_update"]
    out = {
        "metric": "POD TSQR-SVD GB/s & TFLOP/s: mixed-precision vs FP64 at sigma rel err <=1e-6",
        "value": x["tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": x["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"travelling-wave POD {m}x{n} FP32 snapshots (64 waves + noise), "
                               f"mean removed, 99% energy: mixed precision (FP32 leaf QR, FP64 "
                               f"tree and SVD, Rayleigh-Ritz refinement) vs FP64 on the same "
                               f"buffer", "m": m, "n": n, "block_rows": c3["block_rows"],
                   "path": "column-blocked TSQR", "precision": "mixed vs fp64"},
        "gbps": x["gbps"],
        "fp64": {"ms_per_step": f["ms_per_step"], "tflops": f["tflops"], "gbps": f["gbps"],
                 "steps": f["steps"]},
        "speedup_mixed_vs_fp64": c3["speedup_mixed_vs_fp64"],
        "sigma_rel_err_mixed_vs_fp64_run": c3["sigma_rel_err_mixed_vs_fp64_run"],
        "n_r": {"mixed": x["n_r"], "fp64": f["n_r"]},
        "orth_err_U": {"mixed": x["orth_err_U"], "fp64": f["orth_err_U"]},
        "roofline": {"bound": "mfma",
                     "kernel": "k_panel_apply<float> (leaf trailing updates of the FP32 "
                               "column-blocked QR, the 2 m n^2 term)",
                     "achieved": tu["fp32_tflops"], "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": tu["fp32_frac"],
                     "traffic": measured_traffic("blocked_trailing_fp32", (m, n, c3["block_rows"])),
                     "share_of_step": round(x["kernels"]["leaf_trailing_update"]["ms_per_call"] /
                                            x["ms_per_step"], 4)},
        "c3": c3,
    }
    print(f"[bench] headline: mixed {x['ms_per_step']} ms, fp64 {f['ms_per_step']} ms",
          file=sys.stderr, flush=True)
    if args.copy_probe:
        copy_probe()
    if args.dmd_wide:
        out["dmd_wide"] = timed_dmd_wide(api, m, n, 1, 1 if args.warmup else 0)
    if not args.no_c2:
        out["c2"] = timed_c2(api, args)
        print(f"[bench] c2: {out['c2']['ms_per_step']} ms", file=sys.stderr, flush=True)
    if not args.no_spod:
        out["spod"] = timed_spod(api, args.spod_m, args.spod_nt, 256, 128, args.spod_steps,
                                 1 if args.warmup else 0)
        print(f"[bench] spod: {out['spod']['ms_per_step']} ms", file=sys.stderr, flush=True)
    if not args.no_dmd:
        out["dmd"] = timed_dmd(api, args.dmd_m, args.dmd_n, 2, 1 if args.warmup else 0)
        print(f"[bench] dmd: {out['dmd']['ms_per_step']} ms", file=sys.stderr, flush=True)
    if not args.no_ooc:
        out["out_of_core"] = timed_ooc(api, args.ooc_m, args.ooc_n, args.ooc_window, 2)
        print(f"[bench] out-of-core: {out['out_of_core']['s_per_call']} s", file=sys.stderr,
              flush=True)
    if not args.no_batch:
        out["uneven_batch"] = timed_batch(api, args.batch_count, 4, args.batch_steps,
                                          1 if args.warmup else 0)
        print(f"[bench] batch: {out['uneven_batch']['mixed_batched_graph_s']} s", file=sys.stderr,
              flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_c3(m, n, args.cpu_rows)
    print(json.dumps(out), flush=True)


def mixed_summary(x, ms, flops, m, n, s, S_h, nr, orth_err):
    import numpy as np
    nrx = x["nr"]
    Sx = x["S"].cpu().numpy()
    kx = min(nrx, nr)
    return {
        "precision": "mixed (FP32 leaf QR, FP64 tree + SVD, FP64 Rayleigh-Ritz refinement)",
        "storage": "f32",
        "ms_per_step": round(x["ms"], 4),
        "tflops": round(flops / (x["ms"] * 1e-3) / 1e12, 4),
        "gbps": round((2.0 * 4 * m * n + 4.0 * m * nrx) / (x["ms"] * 1e-3) / 1e9, 2),
        "speedup_vs_fp64": round(ms / x["ms"], 3),
        "n_r": nrx,
        "sigma_rel_err_vs_fp64_run": float(np.max(np.abs(Sx[:kx] - S_h[:kx]) / S_h[:kx])) if kx else 0.0,
        "sigma_rel_err_vs_exact": float(np.max(np.abs(Sx[:kx] - s[:kx]) / s[:kx])) if kx else 0.0,
        "orth_err_U": orth_err(x["U"], nrx),
        "jacobi_sweeps_first": x["sweeps"],
        "phase_ms": {"leaf_qr_fp32": round(x["phases"]["leaf_qr"], 4),
                     "tree_combine": round(x["phases"]["tree_combine"], 4),
                     "small_svd": round(x["phases"]["small_svd"], 4),
                     "refine_project_gram_eig": round(x["phases"]["tree_propagate"], 4),
                     "form_u": round(x["phases"]["leaf_apply"], 4)},
    }


if __name__ == "__main__":
    main()
