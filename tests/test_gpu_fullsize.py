"""GPU checks at the full sizes of the benchmarked workloads, in the launch
configurations bench.py times.  The oracle cannot finish these shapes, so
each test checks what holds at any size, or outputs it can recompute one by
one on sampled rows:

* 1,048,576 x 256 FP64 known spectrum, row blocks 4096: sigma against the
  exact spectrum, orthogonality, and sampled rows of U against
  (A v_j) / sigma_j;
* 4,194,304 x 1,808 FP32 travelling waves (column-blocked path): the mixed
  path against the FP64 path on the same buffer, N_r, orthogonality, the
  mean on sampled rows against an FP64 row mean, and sampled rows of U
  against ((D - mu 1^T) v_j) / sigma_j;
* SPOD of 262,144 points x 2,048 snapshots (npwin 256, nolap 128, Hann,
  complex64): the energies against the eigenvalues of Q_f^H Q_f, with the
  spectra Q_f formed independently by torch's FFT, and the modes of sampled
  frequencies against the span of Q_f;
* the 64-instance uneven batch (mixed precision, one graph-captured call):
  every instance against its FP64 solve.

Bars: FP64 1e-12 (sigma) as for the oracle parity; mixed 1e-6 (sigma and
|U^T U - I|_F); complex64 SPOD the FP32 FFT bound 64 log2(npwin) u32 S_1(f).
"""
import math
import sys

import numpy as np
import pytest

from paper_2405_15529_amd import synth
from tests import checks

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def orth_err_dev(U):
    import torch
    Ud = U.double()
    return float(torch.linalg.norm(Ud.T @ Ud - torch.eye(Ud.shape[1], dtype=torch.float64,
                                                           device=U.device)).item())


def test_known_spectrum_1048576x256_fp64():
    import torch
    from paper_2405_15529_amd import api
    m, n = 1_048_576, 256
    say(f"[gpu] full size FP64 {m}x{n} b=4096")
    A, s = synth.graded_fp64_device(m=m, n=n, seed=1)
    ctx = api.Context(0)
    ctx.set_option("block_rows", 4096)
    ctx.set_option("blocked_from", 1025)  # the stacked QR, as bench.py times it
    out = api.pod(A, remove_mean=False, r=0.01, ctx=ctx)
    rc, sweeps = ctx.status()
    nr = out.nr
    S = out.S.cpu().numpy()
    say(f"    rc {rc} sweeps {sweeps} N_r {nr}")
    assert rc == 0 and nr in (32, 33)
    rel = float(np.max(np.abs(S[:nr] - s[:nr]) / s[:nr]))
    nw = float(np.max(np.abs(S - s)) / s[0])
    oe = orth_err_dev(out.U)
    say(f"    sigma rel {rel:.2e} normwise {nw:.2e} |U^T U - I|_F {oe:.2e}")
    assert rel <= 1e-12 and nw <= 1e-12 and oe <= 1e-12
    # sampled rows: u_ij = (A_i . v_j) / sigma_j
    rows = torch.from_numpy(np.random.default_rng(7).choice(m, 256, replace=False)).cuda()
    ref = (A[rows] @ out.VT[:nr].T.contiguous()) / out.S[:nr]
    err = torch.abs(out.U[rows] - ref) * (out.S[:nr] / out.S[0])
    say(f"    sampled rows: max |u - A v / sigma| sigma / sigma_1 {err.max().item():.2e}")
    assert err.max().item() <= 1e-12
    ctx.close()


def test_travelling_waves_4194304x1808_mixed_vs_fp64():
    import torch
    from paper_2405_15529_amd import api
    m, n = 4_194_304, 1808
    say(f"[gpu] full size wide {m}x{n}: mixed and FP64 on the same FP32 buffer")
    D = synth.travelling_waves_device(m, n, seed=2)
    ctx = api.Context(0)
    x = api.pod(D, remove_mean=True, r=0.01, precision="mixed", ctx=ctx)
    rcx, swx = ctx.status()
    Sx = x.S.cpu().numpy()
    nrx = x.nr
    oex = orth_err_dev(x.U)
    rows = torch.from_numpy(np.random.default_rng(3).choice(m, 256, replace=False)).cuda()
    Drow = D[rows].double()
    mu_ref = Drow.mean(dim=1)
    mu_x = x.mean[rows].double()
    refx = ((Drow - mu_ref[:, None]) @ x.VT[:nrx].T.contiguous()) / x.S[:nrx]
    errx = float((torch.abs(x.U[rows].double() - refx).max(dim=0).values /
                  torch.abs(refx).max(dim=0).values).max().item())
    del x
    torch.cuda.empty_cache()
    f = api.pod(D, remove_mean=True, r=0.01, precision="fp64", ctx=ctx)
    rcf, swf = ctx.status()
    Sf = f.S.cpu().numpy()
    nrf = f.nr
    oef = orth_err_dev(f.U)
    mu_f = f.mean[rows].double()
    reff = ((Drow - mu_ref[:, None]) @ f.VT[:nrf].T.contiguous()) / f.S[:nrf]
    errf = float((torch.abs(f.U[rows].double() - reff).max(dim=0).values /
                  torch.abs(reff).max(dim=0).values).max().item())
    say(f"    rc {rcx}/{rcf} sweeps {swx}/{swf} N_r {nrx}/{nrf}")
    assert rcx == 0 and rcf == 0
    assert checks.nr_agrees(nrx, nrf, Sf, 0.01, tie=1e-5), (nrx, nrf)
    k = min(nrx, nrf)
    assert k > 0
    rel = float(np.max(np.abs(Sx[:k] - Sf[:k]) / Sf[:k]))
    say(f"    sigma rel mixed vs FP64 {rel:.2e}; |U^T U - I|_F mixed {oex:.2e} FP64 {oef:.2e}")
    assert rel <= 1e-6 and oex <= 1e-6 and oef <= 1e-6
    # the mean is accumulated in FP64 and stored in FP32 (one rounding)
    emu = max(float((torch.abs(mu_x - mu_ref) / torch.abs(mu_ref).clamp_min(1e-30)).max()),
              float((torch.abs(mu_f - mu_ref) / torch.abs(mu_ref).clamp_min(1e-30)).max()))
    say(f"    sampled mean rel err {emu:.2e}; sampled U rows rel err mixed {errx:.2e} "
        f"FP64 {errf:.2e}")
    assert emu <= 2.0 ** -23
    assert errx <= 1e-5 and errf <= 1e-5
    ctx.close()


def spectra_gram(D, npwin, nolap, keep):
    """Q_f^H Q_f for every frequency and Q_f for the frequencies in `keep`,
    from torch's FFT in FP64: mean over all snapshots removed, Hann window
    over npwin samples with the (npwin - 1) denominator, q = DFT(w x) / sum w,
    bins 1..npwin/2-1 doubled, all scaled by 1 / sqrt(nBlks)."""
    import torch
    m, nt = D.shape
    dev = D.device
    nb = (nt - nolap) // (npwin - nolap)
    nf = npwin // 2 + 1
    j = torch.arange(npwin, dtype=torch.float64, device=dev)
    w = 0.5 - 0.5 * torch.cos(2.0 * math.pi * j / (npwin - 1))
    scale = torch.full((nf,), 2.0, dtype=torch.float64, device=dev)
    scale[0] = 1.0
    scale[-1] = 1.0
    scale = scale / w.sum() / math.sqrt(nb)
    G = torch.zeros((nf, nb, nb), dtype=torch.complex128, device=dev)
    Q = {f: torch.empty((m, nb), dtype=torch.complex128, device=dev) for f in keep}
    step = npwin - nolap
    for p0 in range(0, m, 16384):
        p1 = min(m, p0 + 16384)
        X = D[p0:p1].double()
        X = X - X.mean(dim=1, keepdim=True)
        blocks = torch.stack([X[:, i * step:i * step + npwin] for i in range(nb)], dim=1)
        F = torch.fft.rfft(blocks * w, dim=2) * scale           # rows x nb x nf
        Ff = F.permute(2, 0, 1).contiguous()                    # nf x rows x nb
        Fh = Ff.conj().transpose(1, 2).contiguous()
        G += torch.bmm(Fh, Ff)
        for f in keep:
            Q[f][p0:p1] = Ff[f]
    return G, Q


def test_spod_262144x2048_c64():
    import torch
    from paper_2405_15529_amd import api
    m, nt, npwin, nolap = 262144, 2048, 256, 128
    say(f"[gpu] full size SPOD {m}x{nt} npwin {npwin} nolap {nolap} c64")
    D = torch.from_numpy(synth.spod_field(m, nt, seed=3, nmodes=32)).cuda()
    ctx = api.Context(0)
    out = api.spod(D, npwin=npwin, nolap=nolap, spectra="c64", ctx=ctx)
    rc, sweeps = ctx.status()
    assert rc == 0
    L = out.L.cpu().numpy()
    nf, nb = L.shape
    order = out.order.cpu().numpy()
    keep = sorted({int(order[0]), int(order[1]), 64, nf - 1})
    G, Q = spectra_gram(D, npwin, nolap, keep)
    Lref = np.sort(np.linalg.eigvalsh(G.cpu().numpy()), axis=1)[:, ::-1]
    S = np.sqrt(np.maximum(L, 0.0))
    Sref = np.sqrt(np.maximum(Lref, 0.0))
    bound = 64 * math.log2(npwin) * U32
    err = float(np.max(np.abs(S - Sref) / Sref[:, :1]))
    say(f"    energies: max |S - S_ref| / S_1(f) {err:.2e} (bar {bound:.2e}); sweeps {sweeps}")
    assert err <= bound
    for f in keep:
        U = out.modes[f].to(torch.complex128)
        eye = torch.eye(nb, dtype=torch.complex128, device=U.device)
        oe = torch.linalg.norm(U.conj().T.contiguous() @ U - eye).item()
        Qf = Q[f]
        res = torch.linalg.norm(Qf - U @ (U.conj().T.contiguous() @ Qf)).item()
        rel = res / torch.linalg.norm(Qf).item()
        say(f"    f index {f}: |U^H U - I|_F {oe:.2e}, |Q - U U^H Q| / |Q| {rel:.2e}")
        assert oe <= 1e-5 and rel <= 1e-5
    ctx.close()


def test_uneven_batch_64_mixed_graph_vs_fp64():
    import torch
    from paper_2405_15529_amd import api
    shapes = synth.uneven_batch(count=64, seed=4)
    say(f"[gpu] full size uneven batch: {len(shapes)} instances, "
        f"{sum(mm for mm, _ in shapes)} rows in all")
    A32 = [synth.known_spectrum_device(mm, nn, synth.uneven_spectrum(nn), seed=1000 + i,
                                       dtype=torch.float32) for i, (mm, nn) in enumerate(shapes)]
    ctx = api.Context(0)
    batch = api.PodBatch(A32, remove_mean=False, r=0.01, precision="mixed", use_graph=True,
                         ctx=ctx)
    batch.run()
    rc, _ = ctx.status()
    assert rc == 0
    res = batch.results()
    ctx64 = api.Context(0)
    worst, worst_orth = 0.0, 0.0
    for i, (mm, nn) in enumerate(shapes):
        g64 = api.pod(A32[i].double(), remove_mean=False, r=0.01, ctx=ctx64)
        rc64, _ = ctx64.status()
        assert rc64 == 0
        S64 = g64.S.cpu().numpy()
        Sx = res[i].S.cpu().numpy()
        assert checks.nr_agrees(res[i].nr, g64.nr, S64, 0.01, tie=1e-5), (i, res[i].nr, g64.nr)
        k = min(res[i].nr, g64.nr)
        if k:
            worst = max(worst, float(np.max(np.abs(Sx[:k] - S64[:k]) / S64[:k])))
            worst_orth = max(worst_orth, orth_err_dev(res[i].U))
        del g64
    say(f"    worst sigma rel vs FP64 {worst:.2e}, worst |U^T U - I|_F {worst_orth:.2e}")
    assert worst <= 1e-6 and worst_orth <= 1e-6
    ctx.close()
    ctx64.close()
