"""Python binding of the gfx950 POD / TSQR-SVD library (argument marshalling).

Every function here takes PyTorch tensors that already live on the GPU, hands
their device pointers and the current HIP stream to the C-ABI of
``include/pylom.h``, and returns tensors allocated with PyTorch.  All
arithmetic happens in the library's HIP kernels; nothing is computed here.

Paper: pyLOM, arXiv 2405.15529 -- Alg. 1 (TSQR), Alg. 2 (POD),
Alg. 4 (matmul), Eqs. svdqr1-svdqr3.
"""
from __future__ import annotations

import atexit
import ctypes
import sys
import weakref
from dataclasses import dataclass

import torch

from . import _lib

R32, R64, C64, C128 = 1, 2, 3, 4
FP64, MIXED = 0, 1
_PREC = {"fp64": FP64, "mixed": MIXED}

OK, WNOCONV, WNONFINITE = 0, 1, 2


class PylomError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pylom status {status}: {msg}")
        self.status = status


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return R64
    if t.dtype == torch.float32:
        return R32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _rowmajor(t: torch.Tensor, name: str):
    if t.dim() != 2 or t.stride(1) != 1 or t.stride(0) < t.shape[1]:
        raise ValueError(f"{name} must be a 2-D row-major tensor (stride(1) == 1)")


def _on_gpu(t: torch.Tensor, name: str):
    # a host pointer handed to the kernels would be a GPU page fault
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")


# Every open context, so that all are closed by an exit hook while the HIP
# runtime (and any profiler attached to it) is still alive: a context left to
# the garbage collector at interpreter shutdown would destroy its graphs,
# streams and workspace after the runtime has been torn down.
_live = weakref.WeakSet()


def close_all():
    """Close every open context (registered as an exit hook)."""
    for c in list(_live):
        c.close()


atexit.register(close_all)


class Context:
    """A library context (device workspace + options).  device=-1 creates a
    host-only context: it validates arguments and plans, but runs nothing."""

    def __init__(self, device: int = 0):
        self.lib = _lib.load()
        h = ctypes.c_void_p()
        rc = self.lib.pylom_create(ctypes.byref(h), int(device))
        if rc != 0:
            raise PylomError(rc, self.lib.pylom_strerror(rc).decode())
        self.h = h
        self.device = device
        _live.add(self)

    def close(self):
        if getattr(self, "h", None):
            self.lib.pylom_destroy(self.h)
            self.h = None
        dev = getattr(self, "device", None)
        if _contexts.get(dev) is self:
            del _contexts[dev]

    def __del__(self, _finalizing=sys.is_finalizing):  # pragma: no cover - shutdown order
        # at shutdown the exit hook has already closed every context; never
        # call into the runtime from a finalising interpreter (whose module
        # globals may already be gone, hence the bound default)
        if _finalizing() or not getattr(self, "h", None):
            return
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc: int):
        if rc < 0:
            raise PylomError(rc, self.lib.pylom_last_error(self.h).decode())
        return rc

    def set_option(self, key: str, value: int):
        self.check(self.lib.pylom_set_option(self.h, key.encode(), int(value)))

    def get_option(self, key: str) -> int:
        v = ctypes.c_int64()
        self.check(self.lib.pylom_get_option(self.h, key.encode(), ctypes.byref(v)))
        return v.value

    def bind_stream(self):
        s = torch.cuda.current_stream().cuda_stream
        self.check(self.lib.pylom_set_stream(self.h, ctypes.c_void_p(s)))

    def plan(self, m: int, n: int):
        out = [ctypes.c_int64() for _ in range(4)]
        self.check(self.lib.pylom_plan_query(self.h, m, n, *[ctypes.byref(o) for o in out]))
        return dict(leaves=out[0].value, block_rows=out[1].value, chunk_rows=out[2].value,
                    levels=out[3].value)

    def workspace_bytes(self, m: int, n: int, dtype=R64, precision="fp64") -> int:
        b = ctypes.c_size_t()
        self.check(self.lib.pylom_workspace_query(self.h, dtype, _PREC[precision], m, n, ctypes.byref(b)))
        return b.value

    PHASES = ("leaf_qr", "tree_combine", "small_svd", "tree_propagate", "leaf_apply",
              "front_end")

    def phase_times(self) -> dict:
        """Mean per-phase milliseconds of the timed calls since the last read."""
        buf = (ctypes.c_double * 6)()
        rc = self.lib.pylom_phase_times(self.h, buf, 6)
        if rc < 0:
            raise PylomError(rc, self.lib.pylom_last_error(self.h).decode())
        return {k: buf[i] for i, k in enumerate(self.PHASES)}

    def autotune(self, D: torch.Tensor, precision: str = "fp64", remove_mean: bool = True,
                 reps: int = 2):
        """Time every candidate leaf height of pylom_pod on D and record the
        fastest for this shape class (pylom_autotune); returns (rows, ms)."""
        _rowmajor(D, "D")
        _on_gpu(D, "D")
        m, n = D.shape
        b, t = ctypes.c_int64(), ctypes.c_double()
        self.bind_stream()
        self.check(self.lib.pylom_autotune(self.h, _dtype_code(D), _PREC[precision], m, n,
                                           _ptr(D), D.stride(0), int(bool(remove_mean)), int(reps),
                                           ctypes.byref(b), ctypes.byref(t)))
        return b.value, t.value

    def tune_save(self, path: str):
        self.check(self.lib.pylom_tune_save(self.h, str(path).encode()))

    def tune_load(self, path: str) -> int:
        return self.check(self.lib.pylom_tune_load(self.h, str(path).encode()))

    KERNEL_ROLES = ("working_copy", "leaf_panel_qr", "leaf_trailing_update", "tree_panel_qr",
                    "tree_trailing_update", "small_svd", "tree_propagate", "leaf_apply",
                    "refine", "refine_form_u", "stacked_leaf_qr", "stacked_tree")

    def kernel_times(self) -> dict:
        """Summed milliseconds and launch counts per kernel role since the
        last read (needs the kernel_timing option)."""
        n = len(self.KERNEL_ROLES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        rc = self.lib.pylom_kernel_times(self.h, ms, cnt, n)
        if rc < 0:
            raise PylomError(rc, self.lib.pylom_last_error(self.h).decode())
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.KERNEL_ROLES)}

    def status(self):
        """Synchronise the stream; return (status, sweeps) of the last SVD."""
        sw = ctypes.c_int64()
        rc = self.lib.pylom_check(self.h, ctypes.byref(sw))
        if rc < 0:
            raise PylomError(rc, self.lib.pylom_last_error(self.h).decode())
        return rc, sw.value


_contexts: dict[int, Context] = {}


def context(device: int | None = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    if device not in _contexts:
        _contexts[device] = Context(device)
    return _contexts[device]


@dataclass
class PodResult:
    U: torch.Tensor      # m x N_r spatial modes
    S: torch.Tensor      # n singular values (descending, FP64)
    VT: torch.Tensor     # N_r x n temporal coefficients (FP64)
    mean: torch.Tensor | None
    nr: int
    U_full: torch.Tensor
    VT_full: torch.Tensor


def pod(D: torch.Tensor, remove_mean: bool = True, r: float = 0.01, precision: str = "fp64",
        ctx: Context | None = None, sync: bool = True) -> PodResult:
    """POD of the snapshot matrix D (m x n, rows = points): Alg. 2 + Alg. 1."""
    _rowmajor(D, "D")
    _on_gpu(D, "D")
    ctx = ctx or context(D.device.index)
    m, n = D.shape
    dev = D.device
    U = torch.empty((m, n), dtype=D.dtype, device=dev)
    S = torch.empty(n, dtype=torch.float64, device=dev)
    VT = torch.empty((n, n), dtype=torch.float64, device=dev)
    mean = torch.empty(m, dtype=D.dtype, device=dev) if remove_mean else None
    nr = torch.empty(1, dtype=torch.int64, device=dev)
    ctx.bind_stream()
    rc = ctx.lib.pylom_pod(ctx.h, _dtype_code(D), _PREC[precision], m, n, _ptr(D), D.stride(0),
                           int(bool(remove_mean)), float(r), _ptr(mean), _ptr(U), n, _ptr(S),
                           _ptr(VT), n, _ptr(nr))
    ctx.check(rc)
    k = int(nr.item()) if sync else n
    return PodResult(U=U[:, :k], S=S, VT=VT[:k], mean=mean, nr=k, U_full=U, VT_full=VT)


def ooc_query(m: int, n: int, dtype=R64, ctx: Context | None = None):
    """(device workspace bytes, rows per window, windows) of a pod_host call."""
    ctx = ctx or Context(-1)
    b, wr, nw = ctypes.c_size_t(), ctypes.c_int64(), ctypes.c_int64()
    ctx.check(ctx.lib.pylom_ooc_workspace_query(ctx.h, dtype, m, n, ctypes.byref(b),
                                                ctypes.byref(wr), ctypes.byref(nw)))
    return b.value, wr.value, nw.value


@dataclass
class HostPodResult:
    U: "object"          # m x N_r spatial modes (numpy, storage type)
    S: "object"          # n singular values (numpy FP64)
    VT: "object"         # N_r x n temporal coefficients (numpy FP64)
    mean: "object"       # m row means (numpy, storage type) or None
    nr: int


def pod_host(D, remove_mean: bool = True, r: float = 0.01, ctx: Context | None = None,
             U=None) -> HostPodResult:
    """Out-of-core POD of a snapshot matrix in host memory (a C-contiguous
    numpy array, float64 or float32, m x n): pylom_pod_host streams its rows
    through the device.  U (m x n capacity, same dtype) may be given."""
    import numpy as np
    if not isinstance(D, np.ndarray) or D.ndim != 2 or not D.flags["C_CONTIGUOUS"]:
        raise ValueError("D must be a C-contiguous 2-D numpy array")
    if D.dtype not in (np.float64, np.float32):
        raise TypeError("D must be float64 or float32")
    m, n = D.shape
    ctx = ctx or context(0)
    code = R64 if D.dtype == np.float64 else R32
    if U is None:
        U = np.empty((m, n), dtype=D.dtype)
    if U.shape != (m, n) or U.dtype != D.dtype or not U.flags["C_CONTIGUOUS"]:
        raise ValueError("U must be a C-contiguous m x n array of D's dtype")
    S = np.empty(n)
    VT = np.empty((n, n))
    mean = np.empty(m, dtype=D.dtype) if remove_mean else None
    nr = ctypes.c_int64(0)
    vp = ctypes.c_void_p
    rc = ctx.lib.pylom_pod_host(ctx.h, code, FP64, m, n, vp(D.ctypes.data), n,
                                int(bool(remove_mean)), float(r),
                                vp(mean.ctypes.data if mean is not None else 0),
                                vp(U.ctypes.data), n, vp(S.ctypes.data), vp(VT.ctypes.data), n,
                                ctypes.byref(nr))
    ctx.check(rc)
    k = nr.value
    return HostPodResult(U=U[:, :k], S=S, VT=VT[:k], mean=mean, nr=k)


def tsvd(A: torch.Tensor, r: float = 0.01, precision: str = "fp64", ctx: Context | None = None,
         sync: bool = True) -> PodResult:
    """Tall-skinny SVD without mean removal."""
    _rowmajor(A, "A")
    _on_gpu(A, "A")
    ctx = ctx or context(A.device.index)
    m, n = A.shape
    dev = A.device
    U = torch.empty((m, n), dtype=A.dtype, device=dev)
    S = torch.empty(n, dtype=torch.float64, device=dev)
    VT = torch.empty((n, n), dtype=torch.float64, device=dev)
    nr = torch.empty(1, dtype=torch.int64, device=dev)
    ctx.bind_stream()
    rc = ctx.lib.pylom_tsvd(ctx.h, _dtype_code(A), _PREC[precision], m, n, _ptr(A), A.stride(0),
                            float(r), _ptr(U), n, _ptr(S), _ptr(VT), n, _ptr(nr))
    ctx.check(rc)
    k = int(nr.item()) if sync else n
    return PodResult(U=U[:, :k], S=S, VT=VT[:k], mean=None, nr=k, U_full=U, VT_full=VT)


def tsqr(A: torch.Tensor, want_q: bool = True, ctx: Context | None = None):
    """TSQR (Alg. 1): returns (Q or None, R) with diag(R) >= 0."""
    _rowmajor(A, "A")
    _on_gpu(A, "A")
    ctx = ctx or context(A.device.index)
    m, n = A.shape
    Q = torch.empty((m, n), dtype=A.dtype, device=A.device) if want_q else None
    R = torch.empty((n, n), dtype=torch.float64, device=A.device)
    ctx.bind_stream()
    rc = ctx.lib.pylom_tsqr(ctx.h, _dtype_code(A), FP64, m, n, _ptr(A), A.stride(0), _ptr(Q), n,
                            _ptr(R), n)
    ctx.check(rc)
    return Q, R


def matmul(A: torch.Tensor, B: torch.Tensor, trans_a: bool, ctx: Context | None = None):
    """Alg. 4 on one GPU: A^T B (trans_a) or A B."""
    _rowmajor(A, "A")
    _rowmajor(B, "B")
    _on_gpu(A, "A")
    _on_gpu(B, "B")
    if A.dtype != B.dtype:
        raise TypeError("A and B must have the same dtype")
    ctx = ctx or context(A.device.index)
    if trans_a:
        m, p = A.shape
        if B.shape[0] != m:
            raise ValueError("row counts differ")
        q = B.shape[1]
        C = torch.empty((p, q), dtype=A.dtype, device=A.device)
    else:
        m, p = A.shape
        if B.shape[0] != p:
            raise ValueError("inner dimensions differ")
        q = B.shape[1]
        C = torch.empty((m, q), dtype=A.dtype, device=A.device)
    ctx.bind_stream()
    rc = ctx.lib.pylom_matmul(ctx.h, _dtype_code(A), FP64, int(bool(trans_a)), m, p, q, _ptr(A),
                              A.stride(0), _ptr(B), B.stride(0), _ptr(C), C.stride(0))
    ctx.check(rc)
    return C


def matmul_noalloc(A: torch.Tensor, B: torch.Tensor, trans_a: bool, C: torch.Tensor,
                   ctx: Context | None = None):
    """Alg. 4 into the caller's C without any device allocation by the library
    (pylom_matmul_noalloc); C is (p x q) for trans_a, else (m x q)."""
    for t, nm in ((A, "A"), (B, "B"), (C, "C")):
        _rowmajor(t, nm)
        _on_gpu(t, nm)
    if A.dtype != B.dtype or C.dtype != A.dtype:
        raise TypeError("A, B and C must have the same dtype")
    ctx = ctx or context(A.device.index)
    m, p = A.shape
    q = B.shape[1]
    want = (p, q) if trans_a else (m, q)
    if (B.shape[0] != (m if trans_a else p)) or tuple(C.shape) != want:
        raise ValueError("shapes do not match")
    ctx.bind_stream()
    rc = ctx.lib.pylom_matmul_noalloc(ctx.h, _dtype_code(A), FP64, int(bool(trans_a)), m, p, q,
                                      _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(C),
                                      C.stride(0))
    ctx.check(rc)
    return C


def tree_plan(P: int):
    """The in-device reduction tree for P leaves: list of (level, receiver, sender)."""
    lib = _lib.load()
    cnt = lib.pylom_tree_plan(P, None, 0)
    if cnt < 0:
        raise PylomError(int(cnt), "tree_plan")
    buf = (ctypes.c_int64 * max(1, 3 * cnt))()
    lib.pylom_tree_plan(P, buf, cnt)
    return [(buf[3 * i], buf[3 * i + 1], buf[3 * i + 2]) for i in range(cnt)]


WINDOWS = {"hann": 0, "hamming": 1}


@dataclass
class SpodResult:
    modes: torch.Tensor   # nfreq x m x nblk complex spatial modes (phase-fixed)
    L: torch.Tensor       # nfreq x nblk energies (S^2), descending per frequency
    f: torch.Tensor       # nfreq frequencies f / (dt npwin)
    order: torch.Tensor   # nfreq frequency indices by leading energy


def spod_query(m: int, nt: int, npwin: int, nolap: int, spectra: str = "c64",
               ctx: Context | None = None):
    """(nblocks, nfreq, workspace bytes) of a pylom_spod call of this shape."""
    ctx = ctx or Context(-1)
    nb, nf, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
    code = C64 if spectra == "c64" else C128
    ctx.check(ctx.lib.pylom_spod_query(ctx.h, code, m, nt, npwin, nolap, ctypes.byref(nb),
                                       ctypes.byref(nf), ctypes.byref(b)))
    return nb.value, nf.value, b.value


def spod(D: torch.Tensor, dt: float = 1.0, npwin: int = 256, nolap: int = 128,
         window: str = "hann", remove_mean: bool = True, spectra: str = "c64",
         ctx: Context | None = None) -> SpodResult:
    """SPOD of the FP32 snapshot matrix D (m x nt, rows = points): Alg. 6 with
    the SVD of every frequency's spectral matrix, all frequencies in one batch."""
    _rowmajor(D, "D")
    if D.dtype != torch.float32 or not D.is_cuda:
        raise ValueError("D must be a float32 GPU tensor")
    ctx = ctx or context(D.device.index)
    m, nt = D.shape
    nb, nf, _ = spod_query(m, nt, npwin, nolap, spectra, ctx)
    cdt = torch.complex64 if spectra == "c64" else torch.complex128
    dev = D.device
    modes = torch.empty((nf, m, nb), dtype=cdt, device=dev)
    L = torch.empty((nf, nb), dtype=torch.float64, device=dev)
    f = torch.empty(nf, dtype=torch.float64, device=dev)
    order = torch.empty(nf, dtype=torch.int64, device=dev)
    ctx.bind_stream()
    code = C64 if spectra == "c64" else C128
    rc = ctx.lib.pylom_spod(ctx.h, code, FP64, m, nt, _ptr(D), D.stride(0), float(dt), npwin,
                            nolap, WINDOWS[window], int(bool(remove_mean)), _ptr(modes), _ptr(L),
                            _ptr(f), _ptr(order))
    ctx.check(rc)
    return SpodResult(modes=modes, L=L, f=f, order=order)


DMD_MAX_MODES = 128


@dataclass
class DmdResult:
    phi: torch.Tensor     # m x N_r complex128 exact DMD modes, ordered by |b|
    mu: torch.Tensor      # N_r complex128 eigenvalues of the linear map
    b: torch.Tensor       # N_r complex128 amplitudes (Alg. 5)
    freq: torch.Tensor    # N_r frequencies arg(mu) / (2 pi dt)
    growth: torch.Tensor  # N_r growth rates log|mu| / dt
    nr: int


def dmd_workspace_bytes(m: int, n: int, dtype=R64, remove_mean: bool = False,
                        ctx: Context | None = None) -> int:
    ctx = ctx or Context(-1)
    b = ctypes.c_size_t()
    ctx.check(ctx.lib.pylom_dmd_workspace_query(ctx.h, dtype, m, n, int(bool(remove_mean)),
                                                ctypes.byref(b)))
    return b.value


def dmd(D: torch.Tensor, remove_mean: bool = False, r: float = 0.01, dt: float = 1.0,
        ctx: Context | None = None) -> DmdResult:
    """Exact DMD of the snapshot matrix D (m x N, rows = points): Alg. 3 with
    the TS-SVD of Alg. 1 and the amplitudes of Alg. 5."""
    _rowmajor(D, "D")
    if not D.is_cuda:
        raise ValueError("D must be a GPU tensor")
    ctx = ctx or context(D.device.index)
    m, n = D.shape
    kc = max(1, min(n - 1, DMD_MAX_MODES))
    dev = D.device
    phi = torch.empty((m, kc), dtype=torch.complex128, device=dev)
    mu = torch.empty(kc, dtype=torch.complex128, device=dev)
    b = torch.empty(kc, dtype=torch.complex128, device=dev)
    freq = torch.empty(kc, dtype=torch.float64, device=dev)
    growth = torch.empty(kc, dtype=torch.float64, device=dev)
    nr = torch.zeros(1, dtype=torch.int64, device=dev)
    ctx.bind_stream()
    rc = ctx.lib.pylom_dmd(ctx.h, _dtype_code(D), m, n, _ptr(D), D.stride(0),
                           int(bool(remove_mean)), float(r), float(dt), _ptr(phi), kc, _ptr(mu),
                           _ptr(b), _ptr(freq), _ptr(growth), _ptr(nr))
    ctx.check(rc)
    k = int(nr.item())
    return DmdResult(phi=phi[:, :k], mu=mu[:k], b=b[:k], freq=freq[:k], growth=growth[:k], nr=k)


def tune_block_rows(m: int, n: int, ctx: Context | None = None) -> int:
    """The leaf height the library picks for an m x n problem (host-side model)."""
    ctx = ctx or Context(-1)
    b = ctx.lib.pylom_tune_block_rows(ctx.h, m, n)
    if b < 0:
        raise PylomError(int(b), "tune_block_rows")
    return int(b)


class PodBatch:
    """A batch of POD instances of uneven shapes run by one pylom_pod_batched
    call.  Outputs are allocated once, so that with use_graph the captured
    launch sequence is replayed by every later run()."""

    def __init__(self, Ds, remove_mean=False, r: float = 0.01, precision: str = "fp64",
                 use_graph: bool = True, ctx: Context | None = None):
        if not Ds:
            raise ValueError("empty batch")
        dt = Ds[0].dtype
        for D in Ds:
            _rowmajor(D, "D")
            if D.dtype != dt or not D.is_cuda:
                raise ValueError("all instances must be GPU tensors of one dtype")
        self.ctx = ctx or context(Ds[0].device.index)
        self.precision = precision
        self.use_graph = bool(use_graph)
        self.dtype = _dtype_code(Ds[0])
        rms = remove_mean if isinstance(remove_mean, (list, tuple)) else [remove_mean] * len(Ds)
        rs = r if isinstance(r, (list, tuple)) else [r] * len(Ds)
        self.Ds = list(Ds)
        self.out = []
        arr = (_lib.Problem * len(Ds))()
        for i, D in enumerate(Ds):
            m, n = D.shape
            dev = D.device
            o = dict(U=torch.empty((m, n), dtype=dt, device=dev),
                     S=torch.empty(n, dtype=torch.float64, device=dev),
                     VT=torch.empty((n, n), dtype=torch.float64, device=dev),
                     nr=torch.empty(1, dtype=torch.int64, device=dev),
                     mean=torch.empty(m, dtype=dt, device=dev) if rms[i] else None)
            self.out.append(o)
            arr[i] = _lib.Problem(m, n, D.data_ptr(), D.stride(0), int(bool(rms[i])), float(rs[i]),
                                  o["mean"].data_ptr() if o["mean"] is not None else 0,
                                  o["U"].data_ptr(), n, o["S"].data_ptr(), o["VT"].data_ptr(), n,
                                  o["nr"].data_ptr())
        self.arr = arr

    def run(self):
        self.ctx.bind_stream()
        rc = self.ctx.lib.pylom_pod_batched(self.ctx.h, self.dtype, _PREC[self.precision],
                                            len(self.Ds), ctypes.cast(self.arr, ctypes.c_void_p),
                                            int(self.use_graph))
        self.ctx.check(rc)
        return self

    def results(self):
        res = []
        for o in self.out:
            k = int(o["nr"].item())
            res.append(PodResult(U=o["U"][:, :k], S=o["S"], VT=o["VT"][:k], mean=o["mean"], nr=k,
                                 U_full=o["U"], VT_full=o["VT"]))
        return res
