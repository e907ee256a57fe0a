"""Comparison helpers for GPU-vs-oracle parity (test infrastructure)."""
import numpy as np

EPS64 = 2.0 ** -53


def sigma_errors(S, Sref, nr):
    """(max relative error over the retained modes, max normwise error over all)."""
    S = np.asarray(S, dtype=np.float64)
    Sref = np.asarray(Sref, dtype=np.float64)
    rel = 0.0
    if nr > 0:
        rel = float(np.max(np.abs(S[:nr] - Sref[:nr]) / Sref[:nr]))
    nw = float(np.max(np.abs(S - Sref)) / max(Sref[0], 1e-300))
    return rel, nw


def nr_agrees(nr, nr_ref, Sref, r, tie=1e-10):
    """Equal, or the threshold falls within `tie` of a tail-energy boundary."""
    if nr == nr_ref:
        return True
    e = np.asarray(Sref, dtype=np.float64) ** 2
    tot = e.sum()
    lo = min(nr, nr_ref)
    tail = e[lo:].sum() / tot
    return abs(nr - nr_ref) == 1 and abs(tail - r) <= tie


def orth_error(U):
    U = np.asarray(U, dtype=np.float64)
    k = U.shape[1]
    return float(np.linalg.norm(U.T @ U - np.eye(k)))


def well_separated(Sref, i, gap=1e-3):
    s = Sref
    ok = True
    if i > 0:
        ok &= (s[i - 1] - s[i]) / s[i - 1] >= gap
    if i + 1 < len(s):
        ok &= (s[i] - s[i + 1]) / max(s[i], 1e-300) >= gap
    return bool(ok)


def mode_errors(U, Uref, VT, VTref, Sref, nr, gap=1e-3):
    """Max |u_i - u_ref_i| and |v_i - v_ref_i| (sign aligned) over retained,
    well-separated modes; plus the projector distance of the retained U span."""
    eu = ev = 0.0
    for i in range(nr):
        if not well_separated(Sref, i, gap) or Sref[i] <= 1e3 * len(Sref) * EPS64 * Sref[0]:
            continue
        sg = np.sign(np.dot(U[:, i], Uref[:, i])) or 1.0
        eu = max(eu, float(np.max(np.abs(sg * U[:, i] - Uref[:, i]))))
        ev = max(ev, float(np.max(np.abs(sg * VT[i] - VTref[i]))))
    proj = 0.0
    if nr > 0:
        A = U[:, :nr]
        B = Uref[:, :nr]
        # sine of the largest principal angle: |A - B (B^T A)|_2 (a direct
        # residual; sqrt(1 - cos^2) would amplify rounding to sqrt(eps))
        proj = float(np.linalg.norm(A - B @ (B.T @ A), 2))
    return eu, ev, proj


def sign_convention_holds(VT, nr):
    for i in range(nr):
        j = int(np.argmax(np.abs(VT[i])))
        if VT[i, j] < 0:
            return False
    return True
