"""Pins of the DMD oracle (oracle/dmd.py) against what the mathematics fixes,
independently of the oracle's own formulas:

* exactly linear data d_t = sum_i phi_i b_i lambda_i^t: exact DMD recovers
  every lambda_i, and each mode times its amplitude equals phi_i b_i (the
  product does not depend on how a mode is scaled); the truncated SVD keeps
  exactly the rank of the data;
* a single oscillation x cos(w t) + y sin(w t): mu = e^{+-i w dt}, frequency
  +-w / (2 pi dt) (Eq. freq) and zero growth;
* a decaying real mode: mu = lambda, frequency 0, growth log(lambda) / dt;
* a constant field plus oscillations over whole periods with the mean
  removed over all N snapshots: the mean is the constant, so the dynamics
  are recovered exactly again; without removal the constant is one more
  mode with mu = 1;
* the amplitudes reconstruct the data: Y1 = phi diag(b) V_and.

These fail for a transposed linear map, a dropped S^-1, a wrong sign of the
time index in the Vandermonde matrix or a mean taken over the wrong
columns.
"""
import numpy as np
import pytest

from oracle import dmd as odmd
from paper_2405_15529_amd import synth


def match(mu, lam):
    """Index of the nearest true eigenvalue for every computed one (a
    bijection is asserted)."""
    idx = [int(np.argmin(np.abs(lam - z))) for z in mu]
    assert sorted(idx) == list(range(len(lam)))
    return np.array(idx)


def test_linear_dynamics_recovered():
    D, lam, phi, amp = synth.linear_dynamics(300, 40, seed=1, real_eigs=(0.8,))
    out = odmd.dmd(D, remove_mean=False, r=1e-12)
    assert out["nr"] == len(lam)
    idx = match(out["mu"], lam)
    assert np.max(np.abs(out["mu"] - lam[idx])) <= 1e-12
    mode_amp = out["phi"] * out["b"][None, :]
    ref = phi[:, idx] * amp[idx][None, :]
    assert np.max(np.abs(mode_amp - ref)) <= 1e-10 * np.max(np.abs(ref))
    # sorted by |b|
    assert np.all(np.diff(np.abs(out["b"])) <= 1e-12 * np.abs(out["b"]).max())


def test_single_oscillation_frequency():
    m, N, w, dt = 50, 30, 0.7, 0.25
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal(m), rng.standard_normal(m)
    t = np.arange(N) * dt
    D = np.outer(x, np.cos(w * t)) + np.outer(y, np.sin(w * t))
    out = odmd.dmd(D, r=1e-12, dt=dt)
    assert out["nr"] == 2
    z = np.exp(1j * w * dt)
    assert np.max(np.abs(np.sort_complex(out["mu"]) - np.sort_complex(np.array([z, np.conj(z)])))) <= 1e-12
    assert np.allclose(np.sort(out["freq"]), [-w / (2 * np.pi), w / (2 * np.pi)], atol=1e-12)
    assert np.max(np.abs(out["growth"])) <= 1e-12


def test_decaying_real_mode():
    m, N, lam, dt = 40, 12, 0.9, 0.5
    rng = np.random.default_rng(4)
    x = rng.standard_normal(m)
    D = np.outer(x, lam ** np.arange(N))
    out = odmd.dmd(D, r=1e-12, dt=dt)
    assert out["nr"] == 1
    assert abs(out["mu"][0] - lam) <= 1e-14
    assert abs(out["freq"][0]) <= 1e-14
    assert abs(out["growth"][0] - np.log(lam) / dt) <= 1e-13
    # mode times amplitude is the first snapshot
    np.testing.assert_allclose(np.real(out["phi"][:, 0] * out["b"][0]), x, rtol=0, atol=1e-13)


def test_mean_over_all_snapshots():
    m, N = 60, 48
    rng = np.random.default_rng(5)
    c = rng.standard_normal(m)
    t = np.arange(N)
    ws = [2 * np.pi * 3 / N, 2 * np.pi * 7 / N]   # whole periods over N snapshots
    D = c[:, None] + sum(np.outer(rng.standard_normal(m), np.cos(w * t)) +
                         np.outer(rng.standard_normal(m), np.sin(w * t)) for w in ws)
    out = odmd.dmd(D, remove_mean=True, r=1e-12)
    lam = np.array([np.exp(1j * w) for w in ws] + [np.exp(-1j * w) for w in ws])
    assert out["nr"] == 4
    idx = match(out["mu"], lam)
    assert np.max(np.abs(out["mu"] - lam[idx])) <= 1e-11
    # the removed mean is the constant field (whole periods over all N
    # snapshots; over the first N - 1 it would be off by O(1/N))
    assert np.max(np.abs(out["mean"] - c)) <= 1e-13
    assert np.max(np.abs(D[:, :-1].mean(axis=1) - c)) > 1e-3
    # without mean removal the constant is one more mode, with mu = 1
    keep = odmd.dmd(D, remove_mean=False, r=1e-12)
    assert keep["nr"] == 5 and np.min(np.abs(keep["mu"] - 1.0)) <= 1e-11


def test_amplitudes_reconstruct_first_snapshots():
    D, lam, phi, amp = synth.linear_dynamics(200, 25, seed=7)
    out = odmd.dmd(D, r=1e-12)
    N = D.shape[1]
    Vand = out["mu"][:, None] ** np.arange(N - 1)[None, :]
    rec = (out["phi"] * out["b"][None, :]) @ Vand
    assert np.max(np.abs(rec - D[:, :-1])) <= 1e-10 * np.max(np.abs(D))


def test_eigvec_normalisation():
    rng = np.random.default_rng(8)
    w = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
    v = odmd.normalise_eigvecs(w)
    for i in range(5):
        assert abs(np.linalg.norm(v[:, i]) - 1.0) <= 1e-15
        j = int(np.argmax(np.abs(v[:, i])))
        assert v[j, i].imag == 0.0 and v[j, i].real > 0.0
        # same direction as the input column
        c = np.vdot(v[:, i], w[:, i])
        assert abs(abs(c) - np.linalg.norm(w[:, i])) <= 1e-12 * np.linalg.norm(w[:, i])


def test_empty_basis():
    D = np.repeat(np.arange(1.0, 11.0)[:, None], 8, axis=1)
    out = odmd.dmd(D, remove_mean=True, r=0.01)
    assert out["nr"] == 0


def test_needs_two_snapshots():
    with pytest.raises(ValueError):
        odmd.dmd(np.ones((5, 1)))
