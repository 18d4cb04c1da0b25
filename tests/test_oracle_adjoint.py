"""Pins of the online-loop adjoint oracle (oracle/adjoint.py) against central
finite differences of the oracle's own forward loop, FP64: steps only, one
event, two events, each direction set drawn at random."""
import numpy as np
import pytest

from oracle import adjoint as A
from oracle import rom as O
from paper_2605_28684_amd import workloads as W


def _setup(n=64, r=4, z=3, seed=3):
    prm = O.default_params(r=r, n_s=r, w_init=r, z=z, dt=2e-3, lam=0.7, newton_tol=1e-13,
                           newton_max=30, rom_tol=1e-14, rom_max=30, reorth_every=0)
    x = W.centres(n)
    q0 = 0.4 + 0.3 * np.sin(2 * np.pi * x) + 0.1 * np.cos(6 * np.pi * x + 0.4)
    phys = dict(nu=0.01)
    st = O.offline(W.BURGERS, phys, q0, prm)
    rng = np.random.default_rng(seed)
    q_tgt = q0 + 0.05 * rng.normal(size=n)
    return prm, phys, st, q_tgt, rng


# per input: Richardson-extrapolated central difference step and relative bound
# (y_corr enters through D = diag(1/phi_norm), about 4e4 here, so its step is small;
# the loss barely depends on sigma over a few steps, so its gradient is tiny)
_STEPS = {"a": (1e-3, 1e-5), "Phi": (1e-5, 1e-5), "sigma": (1e-3, 1e-4), "y_corr": (1e-6, 1e-5)}


def _fd_check(n_steps, phi_noise=0.0):
    prm, phys, st, q_tgt, rng = _setup()
    if phi_noise:
        # a non-orthonormal starting basis: terms that vanish when Phi^T Phi = I
        # (the first Gram-Schmidt pass's p1bar) then carry weight
        st["Phi"] = st["Phi"] + phi_noise * rng.normal(size=st["Phi"].shape) / np.sqrt(
            st["Phi"].shape[0])
    n0 = prm["w_init"]
    out, _ = A.online_forward(W.BURGERS, phys, st, prm, n0, n_steps)
    qt = O.reconstruct(out["q_ref"], out["d"], out["Phi"], out["a"])
    grads = dict(zip(("a", "Phi", "sigma", "y_corr"),
                     A.online_vjp(W.BURGERS, phys, st, prm, n0, n_steps, qt - q_tgt)))
    for key, g in grads.items():
        v = rng.normal(size=st[key].shape)
        v /= np.linalg.norm(v)
        dot = float(np.sum(g * v))

        def L(eps):
            s2 = dict(st)
            s2[key] = st[key] + eps * v
            return A.online_loss(W.BURGERS, phys, s2, prm, n0, n_steps, q_tgt)

        h, tol = _STEPS[key]
        f1 = (L(h) - L(-h)) / (2 * h)
        f2 = (L(h / 2) - L(-h / 2)) / h
        fd = (4 * f2 - f1) / 3
        if dot == 0.0:
            assert abs(fd) < 1e-12, (key, fd)
        else:
            assert abs(dot - fd) <= tol * abs(dot), (n_steps, key, dot, fd)
    return out


def test_adjoint_fine_steps_only():
    # w_init = 4, z = 3: the first event follows fine step n = 6
    _fd_check(n_steps=2)


def test_adjoint_one_event():
    _fd_check(n_steps=3)


def test_adjoint_two_events_and_steps_between():
    _fd_check(n_steps=7)


def test_adjoint_sigma_and_ycorr_unused_without_events():
    prm, phys, st, q_tgt, rng = _setup()
    out, _ = A.online_forward(W.BURGERS, phys, st, prm, prm["w_init"], 2)
    qt = O.reconstruct(out["q_ref"], out["d"], out["Phi"], out["a"])
    ab, Phib, sb, yb = A.online_vjp(W.BURGERS, phys, st, prm, prm["w_init"], 2, qt - q_tgt)
    assert np.all(sb == 0.0) and np.all(yb == 0.0)


def test_adjoint_non_orthonormal_basis():
    _fd_check(n_steps=7, phi_noise=0.3)
