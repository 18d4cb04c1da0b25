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


# ---------------------------------------------------------------- whole rollout
def _rollout_case(w_init=5, r=3, n_s=6, hyper="deim", n=48, z=2):
    w = W.euler_adjoint_f32(n_inst=1, n=n, r=r, n_s=n_s, z=z, N_t=20, precision=W.F64)
    prm = w.params()
    prm.update(reorth_every=0, newton_tol=1e-13, rom_tol=1e-14, rom_max=30, newton_max=30,
               w_init=w_init, hyper=hyper)
    return prm, w.phys[0], w.q0.copy(), w.extra["target"][:w.q0.shape[0]]


@pytest.mark.parametrize("case", ["deim_truncated_pod", "deim_w_init_eq_r", "qdeim"])
def test_rollout_vjp_matches_central_differences(case):
    """d L / d q0 through Alg. 1 as a whole (training BE steps, preprocessing,
    POD, a^{w_init}, the first coarse step; then HR-LSPG steps and events), with
    L = 1/2 |q~_end - q_tgt|^2 on the perturbed-Sod recipe of the adjoint
    configuration at 48 cells, against central differences (h = 1e-7) of the
    oracle's own forward with the recorded sample schedule: relative error
    <= 1e-6 on three random directions (measured about 1e-8).  Planted
    mistakes in any single term (the (P^T Phi)^+ adjoint, the D or q_ref terms
    of a step, an event or the seed, the POD's out-of-span term or its sigma
    term, the preprocessing's scale, the first coarse step, an untransposed
    step solve) give 2e-3 or more."""
    kw = dict(deim_truncated_pod={}, deim_w_init_eq_r=dict(w_init=3),
              qdeim=dict(hyper="qdeim", n_s=3))[case]
    prm, phys, q0, tgt = _rollout_case(**kw)
    n_steps = 6
    st, _, sched = A.rollout_forward(W.EULER_RUSANOV, phys, q0, prm, n_steps)
    qt = O.reconstruct(st["q_ref"], st["d"], st["Phi"], st["a"])
    g, _ = A.rollout_vjp(W.EULER_RUSANOV, phys, q0, prm, n_steps, qt - tgt, sched)
    rng = np.random.default_rng(31)
    h = 1e-7
    for _ in range(3):
        v = rng.normal(size=q0.shape)
        Lp = A.rollout_loss(W.EULER_RUSANOV, phys, q0 + h * v, prm, n_steps, tgt, sched)
        Lm = A.rollout_loss(W.EULER_RUSANOV, phys, q0 - h * v, prm, n_steps, tgt, sched)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g @ v) <= 1e-6 * abs(fd), (fd, g @ v)


def test_pinv_vjp_matches_central_differences():
    """The adjoint of M = A^+ (full column rank, n_s > r) against central
    differences of numpy's pinv, on random A, Mbar and directions."""
    rng = np.random.default_rng(5)
    A_ = rng.normal(size=(9, 4))
    Mb = rng.normal(size=(4, 9))
    Ab = A._pinv_vjp(A_, np.linalg.pinv(A_), Mb)
    for _ in range(3):
        V = rng.normal(size=A_.shape)
        h = 1e-6
        fd = np.sum(Mb * (np.linalg.pinv(A_ + h * V) - np.linalg.pinv(A_ - h * V))) / (2 * h)
        assert abs(fd - np.sum(Ab * V)) <= 1e-8 * abs(fd)


def test_pod_vjp_matches_central_differences():
    """The adjoint of the truncated, sign-fixed POD (leading r = 3 of w = 6
    columns) against central differences of the oracle's pod."""
    rng = np.random.default_rng(6)
    X = rng.normal(size=(40, 6)) * np.array([5.0, 3.0, 2.0, 1.0, 0.5, 0.2])
    Phi, s = O.pod(X, 3)
    Pb = rng.normal(size=Phi.shape)
    sb = rng.normal(size=3)
    Xb = A._pod_vjp(X, Phi, Pb, sb)
    for _ in range(3):
        V = rng.normal(size=X.shape)
        h = 1e-6
        Pp, sp_ = O.pod(X + h * V, 3)
        Pm, sm_ = O.pod(X - h * V, 3)
        fd = (np.sum(Pb * (Pp - Pm)) + sb @ (sp_ - sm_)) / (2 * h)
        assert abs(fd - np.sum(Xb * V)) <= 1e-6 * abs(fd)
