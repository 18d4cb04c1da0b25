"""Pins of the explicit path's oracle (oracle/explicit.py): the limited
second-order residual and SSPRK(4,3), against closed forms, invariants and
convergence orders; the explicit Galerkin ROM against the full-order step."""
import numpy as np
import pytest

from oracle import explicit as X
from oracle import fom as F
from oracle import rom as O
from paper_2605_28684_amd import workloads as W

PROBLEMS = [F.BURGERS, F.EULER_RUSANOV, F.EULER_HLLC, F.REACT]


def _phys(problem):
    if problem == F.BURGERS:
        return dict(nu=0.004)
    if problem in (F.EULER_RUSANOV, F.EULER_HLLC):
        return dict(gamma=1.4)
    return W.react10_f32(n_inst=1, n=16).phys[0]


def test_limited_faces_reproduce_linear_data_and_stay_monotone():
    """A linear profile is reconstructed exactly at interior faces (no
    limiting away from extrema); on random data every face state lies between
    the values of the two cells around it and the cell's other neighbour."""
    n = 40
    Q = (3.0 + 0.25 * np.arange(n))[:, None]
    QL, QR = X.limited_faces(Q, periodic=False)
    mid = 0.5 * (Q[:-1, 0] + Q[1:, 0])                       # faces 1/2 .. n-3/2
    assert np.allclose(QL[2:n - 1, 0], mid[1:-1], rtol=0, atol=1e-14)
    assert np.allclose(QR[2:n - 1, 0], mid[1:-1], rtol=0, atol=1e-14)
    rng = np.random.default_rng(5)
    R = rng.normal(size=(60, 3))
    QL, QR = X.limited_faces(R, periodic=True)
    for k in range(61):                                       # face k: cells k-1 | k
        for (val, cell) in ((QL[k], k - 1), (QR[k], k)):
            nb = R[[(cell - 1) % 60, cell % 60, (cell + 1) % 60]]
            assert np.all(val >= nb.min(axis=0) - 1e-15) and np.all(val <= nb.max(axis=0) + 1e-15)


@pytest.mark.parametrize("problem", PROBLEMS)
def test_f2_constant_zigzag_and_conservation(problem):
    """A constant state gives f2 = 0 (no sources for it); a zig-zag state,
    where every cell is a local extremum, limits every slope to zero, so f2
    equals the first-order f; periodic Burgers conserves the sum."""
    ph = _phys(problem)
    nv = F.NVAR[problem]
    n = 32
    rng = np.random.default_rng(6)
    base = W.random_state(problem, [n], seed=7, scale=0.5).reshape(n, nv)
    if problem != F.REACT:
        const = np.tile(base[:1], (n, 1)).reshape(-1)
        assert np.max(np.abs(X.fom_f2(problem, const, ph))) < 1e-10
    sign = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)[:, None]
    zig = np.mean(base, axis=0)[None, :] * (1.0 + 0.1 * sign)  # every cell an extremum
    q = zig.reshape(-1)
    assert np.allclose(X.fom_f2(problem, q, ph), F.fom_f(problem, q, ph), rtol=1e-12,
                       atol=1e-9 * np.max(np.abs(F.fom_f(problem, q, ph))))
    if problem == F.BURGERS:
        qb = rng.normal(size=n)
        assert abs(np.sum(X.fom_f2(problem, qb, ph))) < 1e-10 * n * n


def test_f2_is_second_order_on_a_smooth_monotone_state():
    """Euler, smooth monotone density and pressure ramps (uniform velocity),
    far from the walls: the error of f2 against the exact -dF/dx falls by
    about 4 per halving of dx, the first-order f's by about 2."""
    def state(n):
        x = W.centres(n)
        rho = 1.0 + 0.3 * np.tanh((x - 0.5) / 0.1)
        u = 0.4 * np.ones(n)
        p = 1.0 + 0.2 * np.tanh((x - 0.5) / 0.1)
        return x, W._conserved(rho, u, p)

    def exact(x):
        # F = (rho u, rho u^2 + p, u (E + p)) with u const: dF/dx from d rho/dx, dp/dx
        sech2 = 1.0 / np.cosh((x - 0.5) / 0.1) ** 2
        dr = 0.3 / 0.1 * sech2
        dp = 0.2 / 0.1 * sech2
        u = 0.4
        dE = dp / 0.4 + 0.5 * u * u * dr
        return -np.stack([u * dr, u * u * dr + dp, u * (dE + dp)], axis=1)

    e1, e2 = [], []
    for n in (200, 400, 800):
        x, q = state(n)
        mid = (x > 0.3) & (x < 0.7)
        ex = exact(x)[mid]
        f1 = F.fom_f(F.EULER_RUSANOV, q, dict(gamma=1.4)).reshape(n, 3)[mid]
        f2 = X.fom_f2(F.EULER_RUSANOV, q, dict(gamma=1.4)).reshape(n, 3)[mid]
        e1.append(np.mean(np.abs(f1 - ex)))
        e2.append(np.mean(np.abs(f2 - ex)))
    r1 = np.log2(np.array(e1[:-1]) / np.array(e1[1:]))
    r2 = np.log2(np.array(e2[:-1]) / np.array(e2[1:]))
    assert np.all(r2 > 1.8) and np.all(r1 < 1.3)


def test_ssprk43_stability_polynomial_and_order():
    """On y' = lam y one step multiplies by 1 + z + z^2/2 + z^3/6 + z^4/48
    (z = lam dt), the scheme's stability polynomial; on y' = -y^2 the global
    error at t = 1 falls by about 8 per halving of dt (third order)."""
    for z in (-0.3, -1.7, 0.4 + 0.9j):
        got = X.ssprk43(lambda y: z * y, 1.0 + 0j, 1.0)
        assert abs(got - (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 48)) < 1e-14
    errs = []
    for n in (10, 20, 40):
        y = np.array([1.0])
        for _ in range(n):
            y = X.ssprk43(lambda v: -v * v, y, 1.0 / n)
        errs.append(abs(y[0] - 0.5))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 2.8) and np.all(rates < 3.3)


@pytest.mark.parametrize("problem", [F.BURGERS, F.EULER_HLLC])
def test_explicit_rom_with_full_basis_and_all_rows_is_the_fom_step(problem):
    """Phi = I (r = N), D = 1, q_ref = 0: the explicit Galerkin step (no
    hyper-reduction) and the DEIM-Galerkin step with P = all rows both equal
    the full-order SSPRK(4,3) step."""
    ph = _phys(problem)
    nv = F.NVAR[problem]
    n = 24
    q = W.random_state(problem, [n], seed=8, scale=0.5)
    N = n * nv
    I = np.eye(N)
    dt = 1e-3
    ref = X.fom_step_explicit(problem, q, dt, ph)
    a1 = X.galerkin_hr_explicit_step(problem, ph, np.zeros(N), np.ones(N), I, None, None, q, dt)
    P = np.arange(N)
    a2 = X.galerkin_hr_explicit_step(problem, ph, np.zeros(N), np.ones(N), I, P, O.rebuild(I, P),
                                     q, dt)
    assert np.max(np.abs(a1 - ref)) < 1e-13 * np.max(np.abs(ref))
    assert np.max(np.abs(a2 - ref)) < 1e-12 * np.max(np.abs(ref))


def test_centred_slope_on_quadratic_data():
    """For increasing quadratic data q_i = i^2 the limiter stays inactive and
    the centred slope (q_{i+1} - q_{i-1})/2 = 2i puts the right-face state of
    cell i at i^2 + i (a one-sided slope would give i^2 + i + 1/2)."""
    n = 30
    Q = (np.arange(n, dtype=float) ** 2)[:, None]
    QL, _ = X.limited_faces(Q, periodic=False)
    i = np.arange(2, n - 2)
    assert np.array_equal(QL[i + 1, 0], i ** 2 + i)


@pytest.mark.parametrize("problem", PROBLEMS)
def test_face_flux_reproduces_each_models_first_order_transport(problem):
    """With diffusion, reactions and inflow switched off, -(H(q_i, q_{i+1}) -
    H(q_{i-1}, q_i))/dx from face_flux on cell values is the first-order f of
    the model (so the limited residual changes only the face states)."""
    ph = dict(_phys(problem))
    if problem == F.BURGERS:
        ph["nu"] = 0.0
    if problem == F.REACT:
        ph.update(nu_u=0.0, kappa=0.0, A=0.0, k_in=0.0)
    nv = F.NVAR[problem]
    n = 40
    q = W.random_state(problem, [n], seed=11, scale=0.5)
    if problem == F.REACT:
        q.reshape(n, nv)[:, 11] = 0.8 * np.sin(2 * np.pi * W.centres(n) + 0.4)  # both signs of u
    G = X._ghosted(q.reshape(n, nv), F.PERIODIC[problem])
    H1 = X.face_flux(problem, G[1:-2], G[2:-1], ph)
    f = -(H1[1:] - H1[:-1]) * n
    ref = F.fom_f(problem, q, ph).reshape(n, nv)
    assert np.max(np.abs(f - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_alg1_explicit_path_tracks_the_explicit_fom():
    """Alg. 1 on the explicit path (SSPRK(4,3) DEIM-Galerkin steps with QDEIM +
    FGS sampling, SSPRK(4,3) coarse steps) for the reacting model at small
    size: every step is explicit, the run stays finite, and the adaptive ROM
    follows the explicit full-order trajectory (report-level check: the
    relative error after 30 fine steps stays below 5 %)."""
    w = W.react10_f32(n_inst=1, n=64, r=6, n_s=12, z=3, N_t=50, precision=W.F64)
    w.dt = 2e-5
    w.hyper, w.projection, w.scheme = W.HR_QDEIM_FGS, W.GALERKIN, "ssprk43"
    prm = w.params()
    st, rec = O.adaptive_rom(W.REACT, w.phys[0], w.q0, prm, n_steps=30)
    qf = X.fom_trajectory_explicit(W.REACT, w.q0, w.dt, prm["w_init"] + 30, w.phys[0])[:, -1]
    qr = O.reconstruct(st["q_ref"], st["d"], st["Phi"], st["a"])
    assert np.all(np.isfinite(qr))
    assert np.linalg.norm(qr - qf) / np.linalg.norm(qf) < 0.05
    assert len(rec["events"]) == 10 and all(len(p) == 12 for p in rec["P"])
