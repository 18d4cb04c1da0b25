"""Pins of the oracle's full-order model against closed forms, invariants and
textbook values (CPU only).  Each test would fail on a plausible mistake in the
oracle: a dropped term, a wrong sign, a wrong neighbour or a transposed operand."""
import os

import numpy as np
import pytest

from oracle import fom as F
from oracle import react as R
from oracle import riemann as RS
from paper_2605_28684_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ Burgers
def test_burgers_sum_f_zero_periodic():
    u = W.random_state(W.BURGERS, [257], seed=1)
    f = F.burgers_f(u, 0.01)
    assert abs(np.sum(f)) <= 1e-12 * np.sum(np.abs(f))


def test_godunov_consistency_and_definition():
    rng = np.random.default_rng(3)
    a = rng.normal(size=20000)
    b = rng.normal(size=20000)
    # F(u, u) = g(u) exactly
    assert np.array_equal(F.godunov_burgers(a, a), 0.5 * a * a)
    # textbook Godunov flux for convex g: min of g on [a, b] if a <= b, else max on [b, a]
    g = lambda x: 0.5 * x * x
    ref = np.where(a <= b, g(np.clip(0.0, a, b)), np.maximum(g(a), g(b)))
    assert np.array_equal(F.godunov_burgers(a, b), ref)


@pytest.mark.parametrize("k", [1, 3, 17])
def test_burgers_diffusion_eigenvalue(k):
    n, nu = 128, 0.013
    x = (np.arange(n) + 0.5) / n
    dx = 1.0 / n
    u = np.sin(2 * np.pi * k * x)
    f = F.burgers_f(u, nu, conv=0.0)
    lam = -4.0 / dx ** 2 * np.sin(np.pi * k * dx) ** 2
    np.testing.assert_allclose(f, nu * lam * u, rtol=0, atol=1e-9 * nu * abs(lam))


def test_burgers_constant_state_zero():
    for c in (-0.7, 0.0, 1.3):
        assert np.all(F.burgers_f(np.full(33, c), 0.01) == 0.0)


def test_burgers_upwind_direction():
    # positive velocity: the flux at face i+1/2 is g(u_i) (upwind from the left)
    u = np.array([1.0, 2.0, 3.0, 1.5, 1.2])
    F_ = F.godunov_burgers(u, np.roll(u, -1))
    np.testing.assert_array_equal(F_, 0.5 * u * u)


def test_burgers_newton_conserves_sum_and_converges():
    u0 = W.random_state(W.BURGERS, [200], seed=2)
    s0 = u0.sum()
    u = u0
    for _ in range(50):
        u, it, ok = F.newton_be_step(F.BURGERS, u, 1e-3, dict(nu=0.01))
        assert ok and it <= 10
    assert abs(u.sum() - s0) <= 1e-11 * np.sum(np.abs(u0))


def test_burgers_pure_diffusion_fourier_multiplier():
    n, nu, dt, k = 64, 0.02, 1e-3, 5
    x = (np.arange(n) + 0.5) / n
    u = np.cos(2 * np.pi * k * x)
    phys = dict(nu=nu, conv=0.0)
    u1, it, ok = F.newton_be_step(F.BURGERS, u, dt, phys)
    assert ok and it == 1     # linear problem: exactly one Newton solve
    m = 1.0 / (1.0 + 4 * nu * dt * np.sin(np.pi * k / n) ** 2 * n * n)
    np.testing.assert_allclose(u1, m * u, rtol=0, atol=1e-13)


# ------------------------------------------------------------------ Euler
@pytest.mark.parametrize("flux", [F.rusanov_flux, F.hllc_flux])
def test_euler_flux_consistency(flux):
    U = W.random_state(W.EULER_HLLC, [500], seed=4).reshape(-1, 3)
    np.testing.assert_allclose(flux(U, U, 1.4), F.euler_flux(U, 1.4), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("problem", [F.EULER_RUSANOV, F.EULER_HLLC])
def test_euler_uniform_state_and_wall_fluxes(problem):
    U = np.tile([1.3, 0.4, 2.9], 40)
    assert np.max(np.abs(F.fom_f(problem, U, dict(gamma=1.4)))) < 1e-12
    # sum_i f_i dx = -(F(U_{N-1}) - F(U_0)) with zero-gradient ghosts
    U = W.random_state(problem, [300], seed=5)
    f = F.fom_f(problem, U, dict(gamma=1.4)).reshape(-1, 3)
    Uc = U.reshape(-1, 3)
    wall = F.euler_flux(Uc[[0, -1]], 1.4)
    np.testing.assert_allclose(f.sum(axis=0) / 300, -(wall[1] - wall[0]), rtol=1e-10, atol=1e-11)


def test_hllc_supersonic_is_upwind():
    # both states moving right faster than sound: HLLC returns F(U_L)
    W_ = dict(gamma=1.4)
    UL = np.array([[1.0, 3.0, 1.0 / 0.4 + 0.5 * 9.0]])
    UR = np.array([[0.5, 1.5, 0.5 / 0.4 + 0.5 * 0.5 * 9.0]])
    np.testing.assert_allclose(F.hllc_flux(UL, UR, 1.4), F.euler_flux(UL, 1.4), rtol=1e-14)
    del W_


def test_exact_riemann_textbook_values():
    vals = np.loadtxt(os.path.join(HERE, "golden", "toro_sod_star.txt"))
    p, u, rl, rr = RS.star_densities((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    np.testing.assert_allclose([p, u, rl, rr], vals, rtol=0, atol=6e-6)


def test_exact_riemann_jump_conditions():
    g = 1.4
    WL, WR = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    p, u, rl, rr = RS.star_densities(WL, WR, g)
    S = RS.shock_speed_right(WL, WR, g)
    E = lambda r, v, pp: pp / (g - 1) + 0.5 * r * v * v
    # Rankine-Hugoniot across the right shock: F(U*) - F(U_R) = S (U* - U_R)
    Us = np.array([rr, rr * u, E(rr, u, p)])
    Ur = np.array([0.125, 0.0, E(0.125, 0.0, 0.1)])
    Fs = np.array([rr * u, rr * u * u + p, u * (E(rr, u, p) + p)])
    Fr = np.array([0.0, 0.1, 0.0])
    np.testing.assert_allclose(Fs - Fr, S * (Us - Ur), rtol=1e-12, atol=1e-12)
    # isentropic left fan: p / rho^gamma and u + 2c/(g-1) constant across it
    xi = np.linspace(-1.1, -0.1, 50)
    r_, u_, p_ = RS.sample(WL, WR, xi, g)
    fan = (xi > -np.sqrt(1.4)) & (xi < u - np.sqrt(g * p / rl))
    assert fan.sum() > 10
    np.testing.assert_allclose(p_[fan] / r_[fan] ** g, 1.0, rtol=1e-12)
    c_ = np.sqrt(g * p_[fan] / r_[fan])
    np.testing.assert_allclose(u_[fan] + 2 * c_ / (g - 1), 2 * np.sqrt(1.4) / 0.4, rtol=1e-12)
    # p and u continuous across the contact
    a = RS.sample(WL, WR, [u - 1e-9, u + 1e-9], g)
    assert abs(a[2][0] - a[2][1]) < 1e-12 and abs(a[1][0] - a[1][1]) < 1e-12
    assert abs(a[0][0] - a[0][1]) > 0.1


@pytest.mark.parametrize("problem", [F.EULER_RUSANOV, F.EULER_HLLC])
def test_sod_converges_to_exact_solution(problem):
    errs = []
    for n in (32, 64, 128):
        w = W.sod_hllc_f32(n=n, flux=problem)
        q = w.q0.copy()
        steps = int(round(0.2 / w.dt))
        for _ in range(steps):
            q, _, ok = F.newton_be_step(problem, q, w.dt, dict(gamma=1.4))
            assert ok
        x = (np.arange(n) + 0.5) / n
        rho_ex, _, _ = RS.sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), (x - 0.5) / 0.2)
        errs.append(np.mean(np.abs(q.reshape(-1, 3)[:, 0] - rho_ex)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.05


# ------------------------------------------------------------------ reacting model
def test_react_species_source_sums_to_zero():
    w = W.react10_f32(n_inst=1, n=64)
    Q = W.random_state(W.REACT, [64], seed=7).reshape(-1, 12)
    om = R.species_source(Q, w.phys[0])
    assert np.max(np.abs(om.sum(axis=1))) <= 1e-12 * np.max(np.abs(om))
    assert np.max(np.abs(om)) > 1.0


def test_react_single_bimolecular_reaction_closed_form():
    # one reaction a + b -> c + d at fixed T, no transport, Y_a = Y_b = y0:
    # BE gives y1 = y0 - k dt y1^2, i.e. y1 = (-1 + sqrt(1 + 4 k dt y0)) / (2 k dt)
    base = W.react10_f32(n_inst=1, n=16).phys[0]
    ph = dict(base)
    for key in ("ra", "rb", "pc", "pd", "E", "Q"):
        ph[key] = np.array(base[key])
    ph["A"] = 0.0 * base["A"]
    ph["k_in"] = 0.0
    j = 3
    mask = np.zeros(12)
    mask[j] = 1.0
    ph["A"] = 1e3
    ph["E"] = np.where(mask > 0, np.log(10.0) * 0.5, 1e30)
    ph["Q"] = np.zeros(12)
    n, y0, T, dt = 16, 0.3, 0.8, 1e-3
    Q = np.zeros((n, 12))
    Q[:, ph["ra"][j]] = y0
    Q[:, ph["rb"][j]] = y0
    Q[:, 10] = T
    q1, it, ok = F.newton_be_step(F.REACT, Q.reshape(-1), dt, ph, tol=1e-14, max_it=20)
    assert ok
    k = 1e3 * np.exp(-np.log(10.0) * 0.5 / T)
    y1 = (-1 + np.sqrt(1 + 4 * k * dt * y0)) / (2 * k * dt)
    Q1 = q1.reshape(n, 12)
    np.testing.assert_allclose(Q1[:, ph["ra"][j]], y1, rtol=1e-12)
    np.testing.assert_allclose(Q1[:, ph["pc"][j]], y0 - y1, rtol=1e-12)
    np.testing.assert_allclose(Q1[:, 10], T, rtol=0, atol=1e-15)


def test_react_pure_diffusion_of_temperature():
    base = W.react10_f32(n_inst=1, n=32).phys[0]
    ph = dict(base)
    ph["k_in"] = 0.0
    ph["A"] = 0.0
    n, dt, k = 32, 1e-3, 3
    x = (np.arange(n) + 0.5) / n
    Q = np.zeros((n, 12))
    Q[:, 10] = 1.0 + 0.2 * np.sin(2 * np.pi * k * x)
    q1, it, ok = F.newton_be_step(F.REACT, Q.reshape(-1), dt, ph)
    assert ok and it == 1
    m = 1.0 / (1.0 + 4 * ph["kappa"] * dt * np.sin(np.pi * k / n) ** 2 * n * n)
    np.testing.assert_allclose(q1.reshape(n, 12)[:, 10], 1.0 + 0.2 * m * np.sin(2 * np.pi * k * x),
                               rtol=0, atol=1e-14)


# ------------------------------------------------------------------ Jacobians
def _phys(problem):
    if problem == F.BURGERS:
        return dict(nu=0.01)
    if problem == F.REACT:
        return W.react10_f32(n_inst=1, n=24).phys[0]
    return dict(gamma=1.4)


@pytest.mark.parametrize("problem", [F.BURGERS, F.EULER_RUSANOV, F.EULER_HLLC, F.REACT])
def test_jacobian_matches_central_differences(problem):
    n = 24
    q = W.random_state(problem, [n], seed=11)
    ph = _phys(problem)
    J = F.jacobian_f(problem, q, ph).toarray()
    rng = np.random.default_rng(5)
    for _ in range(3):
        v = rng.normal(size=q.shape)
        h = 1e-6
        fd = (F.fom_f(problem, q + h * v, ph) - F.fom_f(problem, q - h * v, ph)) / (2 * h)
        np.testing.assert_allclose(J @ v, fd, rtol=0, atol=1e-6 * np.max(np.abs(fd)) + 1e-9)


def test_burgers_jacobian_column_sums_vanish():
    q = W.random_state(W.BURGERS, [40], seed=12)
    J = F.jacobian_f(F.BURGERS, q, dict(nu=0.01)).toarray()
    assert np.max(np.abs(J.sum(axis=0))) <= 1e-10 * np.max(np.abs(J))
    # tridiagonal with periodic corners
    nz = np.abs(J) > 0
    i, j = np.nonzero(nz)
    assert np.all(((j - i) % 40 <= 1) | ((i - j) % 40 <= 1))


@pytest.mark.parametrize("problem", [F.BURGERS, F.EULER_RUSANOV])
def test_rollout_vjp_matches_central_differences(problem):
    """<dL/dq0, v> against central differences of L = <gbar, q^T> over a short
    backward-Euler rollout with a tight Newton tolerance (pins the adjoint
    recursion, including the transposes and the step order)."""
    rng = np.random.default_rng(41)
    if problem == F.BURGERS:
        n, phys, dt = 48, dict(nu=0.01), 2e-3
        x = (np.arange(n) + 0.5) / n
        q0 = 0.5 + 0.8 * np.sin(2 * np.pi * x)
    else:
        n, phys, dt = 40, dict(gamma=1.4), 0.064 / 40
        x = (np.arange(n) + 0.5) / n
        rho = 1.0 + 0.3 * np.sin(2 * np.pi * x)
        u = 0.2 * np.cos(2 * np.pi * x)
        p = 1.0 + 0.2 * np.sin(4 * np.pi * x)
        q0 = np.stack([rho, rho * u, p / 0.4 + 0.5 * rho * u * u], axis=1).reshape(-1)
    T = 6
    gbar = rng.normal(size=q0.shape)
    g0 = F.be_rollout_vjp(problem, q0, dt, T, phys, gbar, tol=1e-13, max_it=30)

    def L(q):
        return gbar @ F.fom_trajectory(problem, q, dt, T, phys, tol=1e-13, max_it=30)[:, -1]

    h = 1e-6
    for _ in range(3):
        v = rng.normal(size=q0.shape)
        fd = (L(q0 + h * v) - L(q0 - h * v)) / (2 * h)
        assert abs(g0 @ v - fd) <= 1e-6 * max(1.0, abs(fd)), (g0 @ v, fd)
