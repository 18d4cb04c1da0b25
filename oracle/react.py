"""Oracle: the synthetic stiff ten-species advection-reaction model.  TEST INFRASTRUCTURE ONLY.

The paper's detonation case (Sec. 5.3, App. D) needs a detailed H2-O2 mechanism
and an in-house solver that are not available, so the 10-species workload uses a
synthetic model with the same structure (12 variables per cell: ten mass
fractions Y_1..Y_10, temperature T, velocity u; periodic 1-D domain; transport
plus a stiff Arrhenius source).  All constants are fixed here and in the
workload generator; the mechanism (species indices, activation energies, heat
releases) and the per-instance inflow state arrive as inputs in ``phys``.

Per cell i (dx = 1/N, periodic):
  u:      viscous Burgers, Godunov flux of u^2/2 plus nu_u * second difference
  Y_l, T: conservative upwind advection with face velocity u_f = (u_i+u_{i+1})/2,
          H_{i+1/2} = u_f * (phi_i if u_f >= 0 else phi_{i+1}),
          plus kappa * second difference, plus sources
  rates:  w_j = A exp(-E_j / max(T, T_floor)) Y_{a_j} Y_{b_j}      (j = 1..12)
  omega_l = sum_j w_j ([l in {c_j, d_j}] - [l in {a_j, b_j}])
  S_T     = sum_j Q_j w_j
  inflow: k_in (Y_in - Y_l), k_in (T_in - T) on cells with centre x_i < x_in
"""
import numpy as np

from .fom import godunov_burgers, cmax

T_FLOOR = 1e-2
NSPEC = 10
NREAC = 12


def react_f(Q, phys):
    """f for the synthetic model; Q has shape (N, 12) = [Y_1..Y_10, T, u]."""
    n = Q.shape[0]
    dx = 1.0 / n
    x = (np.arange(n) + 0.5) * dx
    nu_u, kappa, A = phys["nu_u"], phys["kappa"], phys["A"]
    k_in, x_in = phys["k_in"], phys["x_in"]
    ra, rb, pc, pd = phys["ra"], phys["rb"], phys["pc"], phys["pd"]
    E, Qh = phys["E"], phys["Q"]
    Y_in, T_in = phys["Y_in"], phys["T_in"]

    u = Q[:, 11]
    out = np.zeros_like(Q)
    # velocity: viscous Burgers
    up = np.roll(u, -1)
    F = godunov_burgers(u, up)
    du = up - u
    out[:, 11] = -(F - np.roll(F, 1)) / dx + nu_u * (du - np.roll(du, 1)) / (dx * dx)
    # scalars: upwind advection with face velocity, diffusion
    uf = 0.5 * (u + up)
    pos = np.real(uf) >= 0
    for v in range(11):
        phi = Q[:, v]
        phip = np.roll(phi, -1)
        H = uf * np.where(pos, phi, phip)
        dphi = phip - phi
        out[:, v] = -(H - np.roll(H, 1)) / dx + kappa * (dphi - np.roll(dphi, 1)) / (dx * dx)
    # reactions
    T = Q[:, 10]
    Tf = cmax(T, T_FLOOR)
    for j in range(NREAC):
        w = A * np.exp(-E[j] / Tf) * Q[:, ra[j]] * Q[:, rb[j]]
        out[:, ra[j]] -= w
        out[:, rb[j]] -= w
        out[:, pc[j]] += w
        out[:, pd[j]] += w
        out[:, 10] += Qh[j] * w
    # inflow relaxation
    inl = x < x_in
    for l in range(NSPEC):
        out[inl, l] += k_in * (Y_in[l] - Q[inl, l])
    out[inl, 10] += k_in * (T_in - Q[inl, 10])
    return out


def species_source(Q, phys):
    """The reaction part of the species right-hand side only (omega_l per cell)."""
    A, E = phys["A"], phys["E"]
    ra, rb, pc, pd = phys["ra"], phys["rb"], phys["pc"], phys["pd"]
    om = np.zeros((Q.shape[0], NSPEC), dtype=Q.dtype)
    Tf = cmax(Q[:, 10], T_FLOOR)
    for j in range(NREAC):
        w = A * np.exp(-E[j] / Tf) * Q[:, ra[j]] * Q[:, rb[j]]
        om[:, ra[j]] -= w
        om[:, rb[j]] -= w
        om[:, pc[j]] += w
        om[:, pd[j]] += w
    return om
