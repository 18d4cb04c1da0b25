"""Oracle: the explicit full-order model and reduced step of the detonation
case's ROM structure (FP64).  TEST INFRASTRUCTURE ONLY.

The paper's detonation full-order model (App. D) is advanced explicitly by a
four-stage, third-order strong-stability-preserving Runge-Kutta scheme, with a
cell-centred second-order finite-volume discretisation and a Barth-Jespersen
limiter; its reduced model is the DEIM-Galerkin ROM of eq. deim_galerkin_rom
(Sec. 5.3: Galerkin form because the full-order solver is explicit).  Here the
same structure is built on the three model families of this project:

  limited_faces   second-order face states: slope s_i = (q_{i+1} - q_{i-1})/2
                  (in units of cells), limited per cell and variable by the
                  Barth-Jespersen factor psi_i = min(1, min(dmax_i, -dmin_i) /
                  (|s_i|/2)) with dmax_i, dmin_i the largest and smallest
                  neighbour differences (psi = 1 where s_i = 0); left state
                  of face i+1/2 q_i + psi_i s_i/2, right state q_{i+1} -
                  psi_{i+1} s_{i+1}/2
  fom_f2          f with the limited face states fed to each model's two-point
                  face flux (Burgers Godunov, Euler Rusanov/HLLC, the reacting
                  model's transport); diffusion and sources are those of the
                  first-order model: f2 = f - (dH2 - dH1)/dx with dH the face
                  flux differences of the limited and the first-order states
  ssprk43         y1 = y + dt/2 L(y); y2 = y1 + dt/2 L(y1);
                  y3 = 2/3 y + 1/3 y2 + dt/6 L(y2); y+ = y3 + dt/2 L(y3)
                  (Spiteri and Ruuth's SSPRK(4,3), SSP coefficient 2)
  fom_step_explicit  one SSPRK(4,3) step of dq/dt = f2(q)
  galerkin_hr_explicit_step  one SSPRK(4,3) step of eq. deim_galerkin_rom,
                  da/dt = (P^T Phi)^+ P^T D f2(q_ref + D^-1 Phi a); with no
                  hyper-reduction (M = Phi^T, all rows) the full Galerkin ROM

Boundaries follow the models: periodic (Burgers, reacting model) or two
zero-gradient ghost cells at each Euler wall (copies of the end cell).
"""
import numpy as np

from . import fom as F


def _ghosted(Q, periodic):
    """Q (n, nv) with two ghost cells on each side."""
    if periodic:
        return np.concatenate([Q[-2:], Q, Q[:2]], axis=0)
    return np.concatenate([Q[:1], Q[:1], Q, Q[-1:], Q[-1:]], axis=0)


def limited_faces(Q, periodic):
    """(QL, QR), each (n + 1, nv): the left and right states of faces
    i - 1/2, i = 0 .. n (face k sits between cells k - 1 and k)."""
    G = _ghosted(Q, periodic)                    # cell i at G[i + 2]
    c, m, p = G[1:-1], G[:-2], G[2:]             # cells -1 .. n with their neighbours
    s = 0.5 * (p - m)
    dmax = np.maximum(np.maximum(m, c), p) - c
    dmin = np.minimum(np.minimum(m, c), p) - c
    e = 0.5 * np.abs(s)
    with np.errstate(divide="ignore", invalid="ignore"):
        psi = np.where(e > 0, np.minimum(1.0, np.minimum(dmax, -dmin) / np.where(e > 0, e, 1.0)),
                       1.0)
    plus = c + 0.5 * psi * s                     # right-face value of cells -1 .. n
    minus = c - 0.5 * psi * s                    # left-face value of cells -1 .. n
    return plus[:-1], minus[1:]                  # face k: left cell k-1, right cell k


def face_flux(problem, QL, QR, phys):
    """The model's two-point face flux H(QL, QR) for each face (rows)."""
    if problem == F.BURGERS:
        return F.godunov_burgers(QL[:, 0], QR[:, 0])[:, None]
    if problem in (F.EULER_RUSANOV, F.EULER_HLLC):
        flux = F.rusanov_flux if problem == F.EULER_RUSANOV else F.hllc_flux
        return flux(QL, QR, phys["gamma"])
    H = np.zeros_like(QL)
    H[:, 11] = F.godunov_burgers(QL[:, 11], QR[:, 11])
    uf = 0.5 * (QL[:, 11] + QR[:, 11])
    pos = np.real(uf) >= 0
    for v in range(11):
        H[:, v] = uf * np.where(pos, QL[:, v], QR[:, v])
    return H


def fom_f2(problem, q, phys):
    """f of the second-order limited discretisation for one instance."""
    nv = F.NVAR[problem]
    Q = q.reshape(-1, nv)
    n = Q.shape[0]
    per = F.PERIODIC[problem]
    G = _ghosted(Q, per)
    H1 = face_flux(problem, G[1:-2], G[2:-1], phys)        # first-order faces -1/2 .. n-1/2
    QL, QR = limited_faces(Q, per)
    H2 = face_flux(problem, QL, QR, phys)
    dH = (H2[1:] - H2[:-1]) - (H1[1:] - H1[:-1])
    return (F.fom_f(problem, q, phys).reshape(n, nv) - dH * n).reshape(-1)


def ssprk43(L, y, dt):
    """One step of Spiteri and Ruuth's four-stage third-order SSP scheme."""
    y1 = y + 0.5 * dt * L(y)
    y2 = y1 + 0.5 * dt * L(y1)
    y3 = (2.0 / 3.0) * y + (1.0 / 3.0) * y2 + (dt / 6.0) * L(y2)
    return y3 + 0.5 * dt * L(y3)


def fom_step_explicit(problem, q, dt, phys):
    return ssprk43(lambda x: fom_f2(problem, x, phys), q, dt)


def fom_trajectory_explicit(problem, q0, dt, n_steps, phys):
    Q = [q0.copy()]
    q = q0.copy()
    for _ in range(n_steps):
        q = fom_step_explicit(problem, q, dt, phys)
        Q.append(q)
    return np.stack(Q, axis=1)


def galerkin_hr_explicit_step(problem, phys, q_ref, d, Phi, P, M, a, dt):
    """One SSPRK(4,3) step of eq. deim_galerkin_rom; P = None means no
    hyper-reduction (M = Phi^T over all rows)."""
    PhiD = Phi / d[:, None]

    def L(x):
        f = d * fom_f2(problem, q_ref + PhiD @ x, phys)
        return (Phi.T @ f) if P is None else M @ f[P]

    return ssprk43(L, a, dt)
