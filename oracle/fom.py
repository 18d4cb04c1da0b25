"""Oracle: the full-order model (FP64, NumPy/SciPy).  TEST INFRASTRUCTURE ONLY.

State layout: one instance is a flat vector of length N = n_cell * n_var,
cell-major (all variables of cell 0, then cell 1, ...), matching the
block-diagonal layout of the scaling matrix D (paper Sec. 3.1, eq.
scaling_matrix_local_block).

Every function below is written generically over real/complex dtype so that the
Jacobian can be taken by complex-step differentiation: every branch (max, min,
abs, upwinding) is decided on the real part, and the derivative follows the
branch the comparison chose; ties go to the first argument.

Definitions followed
  * semi-discrete system dq/dt = f(q)                 paper Sec. 2, eq. fom_continuous
  * backward-Euler residual r = q - q_prev - dt f(q)  paper Sec. 3.1, eq. be_residual_rom_section
    (the l = 1, alpha_1 = -1, beta_0 = 1 member of eq. fom_lmm)
  * Newton solve of r = 0, tolerance and cap           paper Sec. 5.1 setup (1e-8, 10 iterations)
  * Burgers: first-order upwind convection (read as the conservative Godunov
    flux of g(u) = u^2/2) + centred second difference, periodic     paper Sec. 5.1, eq. burgers_pde_results
  * Euler: cell-centred FV, Rusanov flux with interface speed
    max(|u_L|+c_L, |u_R|+c_R), zero-gradient ghosts, ideal gas       paper App. B, eqs. sod_*
  * Euler HLLC flux (not in the paper): Toro's HLLC with Davis wave-speed
    estimates, used by the 65,536-cell Sod workload
  * gradient of a final-state loss through a backward-Euler rollout (an
    extension beyond the paper): implicit-function adjoint of every step
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

BURGERS, EULER_RUSANOV, EULER_HLLC, REACT = 0, 1, 2, 3
NVAR = {BURGERS: 1, EULER_RUSANOV: 3, EULER_HLLC: 3, REACT: 12}
PERIODIC = {BURGERS: True, EULER_RUSANOV: False, EULER_HLLC: False, REACT: True}

# density / pressure floors used only when primitives are recovered (App. B:
# "small positive floors"; the value is this implementation's reading)
RHO_MIN = 1e-10
P_MIN = 1e-10


# ---------------------------------------------------------------- branch helpers
def cmax(a, b):
    """max(a, b) decided on real parts; ties return the first argument."""
    a, b = np.broadcast_arrays(np.asarray(a), np.asarray(b))
    return np.where(np.real(a) >= np.real(b), a, b)


def cmin(a, b):
    """min(a, b) decided on real parts; ties return the first argument."""
    a, b = np.broadcast_arrays(np.asarray(a), np.asarray(b))
    return np.where(np.real(a) <= np.real(b), a, b)


def cabs(a):
    return np.where(np.real(a) >= 0, a, -a)


# ---------------------------------------------------------------- Burgers
def godunov_burgers(a, b):
    """Godunov flux of g(u) = u^2/2 between left state a and right state b:
    F(a, b) = max(g(max(a, 0)), g(min(b, 0)))."""
    g1 = 0.5 * cmax(a, 0.0) ** 2
    g2 = 0.5 * cmin(b, 0.0) ** 2
    return cmax(g1, g2)


def burgers_f(u, nu, conv=1.0):
    """f(u) for viscous Burgers on the periodic unit interval, N cells.

    f_i = -(F_{i+1/2} - F_{i-1/2})/dx + nu ((u_{i+1}-u_i) - (u_i-u_{i-1}))/dx^2

    conv scales the convective part (1 in every workload; 0 gives pure diffusion,
    used only to pin the diffusion operator against its closed form)."""
    n = u.shape[0]
    dx = 1.0 / n
    up = np.roll(u, -1)
    F = godunov_burgers(u, up)                  # F[i] = F_{i+1/2}
    cterm = -conv * (F - np.roll(F, 1)) / dx
    du = up - u                                 # u_{i+1} - u_i
    diff = nu * (du - np.roll(du, 1)) / (dx * dx)
    return cterm + diff


# ---------------------------------------------------------------- Euler
def euler_primitives(U, gamma):
    """(rho_f, u, p, c) from conserved (rho, m, E) with floors applied on recovery."""
    rho, m, E = U[:, 0], U[:, 1], U[:, 2]
    rf = cmax(rho, RHO_MIN)
    u = m / rf
    p = cmax((gamma - 1.0) * (E - 0.5 * m * u), P_MIN)
    c = np.sqrt(gamma * p / rf)
    return rf, u, p, c


def euler_flux(U, gamma):
    """Physical flux F(U) = (m, m u + p, u (E + p))."""
    rf, u, p, c = euler_primitives(U, gamma)
    m, E = U[:, 1], U[:, 2]
    return np.stack([m, m * u + p, u * (E + p)], axis=1)


def rusanov_flux(UL, UR, gamma):
    """Local Lax-Friedrichs flux, App. B eqs. sod_rusanov_flux / sod_rusanov_speed."""
    _, uL, _, cL = euler_primitives(UL, gamma)
    _, uR, _, cR = euler_primitives(UR, gamma)
    s = cmax(cabs(uL) + cL, cabs(uR) + cR)
    FL = euler_flux(UL, gamma)
    FR = euler_flux(UR, gamma)
    return 0.5 * (FL + FR) - 0.5 * s[:, None] * (UR - UL)


def hllc_waves(UL, UR, gamma):
    """Wave speeds and star states of Toro's HLLC solver with Davis speeds
    S_L = min(u_L-c_L, u_R-c_R), S_R = max(u_L+c_L, u_R+c_R), the contact speed
    S* = (p_R - p_L + rho_L u_L (S_L-u_L) - rho_R u_R (S_R-u_R))
         / (rho_L (S_L-u_L) - rho_R (S_R-u_R))
    and U*_K = rho_K (S_K-u_K)/(S_K-S*) [1, S*, E_K/rho_K + (S*-u_K)(S* + p_K/(rho_K (S_K-u_K)))].
    Returns (SL, Ss, SR, UsL, UsR, FL, FR)."""
    rL, uL, pL, cL = euler_primitives(UL, gamma)
    rR, uR, pR, cR = euler_primitives(UR, gamma)
    SL = cmin(uL - cL, uR - cR)
    SR = cmax(uL + cL, uR + cR)
    num = pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)
    den = rL * (SL - uL) - rR * (SR - uR)
    FL = euler_flux(UL, gamma)
    FR = euler_flux(UR, gamma)
    with np.errstate(divide="ignore", invalid="ignore"):
        Ss = num / den

        def star(U, r, u, p, S):
            fac = r * (S - u) / (S - Ss)
            e = U[:, 2] / r + (Ss - u) * (Ss + p / (r * (S - u)))
            return np.stack([fac, fac * Ss, fac * e], axis=1)

        UsL = star(UL, rL, uL, pL, SL)
        UsR = star(UR, rR, uR, pR, SR)
    return SL, Ss, SR, UsL, UsR, FL, FR


def hllc_flux(UL, UR, gamma):
    """Toro's HLLC flux: F_L if S_L >= 0, F*_L = F_L + S_L (U*_L - U_L) if
    S_L < 0 <= S*, F*_R = F_R + S_R (U*_R - U_R) if S* < 0 <= S_R, else F_R."""
    SL, Ss, SR, UsL, UsR, FL, FR = hllc_waves(UL, UR, gamma)
    with np.errstate(divide="ignore", invalid="ignore"):
        FsL = FL + SL[:, None] * (UsL - UL)
        FsR = FR + SR[:, None] * (UsR - UR)
    sl = np.real(SL)[:, None]
    ss = np.real(Ss)[:, None]
    sr = np.real(SR)[:, None]
    return np.where(sl >= 0, FL, np.where(ss >= 0, FsL, np.where(sr >= 0, FsR, FR)))


def euler_f(U, gamma, flux):
    """f(U) = -(Fhat_{i+1/2} - Fhat_{i-1/2})/dx, zero-gradient ghosts (App. B)."""
    n = U.shape[0]
    dx = 1.0 / n
    Ug = np.concatenate([U[:1], U, U[-1:]], axis=0)     # ghost copies of end cells
    F = flux(Ug[:-1], Ug[1:], gamma)                    # n+1 faces, F[k] at x_{k-1/2}
    return -(F[1:] - F[:-1]) / dx


# ---------------------------------------------------------------- dispatch
def fom_f(problem, q, phys):
    """f(q) for one instance; q flat, cell-major.  phys: dict of physical constants."""
    if problem == BURGERS:
        return burgers_f(q, phys["nu"], phys.get("conv", 1.0))
    if problem in (EULER_RUSANOV, EULER_HLLC):
        U = q.reshape(-1, 3)
        flux = rusanov_flux if problem == EULER_RUSANOV else hllc_flux
        return euler_f(U, phys["gamma"], flux).reshape(-1)
    if problem == REACT:
        from . import react
        return react.react_f(q.reshape(-1, 12), phys).reshape(-1)
    raise ValueError("unknown problem %r" % (problem,))


def be_residual(problem, q, q_prev, dt, phys):
    """Backward-Euler residual r = q - q_prev - dt f(q) (eq. be_residual_rom_section)."""
    return q - q_prev - dt * fom_f(problem, q, phys)


def _n_colors(n_cell):
    for k in (3, 4, 5, 6, 7):
        if n_cell % k == 0:
            return k
    return n_cell


def jacobian_f(problem, q, phys, h=1e-30):
    """Exact J_f = df/dq as a sparse matrix, by complex-step differentiation.

    The stencil of every problem couples a cell only to its two neighbours, so
    columns are grouped by (cell mod K, variable) with K >= 3 dividing the cell
    count (also correct for periodic wrap); each group costs one complex f."""
    nv = NVAR[problem]
    n = q.shape[0]
    nc = n // nv
    if nc < 3:
        raise ValueError("the three-cell stencil needs at least 3 cells")
    K = _n_colors(nc)
    cell = np.arange(n) // nv
    var = np.arange(n) % nv
    rows, cols, vals = [], [], []
    for col in range(K):
        for v in range(nv):
            sel = (cell % K == col) & (var == v)
            qc = q.astype(np.complex128)
            qc[sel] += 1j * h
            df = np.imag(fom_f(problem, qc, phys)) / h
            # row i (cell ci) was perturbed through the unique selected column in
            # cells ci-1, ci, ci+1 (periodic wrap); attribute to that column.
            ci = np.arange(n) // nv
            for off in (-1, 0, 1):
                cj = (ci + off) % nc
                ok = (cj % K == col)
                if K == nc:
                    ok = ok & ((ci + off) % nc == cj)
                jcol = cj * nv + v
                nz = ok & (df != 0.0)
                rows.append(np.nonzero(nz)[0])
                cols.append(jcol[nz])
                vals.append(df[nz])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def jacobian_be(problem, q, dt, phys):
    """J_r = I - dt J_f (eq. be_residual_jacobian_rom_section)."""
    n = q.shape[0]
    return (sp.identity(n, format="csr") - dt * jacobian_f(problem, q, phys)).tocsr()


def newton_be_step(problem, q_prev, dt, phys, tol=1e-8, max_it=10, fixed_iters=False):
    """One backward-Euler step solved by Newton with an exact direct linear solve.

    Iteration: r = r(q); stop if ||r||_inf <= tol; else solve J_r delta = -r and
    q += delta.  At most max_it solves; the initial guess is q_prev.  With
    fixed_iters the stopping test is skipped and exactly max_it solves run.
    Returns (q, n_solves, converged)."""
    q = q_prev.copy()
    for it in range(max_it):
        r = be_residual(problem, q, q_prev, dt, phys)
        if not fixed_iters and np.max(np.abs(r)) <= tol:
            return q, it, True
        J = jacobian_be(problem, q, dt, phys)
        delta = spla.spsolve(J.tocsc(), -r)
        q = q + delta
    if fixed_iters:
        return q, max_it, True
    r = be_residual(problem, q, q_prev, dt, phys)
    return q, max_it, bool(np.max(np.abs(r)) <= tol)


def fom_trajectory(problem, q0, dt, n_steps, phys, tol=1e-8, max_it=10):
    """Fine FOM trajectory [q^0, q^1, ..., q^n_steps] (columns)."""
    Q = [q0.copy()]
    q = q0.copy()
    for _ in range(n_steps):
        q, _, _ = newton_be_step(problem, q, dt, phys, tol, max_it)
        Q.append(q)
    return np.stack(Q, axis=1)


def be_rollout_vjp(problem, q0, dt, n_steps, phys, gbar, tol=1e-8, max_it=10):
    """Gradient of L(q^T) through a backward-Euler rollout q^{k+1} = S(q^k):
    dL/dq^0 = J_r(q^1)^-T ... J_r(q^T)^-T dL/dq^T, where each step's sensitivity
    dq^{k+1}/dq^k = J_r(q^{k+1})^-1 follows from differentiating the converged
    residual q^{k+1} - q^k - dt f(q^{k+1}) = 0 (eq. be_residual_rom_section).
    Every state is kept; the transposed systems are solved exactly."""
    Q = fom_trajectory(problem, q0, dt, n_steps, phys, tol, max_it)
    g = np.asarray(gbar, dtype=np.float64).copy()
    for k in range(n_steps - 1, -1, -1):
        J = jacobian_be(problem, Q[:, k + 1], dt, phys)
        g = spla.spsolve(J.T.tocsc(), g)
    return g


def vjp_f(problem, q, w, phys):
    """Vector-Jacobian product J_f(q)^T w."""
    return jacobian_f(problem, q, phys).T @ w
