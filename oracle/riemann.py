"""Oracle: exact Riemann solver for the 1-D Euler equations (ideal gas).
TEST INFRASTRUCTURE ONLY.

Used to pin the Euler full-order model against the exact Sod solution (paper
Sec. 5.2 / App. B use the Sod problem; the exact solver follows the standard
construction in Toro, "Riemann Solvers and Numerical Methods for Fluid
Dynamics", ch. 4: pressure function f_L + f_R + du = 0 solved by Newton,
then sampling of the self-similar solution).
"""
import numpy as np


def _fk(p, rk, pk, ck, gamma):
    """Pressure function of one side and its derivative (shock if p > pk, else rarefaction)."""
    if p > pk:
        A = 2.0 / ((gamma + 1.0) * rk)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        s = np.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (p + B))
    pr = p / pk
    f = 2.0 * ck / (gamma - 1.0) * (pr ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
    df = 1.0 / (rk * ck) * pr ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(WL, WR, gamma=1.4, tol=1e-15, max_it=100):
    """(p*, u*) of the Riemann problem with primitive states W = (rho, u, p)."""
    rL, uL, pL = WL
    rR, uR, pR = WR
    cL = np.sqrt(gamma * pL / rL)
    cR = np.sqrt(gamma * pR / rR)
    p = max(tol, 0.5 * (pL + pR))
    for _ in range(max_it):
        fL, dL = _fk(p, rL, pL, cL, gamma)
        fR, dR = _fk(p, rR, pR, cR, gamma)
        dp = (fL + fR + uR - uL) / (dL + dR)
        p_new = max(tol, p - dp)
        if abs(p_new - p) <= tol * 0.5 * (p_new + p):
            p = p_new
            break
        p = p_new
    fL, _ = _fk(p, rL, pL, cL, gamma)
    fR, _ = _fk(p, rR, pR, cR, gamma)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    return p, u


def star_densities(WL, WR, gamma=1.4):
    p, u = star_state(WL, WR, gamma)
    out = []
    for (rk, _, pk) in (WL, WR):
        if p > pk:
            g = (gamma - 1.0) / (gamma + 1.0)
            out.append(rk * (p / pk + g) / (g * p / pk + 1.0))
        else:
            out.append(rk * (p / pk) ** (1.0 / gamma))
    return p, u, out[0], out[1]


def sample(WL, WR, xi, gamma=1.4):
    """Primitive solution (rho, u, p) at similarity coordinates xi = (x - x0)/t."""
    rL, uL, pL = WL
    rR, uR, pR = WR
    cL = np.sqrt(gamma * pL / rL)
    cR = np.sqrt(gamma * pR / rR)
    ps, us, rsL, rsR = star_densities(WL, WR, gamma)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for k, s in enumerate(xi):
        if s <= us:                                    # left of contact
            if ps > pL:                                # left shock
                SL = uL - cL * np.sqrt((gamma + 1) / (2 * gamma) * ps / pL + (gamma - 1) / (2 * gamma))
                W = (rL, uL, pL) if s <= SL else (rsL, us, ps)
            else:                                      # left rarefaction
                SHL = uL - cL
                cs = cL * (ps / pL) ** ((gamma - 1) / (2 * gamma))
                STL = us - cs
                if s <= SHL:
                    W = (rL, uL, pL)
                elif s >= STL:
                    W = (rsL, us, ps)
                else:
                    c = 2.0 / (gamma + 1) * (cL + 0.5 * (gamma - 1) * (uL - s))
                    uu = 2.0 / (gamma + 1) * (cL + 0.5 * (gamma - 1) * uL + s)
                    rr = rL * (c / cL) ** (2.0 / (gamma - 1))
                    W = (rr, uu, pL * (c / cL) ** (2 * gamma / (gamma - 1)))
        else:                                          # right of contact
            if ps > pR:                                # right shock
                SR = uR + cR * np.sqrt((gamma + 1) / (2 * gamma) * ps / pR + (gamma - 1) / (2 * gamma))
                W = (rR, uR, pR) if s >= SR else (rsR, us, ps)
            else:                                      # right rarefaction
                SHR = uR + cR
                cs = cR * (ps / pR) ** ((gamma - 1) / (2 * gamma))
                STR = us + cs
                if s >= SHR:
                    W = (rR, uR, pR)
                elif s <= STR:
                    W = (rsR, us, ps)
                else:
                    c = 2.0 / (gamma + 1) * (cR - 0.5 * (gamma - 1) * (uR - s))
                    uu = 2.0 / (gamma + 1) * (-cR + 0.5 * (gamma - 1) * uR + s)
                    rr = rR * (c / cR) ** (2.0 / (gamma - 1))
                    W = (rr, uu, pR * (c / cR) ** (2 * gamma / (gamma - 1)))
        rho[k], u[k], p[k] = W
    del g1
    return rho, u, p


def shock_speed_right(WL, WR, gamma=1.4):
    rR, uR, pR = WR
    cR = np.sqrt(gamma * pR / rR)
    ps, _ = star_state(WL, WR, gamma)
    return uR + cR * np.sqrt((gamma + 1) / (2 * gamma) * ps / pR + (gamma - 1) / (2 * gamma))
