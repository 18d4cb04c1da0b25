"""Oracle: reverse mode of Alg. 1's online loop (FP64).  TEST INFRASTRUCTURE ONLY.

Not in the paper: the gradient of a loss on the adaptive ROM's reconstructed
state with respect to the online state it starts from.  The forward pass is
Alg. 1's online loop for the Galerkin projection (no hyper-reduction, no
re-orthonormalisation):

  fine step     a_{n+1} solves g(a) = a - a_n - dt Phi^T D f(q_ref + D^-1 Phi a) = 0
                (galerkin_step, eq. galerkin_continuous_rom with backward Euler)
  event         y <- BE(y) over z dt (eq. coarse_fom_backward_euler);
                yhat = D (y - q_ref);  Alg. 2: CGS2 projection p = p1 + p2,
                q = yhat - Phi p1 - Phi p2, rho = |q|, core K, its SVD K = Ubar
                Sbar Vbar^T, Phi' = [Phi, q / rho] Ubar[:, :r], sigma' = Sbar[:r];
                state transfer in closed form a' = Ubar[:r, :r]^T a (equal to
                Phi'^T Phi a when q is orthogonal to Phi)

The reverse pass walks the recorded trajectory backwards.  A fine step is
differentiated by the implicit-function theorem at the converged a_{n+1}:
lambda = J_g^-T abar, abar_n = lambda, and Phi receives
dt (D f) lambda^T + dt D^-1 J_f^T (D Phi lambda) a_{n+1}^T.  The core SVD is
differentiated by the standard formula for distinct singular values; the
coarse step by a transposed solve with J_r = I - z dt J_f at the new y.
Functions are checked against central finite differences of online_forward.
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import fom as F
from . import rom as O


def _event_due(n, prm):
    return (n + 1 - prm["w_init"]) % prm["z"] == 0


def online_forward(problem, phys, st, prm, n0, n_steps, record=False):
    """Runs fine steps n0 .. n0 + n_steps - 1 of Alg. 1 (events when due) on a
    copy of st (keys Phi, sigma, a, y_corr, q_ref, d).  Returns (state, record)."""
    st = {k: (np.array(v, dtype=np.float64, copy=True) if isinstance(v, np.ndarray) else v)
          for k, v in st.items()}
    r, dt, z = prm["r"], prm["dt"], prm["z"]
    rec = []
    for n in range(n0, n0 + n_steps):
        a_prev = st["a"]
        a_new, _, ok = O.galerkin_step(problem, phys, st["q_ref"], st["d"], st["Phi"], a_prev,
                                       dt, prm["rom_tol"], prm["rom_max"])
        if record:
            rec.append(("step", dict(a_prev=a_prev, a_new=a_new, Phi=st["Phi"])))
        st["a"] = a_new
        if _event_due(n, prm):
            y_prev = st["y_corr"]
            y_new, _, _ = F.newton_be_step(problem, y_prev, z * dt, phys, prm["newton_tol"],
                                           prm["newton_max"])
            yhat = st["d"] * (y_new - st["q_ref"])
            Phi_old, sig_old, a_old = st["Phi"], st["sigma"], st["a"]
            Phi_new, sig_new, info = O.isvd_update(Phi_old, sig_old, yhat, prm["lam"], r,
                                                   prm["tau_rho"])
            a_new = info["Ubar"][:r, :r].T @ a_old
            if record:
                rec.append(("event", dict(Phi_old=Phi_old, sig_old=sig_old, a_old=a_old,
                                          y_prev=y_prev, y_new=y_new, yhat=yhat, info=info)))
            st.update(Phi=Phi_new, sigma=sig_new, a=a_new, y_corr=y_new)
    return st, rec


def online_loss(problem, phys, st, prm, n0, n_steps, q_tgt):
    """L = 1/2 |q~_end - q_tgt|^2 after the online loop."""
    out, _ = online_forward(problem, phys, st, prm, n0, n_steps)
    qt = O.reconstruct(out["q_ref"], out["d"], out["Phi"], out["a"])
    return 0.5 * float(np.sum((qt - q_tgt) ** 2))


def _step_vjp(problem, phys, st, prm, it, ab, Phib):
    """Reverse of one fine Galerkin step (implicit-function theorem at a_{n+1})."""
    d, q_ref, dt = st["d"], st["q_ref"], prm["dt"]
    Phi, a1 = it["Phi"], it["a_new"]
    PhiD = Phi / d[:, None]
    qt = q_ref + PhiD @ a1
    f = F.fom_f(problem, qt, phys)
    Jf = F.jacobian_f(problem, qt, phys)
    r = Phi.shape[1]
    Jg = np.eye(r) - dt * (Phi.T @ (d[:, None] * (Jf @ PhiD)))
    lam = np.linalg.solve(Jg.T, ab)
    w = Jf.T @ (d * (Phi @ lam))
    Phib = Phib + dt * np.outer(d * f, lam) + dt * np.outer(w / d, a1)
    return lam, Phib


def _svd_vjp(K, U, s, Ub, sb):
    """Reverse of K = U diag(s) V^T (square, distinct s) for the outputs U and
    s: Kbar = U G V^T with G_ii = sbar_i and, for i != j,
    G_ij = s_j (M_ij - M_ji) / (s_j^2 - s_i^2), M = U^T Ubar.  V = K^T U / s for
    the columns with s_j > 0; the others carry no gradient (G_ij = 0)."""
    n = K.shape[0]
    M = U.T @ Ub
    G = np.zeros((n, n))
    V = np.zeros((n, n))
    for j in range(n):
        if s[j] > 0.0:
            V[:, j] = K.T @ U[:, j] / s[j]
        for i in range(n):
            if i == j:
                G[i, i] = sb[i]
            elif s[j] > 0.0:
                G[i, j] = s[j] * (M[i, j] - M[j, i]) / (s[j] ** 2 - s[i] ** 2)
    return U @ G @ V.T


def _event_vjp(problem, phys, st, prm, it, ab, Phib, sb, yb):
    """Reverse of one adaptation event (closed-form transfer, rotation, core SVD,
    CGS2, preprocessing, coarse step)."""
    r, lam_f, dt, z, d = prm["r"], prm["lam"], prm["dt"], prm["z"], st["d"]
    info = it["info"]
    if info["degenerate"]:
        raise ValueError("rho = 0 at an event: the update is not differentiable there")
    Phi, yhat, a_old = it["Phi_old"], it["yhat"], it["a_old"]
    U, s, K = info["Ubar"], info["sbar"], info["K"]
    n = r + 1
    # CGS2 intermediates
    p1 = Phi.T @ yhat
    q1 = yhat - Phi @ p1
    p2 = Phi.T @ q1
    q = q1 - Phi @ p2
    rho = np.linalg.norm(q)
    j = q / rho
    # transfer a' = U[:r, :r]^T a
    Ub = np.zeros((n, n))
    Ub[:r, :r] += np.outer(a_old, ab)
    ab_old = U[:r, :r] @ ab
    # rotation Phi' = [Phi, j] U[:, :r]
    Phib_old = Phib @ U[:r, :r].T
    jb = Phib @ U[r, :r]
    Ub[:r, :r] += Phi.T @ Phib
    Ub[r, :r] += j @ Phib
    # truncation sigma' = s[:r]
    sbf = np.zeros(n)
    sbf[:r] = sb
    Kb = _svd_vjp(K, U, s, Ub, sbf)
    # K = [[lam diag sigma, p], [0, rho]]
    sb_old = lam_f * np.diag(Kb)[:r]
    pb = Kb[:r, r]
    rhob = Kb[r, r]
    # j = q / rho and rho = |q|
    qb = jb / rho
    rhob = rhob - float(jb @ q) / rho ** 2
    qb = qb + rhob * q / rho
    # CGS2 with p = p1 + p2
    p1b = pb.copy()
    p2b = pb.copy()
    q1b = qb.copy()                              # q = q1 - Phi p2
    Phib_old -= np.outer(qb, p2)
    p2b -= Phi.T @ qb
    Phib_old += np.outer(q1, p2b)                # p2 = Phi^T q1
    q1b += Phi @ p2b
    yhatb = q1b.copy()                           # q1 = yhat - Phi p1
    Phib_old -= np.outer(q1b, p1)
    p1b -= Phi.T @ q1b
    Phib_old += np.outer(yhat, p1b)              # p1 = Phi^T yhat
    yhatb += Phi @ p1b
    # yhat = D (y_new - q_ref); y_new = BE(y_prev) over z dt
    yb_new = yb + d * yhatb
    Jr = F.jacobian_be(problem, it["y_new"], z * dt, phys)
    yb_prev = spla.spsolve(Jr.T.tocsc(), yb_new)
    return ab_old, Phib_old, sb_old, yb_prev


def online_vjp(problem, phys, st, prm, n0, n_steps, qbar):
    """Gradient of <qbar, q~_end> through the online loop: returns
    (abar, Phibar, sigmabar, ycorrbar) with respect to the starting a, Phi,
    sigma and y_corr (q_ref and D held fixed)."""
    out, rec = online_forward(problem, phys, st, prm, n0, n_steps, record=True)
    d = out["d"]
    ab = out["Phi"].T @ (qbar / d)
    Phib = np.outer(qbar / d, out["a"])
    sb = np.zeros_like(out["sigma"])
    yb = np.zeros_like(out["y_corr"])
    for kind, it in reversed(rec):
        if kind == "step":
            ab, Phib = _step_vjp(problem, phys, st, prm, it, ab, Phib)
        else:
            ab, Phib, sb, yb = _event_vjp(problem, phys, st, prm, it, ab, Phib, sb, yb)
    return ab, Phib, sb, yb
