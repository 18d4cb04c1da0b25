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

rollout_vjp extends this to the gradient with respect to the initial state q0
of Alg. 1 as a whole, with hyper-reduced LSPG steps (the sample schedule
recorded and held fixed): an HR-LSPG step by the implicit-function theorem on
its vanishing weighted residual (no second derivatives), the adjoint of
(P^T Phi)^+, the q_ref and D terms of every step, event and the loss, and the
offline stage (a^{w_init}, the first coarse step, the truncated POD's SVD
adjoint, the preprocessing's scale and the training BE steps).  Checked
against central finite differences of rollout_forward.
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


def _event_vjp(problem, phys, st, prm, it, ab, Phib, sb, yb, extra=None):
    """Reverse of one adaptation event (closed-form transfer, rotation, core SVD,
    CGS2, preprocessing, coarse step).  With extra (a dict holding "qrb" and
    "db", the gradients of q_ref and of the diagonal of D), the preprocessing
    yhat = D (y_new - q_ref) also adds its terms to them."""
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
    if extra is not None:
        extra["qrb"] -= d * yhatb
        extra["db"] += yhatb * (it["y_new"] - st["q_ref"])
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


# ------------------------------------------------------------------ whole rollout
# The gradient of a final-state loss with respect to the initial state q0,
# through Alg. 1 as a whole: the offline stage (training BE steps,
# preprocessing, POD, a^{w_init}, the first coarse step) and the online loop
# with hyper-reduced LSPG steps.  The sample rows are piecewise constant in
# q0, so they are recorded in a forward run and held fixed (a P schedule);
# q_ref = q0 and D are differentiated.  Re-orthonormalisation must not fire
# (reorth_every = 0).

def rollout_forward(problem, phys, q0, prm, n_steps, P_sched=None, record=False):
    """Alg. 1 from q0: the offline stage, then n_steps fine HR-LSPG steps with
    events when due (closed-form transfer).  Sample rows come from P_sched
    (one array per rebuild, the offline one first) when given.  Returns
    (state, record, P_sched)."""
    if prm["hyper"] == "none":
        raise ValueError("the rollout adjoint covers the hyper-reduced LSPG path")
    nv = F.NVAR[problem]
    r, dt, z, w = prm["r"], prm["dt"], prm["z"], prm["w_init"]
    tol, mx = prm["newton_tol"], prm["newton_max"]
    Q = F.fom_trajectory(problem, q0, dt, w, phys, tol, mx)
    Qt = Q[:, 1:]
    q_ref, d_var = O.preprocess(Qt, q0, nv)
    d = O.dfull(d_var, q0.shape[0] // nv)
    Xh = d[:, None] * (Qt - q_ref[:, None])
    Phi, sigma = O.pod(Xh, r)
    q_last = Qt[:, -1]
    a = Phi.T @ (d * (q_last - q_ref))
    y0, _, _ = F.newton_be_step(problem, q_last, z * dt, phys, tol, mx)
    sched = [] if P_sched is None else list(P_sched)
    k_rb = 0

    def rows(Phi_, y_):
        nonlocal k_rb
        if P_sched is not None:
            P = np.asarray(P_sched[k_rb])
        else:
            P = O.sample_rows(problem, Phi_, y_, prm)
            sched.append(P)
        k_rb += 1
        return P

    P = rows(Phi, y0)
    st = dict(q_ref=q_ref, d_var=d_var, d=d, Phi=Phi, sigma=sigma, a=a, y_corr=y0,
              P=P, M=O.rebuild(Phi, P))
    off = dict(Q=Q, Xh=Xh, d_var=d_var, q_last=q_last, a0=a, Phi0=Phi, y0=y0)
    rec = []
    for n in range(w, w + n_steps):
        a_prev = st["a"]
        a_new, _, ok = O.hr_lspg_step(problem, phys, q_ref, d, st["Phi"], st["P"], st["M"],
                                      a_prev, dt, prm["rom_tol"], prm["rom_max"])
        if record:
            rec.append(("step", dict(a_prev=a_prev, a_new=a_new, Phi=st["Phi"], P=st["P"],
                                     M=st["M"])))
        st["a"] = a_new
        if _event_due(n, prm):
            y_prev = st["y_corr"]
            y_new, _, _ = F.newton_be_step(problem, y_prev, z * dt, phys, tol, mx)
            yhat = d * (y_new - q_ref)
            Phi_old, sig_old, a_old = st["Phi"], st["sigma"], st["a"]
            Phi_new, sig_new, info = O.isvd_update(Phi_old, sig_old, yhat, prm["lam"], r,
                                                   prm["tau_rho"])
            if record:
                rec.append(("event", dict(Phi_old=Phi_old, sig_old=sig_old, a_old=a_old,
                                          y_prev=y_prev, y_new=y_new, yhat=yhat, info=info)))
            P = rows(Phi_new, y_new)
            st.update(Phi=Phi_new, sigma=sig_new, a=info["Ubar"][:r, :r].T @ a_old,
                      y_corr=y_new, P=P, M=O.rebuild(Phi_new, P))
    st["offline"] = off
    return st, rec, sched


def rollout_loss(problem, phys, q0, prm, n_steps, q_tgt, P_sched):
    """L = 1/2 |q~_end - q_tgt|^2 with the sample schedule held fixed."""
    out, _, _ = rollout_forward(problem, phys, q0, prm, n_steps, P_sched)
    qt = O.reconstruct(out["q_ref"], out["d"], out["Phi"], out["a"])
    return 0.5 * float(np.sum((qt - q_tgt) ** 2))


def _pinv_vjp(A, M, Mb):
    """Reverse of M = A^+ for a full-column-rank A (n_s x r):
    Abar = -M^T Mbar M^T + (I - A M) Mbar^T M M^T."""
    return -M.T @ Mb @ M.T + (np.eye(A.shape[0]) - A @ M) @ Mb.T @ (M @ M.T)


def _hr_step_vjp(problem, phys, fixed, prm, it, ab, Phib, qrb, db):
    """Reverse of one HR-LSPG step by the implicit-function theorem.  At the
    converged a_{n+1} the weighted residual b(a) = M P^T D r(q~(a)) vanishes;
    since M P^T Phi = I it equals (a - a_n) - dt M P^T D f(q~(a)), so
    lambda = J_b^-T abar with the Gauss-Newton matrix J_b = M P^T D J_r D^-1 Phi,
    abar_n = lambda, and Phi, q_ref and D receive dt (d(M g)/d theta)^T lambda
    with g = P^T D f(q~): through M = (P^T Phi)^+ and through f at q~."""
    d, q_ref, dt = fixed["d"], fixed["q_ref"], prm["dt"]
    Phi, a1, P, M = it["Phi"], it["a_new"], it["P"], it["M"]
    PhiD = Phi / d[:, None]
    qt = q_ref + PhiD @ a1
    f = F.fom_f(problem, qt, phys)
    Jf = F.jacobian_f(problem, qt, phys)
    Jr = F.jacobian_be(problem, qt, dt, phys)
    As = (d[:, None] * (Jr @ PhiD))[P, :]
    lam = np.linalg.solve((M @ As).T, ab)
    g = d[P] * f[P]
    Ab = _pinv_vjp(Phi[P, :], M, dt * np.outer(lam, g))
    Phib = Phib.copy()
    Phib[P, :] += Ab
    gb = dt * (M.T @ lam)
    db = db.copy()
    db[P] += gb * f[P]
    fb = np.zeros_like(f)
    fb[P] = gb * d[P]
    qtb = Jf.T @ fb
    Phib += np.outer(qtb / d, a1)
    db -= qtb * (Phi @ a1) / d ** 2
    return lam, Phib, qrb + qtb, db


def _pod_vjp(Xh, Phi, Phib, sb):
    """Reverse of (Phi, sigma) = the leading r left singular vectors and values
    of Xh (N x w, distinct nonzero singular values): with the thin SVD
    Xh = U S V^T (U's first r columns equal to Phi), Ubar = [Phibar, 0] and
    sbar padded with zeros,
    Xbar = U (F o (U^T Ubar - Ubar^T U) S + diag(sbar)) V^T + (I - U U^T) Ubar S^-1 V^T,
    F_ij = 1/(s_j^2 - s_i^2) (i != j)."""
    U, s, Vt = np.linalg.svd(Xh, full_matrices=False)
    r = Phi.shape[1]
    sg = np.sign(np.sum(U[:, :r] * Phi, axis=0))
    U[:, :r] *= sg[None, :]
    Vt[:r, :] *= sg[:, None]
    w = s.shape[0]
    Ub = np.zeros_like(U)
    Ub[:, :r] = Phib
    sbf = np.zeros(w)
    sbf[:r] = sb
    Mm = U.T @ Ub
    G = np.diag(sbf)
    for i in range(w):
        for j in range(w):
            if i != j:
                G[i, j] += (Mm[i, j] - Mm[j, i]) * s[j] / (s[j] ** 2 - s[i] ** 2)
    Xb = U @ G @ Vt + (Ub - U @ (U.T @ Ub)) @ (Vt / s[:, None])
    return Xb


def rollout_vjp(problem, phys, q0, prm, n_steps, qbar, P_sched=None):
    """Gradient of <qbar, q~_end> with respect to q0 through Alg. 1 (offline
    stage and online HR-LSPG loop), the sample schedule held fixed.
    Returns (q0bar, P_sched)."""
    nv = F.NVAR[problem]
    out, rec, sched = rollout_forward(problem, phys, q0, prm, n_steps, P_sched, record=True)
    off = out["offline"]
    r, dt, z = prm["r"], prm["dt"], prm["z"]
    d, q_ref = out["d"], out["q_ref"]
    fixed = dict(d=d, q_ref=q_ref)
    # seed: q~ = q_ref + D^-1 Phi a
    ab = out["Phi"].T @ (qbar / d)
    Phib = np.outer(qbar / d, out["a"])
    qrb = qbar.copy()
    db = -qbar * (out["Phi"] @ out["a"]) / d ** 2
    sb = np.zeros(r)
    yb = np.zeros_like(q0)
    extra = dict(qrb=qrb, db=db)
    for kind, it in reversed(rec):
        if kind == "step":
            ab, Phib, extra["qrb"], extra["db"] = _hr_step_vjp(problem, phys, fixed, prm, it, ab,
                                                               Phib, extra["qrb"], extra["db"])
        else:
            ab, Phib, sb, yb = _event_vjp(problem, phys, fixed, prm, it, ab, Phib, sb, yb, extra)
    qrb, db = extra["qrb"], extra["db"]
    Q, Xh, q_last = off["Q"], off["Xh"], off["q_last"]
    w = Q.shape[1] - 1
    Qb = np.zeros_like(Q)
    # a = Phi^T D (q_last - q_ref)
    t = off["Phi0"] @ ab
    Phib = Phib + np.outer(d * (q_last - q_ref), ab)
    Qb[:, w] += d * t
    qrb = qrb - d * t
    db = db + t * (q_last - q_ref)
    # y_corr = BE(q_last) over z dt
    Jr = F.jacobian_be(problem, off["y0"], z * dt, phys)
    Qb[:, w] += spla.spsolve(Jr.T.tocsc(), yb)
    # (Phi, sigma) = POD of Xh = D (Q_train - q_ref)
    Xb = _pod_vjp(Xh, off["Phi0"], Phib, sb)
    Xc = Q[:, 1:] - q_ref[:, None]
    Qb[:, 1:] += d[:, None] * Xb
    qrb = qrb - np.sum(d[:, None] * Xb, axis=1)
    db = db + np.sum(Xb * Xc, axis=1)
    # d_var[v] = 1 / phi_v, phi_v = mean of Xc^2 over the cells and snapshots of v
    n_cell = q0.shape[0] // nv
    dvb = db.reshape(n_cell, nv).sum(axis=0)
    phib = -dvb * off["d_var"] ** 2
    Xv = Xc.reshape(n_cell, nv, w)
    phi = np.mean(Xv ** 2, axis=(0, 2))
    phib = np.where(phi == 0.0, 0.0, phib)
    Xcb = (2.0 / (n_cell * w)) * Xv * phib[None, :, None]
    Qb[:, 1:] += Xcb.reshape(-1, w)
    qrb = qrb - Xcb.reshape(-1, w).sum(axis=1)
    # training steps Q_j = BE(Q_{j-1}), q_ref = q0
    for j in range(w, 0, -1):
        Jr = F.jacobian_be(problem, Q[:, j], dt, phys)
        Qb[:, j - 1] += spla.spsolve(Jr.T.tocsc(), Qb[:, j])
    return Qb[:, 0] + qrb, sched
