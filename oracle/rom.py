"""Oracle: reduced-order model pieces and the adaptive driver (FP64).  TEST INFRASTRUCTURE ONLY.

Each function follows one passage of the paper, in its order and notation:
  preprocess          Sec. 3.1: q_ref = initial state; D = blockdiag of 1/phi_v,norm,
                      phi_v,norm = mean over training snapshots and cells of the
                      squared centred field (eq. variable_normalization, read
                      literally: no square root; centred about q_ref)
  pod                 Sec. 3.1 / Alg. 1 (POD of D(Q_train - q_ref 1^T), leading r)
  isvd_update         Alg. 2 with eqs. isvd_residual .. isvd_truncation; p by
                      classical Gram-Schmidt applied twice (equals Phi^+ y for
                      orthonormal Phi); rho -> 0 guard; SVD of the core K
                      (isvd_core), then the rotation and truncation (isvd_rotate)
  reorth              re-orthonormalisation schedule (not in the paper, which
                      states none is needed; kept as a guard for FP32 storage)
  deim_greedy         greedy DEIM (the interpolation-residual argmax rule of the
                      DEIM reference cited in Sec. 3.2), oversampled to n_s rows
                      by a second least-squares greedy round
  qdeim               QDEIM: pivots of the column-pivoted QR of Phi^T (eq. qdeim_qr)
  fgs                 feature-guided sampling: QDEIM plus the cells of largest
                      feature gradient of the estimated future state (eq. fgs_selection)
  rebuild             (P^T Phi)^+ (eq. qdeim_approximation_phi)
  galerkin_step       backward Euler applied to eq. galerkin_continuous_rom
  hr_lspg_step        Gauss-Newton on eq. hyperreduced_lspg
  wsvd_update         App. A, Alg. A.1 (windowed SVD over the last w snapshots)
  direct_update       App. A, Alg. A.2 (the Direct rule), with orth() read as the
                      Q factor of the thin QR with a positive diagonal of R
  coarse_step         eq. coarse_fom_backward_euler, or the explicit path's SSPRK(4,3)
                      step of size z dt (explicit.py)
  transfer            Alg. 1 state transfer a <- Phi_new^T D (q~ - q_ref)
  adaptive_rom        Alg. 1

Sign convention for singular vectors: a column's entry of largest magnitude is
made positive (lowest index on ties).  Descending singular values.
"""
import numpy as np

from . import explicit as X
from . import fom as F


# ------------------------------------------------------------------ helpers
def sign_fix(U):
    """Flip columns so that each column's largest-|.| entry (first on ties) is positive."""
    U = U.copy()
    idx = np.argmax(np.abs(U), axis=0)
    s = np.sign(U[idx, np.arange(U.shape[1])])
    s[s == 0] = 1.0
    return U * s[None, :]


def dfull(d_var, n_cell):
    """Diagonal of D as a length-N vector (cell-major) from the per-variable scales."""
    return np.tile(np.asarray(d_var, dtype=np.float64), n_cell)


# ------------------------------------------------------------------ Sec. 3.1
def preprocess(Q_train, q0, n_var):
    """(q_ref, d_var): q_ref = q0; d_var[v] = 1/phi_v,norm with phi_v,norm the mean
    of (q_v - q_ref,v)^2 over all cells and training snapshots (1 if zero)."""
    q_ref = np.array(q0, dtype=np.float64)
    X = Q_train - q_ref[:, None]
    n = q_ref.shape[0]
    Xv = X.reshape(n // n_var, n_var, X.shape[1])
    phi = np.mean(Xv ** 2, axis=(0, 2))
    phi = np.where(phi == 0.0, 1.0, phi)
    return q_ref, 1.0 / phi


def pod(Xhat, r):
    """Leading r left singular vectors / values of the preprocessed training matrix."""
    U, s, _ = np.linalg.svd(Xhat, full_matrices=False)
    return sign_fix(U[:, :r]), s[:r].copy()


# ------------------------------------------------------------------ Alg. 2
def isvd_core(Phi, sigma, yhat, lam, tau_rho=1e-12):
    """The first half of one Brand update (Alg. 2): the projection p and the
    residual q by two passes of classical Gram-Schmidt (p = Phi^+ yhat for
    orthonormal Phi, eq. isvd_residual), rho = ||q|| with the rho -> 0 guard,
    the core K (eq. isvd_core_matrix) and its left singular vectors Ubar
    (sign-fixed, descending order) and values sbar.  Returns a dict."""
    N, k = Phi.shape
    p = Phi.T @ yhat
    q = yhat - Phi @ p
    p2 = Phi.T @ q
    q = q - Phi @ p2
    p = p + p2
    rho = np.linalg.norm(q)
    degenerate = rho <= tau_rho * np.linalg.norm(yhat)
    if degenerate:
        rho = 0.0
    K = np.zeros((k + 1, k + 1))
    K[:k, :k] = lam * np.diag(sigma)
    K[:k, k] = p
    K[k, k] = rho
    if degenerate:
        # the residual direction carries nothing: decompose the k x (k+1) block
        # [lambda Sigma, p] so that only directions inside span(Phi) can be kept
        Uk, sk, _ = np.linalg.svd(K[:k, :])
        Ub = np.zeros((k + 1, k + 1))
        Ub[:k, :k] = sign_fix(Uk)
        Ub[k, k] = 1.0
        sb = np.concatenate([sk, [0.0]])
    else:
        Ub, sb, _ = np.linalg.svd(K)
        Ub = sign_fix(Ub)
    return dict(p=p, q=q, rho=rho, K=K, Ubar=Ub, sbar=sb, degenerate=degenerate)


def isvd_rotate(Phi, q, rho, Ubar, r):
    """The second half of Alg. 2: [Phi, q/rho] Ubar (eq. isvd_updated_basis_full)
    truncated to its leading r columns (eq. isvd_truncation); the residual
    direction is zero when rho = 0."""
    j = q / rho if rho > 0.0 else np.zeros(Phi.shape[0])
    Phi_t = np.concatenate([Phi, j[:, None]], axis=1) @ Ubar
    return Phi_t[:, :min(r, Phi.shape[1] + 1)]


def isvd_update(Phi, sigma, yhat, lam, r, tau_rho=1e-12):
    """One Brand update with forgetting factor lam (Alg. 2): isvd_core, then
    isvd_rotate.  Returns (Phi_new, sigma_new, info) where info holds p, q,
    rho, the core K, Ubar and sbar."""
    info = isvd_core(Phi, sigma, yhat, lam, tau_rho)
    Phi_new = isvd_rotate(Phi, info["q"], info["rho"], info["Ubar"], r)
    return Phi_new, info["sbar"][:Phi_new.shape[1]].copy(), info


def reorth(Phi, tau_orth):
    """If max|Phi^T Phi - I| > tau_orth: Cholesky G = L L^T and Phi <- Phi L^{-T}.

    Returns (Phi, L or None)."""
    G = Phi.T @ Phi
    if np.max(np.abs(G - np.eye(G.shape[0]))) <= tau_orth:
        return Phi, None
    L = np.linalg.cholesky(G)
    return np.linalg.solve(L, Phi.T).T, L


# ------------------------------------------------------------------ App. A: windowed rules
def window_matrix(window):
    """The preprocessed window (eq. wsvd_window_matrix): columns oldest first."""
    return np.stack(window, axis=1)


def wsvd_update(Yw, r):
    """Windowed SVD (App. A, Alg. A.1): the leading r left singular vectors of the
    window matrix and its leading r singular values (eq. wsvd_update)."""
    U, s, _ = np.linalg.svd(Yw, full_matrices=False)
    return sign_fix(U[:, :r]), s[:r].copy()


def orth(A):
    """orth(.) of Alg. A.2, read as Gram-Schmidt orthonormalisation of the
    columns: the Q factor of the thin QR factorisation with a positive diagonal
    of R (unique for full column rank, and stable when A is nearly orthonormal,
    as Phi~ is when the window lies near span(Phi))."""
    Q, R = np.linalg.qr(A)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :]


def direct_update(Phi, Yw):
    """Direct update (App. A, Alg. A.2; eqs. direct_optimization and
    direct_update): Z = Phi^+ Yw with Phi^+ = Phi^T for the orthonormal basis,
    Phi~ = Yw Z^+ (pseudo-inverse: singular values below 1e-15 of the largest are
    dropped), then orth."""
    Z = Phi.T @ Yw
    return orth(Yw @ np.linalg.pinv(Z, rcond=1e-15))


# ------------------------------------------------------------------ Sec. 3.2 sampling
def deim_greedy(Phi, n_s):
    """Greedy DEIM row selection with oversampling.

    Round 1 (classic DEIM): p_1 = argmax |phi_1|; for j = 2..r interpolate phi_j on
    the current rows with phi_1..phi_{j-1} and take the argmax of the residual.
    Round 2 (n_s - r more rows, n_s <= 2r): for j = 1..n_s-r fit phi_j by least
    squares on all rows chosen so far with phi_1..phi_{j-1} (no fit for j = 1) and
    take the argmax of the residual.  Rows already chosen are never re-chosen; ties
    go to the lowest row index.  Returns int array of n_s DOF rows in pick order."""
    N, r = Phi.shape
    if not (r <= n_s <= 2 * r) or n_s > N:
        raise ValueError("need r <= n_s <= min(2r, N)")
    chosen = np.zeros(N, dtype=bool)
    P = []

    def pick(res):
        a = np.abs(res)
        a = np.where(chosen, -1.0, a)
        i = int(np.argmax(a))
        chosen[i] = True
        P.append(i)

    pick(Phi[:, 0])
    for j in range(1, r):
        c = np.linalg.solve(Phi[P, :j], Phi[P, j])
        pick(Phi[:, j] - Phi[:, :j] @ c)
    for j in range(0, n_s - r):
        if j == 0:
            pick(Phi[:, 0])
        else:
            c, *_ = np.linalg.lstsq(Phi[P, :j], Phi[P, j], rcond=None)
            pick(Phi[:, j] - Phi[:, :j] @ c)
    return np.array(P, dtype=np.int64)


def qdeim(Phi, m):
    """QDEIM (Sec. 3.2, eq. qdeim_qr): the first m pivots of the column-pivoted
    QR factorisation of Phi^T.  Pivoted QR picks, at step k, the column of the
    trailing block of largest norm, which is the row phi_i of Phi farthest from
    the span of the rows already chosen; that distance is formed here
    explicitly (Gram-Schmidt twice on the chosen rows, FP64).  Ties go to the
    lowest row index."""
    N, r = Phi.shape
    if not (1 <= m <= r):
        raise ValueError("QDEIM gives at most r rows")
    Q = np.zeros((r, 0))
    chosen = np.zeros(N, dtype=bool)
    P = []
    for _ in range(m):
        R = Phi - (Phi @ Q) @ Q.T
        dist = np.where(chosen, -1.0, np.sum(R * R, axis=1))
        i = int(np.argmax(dist))
        chosen[i] = True
        P.append(i)
        v = Phi[i].copy()
        for _ in range(2):
            v = v - Q @ (Q.T @ v)
        Q = np.concatenate([Q, (v / np.linalg.norm(v))[:, None]], axis=1)
    return np.array(P, dtype=np.int64)


# feature map Theta of feature-guided sampling, per problem (variable index):
# Burgers u, Euler density, reacting model temperature
FGS_FEATURE = {F.BURGERS: 0, F.EULER_RUSANOV: 0, F.EULER_HLLC: 0, F.REACT: 10}


def feature_gradient2(problem, y):
    """||grad theta||^2 per cell for theta = Theta(y), the feature variable of
    the problem, by central differences on the unit interval (periodic wrap,
    or the zero-gradient ghosts at the walls of the Euler problems)."""
    nv = F.NVAR[problem]
    th = y.reshape(-1, nv)[:, FGS_FEATURE[problem]]
    n = th.shape[0]
    if F.PERIODIC[problem]:
        tp, tm = np.roll(th, -1), np.roll(th, 1)
    else:
        tp = np.concatenate([th[1:], th[-1:]])
        tm = np.concatenate([th[:1], th[:-1]])
    g = (tp - tm) * (n / 2.0)
    return g * g


def fgs(problem, Phi, y, n_s):
    """Feature-guided sampling (Sec. 3.2, eq. fgs_selection): QDEIM's r rows,
    then the n_s - r cells of largest ||grad theta||^2 (theta of the estimated
    future state y), each contributing its feature-variable row; cells whose
    feature row is already chosen are skipped; ties go to the lowest cell."""
    N, r = Phi.shape
    nv = F.NVAR[problem]
    P = list(qdeim(Phi, r))
    g = feature_gradient2(problem, y)
    taken = set(P)
    for c in np.argsort(-g, kind="stable"):
        if len(P) == n_s:
            break
        row = int(c) * nv + FGS_FEATURE[problem]
        if row not in taken:
            P.append(row)
            taken.add(row)
    return np.array(P, dtype=np.int64)


def sample_rows(problem, Phi, y_corr, prm):
    """The sampling rule of the configuration: greedy DEIM, QDEIM or QDEIM + FGS."""
    if prm["hyper"] == "deim":
        return deim_greedy(Phi, prm["n_s"])
    if prm["hyper"] == "qdeim":
        return qdeim(Phi, prm["n_s"])
    if prm["hyper"] == "qdeim_fgs":
        return fgs(problem, Phi, y_corr, prm["n_s"])
    raise ValueError("unknown sampling %r" % (prm["hyper"],))


def rebuild(Phi, P):
    """(P^T Phi)^+, r x n_s (eq. qdeim_approximation_phi)."""
    return np.linalg.pinv(Phi[P, :])


# ------------------------------------------------------------------ ROM steps
def _stop(delta, a, tol):
    return np.max(np.abs(delta)) <= tol * (1.0 + np.max(np.abs(a)))


def galerkin_step(problem, phys, q_ref, d, Phi, a_prev, dt, tol, max_it):
    """Backward Euler on the Galerkin ROM (eq. galerkin_continuous_rom):
    g(a) = a - a_prev - dt Phi^T D f(q_ref + D^-1 Phi a) = 0, Newton with
    J_g = I - dt Phi^T D J_f D^-1 Phi.  d is the diagonal of D (length N).
    Stops when ||delta||_inf <= tol (1 + ||a||_inf) after the update.
    Returns (a, iterations, converged)."""
    r = Phi.shape[1]
    a = a_prev.copy()
    PhiD = Phi / d[:, None]                       # D^-1 Phi
    for it in range(max_it):
        qt = q_ref + PhiD @ a
        f = F.fom_f(problem, qt, phys)
        g = a - a_prev - dt * (Phi.T @ (d * f))
        Jf = F.jacobian_f(problem, qt, phys)
        Jg = np.eye(r) - dt * (Phi.T @ (d[:, None] * (Jf @ PhiD)))
        delta = np.linalg.solve(Jg, -g)
        a = a + delta
        if _stop(delta, a, tol):
            return a, it + 1, True
    return a, max_it, False


def hr_lspg_step(problem, phys, q_ref, d, Phi, P, M, a_prev, dt, tol, max_it):
    """Hyper-reduced LSPG step (eqs. hyperreduced_lspg, hyperreduced_lspg_stationarity):
    Gauss-Newton on min_a || M P^T D r(q~(a)) ||^2 with r the backward-Euler
    residual (previous state q~_prev = q_ref + D^-1 Phi a_prev) and the Jacobian
    M P^T D J_r D^-1 Phi = M P^T Psi_LSPG.  f and J_f are evaluated on the full
    grid and then sampled.  Returns (a, iterations, converged)."""
    a = a_prev.copy()
    PhiD = Phi / d[:, None]
    qp = q_ref + PhiD @ a_prev
    for it in range(max_it):
        qt = q_ref + PhiD @ a
        res = qt - qp - dt * F.fom_f(problem, qt, phys)
        rho = M @ (d[P] * res[P])
        Jr = F.jacobian_be(problem, qt, dt, phys)
        PsiP = (d[:, None] * (Jr @ PhiD))[P, :]
        A = M @ PsiP
        delta, *_ = np.linalg.lstsq(A, -rho, rcond=None)
        a = a + delta
        if _stop(delta, a, tol):
            return a, it + 1, True
    return a, max_it, False


def transfer(Phi_old, Phi_new, a):
    """Alg. 1 state transfer: a <- Phi_new^T D (q~ - q_ref) = Phi_new^T Phi_old a."""
    return Phi_new.T @ (Phi_old @ a)


def reconstruct(q_ref, d, Phi, a):
    """q~ = q_ref + D^-1 Phi a (eq. trial_approximation)."""
    return q_ref + (Phi @ a) / d


# ------------------------------------------------------------------ Alg. 1
def default_params(**kw):
    p = dict(r=4, n_s=4, w_init=4, N_t=20, z=2, lam=0.5, dt=1e-3,
             newton_tol=1e-8, newton_max=10, rom_tol=1e-12, rom_max=10,
             reorth_every=16, tau_orth=1e-12, tau_rho=1e-12,
             projection="galerkin", hyper="none", update="isvd", window=0, scheme="be")
    p.update(kw)
    return p


def offline(problem, phys, q0, prm):
    """Alg. 1 offline part: training FOM, preprocessing, POD, a^{w_init}, first
    coarse step, first sampling and rebuild."""
    nv = F.NVAR[problem]
    n_cell = q0.shape[0] // nv
    dt, z = prm["dt"], prm["z"]
    tol, mx = prm["newton_tol"], prm["newton_max"]
    explicit = prm.get("scheme", "be") == "ssprk43"
    if explicit:
        Q = X.fom_trajectory_explicit(problem, q0, dt, prm["w_init"], phys)
    else:
        Q = F.fom_trajectory(problem, q0, dt, prm["w_init"], phys, tol, mx)
    Q_train = Q[:, 1:]
    q_ref, d_var = preprocess(Q_train, q0, nv)
    d = dfull(d_var, n_cell)
    Phi, sigma = pod(d[:, None] * (Q_train - q_ref[:, None]), prm["r"])
    q_last = Q_train[:, -1]
    a = Phi.T @ (d * (q_last - q_ref))
    y_corr = coarse_step(problem, phys, q_last, prm)
    st = dict(q_ref=q_ref, d_var=d_var, d=d, Phi=Phi, sigma=sigma, a=a,
              y_corr=y_corr, n_update=0, Q_train=Q_train, P=None, M=None)
    if prm.get("update", "isvd") != "isvd":
        # the window starts from the last training snapshots (at most w of them)
        w = prm["window"]
        st["window"] = [d * (Q_train[:, j] - q_ref)
                        for j in range(max(0, Q_train.shape[1] - w), Q_train.shape[1])]
    if prm["hyper"] != "none":
        st["P"] = sample_rows(problem, Phi, y_corr, prm)
        st["M"] = rebuild(Phi, st["P"])
    return st


def adaptation_event(problem, phys, st, prm):
    """Alg. 1 event: coarse step, preprocess, iSVD, (re-orth), sampling, rebuild, transfer."""
    dt, z = prm["dt"], prm["z"]
    st["y_corr"] = coarse_step(problem, phys, st["y_corr"], prm)
    yhat = st["d"] * (st["y_corr"] - st["q_ref"])
    Phi_old = st["Phi"]
    rule = prm.get("update", "isvd")
    if rule == "isvd":
        Phi, sigma, info = isvd_update(Phi_old, st["sigma"], yhat, prm["lam"], prm["r"],
                                       prm["tau_rho"])
    else:
        # the oldest snapshot leaves the window once it holds w
        st["window"].append(yhat)
        if len(st["window"]) > prm["window"]:
            st["window"].pop(0)
        Yw = window_matrix(st["window"])
        info = None
        if rule == "wsvd":
            Phi, sigma = wsvd_update(Yw, prm["r"])
        elif rule == "direct":
            Phi, sigma = direct_update(Phi_old, Yw), st["sigma"]
        else:
            raise ValueError("unknown update rule %r" % (rule,))
    st["n_update"] += 1
    if prm["reorth_every"] > 0 and st["n_update"] % prm["reorth_every"] == 0:
        Phi, _ = reorth(Phi, prm["tau_orth"])
    st["Phi"], st["sigma"] = Phi, sigma
    if prm["hyper"] != "none":
        st["P"] = sample_rows(problem, Phi, st["y_corr"], prm)
        st["M"] = rebuild(Phi, st["P"])
    st["a"] = transfer(Phi_old, Phi, st["a"])
    return info


def coarse_step(problem, phys, y, prm):
    """The coarse correction step of eq. coarse_fom_backward_euler (step z dt):
    backward Euler by Newton, or, on the explicit path, one SSPRK(4,3) step of
    the limited second-order full-order model."""
    if prm.get("scheme", "be") == "ssprk43":
        return X.fom_step_explicit(problem, y, prm["z"] * prm["dt"], phys)
    y1, _, _ = F.newton_be_step(problem, y, prm["z"] * prm["dt"], phys, prm["newton_tol"],
                                prm["newton_max"])
    return y1


def rom_fine_step(problem, phys, st, prm):
    if prm.get("scheme", "be") == "ssprk43":
        st["a"] = X.galerkin_hr_explicit_step(problem, phys, st["q_ref"], st["d"], st["Phi"],
                                              st["P"], st["M"], st["a"], prm["dt"])
        return 4, True
    if prm["hyper"] != "none":
        a, it, ok = hr_lspg_step(problem, phys, st["q_ref"], st["d"], st["Phi"], st["P"],
                                 st["M"], st["a"], prm["dt"], prm["rom_tol"], prm["rom_max"])
    else:
        a, it, ok = galerkin_step(problem, phys, st["q_ref"], st["d"], st["Phi"], st["a"],
                                  prm["dt"], prm["rom_tol"], prm["rom_max"])
    st["a"] = a
    return it, ok


def adaptive_rom(problem, phys, q0, prm, record_q=False, n_steps=None):
    """Alg. 1.  Runs the fine loop n = w_init .. N_t-1 (or n_steps of it) and
    adapts when (n + 1 - w_init) mod z == 0.  Returns (state, record)."""
    st = offline(problem, phys, q0, prm)
    rec = dict(a=[], sigma=[], P=[], rom_iters=[], events=[], q=[])
    w = prm["w_init"]
    last = prm["N_t"] if n_steps is None else w + n_steps
    for n in range(w, last):
        it, _ = rom_fine_step(problem, phys, st, prm)
        rec["rom_iters"].append(it)
        if (n + 1 - w) % prm["z"] == 0:
            adaptation_event(problem, phys, st, prm)
            rec["events"].append(n + 1)
            rec["sigma"].append(st["sigma"].copy())
            if st["P"] is not None:
                rec["P"].append(st["P"].copy())
        rec["a"].append(st["a"].copy())
        if record_q:
            rec["q"].append(reconstruct(st["q_ref"], st["d"], st["Phi"], st["a"]))
    return st, rec
