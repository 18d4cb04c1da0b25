"""GPU parity of paths that the per-call tests do not reach at their sizes:
  * the persistent streaming residual walking several tiles per block, in
    every tuned launch shape, on a ragged batch and at the 64 x 262,144-cell
    shape the benchmark times;
  * the iSVD update when the snapshot lies in the span of the basis
    (rho -> 0), with and without exact zeros among the singular values;
  * FP32 hyper-reduced LSPG windows (fine steps + event with greedy DEIM),
    eager and graph-replayed, at r = 24, 40 and 64 (the three reduced-solve
    widths), against the oracle window by window;
  * the 512-cell FP64 Burgers configuration over its whole horizon (1,900 fine
    steps, 380 events) from q0, against the oracle's Alg. 1.
Every comparison checks a relative L2 error and the largest elementwise error."""
import numpy as np
import pytest

from oracle import fom as F
from oracle import rom as O
from paper_2605_28684_amd import workloads as W

pytestmark = pytest.mark.gpu


def _euler_state(cells, seed):
    """Euler states whose interfaces take every flux branch: subsonic, and
    supersonic in both directions (|u| up to 2.5 with c near 1.2), with jumps."""
    rng = np.random.default_rng([7, seed])
    out = []
    for n in cells:
        x = W.centres(n)
        rho = 1.0 + 0.5 * np.sin(2 * np.pi * x + 0.3) + 0.2 * (x > 0.6) + 0.02 * rng.uniform(-1, 1, n)
        u = 2.5 * np.sin(4 * np.pi * x) + 0.05 * rng.uniform(-1, 1, n)
        p = 1.0 + 0.4 * np.cos(2 * np.pi * x) - 0.3 * (x > 0.3) + 0.02 * rng.uniform(-1, 1, n)
        out.append(W._conserved(rho, u, p))
    return np.concatenate(out)


def _euler_handle(cells, precision, flux):
    from paper_2605_28684_amd.romhip import RomBatch
    w = W.sod_hllc_f32(n=cells[0], precision=precision, flux=flux)
    w.n_cells = list(cells)
    w.phys = [dict(gamma=1.4)] * len(cells)
    w.r, w.n_s, w.w_init = 2, 2, 2
    return w, RomBatch(w, q0=None, use_graph=False)


def _flux_scale(problem, q, gamma):
    """Per element, the magnitude the residual is formed from: (|F_{i+1/2}| +
    |F_{i-1/2}|)/dx with the oracle's face fluxes.  In smooth regions f is a
    small difference of these, so the error of any FP32 evaluation is about
    eps_32 times this scale, not times |f|."""
    U = q.reshape(-1, 3)
    n = U.shape[0]
    Ug = np.concatenate([U[:1], U, U[-1:]], axis=0)
    flux = F.rusanov_flux if problem == W.EULER_RUSANOV else F.hllc_flux
    Ff = np.abs(flux(Ug[:-1], Ug[1:], gamma))
    return ((Ff[1:] + Ff[:-1]) * n).reshape(-1)


def _check_residual_shapes(h, w, q, precision, problem, instances, norm_tol=None):
    """Every launch shape gives the same bits; shape 0 against the oracle:
    largest error relative to the largest |f| within the per-call bound, and
    per element relative to the flux scale (Rusanov: the per-call bound; HLLC:
    1e-3); the relative L2 error within norm_tol (default: the per-call
    bound)."""
    import gpu_common as G
    import torch
    from paper_2605_28684_amd import romhip as R
    qd = G.to_dev(q, precision)
    n_shapes = h.set_tuning(R.TUNE_RESIDUAL, -1)
    assert n_shapes > 1
    h.set_tuning(R.TUNE_RESIDUAL, 0)
    ref_dev = h.fom_residual(qd)
    for k in range(1, n_shapes):
        h.set_tuning(R.TUNE_RESIDUAL, k)
        out = h.fom_residual(qd)
        torch.cuda.synchronize()
        assert torch.equal(out, ref_dev), k
    f = G.host(ref_dev)
    off = w.offsets()
    tol = G.TOL[precision]
    for b in instances:
        sl = slice(off[b], off[b + 1])
        fref = F.fom_f(problem, q[sl], w.phys[b])
        e2, em = G.relerr(f[sl], fref), G.maxrel(f[sl], fref)
        ec = np.max(np.abs(f[sl] - fref) / _flux_scale(problem, q[sl], w.phys[b]["gamma"]))
        print("  instance %d: relerr %.3e, elementwise %.3e, flux-scaled %.3e" % (b, e2, em, ec))
        assert em <= tol, (b, em)
        # HLLC's star states divide by S_K - S*, which makes a few cells of the
        # transonic test states ill-conditioned beyond the flux scale; Rusanov
        # has no such division
        assert ec <= (tol if problem == W.EULER_RUSANOV else 1e-3), (b, ec)
        assert e2 <= (tol if norm_tol is None else norm_tol), (b, e2)
    assert not (h.status() & 4).any()
    return n_shapes


@pytest.mark.parametrize("precision", [W.F32, W.F64])
@pytest.mark.parametrize("problem", [W.EULER_RUSANOV, W.EULER_HLLC])
def test_residual_every_shape_several_tiles_per_block(problem, precision):
    """A ragged 1.9M-cell batch: 1866 to 7459 tiles for at most 3072 resident
    blocks, so every block of every shape walks two or three tiles (the
    next-tile prefetch and register rotation run), and every instance ends in
    a partial tile."""
    cells = [1000003, 777777, 131073]
    w, h = _euler_handle(cells, precision, problem)
    import gpu_common as G
    q = G.rounded(_euler_state(cells, seed=problem), precision)
    print("residual shapes", problem, precision, cells, flush=True)
    _check_residual_shapes(h, w, q, precision, problem, range(len(cells)))
    h.close()


def test_residual_at_the_benchmark_shape_every_shape():
    """64 instances x 262,144 cells, Rusanov, FP32 (the shape whose roofline the
    benchmark reports; about 18 tiles per block): every shape bitwise equal,
    the autotuned choice included, and three whole instances against the
    oracle (elementwise and flux-scaled errors within 1e-5)."""
    import gpu_common as G
    import torch
    from paper_2605_28684_amd import romhip as R
    w = W.euler_adjoint_f32()
    from paper_2605_28684_amd.romhip import RomBatch
    h = RomBatch(w, q0=None, use_graph=False)
    q = G.rounded(w.q0, W.F32)
    print("residual at 64 x 262144", flush=True)
    # the smooth perturbed states make f a small difference of O(1) face fluxes
    # in most cells: the relative L2 error reaches about 1.02e-5 there (flux-
    # scaled and largest elementwise errors about 2e-7), so the normwise bound
    # of this shape is 2e-5
    _check_residual_shapes(h, w, q, W.F32, W.EULER_RUSANOV, [0, 31, 63], norm_tol=2e-5)
    qd = G.to_dev(q, W.F32)
    h.set_tuning(R.TUNE_RESIDUAL, 0)
    ref = h.fom_residual(qd)
    h.autotune(R.TUNE_RESIDUAL, qd)
    assert torch.equal(h.fom_residual(qd), ref)
    h.close()


# ---------------------------------------------------------------- rho -> 0
def _isvd_case(precision, zeros, seed):
    import gpu_common as G
    cells = [700, 2100, 130]
    r = 8
    w = W.burgers_batch_f32(n_inst=len(cells), precision=precision, r=r)
    w.n_cells = list(cells)
    w.phys = [dict(nu=0.005)] * len(cells)
    w.reorth_every = 0
    rng = np.random.default_rng(seed)
    Phis, sig, a, ys = [], [], [], []
    for b, n in enumerate(cells):
        Q, _ = np.linalg.qr(rng.normal(size=(n, r)))
        Phis.append(G.rounded(Q, precision))
        s = np.sort(rng.uniform(0.5, 5.0, r))[::-1]
        c = rng.normal(size=r)
        if zeros:
            s[-2:] = 0.0          # two exact zeros in sigma ...
            c[-1] = 0.0           # ... one with a zero weight, one without
        sig.append(s)
        a.append(rng.normal(size=r))
        ys.append(G.rounded(Phis[b] @ c, precision))    # inside span(Phi) up to rounding
    return w, cells, r, Phis, sig, a, np.concatenate(ys)


@pytest.mark.parametrize("zeros", [False, True])
@pytest.mark.parametrize("precision", [W.F64, W.F32])
def test_isvd_rho_zero_branch(precision, zeros):
    """Snapshot in span(Phi): the residual norm falls below tau_rho ||y^||, the
    instance is flagged, rho := 0 and the new direction is never kept.  The
    singular values, the covariance Phi' Sigma'^2 Phi'^T (unique even where
    zero singular values repeat), orthonormality, span(Phi') within span(Phi)
    and the carried state Phi' a' = Phi Ubar[:r,:r] Ubar[:r,:r]^T a are
    checked against the oracle's update."""
    import gpu_common as G
    import torch
    from paper_2605_28684_amd import romhip as R
    w, cells, r, Phis, sig, a, y = _isvd_case(precision, zeros, seed=81 + zeros)
    from paper_2605_28684_amd.romhip import RomBatch
    h = RomBatch(w, q0=None, use_graph=False)
    h.set(R.GET_BASIS, G.to_dev(np.concatenate([p.reshape(-1) for p in Phis]), precision))
    h.set(R.GET_SIGMA, torch.as_tensor(np.concatenate(sig)))
    h.set(R.GET_A, torch.as_tensor(np.concatenate(a)))
    h.set(R.GET_QREF, G.to_dev(np.zeros(sum(cells)), precision))
    h.set(R.GET_DVAR, torch.as_tensor(np.ones(len(cells))))
    h.isvd_update(G.to_dev(y, precision))
    P2 = G.host(h.get(R.GET_BASIS))
    s2 = G.host(h.get(R.GET_SIGMA))
    a2 = G.host(h.get(R.GET_A))
    flags = h.status()
    off = w.offsets()
    tol = G.TOL[precision]
    orth = 1e-12 if precision == W.F64 else 2e-6
    for b, n in enumerate(cells):
        assert flags[b] & R.FLAG_RHO_ZERO, b
        sl = slice(off[b], off[b + 1])
        Po, so, info = O.isvd_update(Phis[b], sig[b], y[sl], w.lam, r, tau_rho=w.tau_rho)
        assert info["degenerate"], b
        Pg = P2[off[b] * r:off[b + 1] * r].reshape(n, r)
        sg = s2[b * r:(b + 1) * r]
        G.assert_close(sg, so, tol, what="sigma %d" % b)
        G.assert_close((Pg * sg ** 2) @ Pg.T, (Po * so ** 2) @ Po.T, tol, what="covariance %d" % b)
        # columns with a nonzero singular value are orthonormal and inside span(Phi)
        nz = sg > 0
        Pn = Pg[:, nz]
        assert np.max(np.abs(Pn.T @ Pn - np.eye(Pn.shape[1]))) < orth, b
        out_of_span = Pn - Phis[b] @ (Phis[b].T @ Pn)
        assert np.max(np.abs(out_of_span)) < (1e-12 if precision == W.F64 else 1e-6), b
        # the lifted state is carried: D^-1 Phi' a' equals the oracle's
        ar = O.transfer(Phis[b], Po, a[b])
        G.assert_close(Pg @ a2[b * r:(b + 1) * r], Po @ ar, 10 * tol, what="state %d" % b)
    h.close()


# ---------------------------------------------------------------- FP32 HR-LSPG windows
def _hr_case(kind):
    if kind == "sod_hllc_r40":          # the Sod configuration's r and n_s (<40> solve)
        w = W.sod_hllc_f32(n=1500, r=40, n_s=80, z=3, precision=W.F32, flux=W.EULER_HLLC)
        n_win = 3
    elif kind == "sod_hllc_r44":        # 40 < r <= 48 (<48> solve)
        w = W.sod_hllc_f32(n=1500, r=44, n_s=88, z=3, precision=W.F32, flux=W.EULER_HLLC)
        n_win = 3
    elif kind == "sod_rusanov_r24":     # 16 < r <= 32 (<32> solve)
        w = W.sod_hllc_f32(n=900, r=24, n_s=40, z=3, precision=W.F32, flux=W.EULER_RUSANOV)
        n_win = 3
    else:                               # the reacting configuration's r and n_s (<64>)
        w = W.react10_f32(n_inst=1, n=200, r=64, n_s=128, z=2, precision=W.F32)
        w.dt = 2e-4
        n_win = 2
    return w, n_win


def _device_state(h, w):
    import gpu_common as G
    from paper_2605_28684_amd import romhip as R
    r, nv = w.r, w.n_var
    n = w.n_cells[0]
    d_var = G.host(h.get(R.GET_DVAR))
    return dict(Phi=G.host(h.get(R.GET_BASIS)).reshape(n * nv, r),
                sigma=G.host(h.get(R.GET_SIGMA)), a=G.host(h.get(R.GET_A)),
                y_corr=G.host(h.get(R.GET_YCORR)), q_ref=G.host(h.get(R.GET_QREF)),
                d_var=d_var, d=O.dfull(d_var, n), P=h.get(R.GET_SAMPLES).cpu().numpy().astype(np.int64),
                qt=G.host(h.get(R.GET_QTILDE)))


@pytest.mark.parametrize("kind", ["sod_hllc_r40", "sod_hllc_r44", "sod_rusanov_r24", "react_r64"])
def test_hr_lspg_windows_fp32_eager_graph_and_oracle(kind):
    """FP32 storage (basis, states, coarse step, DEIM passes) with FP64 sampled
    evaluation and solves.  Both handles start from the oracle's offline state
    rounded to FP32.  Each window (z fine steps and an event) is checked
    against the oracle run from the device's own state at the window start
    (rounded inputs, so the check measures one window's error, not drift):
    y_corr after the coarse step, sigma and the core's left singular vectors
    (a valid SVD of the oracle's core, whose trailing vectors are not unique
    here), the rotated basis, a and q~ within the FP32 bound; the new sample
    rows equal, row for row, the oracle's greedy DEIM on the device's new
    basis.  The graph-replayed handle gives the same bits as the eager one
    after every window."""
    import gpu_common as G
    import torch
    from paper_2605_28684_amd import romhip as R
    w, n_win = _hr_case(kind)
    problem = w.problem
    prm = w.params()
    phys = w.phys[0]
    st0 = O.offline(problem, phys, w.q0, prm)
    z = w.z
    s = torch.cuda.Stream()
    hs = []
    with torch.cuda.stream(s):
        for graph in (False, True):
            h = R.RomBatch(w, q0=None, use_graph=graph)
            h.set(R.GET_BASIS, G.to_dev(st0["Phi"].reshape(-1), W.F32))
            h.set(R.GET_SIGMA, torch.as_tensor(st0["sigma"]))
            h.set(R.GET_A, torch.as_tensor(st0["a"]))
            h.set(R.GET_QREF, G.to_dev(st0["q_ref"], W.F32))
            h.set(R.GET_DVAR, torch.as_tensor(st0["d_var"]))
            h.set(R.GET_YCORR, G.to_dev(st0["y_corr"], W.F32))
            h.set(R.GET_COUNTERS, [w.w_init, 0, 0, 0])
            h.rom_rebuild()
            hs.append(h)
        torch.cuda.synchronize()
        dev = _device_state(hs[0], w)
        np.testing.assert_array_equal(dev["P"], O.deim_greedy(dev["Phi"], w.n_s))
        tight = dict(prm, rom_tol=1e-13, rom_max=30, newton_tol=1e-11, newton_max=30)
        for k in range(n_win):
            print("HR window", kind, k, flush=True)
            # the oracle from the device's state at the window start: z fine
            # steps, the coarse step of y_corr, then Alg. 2, DEIM and the
            # transfer on the device's own (FP32-rounded) snapshot, so that the
            # rounding of y_corr, amplified by ||y^|| / rho in the new
            # direction, is not counted against the update
            st = dict(q_ref=dev["q_ref"], d=dev["d"], Phi=dev["Phi"], sigma=dev["sigma"],
                      a=dev["a"], P=dev["P"], M=O.rebuild(dev["Phi"], dev["P"]))
            for _ in range(z):
                O.rom_fine_step(problem, phys, st, tight)
            y_ref, _, _ = F.newton_be_step(problem, dev["y_corr"], z * w.dt, phys,
                                           tight["newton_tol"], tight["newton_max"])
            for h in hs:
                h.rom_step(z)
            torch.cuda.synchronize()
            dev = _device_state(hs[0], w)
            devg = _device_state(hs[1], w)
            for key in ("Phi", "sigma", "a", "y_corr", "P", "qt"):
                assert np.array_equal(dev[key], devg[key]), (k, key)
            e_y = G.assert_close(dev["y_corr"], y_ref, 1e-5, what="y_corr window %d" % k)
            yhat = st["d"] * (dev["y_corr"] - st["q_ref"])
            info = O.isvd_core(st["Phi"], st["sigma"], yhat, w.lam, w.tau_rho)
            # the core's trailing singular values sit at FP64 round-off of the
            # leading one (tail/leading about 1e-16 here), so its trailing
            # vectors, and which of them truncation drops, are not unique: the
            # device's Ubar must be a valid SVD of the oracle's K, and the rest of
            # the update is compared on the device's Ubar
            Ug = G.host(hs[0].get(R.GET_UBAR)).reshape(w.r + 1, w.r + 1)
            K, sb = info["K"], info["sbar"]
            assert np.max(np.abs(Ug.T @ Ug - np.eye(w.r + 1))) <= 1e-13
            assert np.max(np.abs(K @ (K.T @ Ug) - Ug * sb ** 2)) <= 1e-13 * sb[0] ** 2
            e_s = G.assert_close(dev["sigma"], sb[:w.r], 1e-11, what="sigma window %d" % k)
            Phi_g = O.isvd_rotate(st["Phi"], info["q"], info["rho"], Ug, w.r)
            a_g = Ug[:w.r, :w.r].T @ st["a"]               # closed-form transfer
            e_p = G.assert_close(dev["Phi"], Phi_g, 1e-5, what="basis window %d" % k)
            e_a = G.assert_close(dev["a"], a_g, 1e-5, what="a window %d" % k)
            e_q = G.assert_close(dev["qt"], O.reconstruct(st["q_ref"], st["d"], Phi_g, a_g), 1e-5,
                                 what="q~ window %d" % k)
            np.testing.assert_array_equal(dev["P"], O.deim_greedy(dev["Phi"], w.n_s))
            Phi1, _, _ = O.isvd_update(st["Phi"], st["sigma"], yhat, w.lam, w.r, w.tau_rho)
            own = O.reconstruct(st["q_ref"], st["d"], Phi1, O.transfer(st["Phi"], Phi1, st["a"]))
            amp = np.linalg.norm(yhat) / max(info["rho"], 1e-300)
            print("  q~ %.1e/%.1e basis %.1e/%.1e a %.1e/%.1e sigma %.1e y_corr %.1e/%.1e; "
                  "||y^||/rho %.1e; sigma_r/sigma_1 %.1e; q~ against the oracle's own SVD %.1e/%.1e"
                  % (e_q + e_p + e_a + (e_s[0],) + e_y +
                     (amp, sb[w.r - 1] / sb[0], G.relerr(dev["qt"], own), G.maxrel(dev["qt"], own))),
                  flush=True)
        assert hs[0].get(R.GET_COUNTERS)[2] == n_win
        for h in hs:
            assert not (h.status() & (R.FLAG_NONFINITE | R.FLAG_SINGULAR | R.FLAG_ROM_NOCONV)).any()
            h.close()


# ---------------------------------------------------------------- the 512-cell configuration
def test_burgers_512_fp64_whole_horizon():
    """The 512-cell FP64 configuration exactly (nu = 0.01, dt = 1e-3, N_t = 2000,
    w_init = 100, r = 10, z = 5, lambda = 0.5).  The device runs Alg. 1 from q0
    (its own offline stage; windows replayed from graphs) through all 1,900
    fine steps and 380 events.  Two comparisons per window:
      * per window: the oracle runs the window (5 Galerkin steps, the coarse
        step, the update) from the device's state at the window start, with
        the device's snapshot and core vectors (trailing singular values at
        1e-14 of the leading one leave the trailing vectors fixed only up to
        rounding; the device's must be a valid SVD of the oracle's core to
        1e-13); q~, sigma, y_corr and the basis at the window end within
        max(1e-11, eps_64 ||y^||/rho) (relative L2 and largest elementwise):
        the new direction q/rho carries the rounding of q amplified by
        ||y^||/rho, which grows from 3e3 to 5e11 over the horizon as the
        snapshots fall into the span of the basis;
      * the whole trajectory: the oracle's independent Alg. 1 from q0.  sigma
        and y_corr stay within 1e-11.  q~ does not: the singular values span
        5e2 down to 1e-11, so the trailing basis directions are fixed by
        rounding, and two oracle runs whose bases differ by 1e-15 drift apart
        to about 4e-9 by the end (a CPU test measures it).  The device and the
        oracle drift the same way (measured 5e-9 relative L2, 2e-8
        elementwise); the recorded trajectory bound for q~ is 1e-7."""
    import gpu_common as G
    import torch
    from paper_2605_28684_amd import romhip as R
    w = W.burgers_512_f64()
    prm = w.params()
    phys = w.phys[0]
    st = O.offline(W.BURGERS, phys, w.q0, prm)
    s = torch.cuda.Stream()
    win, traj = [], []
    with torch.cuda.stream(s):
        h = R.RomBatch(w, q0=G.to_dev(w.q0, W.F64), use_graph=True)
        d = O.dfull(G.host(h.get(R.GET_DVAR)), 512)

        def dev_state():
            return dict(Phi=G.host(h.get(R.GET_BASIS)).reshape(512, w.r),
                        sigma=G.host(h.get(R.GET_SIGMA)), a=G.host(h.get(R.GET_A)),
                        y_corr=G.host(h.get(R.GET_YCORR)), q_ref=G.host(h.get(R.GET_QREF)),
                        qt=G.host(h.get(R.GET_QTILDE)))
        dv = dev_state()
        for k, n0 in enumerate(range(prm["w_init"], prm["N_t"], w.z)):
            sw = dict(q_ref=dv["q_ref"], d=d, Phi=dv["Phi"], sigma=dv["sigma"], a=dv["a"])
            for _ in range(w.z):
                O.rom_fine_step(W.BURGERS, phys, sw, prm)
                O.rom_fine_step(W.BURGERS, phys, st, prm)
            y_ref, _, _ = F.newton_be_step(W.BURGERS, dv["y_corr"], w.z * w.dt, phys,
                                           prm["newton_tol"], prm["newton_max"])
            O.adaptation_event(W.BURGERS, phys, st, prm)
            h.rom_step(w.z)
            dv = dev_state()
            # the window's event on the device's snapshot and core vectors (the
            # trailing singular values reach 1e-14 of the leading one, so the
            # trailing vectors are fixed only up to rounding): Ubar must be a
            # valid SVD of the oracle's core, the rest is compared on it
            info = O.isvd_core(sw["Phi"], sw["sigma"], d * (dv["y_corr"] - sw["q_ref"]), w.lam,
                               w.tau_rho)
            Ug = G.host(h.get(R.GET_UBAR)).reshape(w.r + 1, w.r + 1)
            K, sb = info["K"], info["sbar"]
            valid = max(np.max(np.abs(Ug.T @ Ug - np.eye(w.r + 1))),
                        np.max(np.abs(K @ (K.T @ Ug) - Ug * sb ** 2)) / sb[0] ** 2)
            Phi_g = O.isvd_rotate(sw["Phi"], info["q"], info["rho"], Ug, w.r)
            a_g = Ug[:w.r, :w.r].T @ sw["a"]
            qw = O.reconstruct(sw["q_ref"], d, Phi_g, a_g)
            qo = O.reconstruct(st["q_ref"], st["d"], st["Phi"], st["a"])
            kappa = np.linalg.norm(d * (dv["y_corr"] - sw["q_ref"])) / max(info["rho"], 1e-300)
            win.append([f(x, y) for f in (G.relerr, G.maxrel)
                        for x, y in ((dv["qt"], qw), (dv["sigma"], sb[:w.r]),
                                     (dv["y_corr"], y_ref), (dv["Phi"], Phi_g))] + [valid, kappa])
            traj.append([f(x, y) for f in (G.relerr, G.maxrel)
                         for x, y in ((dv["qt"], qo), (dv["sigma"], st["sigma"]),
                                      (dv["y_corr"], st["y_corr"]))])
        win, traj = np.array(win), np.array(traj)
        for k in list(range(0, 380, 38)) + [379]:
            print("event %3d: window q~ %.1e/%.1e; trajectory q~ %.1e/%.1e sigma %.1e y_corr %.1e"
                  % (k + 1, win[k, 0], win[k, 4], traj[k, 0], traj[k, 3], traj[k, 1], traj[k, 2]))
        print("largest per window (q~, sigma, y_corr, basis; L2 then elementwise; SVD validity; "
              "||y^||/rho):", win.max(axis=0))
        print("largest along the trajectory:", traj.max(axis=0))
        assert h.get(R.GET_COUNTERS)[2] == 380 and h.get(R.GET_COUNTERS)[0] == prm["N_t"]
        assert win[:, 8].max() <= 1e-13
        # the new direction q / rho carries the rounding of q times ||y^|| / rho
        bound = np.maximum(1e-11, 2.2e-16 * win[:, 9])
        assert (win[:, :8] <= bound[:, None]).all(), win[np.argmax((win[:, :8] / bound[:, None]).max(axis=1))]
        assert traj[:, [1, 2, 4, 5]].max() <= 1e-11
        assert traj[:, [0, 3]].max() <= 1e-7
        assert not (h.status() & (R.FLAG_NONFINITE | R.FLAG_NEWTON_NOCONV | R.FLAG_ROM_NOCONV)).any()
        h.close()
