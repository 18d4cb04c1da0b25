"""GPU parity of the rollout adjoint (rom_rollout_vjp): the gradient of a
final-state loss with respect to the initial state q0 through Alg. 1 as a
whole (offline stage and HR-LSPG online loop, sample rows of the run held
fixed), on the perturbed-Sod recipe of the adjoint configuration at reduced
sizes: against the oracle's reverse mode, against central differences of the
device's own forward runs on 16 directions, checkpoint invariance, the FP32
path, and the autograd Function."""
import numpy as np
import pytest

from oracle import adjoint as A
from oracle import rom as O
from paper_2605_28684_amd import workloads as W

pytestmark = pytest.mark.gpu


def _workload(n_cells, precision=W.F64, r=3, n_s=6, w_init=5, z=2, hyper=W.HR_DEIM):
    w = W.euler_adjoint_f32(n_inst=len(n_cells), n=max(n_cells), r=r, n_s=n_s, z=z, N_t=40,
                            precision=precision)
    # ragged instances: each the recipe's state on its own grid
    if len(set(n_cells)) > 1:
        q0, tgt = [], []
        for b, n in enumerate(n_cells):
            wb = W.euler_adjoint_f32(n_inst=b + 1, n=n, r=r, n_s=n_s, z=z, N_t=40,
                                     precision=precision)
            o = wb.offsets()
            q0.append(wb.q0[o[b]:o[b + 1]])
            tgt.append(wb.extra["target"][o[b]:o[b + 1]])
        w.q0, w.extra["target"] = np.concatenate(q0), np.concatenate(tgt)
        w.n_cells = list(n_cells)
        w.phys = [dict(gamma=1.4)] * len(n_cells)
    w.w_init, w.hyper, w.reorth_every = w_init, hyper, 0
    f64 = precision == W.F64
    w.newton_tol = 1e-13 if f64 else 1e-5
    w.rom_tol = 1e-14 if f64 else 1e-6
    w.newton_max, w.rom_max = 30, 30
    return w


@pytest.mark.parametrize("cells", [[48], [48, 37]])
def test_rollout_vjp_matches_oracle_fp64(cells):
    """d<qbar, q~_end>/d q0 for 6 fine steps (3 events) after the offline
    stage, with the oracle's loss cotangent q~_end - q_tgt: the sample rows of
    the last window bit-exact, q~_end within 1e-11 and the gradient within
    1e-9 (relative L2 and elementwise; see the design notes' parity bounds)."""
    import gpu_common as G
    from paper_2605_28684_amd import romhip as R
    w = _workload(cells)
    n_steps = 6
    prm = w.params()
    off = w.offsets()
    qbar, refs, P_end, qt_ref = [], [], [], []
    for b in range(w.n_inst):
        q0 = w.q0[off[b]:off[b + 1]]
        st, _, sched = A.rollout_forward(w.problem, w.phys[b], q0, prm, n_steps)
        qt = O.reconstruct(st["q_ref"], st["d"], st["Phi"], st["a"])
        qb = qt - w.extra["target"][off[b]:off[b + 1]]
        g, _ = A.rollout_vjp(w.problem, w.phys[b], q0, prm, n_steps, qb, sched)
        qbar.append(qb)
        refs.append(g)
        P_end.append(sched[-1])
        qt_ref.append(qt)
    h = R.RomBatch(w, q0=None, use_graph=False)
    q0d = G.to_dev(w.q0, W.F64)
    gq = G.host(h.rollout_vjp(q0d, n_steps, G.to_dev(np.concatenate(qbar), W.F64)))
    np.testing.assert_array_equal(h.get(R.GET_SAMPLES).cpu().numpy(), np.concatenate(P_end))
    qt_dev = G.host(h.get(R.GET_QTILDE))
    for b in range(w.n_inst):
        G.assert_close(qt_dev[off[b]:off[b + 1]], qt_ref[b], 1e-11, what="q~ end %d" % b)
        G.assert_close(gq[off[b]:off[b + 1]], refs[b], 1e-9, what="dL/dq0 %d" % b)
    assert not (h.status() & (R.FLAG_SINGULAR | R.FLAG_NONFINITE)).any()
    h.close()


def test_rollout_vjp_central_differences_on_device_fp64():
    """The adjoint configuration's check at reduced size: 16 directions
    v ~ N(0, I), h = 1e-6, L = 1/2 |q~_end - q_tgt|^2 from the device's own
    forward runs (rom_offline + rom_step); the sample rows of every perturbed
    run equal the unperturbed run's, and each directional derivative matches
    within 1e-5 relative (FD truncation about 5e-7 here)."""
    import gpu_common as G
    import torch
    from paper_2605_28684_amd import romhip as R
    w = _workload([48])
    n_steps = 6
    tgt = w.extra["target"]
    h = R.RomBatch(w, q0=None, use_graph=False)

    def loss(q0):
        h.offline(G.to_dev(q0, W.F64))
        h.rom_step(n_steps)
        qt = G.host(h.get(R.GET_QTILDE))
        return 0.5 * float(np.sum((qt - tgt) ** 2)), qt, h.get(R.GET_SAMPLES).cpu().numpy()

    L0, qt0, P0 = loss(w.q0)
    g = G.host(h.rollout_vjp(G.to_dev(w.q0, W.F64), n_steps, G.to_dev(qt0 - tgt, W.F64)))
    rng = np.random.default_rng(2000)
    worst = 0.0
    for _ in range(16):
        v = rng.normal(size=w.q0.shape)
        Lp, _, Pp = loss(w.q0 + 1e-6 * v)
        Lm, _, Pm = loss(w.q0 - 1e-6 * v)
        np.testing.assert_array_equal(Pp, P0)
        np.testing.assert_array_equal(Pm, P0)
        fd = (Lp - Lm) / 2e-6
        worst = max(worst, abs(fd - g @ v) / abs(fd))
    print("  parity FD 16 directions: worst relative %.3e" % worst)
    assert worst <= 1e-5
    torch.cuda.synchronize()
    h.close()


def test_rollout_vjp_checkpoint_invariance_and_end_state():
    """Any checkpoint count gives bitwise the same gradient, and the handle
    ends at the state rom_offline + rom_step reach."""
    import gpu_common as G
    from paper_2605_28684_amd import romhip as R
    w = _workload([64, 41])
    n_steps = 7
    h = R.RomBatch(w, q0=None, use_graph=False)
    q0d = G.to_dev(w.q0, W.F64)
    gbar = G.to_dev(np.random.default_rng(4).normal(size=w.q0.shape), W.F64)
    outs = [G.host(h.rollout_vjp(q0d, n_steps, gbar, n_ckpt=c)) for c in (0, 1, 3, 7)]
    end = G.host(h.get(R.GET_QTILDE))
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    h.offline(q0d)
    h.rom_step(n_steps)
    np.testing.assert_array_equal(G.host(h.get(R.GET_QTILDE)), end)
    h.close()


def test_rollout_vjp_fp32_storage_near_oracle():
    """FP32 states and basis (the adjoint configuration's precision) against the
    FP64 oracle at 48 cells: relative L2 within 1e-5 (measured 8e-7)."""
    import gpu_common as G
    from paper_2605_28684_amd import romhip as R
    w = _workload([48], precision=W.F32)
    n_steps = 6
    w64 = _workload([48])
    prm = w64.params()
    st, _, sched = A.rollout_forward(w.problem, w.phys[0], w.q0, prm, n_steps)
    qt = O.reconstruct(st["q_ref"], st["d"], st["Phi"], st["a"])
    qb = qt - w.extra["target"]
    ref, _ = A.rollout_vjp(w.problem, w.phys[0], w.q0, prm, n_steps, qb, sched)
    h = R.RomBatch(w, q0=None, use_graph=False)
    gq = G.host(h.rollout_vjp(G.to_dev(w.q0, W.F32), n_steps, G.to_dev(qb, W.F32)))
    e = G.relerr(gq, ref)
    print("  parity dL/dq0 FP32 storage: relerr %.3e" % e)
    assert e <= 1e-5
    h.close()


def test_rom_rollout_autograd_function_fp64():
    """RomRollout: torch.autograd.grad of the misfit loss through the Function
    equals rom_rollout_vjp with the same cotangent."""
    import gpu_common as G
    import torch
    from paper_2605_28684_amd import romhip as R
    w = _workload([48])
    n_steps = 4
    h = R.RomBatch(w, q0=None, use_graph=False)
    q0 = G.to_dev(w.q0, W.F64).requires_grad_(True)
    tgt = G.to_dev(w.extra["target"], W.F64)
    q = R.RomRollout.apply(q0, h, n_steps)
    L = 0.5 * torch.sum((q - tgt) ** 2)
    (g,) = torch.autograd.grad(L, q0)
    ref = h.rollout_vjp(q0.detach(), n_steps, (q - tgt).detach().contiguous())
    np.testing.assert_array_equal(G.host(g), G.host(ref))
    h.close()


def test_rollout_vjp_refuses_other_paths():
    import gpu_common as G
    from paper_2605_28684_amd import romhip as R
    w = _workload([48])
    w.projection = W.GALERKIN
    h = R.RomBatch(w, q0=None, use_graph=False)
    q0 = G.to_dev(w.q0, W.F64)
    with pytest.raises(R.RomError) as e:
        h.rollout_vjp(q0, 4, q0)
    assert e.value.code == R.ROM_E_UNSUPPORTED
    h.close()


def test_rollout_vjp_central_differences_full_instance_size_fp64():
    """The adjoint configuration's recipe at its real instance size (N = 262,144
    cells, w_init = 10, z = 10, greedy DEIM with n_s = 2r) for 4 instances,
    FP64, through one event (12 fine steps): 16 directions v ~ N(0, I) with
    h = 1e-6 against the device's own forward runs; the sample rows of the
    perturbed runs equal the unperturbed run's, and every directional
    derivative matches within 1e-4 relative (measured 1.8e-5; central
    differences of this loss at h = 1e-6 carry truncation errors up to 2e-5,
    as the oracle's own differences against its limit show).  The rank is 6: at the
    configuration's rank 10 the training matrix's singular values span ten
    decades (sigma_10 / sigma_1 = 1.8e-10) and the core's last two at the first
    event are 3e-9 of the first apart, so the loss has curvature that central
    differences at h = 1e-6 resolve to about 1e-2 only (the oracle's own
    differences move towards its adjoint as h shrinks)."""
    import torch
    from paper_2605_28684_amd import romhip as R
    r, n_steps, case = 6, 12, "r6"
    w = W.euler_adjoint_f32(n_inst=4, n=262144, r=r, n_s=2 * r, precision=W.F64)
    w.w_init = 10
    w.reorth_every = 0
    w.newton_tol, w.rom_tol = 1e-12, 1e-13
    w.newton_max, w.rom_max = 30, 30
    tgt = torch.as_tensor(w.extra["target"], dtype=torch.float64, device="cuda")
    h = R.RomBatch(w, q0=None, use_graph=False)
    q0 = torch.as_tensor(w.q0, dtype=torch.float64, device="cuda")

    def loss(x):
        h.offline(x)
        h.rom_step(n_steps)
        d = h.get(R.GET_QTILDE) - tgt
        return 0.5 * float(torch.sum(d * d)), d.clone(), h.get(R.GET_SAMPLES).cpu().numpy()

    _, d0, P0 = loss(q0)
    g = h.rollout_vjp(q0, n_steps, d0)
    gen = torch.Generator(device="cuda").manual_seed(2000)
    worst = 0.0
    for _ in range(16):
        v = torch.randn(q0.shape, generator=gen, dtype=torch.float64, device="cuda")
        Lp, _, Pp = loss(q0 + 1e-6 * v)
        Lm, _, Pm = loss(q0 - 1e-6 * v)
        np.testing.assert_array_equal(Pp, P0)
        np.testing.assert_array_equal(Pm, P0)
        fd = (Lp - Lm) / 2e-6
        ad = float(torch.dot(g, v))
        worst = max(worst, abs(fd - ad) / abs(fd))
    print("  parity FD 16 directions, 4 x 262,144 cells, %s: worst relative %.3e" % (case, worst))
    assert worst <= 1e-4
    assert not (h.status() & (R.FLAG_SINGULAR | R.FLAG_NONFINITE)).any()
    h.close()
