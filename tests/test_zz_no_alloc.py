"""The allocation-free rollout adjoint (fom_rollout_vjp_noalloc) against the
allocating entry point (fom_rollout_vjp): same kernels, so the gradients must be
bitwise equal, on two calls in a row through the shared device array, the
second on a smaller batch and a shorter rollout."""
import numpy as np
import pytest

from paper_2605_28684_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(problem, cells, precision, seed):
    import gpu_common as G
    if problem == W.BURGERS:
        w = W.burgers_batch_f32(n_inst=len(cells), precision=precision)
        w.phys = [dict(nu=0.004 + 0.002 * b) for b in range(len(cells))]
    else:
        w = W.sod_hllc_f32(n=cells[0], precision=precision, flux=problem)
        w.phys = [dict(gamma=1.4)] * len(cells)
    w.n_cells = list(cells)
    w.hyper, w.projection = W.HR_DEIM, W.LSPG
    w.r, w.n_s, w.w_init = 2, 2, 2
    w.newton_tol = 1e-12 if precision == W.F64 else 1e-5
    w.newton_max = 20
    q = G.rounded(W.random_state(problem, cells, seed=seed, scale=0.5), precision)
    g = G.rounded(np.random.default_rng(seed + 1).normal(size=q.shape), precision)
    dt = 2e-3 if problem == W.BURGERS else 0.064 / 96
    return w, q, g, dt


@pytest.mark.parametrize("problem,precision", [(W.EULER_RUSANOV, W.F32), (W.BURGERS, W.F64)])
def test_noalloc_rollout_vjp_matches_allocating_call(problem, precision):
    import gpu_common as G
    import torch
    from paper_2605_28684_amd import romhip as R
    runs = [([700, 517, 96], 9, 0), ([96, 60], 5, 2)]   # second call: smaller batch, shorter
    handles = []
    for k, (cells, T, ck) in enumerate(runs):
        w, q0, gbar, dt = _case(problem, cells, precision, seed=60 + k)
        h = R.RomBatch(w, q0=None, use_graph=False)
        handles.append(h)
        qd, gd = G.to_dev(q0, precision), G.to_dev(gbar, precision)
        out = torch.full_like(qd, float("nan"))
        print("noalloc call", k, "problem", problem, "cells", cells, "T", T, "n_ckpt", ck,
              flush=True)
        h.fom_rollout_vjp_noalloc(qd, T, dt, gd, n_ckpt=ck, out=out)
        got = G.host(out)
        ref = G.host(h.fom_rollout_vjp(qd, T, dt, gd, n_ckpt=ck))
        assert np.isfinite(got).all()
        assert np.array_equal(got, ref), (k, np.abs(got - ref).max())
        assert np.array_equal(G.host(qd), q0) and np.array_equal(G.host(gd), gbar)
    # a plan beyond the 32 MiB array is refused before anything is enqueued
    h = handles[0]
    w, q0, gbar, dt = _case(problem, runs[0][0], precision, seed=60)
    qd, gd = G.to_dev(q0, precision), G.to_dev(gbar, precision)
    st = h.total_dof * (8 if precision == W.F64 else 4)
    T = (32 << 20) // st + 10
    with pytest.raises(R.RomError) as e:
        h.fom_rollout_vjp_noalloc(qd, T, dt, gd, n_ckpt=1, out=torch.empty_like(qd))
    assert e.value.code == R.ROM_E_INVAL
    for h in handles:
        h.close()
