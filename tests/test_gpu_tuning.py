"""GPU checks of the tuning targets: every greedy DEIM pass split gives the
same rows and (P^T Phi)^+ bit for bit; every solver part size solves the
backward-Euler step to the oracle's tolerance; autotuning and the JSON cache
set valid choices, the second time from the cache."""
import numpy as np
import pytest

from oracle import fom as F
from oracle import rom as O
from paper_2605_28684_amd import workloads as W

pytestmark = pytest.mark.gpu


def _orth(N, r, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(N, r)) * rng.uniform(0.3, 2.0, size=(N, 1)))
    return Q


def _sod(cells, r, n_s, precision):
    w = W.sod_hllc_f32(n=cells[0], r=r, n_s=n_s, precision=precision)
    w.n_cells = list(cells)
    w.phys = [dict(gamma=1.4)] * len(cells)
    w.w_init = r
    return w


@pytest.mark.parametrize("precision", [W.F64, W.F32])
def test_deim_pass_splits_are_bitwise_identical(precision):
    """Ragged instances of 2300 and 5001 cells (several 2048-row pass tiles,
    ragged tails), r = 9, n_s = 18: the rows and the pseudo-inverse of every
    split equal those of the default split bit for bit, and the rows are the
    oracle's."""
    import gpu_common as G
    import torch
    from paper_2605_28684_amd import romhip as R
    cells = [2300, 5001]
    r, ns = 9, 18
    w = _sod(cells, r, ns, precision)
    h = R.RomBatch(w, q0=None, use_graph=False)
    Phis = [G.rounded(_orth(3 * n, r, 70 + b), precision) for b, n in enumerate(cells)]
    h.set(R.GET_BASIS, G.to_dev(np.concatenate([p.reshape(-1) for p in Phis]), precision))
    h.set(R.GET_SIGMA, torch.as_tensor(np.ones(2 * r)))
    h.set(R.GET_A, torch.as_tensor(np.zeros(2 * r)))
    h.set(R.GET_QREF, G.to_dev(np.zeros(3 * sum(cells)), precision))
    h.set(R.GET_DVAR, torch.as_tensor(np.ones(6)))
    n = h.set_tuning(R.TUNE_DEIM_PASS, -1)
    assert n == 3
    out = []
    for c in range(n):
        h.set_tuning(R.TUNE_DEIM_PASS, c)
        h.rom_rebuild()
        out.append((h.get(R.GET_SAMPLES).cpu().numpy(), G.host(h.get(R.GET_PINV))))
    for P, M in out[1:]:
        np.testing.assert_array_equal(P, out[0][0])
        np.testing.assert_array_equal(M, out[0][1])
    P0 = out[0][0].reshape(2, ns)
    for b in range(2):
        np.testing.assert_array_equal(P0[b], O.deim_greedy(Phis[b], ns))
    h.close()


@pytest.mark.parametrize("precision", [W.F64, W.F32])
def test_solver_part_sizes_solve_the_step(precision):
    """Each part size (16, 8, 32 cells) gives a backward-Euler step on a ragged
    Euler batch (300, 517, 64 cells) within 1e-11 (FP64) / 1e-5 (FP32) of the
    oracle's Newton step, with the same Newton iteration counts in FP64."""
    import gpu_common as G
    import torch
    from paper_2605_28684_amd import romhip as R
    cells = [300, 517, 64]
    w = _sod(cells, 2, 2, precision)
    w.hyper, w.projection = W.HR_DEIM, W.LSPG
    w.newton_tol = 1e-10 if precision == W.F64 else 1e-5
    h = R.RomBatch(w, q0=None, use_graph=False)
    q = G.rounded(W.random_state(W.EULER_HLLC, cells, seed=3, scale=0.5), precision)
    dt = 0.064 / 512
    off = w.offsets()
    refs = []
    for b in range(3):
        ref, n_ref, ok = F.newton_be_step(W.EULER_HLLC, q[off[b]:off[b + 1]], dt, w.phys[b],
                                          tol=w.newton_tol, max_it=10)
        assert ok
        refs.append((ref, n_ref))
    n = h.set_tuning(R.TUNE_BT_PART, -1)
    assert n == 3
    for c in range(n):
        h.set_tuning(R.TUNE_BT_PART, c)
        it = torch.zeros(3, dtype=torch.int32, device="cuda")
        q1 = G.host(h.fom_step(G.to_dev(q, precision), dt, iters=it))
        its = it.cpu().numpy()
        for b in range(3):
            if precision == W.F64:
                assert int(its[b]) == refs[b][1], (c, b, its[b], refs[b][1])
            G.assert_close(q1[off[b]:off[b + 1]], refs[b][0],
                           1e-11 if precision == W.F64 else 1e-5, what="part %d inst %d" % (c, b))
    assert not (h.status() & 1).any()
    h.close()


def test_autotune_and_cache_round_trip(tmp_path):
    """On the Sod shape with greedy DEIM: the cache tunes the residual, the DEIM
    split and the part size once, and a second handle gets the same choices
    from the file without timing them."""
    import gpu_common as G
    from paper_2605_28684_amd import romhip as R
    from paper_2605_28684_amd import tuning as T
    w = W.sod_hllc_f32(n=8192, r=8, n_s=16, z=3, N_t=40)
    q0 = G.to_dev(w.q0, W.F32)
    path = str(tmp_path / "tune.json")
    h = R.RomBatch(w, q0=q0, use_graph=False)
    done = T.TuningCache(path).apply(h, q=q0)
    assert set(done) == {"residual", "deim_pass", "bt_part"}
    assert all(v[1] == "tuned" for v in done.values())
    h.rom_step(2 * w.z)
    assert not (h.status() & (R.FLAG_NONFINITE | R.FLAG_SINGULAR)).any()
    h2 = R.RomBatch(w, q0=q0, use_graph=False)
    done2 = T.TuningCache(path).apply(h2, q=q0)
    assert {k: v[0] for k, v in done2.items()} == {k: v[0] for k, v in done.items()}
    assert all(v[1] == "cache" for v in done2.values())
    h.close()
    h2.close()
