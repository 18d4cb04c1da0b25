"""GPU parity of QDEIM (eq. qdeim_qr) and feature-guided sampling (eq.
fgs_selection) against the oracle: sample rows bit-exact on identical basis
and correction-state input (ragged instances over several pass tiles, up to
r = 64), (P^T Phi)^+ within FP64 round-off, and Alg. 1 with these samplers
(LSPG steps and events) from the oracle's offline state."""
import numpy as np
import pytest

from oracle import rom as O
from paper_2605_28684_amd import workloads as W

pytestmark = pytest.mark.gpu


def _orth(N, r, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(N, r)) * rng.uniform(0.3, 2.0, size=(N, 1)))
    return Q


def _load(h, w, Phis, precision, y=None):
    import gpu_common as G
    import torch
    from paper_2605_28684_amd import romhip as R
    r, n_inst, nv = w.r, w.n_inst, w.n_var
    rng = np.random.default_rng(2)
    h.set(R.GET_BASIS, G.to_dev(np.concatenate([p.reshape(-1) for p in Phis]), precision))
    h.set(R.GET_SIGMA, torch.as_tensor(np.ones(n_inst * r)))
    h.set(R.GET_A, torch.as_tensor(rng.normal(size=n_inst * r)))
    h.set(R.GET_QREF, G.to_dev(np.zeros(sum(w.n_cells) * nv), precision))
    h.set(R.GET_DVAR, torch.as_tensor(np.ones(n_inst * nv)))
    if y is not None:
        h.set(R.GET_YCORR, G.to_dev(y, precision))


def _sod(cells, r, n_s, precision, hyper):
    w = W.sod_hllc_f32(n=cells[0], r=r, n_s=n_s, precision=precision)
    w.n_cells = list(cells)
    w.phys = [dict(gamma=1.4)] * len(cells)
    w.hyper = hyper
    w.w_init = r
    return w


@pytest.mark.parametrize("r", [7, 64])
@pytest.mark.parametrize("precision", [W.F64, W.F32])
def test_qdeim_rows_bit_exact_and_pinv(precision, r):
    """Ragged instances of 900 / 2300 (r = 7) or 700 / 1501 (r = 64) cells of
    three variables: several 2048-row pass tiles with ragged tails."""
    import gpu_common as G
    from paper_2605_28684_amd import romhip as R
    cells = [900, 2300] if r == 7 else [700, 1501]
    w = _sod(cells, r, r, precision, W.HR_QDEIM)
    h = R.RomBatch(w, q0=None, use_graph=False)
    Phis = [G.rounded(_orth(3 * n, r, 90 + b), precision) for b, n in enumerate(cells)]
    _load(h, w, Phis, precision)
    h.rom_rebuild()
    P = h.get(R.GET_SAMPLES).cpu().numpy().reshape(2, r)
    M = G.host(h.get(R.GET_PINV)).reshape(2, r, r)
    for b in range(2):
        ref = O.qdeim(Phis[b], r)
        np.testing.assert_array_equal(P[b], ref)
        G.assert_close(M[b], O.rebuild(Phis[b], ref), 1e-11, what="pinv %d" % b)
    assert not (h.status() & R.FLAG_SINGULAR).any()
    h.close()


def _front_state(problem, cells, seed):
    """Correction states with one sharp front of the feature variable per
    instance (a different place per instance) on a smooth random background."""
    nv = W.NVAR[problem]
    base = W.random_state(problem, cells, seed=seed, scale=0.5)
    out, o = [], 0
    feat = O.FGS_FEATURE[problem]
    for b, n in enumerate(cells):
        y = base[o:o + n * nv].reshape(n, nv).copy()
        x = W.centres(n)
        y[:, feat] += 0.3 * np.tanh((x - 0.3 - 0.2 * b) / 0.01)
        out.append(y.reshape(-1))
        o += n * nv
    return np.concatenate(out)


@pytest.mark.parametrize("problem", [W.BURGERS, W.EULER_RUSANOV, W.REACT])
@pytest.mark.parametrize("precision", [W.F64, W.F32])
def test_fgs_rows_bit_exact(precision, problem):
    """QDEIM's r rows, then the feature rows of the cells of largest squared
    feature gradient of y_corr (Burgers u, Euler density, reacting-model
    temperature), on a ragged pair of instances with one sharp front each."""
    import gpu_common as G
    from paper_2605_28684_amd import romhip as R
    nv = W.NVAR[problem]
    cells = [700, 1300] if nv < 12 else [200, 331]
    r, n_s = 6, 11
    if problem == W.BURGERS:
        w = W.burgers_batch_f32(n_inst=2, r=r, precision=precision)
        w.n_cells, w.phys = cells, [dict(nu=0.01)] * 2
        w.projection = W.LSPG
    elif problem == W.REACT:
        w = W.react10_f32(n_inst=2, n=cells[0], r=r, n_s=n_s, precision=precision)
        w.n_cells = cells
    else:
        w = _sod(cells, r, n_s, precision, W.HR_QDEIM_FGS)
    w.hyper, w.n_s, w.w_init = W.HR_QDEIM_FGS, n_s, r
    h = R.RomBatch(w, q0=None, use_graph=False)
    Phis = [G.rounded(_orth(nv * n, r, 95 + b), precision) for b, n in enumerate(cells)]
    y = G.rounded(_front_state(problem, cells, seed=9), precision)
    _load(h, w, Phis, precision, y)
    h.rom_rebuild()
    P = h.get(R.GET_SAMPLES).cpu().numpy().reshape(2, n_s)
    off = w.offsets()
    for b in range(2):
        ref = O.fgs(problem, Phis[b], y[off[b]:off[b + 1]], n_s)
        np.testing.assert_array_equal(P[b], ref)
        assert len(set(P[b].tolist())) == n_s
    h.close()


@pytest.mark.parametrize("kind", ["sod_qdeim", "react_fgs"])
def test_alg1_with_qdeim_and_fgs_fp64(kind):
    """Alg. 1 with LSPG steps and QDEIM (the paper's LSPG-QDEIM, on the Sod
    problem with Rusanov fluxes) or QDEIM + FGS (reacting model) from the
    oracle's offline state: sample rows bit-exact after every event, q~ and
    sigma within 1e-11."""
    import gpu_common as G
    import torch
    from paper_2605_28684_amd import romhip as R
    if kind == "sod_qdeim":
        w = W.sod_hllc_f32(n=128, r=5, n_s=5, z=3, precision=W.F64, flux=W.EULER_RUSANOV, N_t=40)
        w.hyper = W.HR_QDEIM
    else:
        w = W.react10_f32(n_inst=1, n=48, r=6, n_s=10, z=3, N_t=40, precision=W.F64)
        w.dt = 2e-4
        w.hyper = W.HR_QDEIM_FGS
    w.rom_tol = 1e-13
    prm = w.params()
    problem, phys = w.problem, w.phys[0]
    h = R.RomBatch(w, q0=G.to_dev(w.q0, W.F64), use_graph=False)
    st = O.offline(problem, phys, w.q0, prm)
    h.set(R.GET_BASIS, G.to_dev(st["Phi"].reshape(-1), W.F64))
    h.set(R.GET_SIGMA, torch.as_tensor(st["sigma"]))
    h.set(R.GET_A, torch.as_tensor(st["a"]))
    h.set(R.GET_YCORR, G.to_dev(st["y_corr"], W.F64))
    h.set(R.GET_DVAR, torch.as_tensor(st["d_var"]))
    h.set(R.GET_COUNTERS, [w.w_init, 0, 0, 0])
    h.rom_rebuild()
    np.testing.assert_array_equal(h.get(R.GET_SAMPLES).cpu().numpy(), st["P"])
    events = 0
    for k in range(9):
        h.rom_step(1)
        n = prm["w_init"] + k
        O.rom_fine_step(problem, phys, st, prm)
        if (n + 1 - prm["w_init"]) % prm["z"] == 0:
            O.adaptation_event(problem, phys, st, prm)
            events += 1
            np.testing.assert_array_equal(h.get(R.GET_SAMPLES).cpu().numpy(), st["P"])
        ref = O.reconstruct(st["q_ref"], st["d"], st["Phi"], st["a"])
        G.assert_close(G.host(h.get(R.GET_QTILDE)), ref, 1e-11, what="q~ %d" % k)
        G.assert_close(G.host(h.get(R.GET_SIGMA)), st["sigma"], 1e-11, what="sigma %d" % k)
    assert events == 3
    assert not (h.status() & (R.FLAG_NONFINITE | R.FLAG_SINGULAR | R.FLAG_ROM_NOCONV)).any()
    h.close()
