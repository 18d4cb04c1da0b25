"""rom_save / rom_load: a saved state resumed on a new handle (or rewound on
the same one) continues with the same bits as the uninterrupted run, on the
overlapped Galerkin windows (FP32, graphs), on hyper-reduced LSPG windows
(FP32, DEIM, graphs), on eager FP64 Galerkin steps and with the Direct rule
(whose snapshot window is part of the state); mismatched or damaged
states are refused without touching the handle."""
import numpy as np
import pytest

from paper_2605_28684_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(kind):
    if kind == "burgers_f32_graph":
        w = W.burgers_batch_f32(n_inst=5, r=32)
        w.n_cells = [2048, 4096, 700, 1024, 3000]
        w.phys = [dict(nu=0.002 + 0.002 * b) for b in range(5)]
        w.q0 = np.concatenate([0.3 * np.sin(2 * np.pi * W.centres(n) + b) + 0.5
                               for b, n in enumerate(w.n_cells)])
        return w, True
    if kind == "sod_hr_f32_graph":
        return W.sod_hllc_f32(n=1500, r=12, n_s=20, z=3, precision=W.F32), True
    w = W.burgers_512_f64(n=256, N_t=200, w_init=20, r=6, z=5)
    if kind == "burgers_direct_f64":
        w.update, w.window = "direct", 8
    return w, False


def _state(h):
    import torch
    from paper_2605_28684_amd import romhip as R
    torch.cuda.synchronize()
    out = {k: h.get(getattr(R, k)).cpu().numpy().copy()
           for k in ("GET_BASIS", "GET_SIGMA", "GET_A", "GET_QTILDE", "GET_YCORR", "GET_SAMPLES",
                     "GET_PINV")}
    out["counters"] = list(h.get(R.GET_COUNTERS))
    out["flags"] = h.status().copy()
    if h.cfg.update_rule != R.UPDATE_ISVD:
        out["window"] = h.get(R.GET_WINDOW).cpu().numpy().copy()
    return out


@pytest.mark.parametrize("kind", ["burgers_f32_graph", "sod_hr_f32_graph", "burgers_f64_eager",
                                  "burgers_direct_f64"])
def test_save_load_resume_is_bitwise(kind):
    import torch
    from paper_2605_28684_amd import romhip as R
    w, graph = _case(kind)
    dt = torch.float64 if w.precision == W.F64 else torch.float32
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        h1 = R.RomBatch(w, q0=torch.as_tensor(w.q0, dtype=dt, device="cuda"), use_graph=graph)
        h1.rom_step(2 * w.z)
        blob = h1.save()
        before = _state(h1)
        n = 3 * w.z
        h1.rom_step(n)                               # the uninterrupted run
        ref = _state(h1)
        h2 = R.RomBatch(w, q0=None, use_graph=graph)
        h2.load(blob)                                # resume on a fresh handle
        assert _state(h2)["counters"] == before["counters"]
        h2.rom_step(n)
        got = _state(h2)
        h1.load(blob)                                # rewind the same handle
        h1.rom_step(n)
        again = _state(h1)
        for k in ref:
            assert np.array_equal(np.asarray(ref[k]), np.asarray(got[k])), k
            assert np.array_equal(np.asarray(ref[k]), np.asarray(again[k])), k
        assert ref["counters"][2] == 5
        h1.close()
        h2.close()


def test_load_refuses_mismatched_or_damaged_states():
    import torch
    from paper_2605_28684_amd import romhip as R
    w, _ = _case("burgers_f64_eager")
    h = R.RomBatch(w, q0=torch.as_tensor(w.q0, dtype=torch.float64, device="cuda"),
                   use_graph=False)
    h.rom_step(3)
    blob = h.save()
    keep = _state(h)
    other = W.burgers_512_f64(n=256, N_t=200, w_init=20, r=7, z=5)   # another r
    h_other = R.RomBatch(other, q0=None, use_graph=False)
    with pytest.raises(R.RomError) as e:
        h_other.load(blob[:blob.numel()])
    assert e.value.code == R.ROM_E_INVAL
    with pytest.raises(R.RomError) as e:
        h.load(blob[:blob.numel() - 8])              # truncated
    assert e.value.code == R.ROM_E_INVAL
    bad = blob.clone()
    bad[0] ^= 1                                      # damaged magic
    with pytest.raises(R.RomError) as e:
        h.load(bad)
    assert e.value.code == R.ROM_E_INVAL
    with pytest.raises(R.RomError) as e:             # a destination that is too small
        h.save(out=torch.empty(16, dtype=torch.uint8, device="cuda"))
    assert e.value.code == R.ROM_E_INVAL
    after = _state(h)
    for k in keep:
        assert np.array_equal(np.asarray(keep[k]), np.asarray(after[k])), k
    h.close()
    h_other.close()
