"""Benchmark of the adaptive-ROM hot path on one MI355X.

Workload (the batched Burgers configuration): 256 instances, N_i drawn from
{2048, 4096, 8192, 16384}, nu log-uniform in [1e-3, 1e-2], four seeded sine
modes, FP32 state and basis with FP64 core SVD / reduced solves, r = 32, an
iSVD update every z = 4 steps, full Galerkin reduced model.

A "step" is one adaptation window for the whole batch: z fine reduced steps of
every instance plus one adaptation event (coarse backward-Euler full-order step
of the correction state, iSVD update with re-orthonormalisation schedule,
rebuild, state transfer), replayed from a HIP graph.  The offline stage
(training steps, POD) runs before the timed region.

value        = instances x fine steps / second (events amortised in), batched path
plain        = the same kernels launched per instance from a host loop (no graph)
roofline     = dominant kernel of the step, timed live with HIP events on the
               launch stream, against the 8 TB/s HBM peak
fom_residual = R(q) on the 64 x 262,144-cell Euler (Rusanov, FP32) shape:
               cell-updates/s and fraction of the HBM roofline (24 B/cell)
cpu_baseline = the FP64 CPU oracle timed on a bounded sample of the same workload
               (cores = BLAS threads it used; affinity_cores and cpu_model describe the host)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "adaptive-ROM steps/s + FOM cell-updates/s (% HBM roofline), batched vs plain"
HBM_PEAK_GBS = 8000.0
MFMA_F32_TFLOPS = 157.3

# HBM traffic per launch from rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE
# in KiB per dispatch, bench.py --only galerkin / --only residual), each scaled
# by what the same counter reads for a plain 512 MiB device copy (bench.py --only
# copy: FETCH_SIZE reads 262157 KiB for 524288 KiB moved, WRITE_SIZE exactly
# 524288 KiB).  Valid only for the kernel version they were taken on; the
# summaries of those runs are kept in the profiles directory.
COPY_SCALE = {"fetch": 524288.0 / 262157.4, "write": 1.0}
MEASURED_KIB = {
    "k_galerkin_mfma<32>": {"fetch": 133445.3, "write": 4245.8},
    # streaming Euler residual on the 64 x 262,144-cell shape, every launch shape
    # of the autotuner (bench.py --only residual walks them in order)
    "k_residual_euler/0": {"fetch": 101937.4, "write": 196608.3},
    "k_residual_euler/1": {"fetch": 101935.0, "write": 196608.0},
    "k_residual_euler/2": {"fetch": 105509.1, "write": 196609.4},
    "k_residual_euler/3": {"fetch": 105509.1, "write": 196608.4},
    "k_residual_euler/4": {"fetch": 105509.0, "write": 196608.0},
    "k_residual_euler/5": {"fetch": 112667.6, "write": 196608.9},
    "k_residual_euler/6": {"fetch": 112674.0, "write": 196608.5},
    "k_residual_euler/7": {"fetch": 101944.8, "write": 204654.5},
    "k_residual_euler/8": {"fetch": 105521.6, "write": 205916.6},
    "k_residual_euler/9": {"fetch": 105512.3, "write": 203707.4},
    "k_residual_euler/10": {"fetch": 112684.5, "write": 230598.9},
    "k_residual_euler/11": {"fetch": 112682.3, "write": 232216.8},
}


def traffic_bytes(key):
    m = MEASURED_KIB.get(key)
    if m is None:
        return None
    return int(1024 * (m["fetch"] * COPY_SCALE["fetch"] + m["write"] * COPY_SCALE["write"]))


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--plain-inst", type=int, default=32,
                   help="instances timed on the plain per-instance path")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--no-configs", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=20.0)
    p.add_argument("--only", choices=["all", "copy", "galerkin", "residual", "windows", "adjoint",
                                      "rollout", "configs"],
                   default="all",
                   help="profiling runs: 'copy' times a plain 512 MiB device copy (the "
                        "reference for counter scaling), 'galerkin' only the Galerkin pass, "
                        "'residual' only R(q), 'windows' the offline stage plus --warmup and "
                        "--steps adaptation windows, 'adjoint' the online adjoint, 'rollout' "
                        "the 64 x 262,144 Euler rollout adjoint through Alg. 1 over --steps "
                        "fine steps (0: the full 990), 'configs' the other configurations' "
                        "figures; 'all' is the benchmark")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, budget_s):
    """The FP64 oracle on a bounded sample: instances of the same workload, the
    offline stage untimed, then whole adaptation windows timed until the budget."""
    import numpy as np
    from oracle import rom as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    prm = w.params()
    order = np.argsort(np.asarray(w.n_cells))
    picks = [int(order[len(order) * k // 4]) for k in range(4)]  # spread over the size mix
    steps = 0
    cells = 0
    t_total = 0.0
    for b in picks:
        q0 = w.instance(b)
        st = O.offline(W.BURGERS, w.phys[b], q0, prm)
        n = prm["w_init"]
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s / len(picks):
            for _ in range(prm["z"]):
                O.rom_fine_step(W.BURGERS, w.phys[b], st, prm)
                if (n + 1 - prm["w_init"]) % prm["z"] == 0:
                    O.adaptation_event(W.BURGERS, w.phys[b], st, prm)
                n += 1
                steps += 1
                cells += w.n_cells[b]
        t_total += time.perf_counter() - t0
    mean_cells = float(np.mean(w.n_cells))
    # scale to the workload's size mix: time per instance-step grows with N
    per_cell_step = t_total / cells
    value = 1.0 / (per_cell_step * mean_cells)
    return dict(value=value, unit="steps/s", cores=int(threads), kind="oracle",
                affinity_cores=len(os.sched_getaffinity(0)), cpu_model=_cpu_model(),
                sample="%d instance-steps of 4 instances (N=%s) in whole windows, %.1f s; "
                       "scaled by mean N of the batch" % (steps, [w.n_cells[b] for b in picks],
                                                         t_total))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _timed(torch, fn, reps):
    """Mean ms per call of fn (enqueued on the current stream), after one warm-up."""
    fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _or_all(flags):
    acc = 0
    for x in flags:
        acc |= int(x)
    return acc


def _timed_once(torch, fn):
    """ms of one call of fn (enqueued on the current stream)."""
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    fn()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def config_measurements(torch, W, R):
    """The other configurations' figures: C1 (the FP64 parity anchor, steps/s), C3
    (one Sod/HLLC instance with HR-LSPG: windows and the cost split of an event),
    C5 (32 reacting instances with HR-LSPG: windows and R(q), which is
    MALL-resident at 101 MB) and C4 (64 Euler instances: the full-order step and
    the checkpointed rollout adjoint)."""
    out = {}
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        # C1
        w = W.burgers_512_f64()
        h = R.RomBatch(w, q0=torch.as_tensor(w.q0, dtype=torch.float64, device="cuda"),
                       use_graph=True)
        nwin = 20
        ms = _timed(torch, lambda: h.rom_step(w.z * nwin), 1) / nwin
        out["C1_burgers_512_f64"] = dict(ms_per_window=round(ms, 4),
                                         steps_per_s=w.z / (ms * 1e-3))
        h.close()
        # C3
        w = W.sod_hllc_f32()
        h = R.RomBatch(w, q0=torch.as_tensor(w.q0, dtype=torch.float32, device="cuda"),
                       use_graph=True)
        ms_win = _timed(torch, lambda: h.rom_step(w.z * 5), 1) / 5
        y = h.get(R.GET_YCORR).clone()
        y2 = torch.empty_like(y)
        ms_coarse = _timed(torch, lambda: h.fom_step(y, w.z * w.dt, out=y2), 3)
        ms_isvd = _timed(torch, lambda: h.isvd_update(y2), 3)
        ms_rebuild = _timed(torch, lambda: h.rom_rebuild(), 3)
        split_choice = h.autotune(R.TUNE_DEIM_PASS)
        ms_rebuild_tuned = _timed(torch, lambda: h.rom_rebuild(), 3)
        h.set_tuning(R.TUNE_DEIM_PASS, 0)
        out["C3_sod_hllc_65536_f32"] = dict(
            ms_per_window=round(ms_win, 4), steps_per_s=w.z / (ms_win * 1e-3),
            event_split_ms=dict(coarse_step=round(ms_coarse, 4), isvd_update=round(ms_isvd, 4),
                                deim_rebuild=round(ms_rebuild, 4)),
            deim_pass_tuned=dict(choice=split_choice, rebuild_ms=round(ms_rebuild_tuned, 4)))
        h.close()
        # C5
        w = W.react10_f32()
        q = torch.as_tensor(w.q0, dtype=torch.float32, device="cuda")
        h = R.RomBatch(w, q0=q, use_graph=True)
        ms_win = _timed(torch, lambda: h.rom_step(w.z * 3), 1) / 3
        ms_res = h.profile(R.PROF_RESIDUAL, 20, q)
        cells = sum(w.n_cells)
        cu = cells / (ms_res * 1e-3)
        out["C5_react10_32x32768_f32"] = dict(
            ms_per_window=round(ms_win, 4),
            instance_steps_per_s=w.n_inst * w.z / (ms_win * 1e-3),
            residual_cell_updates_per_s=cu,
            residual_frac_of_peak=round(cu / (HBM_PEAK_GBS * 1e9 / 96.0), 4),
            residual_note="96 B per cell; 101 MB per evaluation is MALL-resident")
        h.close()
        # C4: 64 Euler (Rusanov) instances of 262,144 cells, the full-order rollout
        # and its checkpointed adjoint
        w = W.euler_adjoint_f32(n_inst=64, n=262144)
        h = R.RomBatch(w, q0=None, use_graph=False)
        q0 = torch.as_tensor(w.q0, dtype=torch.float32, device="cuda")
        gbar = q0 - torch.as_tensor(w.extra["target"], dtype=torch.float32, device="cuda")
        q = q0.clone()
        gq = torch.empty_like(q0)
        ms_step = _timed(torch, lambda: h.fom_step(q, w.dt, out=q), 5)
        # the solver part size chosen by timing (candidate 0 is the default above)
        part_choice = h.autotune(R.TUNE_BT_PART, q0)
        ms_step_tuned = _timed(torch, lambda: h.fom_step(q, w.dt, out=q), 5)
        h.set_tuning(R.TUNE_BT_PART, 0)
        n_steps, n_ckpt = 16, 4
        ms_vjp = _timed(torch, lambda: h.fom_rollout_vjp(q0, n_steps, w.dt, gbar, n_ckpt=n_ckpt,
                                                     out=gq), 2)
        cells = sum(w.n_cells)
        out["C4_euler_rusanov_64x262144_f32"] = dict(
            fom_step_ms=round(ms_step, 4), fom_step_cell_updates_per_s=cells / (ms_step * 1e-3),
            fom_step_tuned_part_choice=part_choice, fom_step_tuned_ms=round(ms_step_tuned, 4),
            rollout_vjp_ms_per_step=round(ms_vjp / n_steps, 4),
            rollout_vjp_steps=n_steps, rollout_vjp_checkpoints=n_ckpt,
            note="backward-Euler Newton steps at dt = 0.064/N; the adjoint call runs the "
                 "forward pass, the checkpointed recomputation and the transposed solves")
        h.close()
        # the adaptive ROM's rollout adjoint at the full horizon: dL/dq0 through the
        # offline stage (10 training steps, POD) and 990 HR-LSPG steps with 99
        # events, 32 checkpoint segments (re-orthonormalisation off, so that no
        # update falls outside what the adjoint differentiates)
        w.reorth_every = 0
        h = R.RomBatch(w, q0=None, use_graph=False)
        T = w.N_t - w.w_init
        tgt = torch.as_tensor(w.extra["target"], dtype=torch.float32, device="cuda")

        def forward():
            h.offline(q0)
            h.rom_step(T)

        forward()   # warm-up
        torch.cuda.synchronize()
        ms_fwd = _timed_once(torch, forward)
        gq_rom = torch.empty_like(q0)
        gb = (h.get(R.GET_QTILDE) - tgt).contiguous()
        ms_adj = _timed_once(torch, lambda: h.rollout_vjp(q0, T, gb, n_ckpt=32, out=gq_rom))
        fl = h.status()
        out["C4_euler_rusanov_64x262144_f32"].update(
            rom_rollout_forward_ms=round(ms_fwd, 2), rom_rollout_vjp_ms=round(ms_adj, 2),
            rom_rollout_steps=T, rom_rollout_events=T // w.z, rom_rollout_segments=32,
            rom_rollout_vjp_over_forward=round(ms_adj / ms_fwd, 3),
            rom_rollout_flags_or=_or_all(fl),
            rom_rollout_note="dL/dq0 through Alg. 1 (offline stage, HR-LSPG steps with "
                             "greedy DEIM rows held fixed, iSVD events); the adjoint call "
                             "includes its own forward pass and the recomputation")
        h.close()
        # the explicit path (Sec. 5.3, App. D) on the reacting shape: SSPRK(4,3)
        # DEIM-Galerkin fine steps on the limited second-order f, QDEIM + FGS rows
        # (n_s = 2r), coarse SSPRK(4,3) steps of z dt; iSVD against Direct updates
        # (the comparison of the paper's detonation timing table).  dt is set
        # inside the explicit stability limit of 32,768 cells with diffusion 1e-3.
        expl = {}
        for rule in ("isvd", "direct"):
            w = W.react10_f32()
            w.projection, w.scheme, w.hyper = W.GALERKIN, "ssprk43", W.HR_QDEIM_FGS
            w.dt = 2e-8
            w.update, w.window = rule, (w.r if rule == "direct" else 0)
            h = R.RomBatch(w, q0=torch.as_tensor(w.q0, dtype=torch.float32, device="cuda"),
                           use_graph=rule == "isvd")
            ms = _timed(torch, lambda: h.rom_step(w.z * 3), 1) / 3
            expl[rule] = dict(ms_per_window=round(ms, 4),
                              instance_steps_per_s=w.n_inst * w.z / (ms * 1e-3),
                              flags_or=_or_all(h.status()))
            h.close()
        out["explicit_path_react10_32x32768_f32"] = dict(
            expl, dt=2e-8, r=64, n_s=128, z=10, direct_window=64)
        # cost of one basis update per rule (App. A) on the batched Burgers shape
        # and the Sod shape: iSVD (Alg. 2), windowed SVD (Alg. A.1), Direct (Alg. A.2)
        rules = {}
        for name, mk, window in (("C2_burgers_batch_f32", W.burgers_batch_f32, 40),
                                 ("C3_sod_hllc_65536_f32", W.sod_hllc_f32, 48)):
            per = {}
            for rule in ("isvd", "wsvd", "direct"):
                w = mk()
                w.update, w.window = rule, window
                h = R.RomBatch(w, q0=torch.as_tensor(w.q0, dtype=torch.float32, device="cuda"),
                               use_graph=False)
                y = h.get(R.GET_YCORR).clone()
                per[rule] = round(_timed(torch, lambda: h.isvd_update(y), 3), 4)
                h.close()
            rules[name] = dict(ms_per_update=per, window=window, r=mk().r)
        out["update_rules"] = rules
        # cost of one rebuild per sampling rule (Sec. 3.2) on the Sod and reacting shapes
        samplers = {}
        for name, mk, r in (("C3_sod_hllc_65536_f32", W.sod_hllc_f32, 40),
                            ("C5_react10_32x32768_f32", W.react10_f32, 64)):
            per = {}
            for label, hyper, n_s in (("deim", W.HR_DEIM, 2 * r), ("qdeim", W.HR_QDEIM, r),
                                      ("qdeim_fgs", W.HR_QDEIM_FGS, 2 * r)):
                w = mk()
                w.hyper, w.n_s = hyper, n_s
                h = R.RomBatch(w, q0=torch.as_tensor(w.q0, dtype=torch.float32, device="cuda"),
                               use_graph=False)
                per[label] = dict(n_s=n_s, ms_per_rebuild=round(_timed(torch, h.rom_rebuild, 3), 4))
                h.close()
            samplers[name] = per
        out["samplers"] = samplers
    return out


def adjoint_ms(torch, h, w, n_win):
    """Wall time per window of rom_online_vjp over n_win whole windows (the forward
    pass, its checkpointed recomputation and the reverse pass; the call
    synchronises), after one untimed call."""
    qbar = torch.full((h.total_dof,), 1e-3, dtype=torch.float32, device="cuda")
    h.online_vjp(w.z, qbar)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.online_vjp(w.z * n_win, qbar)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / n_win


def profile_only(args, torch, W, R):
    """One kernel family at a time, for rocprofv3 counter runs."""
    reps = max(args.steps, 1)
    if args.only == "copy":
        n = 128 * 1024 * 1024                      # 512 MiB of float32 each way
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(reps):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy: %d x %d bytes" % (reps, 4 * n))
    elif args.only == "windows":
        w = W.burgers_batch_f32()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            h = R.RomBatch(w, q0=torch.as_tensor(w.q0, dtype=torch.float32, device="cuda"),
                           use_graph=True)
            h.rom_step(w.z * args.warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if args.steps:
                h.rom_step(w.z * args.steps)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            h.close()
        log("windows: %d after %d warm-up, %.3f ms each" % (
            args.steps, args.warmup, 1e3 * (t1 - t0) / max(args.steps, 1)))
    elif args.only == "configs":
        log("other configurations: " + json.dumps(config_measurements(torch, W, R)))
    elif args.only == "adjoint":
        w = W.burgers_batch_f32()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            h = R.RomBatch(w, q0=torch.as_tensor(w.q0, dtype=torch.float32, device="cuda"),
                           use_graph=False)
            ms = adjoint_ms(torch, h, w, max(args.steps, 1))
            h.close()
        log("online adjoint: %d window(s), %.3f ms per window" % (max(args.steps, 1), ms))
    elif args.only == "rollout":
        w = W.euler_adjoint_f32(n_inst=64, n=262144)
        w.reorth_every = 0
        T = args.steps if args.steps > 0 else w.N_t - w.w_init
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            h = R.RomBatch(w, q0=None, use_graph=False)
            q0 = torch.as_tensor(w.q0, dtype=torch.float32, device="cuda")
            tgt = torch.as_tensor(w.extra["target"], dtype=torch.float32, device="cuda")
            h.offline(q0)
            h.rom_step(T)
            gb = (h.get(R.GET_QTILDE) - tgt).contiguous()
            gq = torch.empty_like(q0)
            ms = _timed_once(torch, lambda: h.rollout_vjp(q0, T, gb, out=gq))
            h.close()
        log("rollout adjoint: %d fine steps, %.2f ms" % (T, ms))
    elif args.only == "galerkin":
        w = W.burgers_batch_f32()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            h = R.RomBatch(w, q0=torch.as_tensor(w.q0, dtype=torch.float32, device="cuda"),
                           use_graph=True)
            ms = h.profile(R.PROF_GALERKIN_PASS, reps)
            h.close()
        log("galerkin pass: %.5f ms per launch" % ms)
    else:
        # every launch shape in turn, reps launches each (dispatch order: shape
        # 0's launches first), so counter runs give the traffic of each shape
        we = W.euler_adjoint_f32(n_inst=64, n=262144)
        he = R.RomBatch(we, q0=None, use_graph=False)
        qe = torch.as_tensor(we.q0, dtype=torch.float32, device="cuda")
        for i in range(he.set_tuning(R.TUNE_RESIDUAL, -1)):
            he.set_tuning(R.TUNE_RESIDUAL, i)
            ms = he.profile(R.PROF_RESIDUAL, reps, qe)
            log("residual shape %d: %.5f ms per launch" % (i, ms))
        he.close()
    return 0


def main():
    args = parse()
    if args.gpus != 1:
        log("bench.py runs on one GPU only: this build has no multi-GPU path "
            "(instances would shard across GPUs with no communication).")
        sys.exit(2)
    import numpy as np
    import torch
    global W
    from paper_2605_28684_amd import workloads as W
    from paper_2605_28684_amd import romhip as R

    torch.cuda.set_device(0)
    if args.only != "all":
        return profile_only(args, torch, W, R)
    w = W.burgers_batch_f32()
    z = w.z
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        # FOM residual roofline on the 64 x 262,144 Euler shape (403 MB per evaluation),
        # measured first, on a GPU that has not yet run the minute of batched work
        # below (measured later in the run, the same launches take about 3% longer)
        we = W.euler_adjoint_f32(n_inst=64, n=262144)
        he = R.RomBatch(we, q0=None, use_graph=False)
        qe = torch.as_tensor(we.q0, dtype=torch.float32, device="cuda")
        shape = he.autotune(R.TUNE_RESIDUAL, qe)
        he.profile(R.PROF_RESIDUAL, 3, qe)
        ms_res = he.profile(R.PROF_RESIDUAL, 50, qe)
        cells = 64 * 262144
        res_bytes = cells * 3 * 4 * 2
        res_gbs = res_bytes / (ms_res * 1e-3) / 1e9
        fom = dict(workload="euler_rusanov_64x262144_f32", ms_per_launch=round(ms_res, 5),
                   cell_updates_per_s=cells / (ms_res * 1e-3), achieved_GBs=round(res_gbs, 1),
                   frac_hbm=round(res_gbs / HBM_PEAK_GBS, 4), bytes_per_launch=res_bytes,
                   tuned_shape=int(shape), traffic=traffic_bytes("k_residual_euler/%d" % shape))
        ms_vjp = he.profile(R.PROF_RESIDUAL_VJP, 20, qe)
        fom["vjp_ms_per_launch"] = round(ms_vjp, 5)
        fom["vjp_frac_hbm"] = round(cells * 3 * 4 * 3 / (ms_vjp * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        he.close()
        log("R(q): %.4f ms, %.3g cell-updates/s, %.1f%% of HBM" % (ms_res, fom["cell_updates_per_s"],
                                                                100 * fom["frac_hbm"]))

        q0 = torch.as_tensor(w.q0, dtype=torch.float32, device="cuda")
        t0 = time.time()
        h = R.RomBatch(w, q0=q0, use_graph=True)
        torch.cuda.synchronize()
        log("offline stage: %.2f s (%d instances, %d DOF)" % (time.time() - t0, w.n_inst,
                                                             h.total_dof))
        # warmup (first window captures the graph)
        h.rom_step(z * args.warmup)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(s)
        h.rom_step(z * args.steps)
        ev1.record(s)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        ms_per_step = ms / args.steps
        value = w.n_inst * z * args.steps / (ms / 1e3)
        flags = h.status()
        log("batched: %.3f ms per window, %.4g instance-steps/s, flags %s"
            % (ms_per_step, value, np.unique(flags).tolist()))

        # dominant kernel: the fused Galerkin pass (one launch = one pass over the basis)
        reps = 50
        ms_pass = h.profile(R.PROF_GALERKIN_PASS, reps)
        r = w.r
        tot = h.total_dof
        bytes_pass = tot * r * 4 + tot * 4 + 2 * 2 * r * 4 * w.n_inst  # basis, q_ref, halo rows
        achieved = bytes_pass / (ms_pass * 1e-3) / 1e9
        kname = "k_galerkin_mfma<%d>" % r          # the name kernel traces give it
        roofline = dict(kernel=kname, bound="hbm", achieved=round(achieved, 1),
                        peak=HBM_PEAK_GBS, unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                        traffic=traffic_bytes(kname), ms_per_launch=round(ms_pass, 5),
                        bytes_per_launch=int(bytes_pass))
        # the same pass against the FP32 MFMA peak: 2 N r^2 flops per launch
        flops_pass = 2.0 * tot * r * r
        roofline_mfma = dict(kernel=kname, bound="mfma",
                             achieved=round(flops_pass / (ms_pass * 1e-3) / 1e12, 2),
                             peak=MFMA_F32_TFLOPS, unit="TFLOP/s",
                             frac=round(flops_pass / (ms_pass * 1e-3) / 1e12 / MFMA_F32_TFLOPS, 4))
        ms_proj = h.profile(R.PROF_ISVD_PROJECT, reps, h.get(R.GET_YCORR))
        # the online adjoint (extension): gradient through whole windows
        adj_ms = adjoint_ms(torch, h, w, 2)
        log("online adjoint: %.3f ms per window" % adj_ms)
        h.close()

        # plain path: the same kernels per instance in a host loop, no graph
        plain = None
        if not args.no_plain:
            idx = np.linspace(0, w.n_inst - 1, args.plain_inst).round().astype(int)
            hs = []
            for b in idx:
                wb = W.burgers_batch_f32()
                wb.n_cells = [w.n_cells[b]]
                wb.phys = [w.phys[b]]
                wb.q0 = w.instance(b)
                hs.append(R.RomBatch(wb, q0=torch.as_tensor(wb.q0, dtype=torch.float32,
                                                              device="cuda"), use_graph=False))
            torch.cuda.synchronize()
            for hb in hs:
                hb.rom_step(z)
            torch.cuda.synchronize()
            nwin = max(1, args.steps // 4)
            ev0.record(s)
            for _ in range(nwin):
                for hb in hs:
                    hb.rom_step(z)
            ev1.record(s)
            torch.cuda.synchronize()
            pms = ev0.elapsed_time(ev1)
            sub_cells = sum(w.n_cells[b] for b in idx)
            # per-instance time scales with N: extrapolate by the batch's total cells
            plain_value = len(idx) * z * nwin / (pms / 1e3) * (sub_cells / len(idx)) / np.mean(w.n_cells)
            plain = dict(value=plain_value, unit="steps/s", instances_timed=int(len(idx)),
                         windows=nwin, speedup_batched=round(value / plain_value, 2))
            for hb in hs:
                hb.close()
            log("plain: %.4g instance-steps/s (speed-up %.2fx)" % (plain_value, value / plain_value))

    configs = None
    if not args.no_configs:
        configs = config_measurements(torch, W, R)
        log("other configurations: %s" % json.dumps(configs))

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, args.cpu_seconds)
        log("cpu baseline: %.4g steps/s on %d threads" % (cpu["value"], cpu["cores"]))

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "burgers_batch_f32", "n_inst": w.n_inst,
                   "cells_total": int(sum(w.n_cells)), "r": w.r, "z": w.z, "dt": w.dt,
                   "lambda": w.lam, "projection": "galerkin", "step": "one adaptation window "
                   "(z fine steps + event) of all instances", "parallelism": "single GPU, batch"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "plain": plain,
        "fom_residual": fom,
        "isvd_project_ms": round(ms_proj, 5),
        "roofline_mfma": roofline_mfma,
        "other_configs": configs,
        "online_adjoint": {"ms_per_window": round(adj_ms, 3), "windows": 2,
                           "what": "rom_online_vjp: forward recording the horizon (sqrt(T) "
                                   "checkpoints and recomputation when memory is short), "
                                   "reverse (transposed reduced solves, iSVD backward, "
                                   "transposed banded solves)"},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
