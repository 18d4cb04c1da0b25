"""Python binding of the romhip C interface (ctypes; argument marshalling only).

Every call forwards device pointers of torch tensors and the current HIP stream
to ``libromhip.so``; all arithmetic runs in the library's HIP kernels.  The
library must have been built (``paper_2605_28684_amd.build``); importing this
module on a machine without it raises immediately.

The functions mirror the C entry points of ``include/romhip.h``:
``rom_create``, ``rom_destroy``, ``fom_residual``, ``fom_step``,
``isvd_update``, ``rom_rebuild``, ``rom_step``, ``rom_get``, ``rom_set``,
``rom_get_status``, ``fom_residual_vjp``, ``fom_step_vjp``; ``RomBatch`` bundles
a handle with its layout.
"""
import ctypes
import os

import numpy as np
import torch

from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libromhip.so")

ROM_OK = 0
ROM_E_INVAL, ROM_E_NOMEM, ROM_E_DEVICE, ROM_E_STATE, ROM_E_UNSUPPORTED = -1, -2, -3, -6, -7
STATUS = {0: "ROM_OK", -1: "ROM_E_INVAL", -2: "ROM_E_NOMEM", -3: "ROM_E_DEVICE",
          -6: "ROM_E_STATE", -7: "ROM_E_UNSUPPORTED"}
FLAG_NEWTON_NOCONV, FLAG_FLOOR, FLAG_NONFINITE, FLAG_RHO_ZERO = 1, 2, 4, 8
FLAG_SINGULAR, FLAG_ROM_NOCONV, FLAG_REORTH = 16, 32, 64
GET_BASIS, GET_SIGMA, GET_A, GET_QTILDE, GET_SAMPLES, GET_YCORR = 0, 1, 2, 3, 4, 5
GET_QREF, GET_DVAR, GET_PINV, GET_COUNTERS, GET_UBAR, GET_WINDOW = 6, 7, 8, 9, 10, 11
UPDATE_ISVD, UPDATE_WSVD, UPDATE_DIRECT = 0, 1, 2
SCHEME_BE, SCHEME_SSPRK43 = 0, 1
N_COUNTERS = 6


class RomError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class rom_config(ctypes.Structure):
    _fields_ = [("problem", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("projection", ctypes.c_int32), ("hyper", ctypes.c_int32),
                ("n_inst", ctypes.c_int32),
                ("n_cells", ctypes.POINTER(ctypes.c_int64)),
                ("phys", ctypes.POINTER(ctypes.c_double)),
                ("n_phys", ctypes.c_int32),
                ("r", ctypes.c_int32), ("n_s", ctypes.c_int32), ("w_init", ctypes.c_int32),
                ("z", ctypes.c_int32),
                ("newton_max", ctypes.c_int32), ("rom_max", ctypes.c_int32),
                ("reorth_every", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("update_rule", ctypes.c_int32), ("window", ctypes.c_int32),
                ("scheme", ctypes.c_int32),
                ("lambda_", ctypes.c_double), ("dt", ctypes.c_double),
                ("newton_tol", ctypes.c_double), ("rom_tol", ctypes.c_double),
                ("tau_orth", ctypes.c_double), ("tau_rho", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libromhip.so is not built (run paper_2605_28684_amd.build): " + LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "rom_create": [ctypes.POINTER(rom_config), vp, vp, ctypes.POINTER(vp)],
        "rom_destroy": [vp],
        "fom_residual": [vp, vp, vp, d, vp, vp],
        "fom_step": [vp, vp, d, vp, vp, vp],
        "isvd_update": [vp, vp, vp],
        "rom_rebuild": [vp, vp],
        "rom_step": [vp, i32, vp],
        "rom_get": [vp, i32, vp, vp],
        "rom_set": [vp, i32, vp, vp],
        "rom_get_status": [vp, vp],
        "rom_save": [vp, vp, ctypes.POINTER(ctypes.c_size_t), vp],
        "rom_load": [vp, vp, ctypes.c_size_t, vp],
        "rom_clear_status": [vp, vp],
        "fom_residual_vjp": [vp, vp, vp, d, vp, vp, vp, vp],
        "fom_step_vjp": [vp, vp, d, vp, vp, vp],
        "fom_rollout_vjp": [vp, vp, i32, d, i32, vp, vp, vp],
        "fom_rollout_vjp_noalloc": [vp, vp, i32, d, i32, vp, vp, vp],
        "rom_online_vjp": [vp, i32, i32, vp, vp, vp, vp, vp, vp],
        "rom_offline": [vp, vp, vp],
        "rom_rollout_vjp": [vp, vp, i32, i32, vp, vp, vp],
        "rom_autotune": [vp, i32, vp, ctypes.POINTER(i32), vp],
        "rom_set_tuning": [vp, i32, i32, ctypes.POINTER(i32)],
        "rom_query": [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32),
                      ctypes.POINTER(i32)],
        "rom_profile": [vp, i32, i32, vp, ctypes.POINTER(d), vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.rom_last_error.argtypes = []
    lib.rom_last_error.restype = ctypes.c_char_p
    return lib


LIB = _load()
SYMBOLS = ("rom_create", "rom_destroy", "fom_residual", "fom_step", "isvd_update", "rom_rebuild",
           "rom_step", "rom_get", "rom_set", "rom_save", "rom_load", "rom_get_status", "rom_clear_status",
           "fom_residual_vjp", "fom_step_vjp", "fom_rollout_vjp", "fom_rollout_vjp_noalloc",
           "rom_online_vjp", "rom_offline", "rom_rollout_vjp", "rom_autotune",
           "rom_set_tuning", "rom_query", "rom_profile", "rom_last_error")
TUNE_RESIDUAL, TUNE_DEIM_PASS, TUNE_BT_PART = 0, 1, 2
PROF_RESIDUAL, PROF_GALERKIN_PASS, PROF_ISVD_PROJECT, PROF_RESIDUAL_VJP, PROF_FOM_STEP = range(5)


def _check(code):
    if code != ROM_OK:
        raise RomError(code, LIB.rom_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor required")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor required")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_config(w: W.Workload, use_graph=True, precision=None, **over):
    """rom_config from a workload (host arrays kept alive on the returned object)."""
    cfg = rom_config()
    prec = w.precision if precision is None else precision
    cfg.problem, cfg.precision = w.problem, prec
    cfg.projection, cfg.hyper = w.projection, w.hyper
    cfg.n_inst = w.n_inst
    nc = np.ascontiguousarray(np.asarray(w.n_cells, dtype=np.int64))
    ph = np.ascontiguousarray(w.phys_vector())
    cfg.n_cells = nc.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    cfg.phys = ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    cfg.n_phys = ph.shape[1]
    cfg.r, cfg.n_s, cfg.w_init, cfg.z = w.r, w.n_s, w.w_init, w.z
    cfg.newton_max, cfg.rom_max, cfg.reorth_every = w.newton_max, w.rom_max, w.reorth_every
    cfg.use_graph = 1 if use_graph else 0
    cfg.update_rule = {"isvd": UPDATE_ISVD, "wsvd": UPDATE_WSVD, "direct": UPDATE_DIRECT}[w.update]
    cfg.window = w.window
    cfg.scheme = {"be": SCHEME_BE, "ssprk43": SCHEME_SSPRK43}[w.scheme]
    cfg.lambda_, cfg.dt = w.lam, w.dt
    cfg.newton_tol, cfg.rom_tol = w.newton_tol, w.rom_tol
    cfg.tau_orth, cfg.tau_rho = w.tau_orth, w.tau_rho
    for k, v in over.items():
        setattr(cfg, "lambda_" if k == "lam" else k, v)
    cfg._keep = (nc, ph)
    return cfg


def torch_dtype(precision):
    return torch.float64 if precision == W.F64 else torch.float32


class RomBatch:
    """A batch handle plus its layout.  q0: device tensor of the initial states
    (or None to create a handle for full-order calls / rom_set only)."""

    def __init__(self, w: W.Workload, q0=None, use_graph=True, precision=None, **over):
        self.w = w
        self.cfg = make_config(w, use_graph=use_graph, precision=precision, **over)
        self.precision = self.cfg.precision
        self.dtype = torch_dtype(self.precision)
        self.h = ctypes.c_void_p()
        _check(LIB.rom_create(ctypes.byref(self.cfg), _ptr(q0), _stream(), ctypes.byref(self.h)))
        td, nv, r, ns = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(LIB.rom_query(self.h, ctypes.byref(td), ctypes.byref(nv), ctypes.byref(r),
                             ctypes.byref(ns)))
        self.total_dof, self.n_var, self.r, self.n_s = td.value, nv.value, r.value, ns.value
        self.n_inst = w.n_inst

    def close(self):
        if self.h:
            LIB.rom_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self, n, dtype=None):
        return torch.empty(n, dtype=self.dtype if dtype is None else dtype, device="cuda")

    # ---- full-order model
    def fom_residual(self, q, q_prev=None, dt=0.0, out=None):
        out = self._new(self.total_dof) if out is None else out
        _check(LIB.fom_residual(self.h, _ptr(q), _ptr(q_prev), float(dt), _ptr(out), _stream()))
        return out

    def fom_step(self, q_prev, dt, out=None, iters=None):
        out = self._new(self.total_dof) if out is None else out
        _check(LIB.fom_step(self.h, _ptr(q_prev), float(dt), _ptr(out), _ptr(iters), _stream()))
        return out

    def fom_residual_vjp(self, q, gbar, q_prev=None, dt=0.0, gq=None, gq_prev=None):
        gq = self._new(self.total_dof) if gq is None else gq
        if q_prev is not None and gq_prev is None:
            gq_prev = self._new(self.total_dof)
        _check(LIB.fom_residual_vjp(self.h, _ptr(q), _ptr(q_prev), float(dt), _ptr(gbar), _ptr(gq),
                                    _ptr(gq_prev), _stream()))
        return gq, gq_prev

    def fom_step_vjp(self, q, dt, gbar, out=None):
        out = self._new(self.total_dof) if out is None else out
        _check(LIB.fom_step_vjp(self.h, _ptr(q), float(dt), _ptr(gbar), _ptr(out), _stream()))
        return out

    def fom_rollout_vjp(self, q0, n_steps, dt, gbar, n_ckpt=0, out=None):
        out = self._new(self.total_dof) if out is None else out
        _check(LIB.fom_rollout_vjp(self.h, _ptr(q0), int(n_steps), float(dt), int(n_ckpt),
                                   _ptr(gbar), _ptr(out), _stream()))
        return out

    def fom_rollout_vjp_noalloc(self, q0, n_steps, dt, gbar, n_ckpt=0, out=None):
        """fom_rollout_vjp with its checkpoints in the library's static device
        array (no allocation inside the call; out must be given to allocate
        nothing at all)."""
        out = self._new(self.total_dof) if out is None else out
        _check(LIB.fom_rollout_vjp_noalloc(self.h, _ptr(q0), int(n_steps), float(dt), int(n_ckpt),
                                           _ptr(gbar), _ptr(out), _stream()))
        return out

    def online_vjp(self, n_fine, qbar, n_ckpt=0):
        """Gradient of <qbar, q~_end> over n_fine online steps (events included)
        with respect to the starting (a, Phi, sigma, y_corr); FP64 tensors.
        Advances the state as rom_step(n_fine) would."""
        import torch
        B, r, tot = self.n_inst, self.r, self.total_dof
        dev = torch.device("cuda", torch.cuda.current_device())
        ab = torch.empty(B * r, dtype=torch.float64, device=dev)
        pb = torch.empty(tot * r, dtype=torch.float64, device=dev)
        sb = torch.empty(B * r, dtype=torch.float64, device=dev)
        yb = torch.empty(tot, dtype=torch.float64, device=dev)
        _check(LIB.rom_online_vjp(self.h, int(n_fine), int(n_ckpt), _ptr(qbar), _ptr(ab),
                                  _ptr(pb), _ptr(sb), _ptr(yb), _stream()))
        return ab, pb, sb, yb

    def offline(self, q0):
        """Alg. 1's offline stage from q0 on this handle (as rom_create with q0)."""
        _check(LIB.rom_offline(self.h, _ptr(q0), _stream()))

    def rollout_vjp(self, q0, n_steps, gbar, n_ckpt=0, out=None):
        """Gradient of <gbar, q~_end> with respect to q0 through the offline
        stage and n_steps HR-LSPG fine steps (events included), the sample rows
        of the forward run held fixed.  Leaves the handle at the end state."""
        out = self._new(self.total_dof) if out is None else out
        _check(LIB.rom_rollout_vjp(self.h, _ptr(q0), int(n_steps), int(n_ckpt), _ptr(gbar),
                                   _ptr(out), _stream()))
        return out

    # ---- reduced model
    def isvd_update(self, y):
        _check(LIB.isvd_update(self.h, _ptr(y), _stream()))

    def rom_rebuild(self):
        _check(LIB.rom_rebuild(self.h, _stream()))

    def rom_step(self, n_fine):
        _check(LIB.rom_step(self.h, int(n_fine), _stream()))

    _SIZES = {GET_BASIS: ("T", "dof*r"), GET_SIGMA: ("f64", "B*r"), GET_A: ("f64", "B*r"),
              GET_QTILDE: ("T", "dof"), GET_SAMPLES: ("i32", "B*ns"), GET_YCORR: ("T", "dof"),
              GET_QREF: ("T", "dof"), GET_DVAR: ("f64", "B*nv"), GET_PINV: ("f64", "B*r*ns"),
              GET_UBAR: ("f64", "B*n*n"), GET_WINDOW: ("T", "w*dof")}

    def _shape(self, what):
        kind, n = self._SIZES[what]
        size = {"dof*r": self.total_dof * self.r, "B*r": self.n_inst * self.r,
                "dof": self.total_dof, "B*ns": self.n_inst * max(self.n_s, 1),
                "B*nv": self.n_inst * self.n_var, "B*r*ns": self.n_inst * self.r * max(self.n_s, 1),
                "B*n*n": self.n_inst * (self.r + 1) ** 2,
                "w*dof": max(self.cfg.window, 0) * self.total_dof}[n]
        dt = {"T": self.dtype, "f64": torch.float64, "i32": torch.int32}[kind]
        return size, dt

    def get(self, what):
        if what == GET_COUNTERS:
            buf = (ctypes.c_int64 * N_COUNTERS)()
            _check(LIB.rom_get(self.h, what, ctypes.cast(buf, ctypes.c_void_p), _stream()))
            return list(buf)
        n, dt = self._shape(what)
        out = self._new(n, dt)
        _check(LIB.rom_get(self.h, what, _ptr(out), _stream()))
        return out

    def set(self, what, src):
        if what == GET_COUNTERS:
            vals = [int(x) for x in src]
            cur = self.get(GET_COUNTERS)
            buf = (ctypes.c_int64 * N_COUNTERS)(*(vals + cur[len(vals):]))
            _check(LIB.rom_set(self.h, what, ctypes.cast(buf, ctypes.c_void_p), _stream()))
            return
        n, dt = self._shape(what)
        src = src.to(device="cuda", dtype=dt).contiguous()
        if src.numel() != n:
            raise ValueError("expected %d elements, got %d" % (n, src.numel()))
        _check(LIB.rom_set(self.h, what, _ptr(src), _stream()))
        torch.cuda.current_stream().synchronize()

    def save(self, out=None):
        """The handle's online state as a device byte tensor (rom_save)."""
        n = ctypes.c_size_t(0)
        _check(LIB.rom_save(self.h, None, ctypes.byref(n), _stream()))
        if out is None:
            out = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        n = ctypes.c_size_t(out.numel())
        _check(LIB.rom_save(self.h, _ptr(out), ctypes.byref(n), _stream()))
        return out

    def load(self, blob):
        """Restore a state written by save() (rom_load; synchronises the stream)."""
        _check(LIB.rom_load(self.h, _ptr(blob), ctypes.c_size_t(blob.numel()), _stream()))

    def autotune(self, what, q=None):
        """Pick the fastest candidate of a tuning target; returns its index."""
        c = ctypes.c_int32()
        _check(LIB.rom_autotune(self.h, int(what), _ptr(q) if q is not None else None,
                                ctypes.byref(c), _stream()))
        return c.value

    def set_tuning(self, what, choice):
        """Force a launch shape (choice < 0 only queries); returns the candidate count."""
        n = ctypes.c_int32()
        _check(LIB.rom_set_tuning(self.h, int(what), int(choice), ctypes.byref(n)))
        return n.value

    def profile(self, stage, reps, q=None):
        """Mean milliseconds per launch of one hot-path stage (HIP events on the current stream)."""
        ms = ctypes.c_double()
        _check(LIB.rom_profile(self.h, int(stage), int(reps), _ptr(q), ctypes.byref(ms), _stream()))
        return ms.value

    def status(self):
        buf = np.zeros(self.n_inst, dtype=np.uint32)
        _check(LIB.rom_get_status(self.h, ctypes.c_void_p(buf.ctypes.data)))
        return buf

    def clear_status(self):
        _check(LIB.rom_clear_status(self.h, _stream()))


class FomResidual(torch.autograd.Function):
    """f(q) of a handle's batch as a differentiable op; the backward pass is the
    hand-written adjoint J_f(q)^T g (fom_residual_vjp)."""

    @staticmethod
    def forward(ctx, q, handle):
        q = q.contiguous()
        ctx.save_for_backward(q)
        ctx.handle = handle
        return handle.fom_residual(q)

    @staticmethod
    def backward(ctx, g):
        (q,) = ctx.saved_tensors
        gq, _ = ctx.handle.fom_residual_vjp(q, g.contiguous())
        return gq, None


class FomRollout(torch.autograd.Function):
    """q^T after n_steps backward-Euler steps of size dt from q0 (fom_step); the
    backward pass is the checkpointed rollout adjoint (fom_rollout_vjp)."""

    @staticmethod
    def forward(ctx, q0, handle, n_steps, dt, n_ckpt=0):
        q0 = q0.contiguous()
        q = q0.clone()
        for _ in range(int(n_steps)):
            handle.fom_step(q, dt, out=q)
        ctx.save_for_backward(q0)
        ctx.handle, ctx.n_steps, ctx.dt, ctx.n_ckpt = handle, int(n_steps), float(dt), int(n_ckpt)
        return q

    @staticmethod
    def backward(ctx, g):
        (q0,) = ctx.saved_tensors
        gq0 = ctx.handle.fom_rollout_vjp(q0, ctx.n_steps, ctx.dt, g.contiguous(), ctx.n_ckpt)
        return gq0, None, None, None, None


class RomRollout(torch.autograd.Function):
    """q~ after Alg. 1 run from the initial state q0: the offline stage, then
    n_steps hyper-reduced LSPG fine steps with their events.  The backward pass
    is rom_rollout_vjp (the sample rows of the run held fixed), which reruns
    the rollout from q0 with checkpoints.  The handle's state is overwritten."""

    @staticmethod
    def forward(ctx, q0, handle, n_steps, n_ckpt=0):
        qd = q0.detach().contiguous().to(handle.dtype)
        handle.offline(qd)
        handle.rom_step(int(n_steps))
        q = handle.get(GET_QTILDE).clone()
        ctx.save_for_backward(qd)
        ctx.handle, ctx.n_steps, ctx.n_ckpt, ctx.dtype = handle, int(n_steps), int(n_ckpt), q0.dtype
        return q.to(q0.dtype)

    @staticmethod
    def backward(ctx, g):
        (qd,) = ctx.saved_tensors
        h = ctx.handle
        gq = h.rollout_vjp(qd, ctx.n_steps, g.contiguous().to(h.dtype), ctx.n_ckpt)
        return gq.to(ctx.dtype), None, None, None


class RomOnline(torch.autograd.Function):
    """q~ at the end of n_fine online steps of Alg. 1 (Galerkin steps and the
    adaptation events that fall due) from the reduced state (a, Phi, sigma,
    y_corr); the backward pass is the checkpointed online adjoint
    (rom_online_vjp), which restarts from the saved inputs.  The handle's state
    is overwritten by the inputs in both passes; q_ref, D and the fine-step
    counter it holds at the first call are kept."""

    @staticmethod
    def forward(ctx, a, Phi, sigma, y_corr, handle, n_fine, n_ckpt=0):
        counters = list(handle.get(GET_COUNTERS))
        handle.set(GET_A, a.detach().contiguous())
        handle.set(GET_BASIS, Phi.detach().contiguous())
        handle.set(GET_SIGMA, sigma.detach().contiguous())
        handle.set(GET_YCORR, y_corr.detach().contiguous())
        handle.rom_step(int(n_fine))
        q = handle.get(GET_QTILDE).clone()
        ctx.save_for_backward(a.detach(), Phi.detach(), sigma.detach(), y_corr.detach())
        ctx.handle, ctx.n_fine, ctx.n_ckpt, ctx.counters = handle, int(n_fine), int(n_ckpt), counters
        return q

    @staticmethod
    def backward(ctx, g):
        a, Phi, sigma, y_corr = ctx.saved_tensors
        h = ctx.handle
        h.set(GET_COUNTERS, ctx.counters)
        h.set(GET_A, a.contiguous())
        h.set(GET_BASIS, Phi.contiguous())
        h.set(GET_SIGMA, sigma.contiguous())
        h.set(GET_YCORR, y_corr.contiguous())
        ab, pb, sb, yb = h.online_vjp(ctx.n_fine, g.contiguous().to(h.dtype), ctx.n_ckpt)
        return (ab.to(a.dtype).view_as(a), pb.to(Phi.dtype).view_as(Phi),
                sb.to(sigma.dtype).view_as(sigma), yb.to(y_corr.dtype).view_as(y_corr),
                None, None, None)
