"""Seeded synthetic workloads (initial states, physical constants, ROM settings).

This module holds no arithmetic of the method: it only draws the seeded inputs
that both the HIP path and the CPU checker consume.  Random numbers come from
``numpy.random.default_rng([workload_id, stream])``.

Workloads (sizes and settings of the five benchmark problems):
  1 burgers_512_f64      viscous Burgers, N = 512, FP64, Galerkin, r = 10
  2 burgers_batch_f32    256 Burgers instances, N in {2048..16384}, FP32, r = 32
  3 sod_hllc_f32         Sod shock tube, N = 65,536, HLLC, HR-LSPG + DEIM, r = 40
  4 euler_adjoint_f32    64 perturbed Sod instances, N = 262,144, Rusanov
  5 react10_f32          32 instances of the 12-variable reacting model, N = 32,768
Smaller variants (fewer instances / cells) are produced by the same recipes for
tests; they keep the value distributions and structure of the full sizes.
"""
from dataclasses import dataclass, field
import numpy as np

BURGERS, EULER_RUSANOV, EULER_HLLC, REACT = 0, 1, 2, 3
NVAR = {BURGERS: 1, EULER_RUSANOV: 3, EULER_HLLC: 3, REACT: 12}
F32, F64 = 0, 1
GALERKIN, LSPG = 0, 1
HR_NONE, HR_DEIM, HR_QDEIM, HR_QDEIM_FGS = 0, 1, 2, 3

# packed per-instance constant vector layout of the reacting model
REACT_NPHYS = 6 + 10 + 6 * 12


@dataclass
class Workload:
    name: str
    problem: int
    precision: int
    projection: int
    hyper: int
    n_cells: list
    phys: list                     # one dict per instance (checker side)
    q0: np.ndarray                 # concatenated initial states (float64)
    r: int
    n_s: int
    w_init: int
    z: int
    N_t: int
    lam: float
    dt: float
    newton_tol: float
    newton_max: int = 10
    rom_tol: float = 1e-12
    rom_max: int = 10
    reorth_every: int = 16
    tau_orth: float = 1e-12
    tau_rho: float = 1e-12
    update: str = "isvd"           # basis update rule: isvd | wsvd | direct
    window: int = 0                # snapshot window of the windowed rules
    scheme: str = "be"             # time scheme: be (backward Euler) | ssprk43 (explicit path)
    extra: dict = field(default_factory=dict)

    @property
    def n_var(self):
        return NVAR[self.problem]

    @property
    def n_inst(self):
        return len(self.n_cells)

    def offsets(self):
        """DOF offsets of each instance in the concatenated state."""
        o = [0]
        for n in self.n_cells:
            o.append(o[-1] + n * self.n_var)
        return o

    def instance(self, b, arr=None):
        o = self.offsets()
        a = self.q0 if arr is None else arr
        return a[o[b]:o[b + 1]]

    def phys_vector(self):
        """Per-instance physical constants packed as doubles for the C interface."""
        rows = []
        for ph in self.phys:
            if self.problem == BURGERS:
                rows.append([ph["nu"]])
            elif self.problem in (EULER_RUSANOV, EULER_HLLC):
                rows.append([ph["gamma"]])
            else:
                v = [ph["nu_u"], ph["kappa"], ph["A"], ph["k_in"], ph["x_in"], ph["T_in"]]
                v += list(ph["Y_in"])
                for key in ("ra", "rb", "pc", "pd"):
                    v += [float(x) for x in ph[key]]
                v += list(ph["E"]) + list(ph["Q"])
                rows.append(v)
        return np.asarray(rows, dtype=np.float64)

    def params(self):
        """Adaptive-ROM settings as a plain dict (checker side)."""
        return dict(r=self.r, n_s=self.n_s, w_init=self.w_init, N_t=self.N_t, z=self.z,
                    lam=self.lam, dt=self.dt, newton_tol=self.newton_tol,
                    newton_max=self.newton_max, rom_tol=self.rom_tol, rom_max=self.rom_max,
                    reorth_every=self.reorth_every, tau_orth=self.tau_orth,
                    tau_rho=self.tau_rho, update=self.update, window=self.window,
                    scheme=self.scheme,
                    projection="lspg" if self.projection == LSPG else "galerkin",
                    hyper={HR_NONE: "none", HR_DEIM: "deim", HR_QDEIM: "qdeim",
                           HR_QDEIM_FGS: "qdeim_fgs"}[self.hyper])


def centres(n):
    return (np.arange(n) + 0.5) / n


def _sod_state(x, gamma=1.4):
    rho = np.where(x < 0.5, 1.0, 0.125)
    p = np.where(x < 0.5, 1.0, 0.1)
    u = np.zeros_like(x)
    return rho, u, p


def _conserved(rho, u, p, gamma=1.4):
    U = np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u], axis=1)
    return U.reshape(-1)


# ----------------------------------------------------------------- workload 1
def burgers_512_f64(n=512, N_t=2000, w_init=100, r=10, z=5):
    x = centres(n)
    rng = np.random.default_rng([1, 0])
    u0 = 0.5 + np.sin(2 * np.pi * x) + rng.normal(0.0, 1e-3, n)
    return Workload("burgers_512_f64", BURGERS, F64, GALERKIN, HR_NONE, [n],
                    [dict(nu=0.01)], u0, r=r, n_s=r, w_init=w_init, z=z, N_t=N_t,
                    lam=0.5, dt=1e-3, newton_tol=1e-8, rom_tol=1e-12,
                    tau_orth=1e-12, tau_rho=1e-12)


# ----------------------------------------------------------------- workload 2
def burgers_batch_f32(n_inst=256, sizes=(2048, 4096, 8192, 16384), r=32, z=4, N_t=5000,
                      w_init=None, precision=F32):
    rng = np.random.default_rng([2, 0])
    n_cells = [int(s) for s in rng.choice(np.asarray(sizes), size=n_inst)]
    nus = 10.0 ** rng.uniform(-3.0, -2.0, size=n_inst)
    q0, phys = [], []
    for b in range(n_inst):
        x = centres(n_cells[b])
        A = rng.uniform(0.0, 1.0, 4)
        ph = rng.uniform(0.0, 2 * np.pi, 4)
        u = sum(A[m] * np.sin(2 * np.pi * (m + 1) * x + ph[m]) for m in range(4))
        q0.append(u)
        phys.append(dict(nu=float(nus[b])))
    f64 = precision == F64
    return Workload("burgers_batch_f32", BURGERS, precision, GALERKIN, HR_NONE, n_cells, phys,
                    np.concatenate(q0), r=r, n_s=r, w_init=r if w_init is None else w_init,
                    z=z, N_t=N_t, lam=0.5, dt=1e-4,
                    newton_tol=1e-8 if f64 else 1e-5, rom_tol=1e-12 if f64 else 1e-6,
                    tau_orth=1e-12 if f64 else 1e-6, tau_rho=1e-12 if f64 else 1e-6)


# ----------------------------------------------------------------- workload 3
def sod_hllc_f32(n=65536, r=40, n_s=80, z=10, precision=F32, flux=EULER_HLLC, N_t=None):
    x = centres(n)
    rho, u, p = _sod_state(x)
    dt = 0.064 / n
    steps = int(round(0.2 / dt)) if N_t is None else N_t
    f64 = precision == F64
    return Workload("sod_hllc_f32", flux, precision, LSPG, HR_DEIM, [n], [dict(gamma=1.4)],
                    _conserved(rho, u, p), r=r, n_s=n_s, w_init=r, z=z, N_t=steps, lam=0.01,
                    dt=dt, newton_tol=1e-8 if f64 else 1e-5, rom_tol=1e-12 if f64 else 1e-6,
                    tau_orth=1e-12 if f64 else 1e-6, tau_rho=1e-12 if f64 else 1e-6)


# ----------------------------------------------------------------- workload 4
def _perturbed_sod(n, rng):
    x = centres(n)
    rho, u, p = _sod_state(x)
    a = rng.uniform(-1, 1, 4)
    b = rng.uniform(-1, 1, 4)
    ph = rng.uniform(0, 2 * np.pi, 4)
    ps = rng.uniform(0, 2 * np.pi, 4)
    pert = sum(a[m] * np.sin(2 * np.pi * (m + 1) * x + ph[m]) for m in range(4))
    upert = sum(b[m] * np.sin(2 * np.pi * (m + 1) * x + ps[m]) for m in range(4))
    rho = rho * (1 + 0.01 * pert)
    p = p * (1 + 0.01 * pert)
    u = 0.05 + 0.01 * upert
    return _conserved(rho, u, p)


def euler_adjoint_f32(n_inst=64, n=262144, r=10, n_s=20, z=10, N_t=1000, precision=F32):
    q0, tgt = [], []
    for b in range(n_inst):
        q0.append(_perturbed_sod(n, np.random.default_rng([4, 1 + b])))
        tgt.append(_perturbed_sod(n, np.random.default_rng([4, 1000 + b])))
    f64 = precision == F64
    w = Workload("euler_adjoint_f32", EULER_RUSANOV, precision, LSPG, HR_DEIM, [n] * n_inst,
                 [dict(gamma=1.4)] * n_inst, np.concatenate(q0), r=r, n_s=n_s, w_init=r, z=z,
                 N_t=N_t, lam=0.01, dt=0.064 / n, newton_tol=1e-8 if f64 else 1e-5,
                 rom_tol=1e-12 if f64 else 1e-6, tau_orth=1e-12 if f64 else 1e-6,
                 tau_rho=1e-12 if f64 else 1e-6)
    w.extra["target"] = np.concatenate(tgt)
    w.extra["fd_directions"] = 16
    w.extra["fd_h"] = 1e-6
    return w


# ----------------------------------------------------------------- workload 5
def react_mechanism():
    """Synthetic 12-reaction mechanism on 10 species (stream 0 of workload 5)."""
    rng = np.random.default_rng([5, 0])
    ra, rb, pc, pd = [], [], [], []
    for _ in range(12):
        s = rng.choice(10, size=4, replace=False)
        ra.append(int(s[0])); rb.append(int(s[1])); pc.append(int(s[2])); pd.append(int(s[3]))
    xi = rng.uniform(0.0, 1.0, 12)
    xq = rng.uniform(0.0, 1.0, 12)
    return dict(ra=np.array(ra), rb=np.array(rb), pc=np.array(pc), pd=np.array(pd),
                E=np.log(10.0) * (4.0 - 3.0 * xi), Q=0.05 * xq)


def react10_f32(n_inst=32, n=32768, r=64, n_s=128, z=10, N_t=2000, precision=F32):
    mech = react_mechanism()
    q0, phys = [], []
    x = centres(n)
    for b in range(n_inst):
        rng = np.random.default_rng([5, 1 + b])
        zeta = rng.uniform(-1, 1, 3)
        Y_in = np.zeros(10)
        Y_in[0] = 0.5 * (1 + 0.05 * zeta[0])
        Y_in[1] = 0.5 * (1 + 0.05 * zeta[1])
        Y_in /= Y_in.sum()
        T_in = 0.2 * (1 + 0.05 * zeta[2])
        ph = dict(nu_u=1e-3, kappa=1e-3, A=1e7, k_in=50.0, x_in=0.05, T_in=T_in, Y_in=Y_in)
        ph.update(mech)
        phys.append(ph)
        Q = np.zeros((n, 12))
        Q[:, :10] = Y_in[None, :]
        Q[:, 10] = 0.2 + 0.8 * np.exp(-((x - 0.5) / 0.02) ** 2)
        Q[:, 11] = 1.0 + 0.1 * np.sin(2 * np.pi * x)
        q0.append(Q.reshape(-1))
    f64 = precision == F64
    return Workload("react10_f32", REACT, precision, LSPG, HR_DEIM, [n] * n_inst, phys,
                    np.concatenate(q0), r=r, n_s=n_s, w_init=r, z=z, N_t=N_t, lam=0.5,
                    dt=1e-4, newton_tol=1e-8 if f64 else 1e-5, rom_tol=1e-12 if f64 else 1e-6,
                    tau_orth=1e-12 if f64 else 1e-6, tau_rho=1e-12 if f64 else 1e-6)


def random_state(problem, n_cells, seed, scale=1.0):
    """Smooth random states of the right physical range for per-call tests
    (positive density/pressure for Euler, positive T for the reacting model)."""
    rng = np.random.default_rng([99, seed])
    out = []
    for n in n_cells:
        x = centres(n)
        def smooth():
            A = rng.uniform(-1, 1, 3)
            ph = rng.uniform(0, 2 * np.pi, 3)
            return sum(A[m] * np.sin(2 * np.pi * (m + 1) * x + ph[m]) for m in range(3)) / 3
        if problem == BURGERS:
            out.append(scale * (smooth() + 0.3 * rng.normal(size=n)))
        elif problem in (EULER_RUSANOV, EULER_HLLC):
            rho = 1.0 + 0.5 * smooth() + 0.05 * rng.uniform(-1, 1, n)
            u = 0.5 * smooth() + 0.05 * rng.uniform(-1, 1, n)
            p = 1.0 + 0.5 * smooth() + 0.05 * rng.uniform(-1, 1, n)
            out.append(_conserved(rho, u, p))
        else:
            Q = np.zeros((n, 12))
            Q[:, :10] = rng.uniform(0.0, 0.3, (n, 10))
            Q[:, 10] = 0.5 + 0.3 * smooth() + 0.05 * rng.uniform(-1, 1, n)
            Q[:, 11] = 1.0 + 0.3 * smooth() + 0.05 * rng.uniform(-1, 1, n)
            out.append(Q.reshape(-1))
    return np.concatenate(out)
