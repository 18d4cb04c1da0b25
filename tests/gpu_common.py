"""Helpers shared by the GPU parity tests (imported only by tests marked gpu)."""
import numpy as np
import torch

from paper_2605_28684_amd import workloads as W

TOL = {W.F64: 1e-11, W.F32: 1e-5}


def relerr(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return np.linalg.norm(x - ref) / (den if den > 0 else 1.0)


def maxrel(x, ref):
    """Largest elementwise error relative to the largest reference entry."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref)) if ref.size else 0.0
    return np.max(np.abs(x - ref)) / (den if den > 0 else 1.0) if ref.size else 0.0


def assert_close(x, ref, tol, elem_tol=None, what=""):
    """Relative L2 error <= tol and largest elementwise error <= elem_tol (default
    tol) times the largest reference entry; an error confined to a few entries
    is not diluted by the norm.  Returns both errors."""
    e2, em = relerr(x, ref), maxrel(x, ref)
    et = tol if elem_tol is None else elem_tol
    print("  parity %s: relerr %.3e elementwise %.3e (bound %.1e)" % (what, e2, em, tol))
    assert e2 <= tol and em <= et, "%s: relerr %.3e (bound %.1e), max elementwise %.3e (bound %.1e)" % (
        what, e2, tol, em, et)
    return e2, em


def to_dev(a, precision):
    dt = torch.float64 if precision == W.F64 else torch.float32
    return torch.as_tensor(np.asarray(a), dtype=dt, device="cuda").contiguous()


def rounded(a, precision):
    """The values the device sees, upcast to float64 for the checker."""
    if precision == W.F64:
        return np.asarray(a, dtype=np.float64)
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def phys_of(w, b):
    return w.phys[b]


def align_signs(A, ref):
    """Flip columns of A to match the signs of ref (for singular vectors)."""
    s = np.sign(np.sum(A * ref, axis=0))
    s[s == 0] = 1.0
    return A * s[None, :]
