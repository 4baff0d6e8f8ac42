"""Helpers shared by the GPU parity tests (comparison norms and tensors)."""
import sys

import numpy as np

MVM_TOL = 1e-10        # componentwise, relative to (K|v|)_j, and normwise
SOLVE_TOL = 1e-8       # relative 2-norm error of the CG solution vs Cholesky


def torch_dev():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a visible GPU")
    return torch, torch.device("cuda:0")


def to_gpu(a):
    torch, dev = torch_dev()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def to_np(t):
    return t.detach().cpu().numpy()


def mvm_errors(y, yref, yabs):
    """(componentwise error / (K|v|), normwise relative error)."""
    y = np.asarray(y)
    yref = np.asarray(yref)
    yabs = np.asarray(yabs)
    comp = float(np.max(np.abs(y - yref) / np.maximum(yabs, 1e-300)))
    nrm = float(np.linalg.norm(y - yref) / max(np.linalg.norm(yref), 1e-300))
    return comp, nrm


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def converged(solvers, status, passed):
    """One round of the stop rule of gp_cg_solve for hand-driven solvers: a
    solver whose columns all converged by the recurrence (status 0) has its
    residual recomputed (mm_solver_check); a miss restarts it with tighter
    tolerances.  passed[k] records the solvers done; True when all are."""
    for k, (s, st) in enumerate(zip(solvers, status)):
        if not passed[k] and st == 0:
            passed[k] = s.check(tighten=True)[0]
    return all(passed)
