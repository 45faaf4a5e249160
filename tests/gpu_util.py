"""Helpers shared by the GPU tests: device copies of synthetic inputs and
oracle references.  (Test infrastructure; imports the oracle.)"""
import numpy as np

from oracle import oracle as O


def dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device="cuda")


def colmajor(B):
    """(order, nrhs) float64 device tensor laid out column by column."""
    import torch
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        return dev(B)
    return torch.as_tensor(np.ascontiguousarray(B.T), device="cuda").t()


def factor_solve(kkt, inp, B):
    rc = kkt.factor(dev(inp.W_val), dev(inp.Sigma), dev(inp.J_val), inp.rho)
    X, info = kkt.solve(colmajor(B))
    return rc, X.cpu().numpy(), info


def form_id(form):
    return O.CONDENSED if form == "condensed" else O.STABILIZED


def omega_cpu(inp, form, X, B):
    """Backward error of X measured in FP64 on the CPU against the oracle's K."""
    K = O.assemble(inp, form_id(form))
    return float(O.backward_error(K, X, B).max())


def kappa_inf(inp, form):
    Kd = O.assemble(inp, form_id(form)).dense()
    return float(np.abs(Kd).sum(1).max() * np.abs(np.linalg.inv(Kd)).sum(1).max())
