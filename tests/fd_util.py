"""Finite-difference bar and sample of the config-5 adjoint checks (test
infrastructure, shared by the oracle pin and the GPU test)."""
import numpy as np


def fd_tolerance(g, Wt, X, h):
    """Bar for a central difference of loss = sum(w * x) at step h, reading
    C13 recalibrated: the relative 1e-4 plus the rounding noise of the two
    losses, 2000 u sum|w x| / h (at config 5 the oracle's own differences
    reach 350 u sum|w x| / h; first-guess 1e-6 max|g| was 100x too tight)."""
    return 1e-4 * np.abs(g) + 2e3 * np.finfo(float).eps * np.sum(np.abs(Wt * X)) / h


def config5_fd_cases(inp, rng, count=50):
    """The config-5 sample: `count` stored entries each of W, Sigma, J and
    `count` (row, column) entries of B, drawn without replacement."""
    n = inp.n
    return {"W_val": rng.choice(len(inp.W_val), count, replace=False),
            "Sigma": rng.choice(n, count, replace=False),
            "J_val": rng.choice(len(inp.J_val), count, replace=False),
            "B": np.stack([rng.choice(n, count, replace=False), rng.integers(0, 16, count)], axis=1)}
