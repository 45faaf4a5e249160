"""Dense brute-force LDL^T for tiny systems (test infrastructure only).

Right-looking elimination of a dense symmetric matrix with no pivoting and the
same static-pivot rule as the sparse oracle (Sec. 3.1: a pivot below the
threshold is replaced by the threshold, signed by its block).  Without
pivoting the factorization of a given symmetric ordering is unique, so this
is an independent second computation of the sparse oracle's L and D.
"""
from __future__ import annotations

import numpy as np


def ldl(A: np.ndarray, signs=None, pivot_thr: float = 0.0):
    """A (N x N, symmetric, already permuted) -> (L unit lower, D, nperturbed)."""
    A = np.array(A, dtype=np.float64, copy=True)
    N = A.shape[0]
    L = np.eye(N)
    D = np.zeros(N)
    npert = 0
    for k in range(N):
        d = A[k, k]
        if pivot_thr > 0.0 and abs(d) < pivot_thr:
            s = 1 if signs is None else int(signs[k])
            d = pivot_thr if s > 0 else -pivot_thr
            npert += 1
        D[k] = d
        col = A[k + 1:, k].copy()
        L[k + 1:, k] = col / d
        A[k + 1:, k + 1:] -= np.outer(col, col) / d
    return L, D, npert
