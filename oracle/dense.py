"""Dense brute-force LDL^T for tiny systems (test infrastructure only).

Right-looking elimination of a dense symmetric matrix with no pivoting and the
same static-pivot rule as the sparse oracle (Sec. 3.1: a pivot below the
threshold is replaced by the threshold, signed by its block).  Without
pivoting the factorization of a given symmetric ordering is unique, so this
is an independent second computation of the sparse oracle's L and D.
"""
from __future__ import annotations

import numpy as np


def ldl(A: np.ndarray, signs=None, pivot_thr=0.0):
    """A (N x N, symmetric, already permuted) -> (L unit lower, D, nperturbed).
    pivot_thr: one threshold, or a (primal, dual) pair chosen by signs[k]."""
    tp, td = (pivot_thr, pivot_thr) if np.ndim(pivot_thr) == 0 else pivot_thr
    A = np.array(A, dtype=np.float64, copy=True)
    N = A.shape[0]
    L = np.eye(N)
    D = np.zeros(N)
    npert = 0
    for k in range(N):
        d = A[k, k]
        s = 1 if signs is None else int(signs[k])
        t = tp if s > 0 else td
        if t > 0.0 and abs(d) < t:
            d = t if s > 0 else -t
            npert += 1
        D[k] = d
        col = A[k + 1:, k].copy()
        L[k + 1:, k] = col / d
        A[k + 1:, k + 1:] -= np.outer(col, col) / d
    return L, D, npert
