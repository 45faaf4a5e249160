"""Seeded synthetic inputs for the NCL KKT systems.

This module only draws the raw data the method consumes — the Hessian block W
(lower CSC), the barrier diagonal Sigma, the Jacobian J (CSR), the penalty rho
and right-hand sides.  It never forms K or any product of the method: the
library and the CPU oracle each do that themselves from these arrays.

Shapes follow the paper's OPF/COPS-style workloads (Sec. 5.2): a sparse
Hessian with small dense per-bus blocks, a Jacobian with a handful of nonzeros
per row on node/edge incidence, a barrier diagonal spanning many decades and
penalties stepped over 1e2..1e8 (Algorithm 1 multiplies rho by 10).  The PGLIB
and COPS instances themselves are not available; these generators stand in for
them.

Every generator takes a seed and draws from numpy's PCG64 in a fixed order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


@dataclass
class KKTInput:
    """Raw data of one KKT system.

    W is stored as lower-triangular CSC (colptr, rowidx sorted per column,
    values), 0-based int32.  J is CSR (rowptr, colidx sorted per row, values).
    Sigma has length n, rhs is (size, nrhs) column-major-compatible float64.
    """
    n: int
    m: int
    W_colptr: np.ndarray
    W_rowidx: np.ndarray
    W_val: np.ndarray
    Sigma: np.ndarray
    J_rowptr: np.ndarray
    J_colidx: np.ndarray
    J_val: np.ndarray
    rho: float
    meta: dict = field(default_factory=dict)

    def with_values(self, W_val=None, Sigma=None, J_val=None, rho=None):
        return KKTInput(self.n, self.m, self.W_colptr, self.W_rowidx,
                        self.W_val if W_val is None else W_val,
                        self.Sigma if Sigma is None else Sigma,
                        self.J_rowptr, self.J_colidx,
                        self.J_val if J_val is None else J_val,
                        self.rho if rho is None else float(rho), dict(self.meta))


def _lower_csc(n, rows, cols, vals):
    """COO (row >= col) -> sorted lower CSC with int32 indices; duplicates summed."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    assert np.all(rows >= cols)
    A = sp.coo_matrix((np.asarray(vals, dtype=np.float64), (rows, cols)), shape=(n, n)).tocsc()
    A.sum_duplicates()
    A.sort_indices()
    return (A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64))


def _csr(m, n, rows, cols, vals):
    A = sp.coo_matrix((np.asarray(vals, dtype=np.float64),
                       (np.asarray(rows, dtype=np.int64), np.asarray(cols, dtype=np.int64))),
                      shape=(m, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return (A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64))


# ---------------------------------------------------------------------------
# Workload A: grid Laplacian Hessian + banded Jacobian (n = 2000, m = 1000)
# ---------------------------------------------------------------------------

def grid_banded(seed: int = 1, nr: int = 40, nc: int = 50, m: int = 1000, per_row: int = 4,
                band: int = 50, rho: float = 1e4, sigma_lo: float = -8.0, sigma_hi: float = 2.0,
                shift: float = 1.0) -> KKTInput:
    """5-point Dirichlet Laplacian of an nr x nc grid plus shift*I (node k = r*nc + c),
    m Jacobian rows with `per_row` N(0,1) entries in distinct columns drawn uniformly from
    the window [lo, lo+band), lo = clamp(2i - band/2, 0, n - band); Sigma log-uniform in
    [10^sigma_lo, 10^sigma_hi].  Draw order: J columns row by row, J values, Sigma."""
    rng = np.random.default_rng(seed)
    n = nr * nc
    rows, cols, vals = [], [], []
    for r in range(nr):
        for c in range(nc):
            k = r * nc + c
            rows.append(k); cols.append(k); vals.append(4.0 + shift)
            if c + 1 < nc:
                rows.append(k + 1); cols.append(k); vals.append(-1.0)
            if r + 1 < nr:
                rows.append(k + nc); cols.append(k); vals.append(-1.0)
    Wp, Wi, Wx = _lower_csc(n, rows, cols, vals)
    jr, jc = [], []
    for i in range(m):
        lo = min(max(2 * i - band // 2, 0), n - band)
        sel = np.sort(rng.choice(band, size=per_row, replace=False)) + lo
        jr.extend([i] * per_row)
        jc.extend(sel.tolist())
    jv = rng.standard_normal(len(jr))
    Jp, Jj, Jx = _csr(m, n, jr, jc, jv)
    Sigma = 10.0 ** rng.uniform(sigma_lo, sigma_hi, size=n)
    return KKTInput(n, m, Wp, Wi, Wx, Sigma, Jp, Jj, Jx, float(rho),
                    meta={"workload": f"grid{nr}x{nc}-banded", "seed": seed})


# ---------------------------------------------------------------------------
# Workload B: OPF-shaped network (Delaunay graph, 4 vars/node + edge vars)
# ---------------------------------------------------------------------------

def _haar_blocks(rng, count):
    """count random 4x4 orthogonal matrices (QR of Gaussians with the sign fix)."""
    G = rng.standard_normal((count, 4, 4))
    Q, R = np.linalg.qr(G)
    s = np.sign(np.einsum("kii->ki", R))
    s[s == 0] = 1.0
    return Q * s[:, None, :]


def opf_network(N: int = 100_000, seed: int = 2, n_edge_vars: int | None = None,
                eig_lo: float = -2.0, eig_hi: float = 2.0, coupling_std: float = 0.1,
                rho: float = 1e2, sigma_lo: float = -8.0, sigma_hi: float = 8.0,
                sigma_seed: int | None = None) -> KKTInput:
    """N uniform points in the unit square, Delaunay edges E.  Node u owns variables
    4u..4u+3; n_edge_vars (default N) edges chosen uniformly without replacement own one
    variable each, numbered 4N + t.  W = per-node SPD 4x4 blocks Q diag(10^U(eig_lo,eig_hi)) Q^T
    + per-edge 4x4 node-node coupling blocks with N(0, coupling_std^2) entries + the diagonal
    compensation diag(sum_j |C_ij|), which keeps the coupling part diagonally dominant so
    W is SPD on the node variables; edge variables have no W entries.  J has one row per
    Delaunay edge with N(0,1) values on the 8 endpoint variables (and on the edge variable
    when that edge owns one).  Sigma is log-uniform; it is drawn from its own seed when
    `sigma_seed` is given (the refactor sequence redraws it per step)."""
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    pts = rng.uniform(size=(N, 2))
    tri = Delaunay(pts).simplices.astype(np.int64)
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [0, 2]]])
    e.sort(axis=1)
    e = np.unique(e, axis=0)                      # undirected edges (u < v), lexicographic
    E = e.shape[0]
    ne = N if n_edge_vars is None else int(n_edge_vars)
    ne = min(ne, E)
    owner = rng.choice(E, size=ne, replace=False)  # edge t = owner[k] owns var 4N + k
    n = 4 * N + ne

    # per-node SPD blocks
    Q = _haar_blocks(rng, N)
    lam = 10.0 ** rng.uniform(eig_lo, eig_hi, size=(N, 4))
    B = np.einsum("kij,kj,klj->kil", Q, lam, Q)
    # coupling blocks C_uv (rows of node v, cols of node u, u < v)
    C = rng.standard_normal((E, 4, 4)) * coupling_std
    comp = np.zeros(4 * N)
    absC = np.abs(C)
    np.add.at(comp, (4 * e[:, 1])[:, None] + np.arange(4)[None, :], absC.sum(axis=2))
    np.add.at(comp, (4 * e[:, 0])[:, None] + np.arange(4)[None, :], absC.sum(axis=1))

    a, b = np.tril_indices(4)
    rows = [(4 * np.arange(N))[:, None] + a[None, :]]
    cols = [(4 * np.arange(N))[:, None] + b[None, :]]
    bv = B[:, a, b].copy()
    diag_mask = (a == b)
    bv[:, diag_mask] += comp.reshape(N, 4)
    vals = [bv]
    ia, ib = np.meshgrid(np.arange(4), np.arange(4), indexing="ij")
    rows.append((4 * e[:, 1])[:, None] + ia.reshape(1, -1))
    cols.append((4 * e[:, 0])[:, None] + ib.reshape(1, -1))
    vals.append(C.reshape(E, 16))
    Wp, Wi, Wx = _lower_csc(n, np.concatenate([r.ravel() for r in rows]),
                            np.concatenate([c.ravel() for c in cols]),
                            np.concatenate([v.ravel() for v in vals]))

    # Jacobian: one row per edge on its 8 endpoint vars (+ owned edge var)
    ev = np.full(E, -1, dtype=np.int64)
    ev[owner] = 4 * N + np.arange(ne)
    jr = [np.repeat(np.arange(E), 8)]
    jc = [np.concatenate([(4 * e[:, 0])[:, None] + np.arange(4), (4 * e[:, 1])[:, None] + np.arange(4)],
                         axis=1).ravel()]
    has = ev >= 0
    jr.append(np.nonzero(has)[0])
    jc.append(ev[has])
    jr = np.concatenate(jr); jc = np.concatenate(jc)
    jv = rng.standard_normal(jr.size)
    Jp, Jj, Jx = _csr(E, n, jr, jc, jv)

    srng = rng if sigma_seed is None else np.random.default_rng(sigma_seed)
    Sigma = 10.0 ** srng.uniform(sigma_lo, sigma_hi, size=n)
    return KKTInput(n, E, Wp, Wi, Wx, Sigma, Jp, Jj, Jx, float(rho),
                    meta={"workload": f"opf-delaunay-N{N}", "seed": seed, "N": N, "E": E})


def opf_sequence_values(inp: KKTInput, k: int, steps: int = 30, rho_lo: float = 2.0,
                        rho_hi: float = 8.0, sigma_lo: float = -8.0, sigma_hi: float = 8.0,
                        seed_base: int = 2000):
    """Sigma and rho of refactor k of the OPF sequence: Sigma log-uniform in
    [10^sigma_lo, 10^sigma_hi] from seed seed_base + k, rho = 10^(rho_lo + (rho_hi-rho_lo) k/(steps-1))."""
    rng = np.random.default_rng(seed_base + k)
    Sigma = 10.0 ** rng.uniform(sigma_lo, sigma_hi, size=inp.n)
    rho = 10.0 ** (rho_lo + (rho_hi - rho_lo) * k / max(steps - 1, 1))
    return Sigma, float(rho)


# ---------------------------------------------------------------------------
# Right-hand sides and small random systems for tests
# ---------------------------------------------------------------------------

def rhs(size: int, nrhs: int = 1, seed: int = 0) -> np.ndarray:
    """(size, nrhs) N(0,1) right-hand sides, Fortran order (column-major)."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((size, nrhs)))


def random_system(n: int, m: int, seed: int = 0, w_density: float = 0.15, j_per_row: int = 3,
                  rho: float = 10.0, sigma_lo: float = -2.0, sigma_hi: float = 1.0,
                  spd: bool = True, empty_w_rows=(), empty_j_cols=(), zero_sigma=()) -> KKTInput:
    """Small random system: W lower with random off-diagonal pattern of the given density
    (values N(0,1)) and a diagonal that is made dominant when `spd` (else N(0,1));
    J with j_per_row distinct random columns per row.  Rows/columns listed in
    `empty_w_rows` get no W entries at all, columns in `empty_j_cols` get no J entries,
    and entries listed in `zero_sigma` get Sigma = 0 (used to force exact zero pivots)."""
    rng = np.random.default_rng(seed)
    mask = rng.uniform(size=(n, n)) < w_density
    mask = np.tril(mask, -1)
    ii, jj = np.nonzero(mask)
    off = rng.standard_normal(ii.size)
    keep = ~(np.isin(ii, empty_w_rows) | np.isin(jj, empty_w_rows))
    ii, jj, off = ii[keep], jj[keep], off[keep]
    rowsum = np.zeros(n)
    np.add.at(rowsum, ii, np.abs(off)); np.add.at(rowsum, jj, np.abs(off))
    if spd:
        dg = rowsum + 1.0 + rng.uniform(size=n)
    else:
        dg = rng.standard_normal(n)
    dmask = ~np.isin(np.arange(n), empty_w_rows)
    rows = np.concatenate([ii, np.arange(n)[dmask]])
    cols = np.concatenate([jj, np.arange(n)[dmask]])
    vals = np.concatenate([off, dg[dmask]])
    Wp, Wi, Wx = _lower_csc(n, rows, cols, vals)
    allowed = np.setdiff1d(np.arange(n), np.asarray(empty_j_cols, dtype=np.int64))
    jr, jc = [], []
    for r in range(m):
        k = min(j_per_row, allowed.size)
        sel = np.sort(rng.choice(allowed, size=k, replace=False))
        jr.extend([r] * k); jc.extend(sel.tolist())
    jv = rng.standard_normal(len(jr))
    Jp, Jj, Jx = _csr(m, n, jr, jc, jv)
    Sigma = 10.0 ** rng.uniform(sigma_lo, sigma_hi, size=n)
    Sigma[np.asarray(zero_sigma, dtype=np.int64)] = 0.0
    return KKTInput(n, m, Wp, Wi, Wx, Sigma, Jp, Jj, Jx, float(rho),
                    meta={"workload": f"random-n{n}-m{m}", "seed": seed})


def batched_sizes(count: int = 256, lo: int = 125, hi: int = 5000, seed: int = 4):
    """Node counts N_s = round(10^U(log10 lo, log10 hi)) of the batched workload."""
    rng = np.random.default_rng(seed)
    return np.rint(10.0 ** rng.uniform(np.log10(lo), np.log10(hi), size=count)).astype(np.int64)


def batched_system(s: int, N_s: int) -> KKTInput:
    """System s of the batched workload: the OPF network generator at N_s nodes (seed
    4000 + s) with rho log-uniform in [1e2, 1e6] and Sigma log-uniform in [1e-6, 1e6]."""
    rng = np.random.default_rng(4000 + s)
    rho = 10.0 ** rng.uniform(2.0, 6.0)
    inp = opf_network(N=int(N_s), seed=4000 + s, rho=rho, sigma_lo=-6.0, sigma_hi=6.0,
                      sigma_seed=100000 + s)
    inp.meta["batch_index"] = s
    return inp


def slack_sigma(m: int, seed: int = 9, ineq_fraction: float = 1.0 / 3.0, lo: float = -4.0,
                hi: float = 4.0) -> np.ndarray:
    """Slack barrier values for the rows of J of a problem with inequality
    constraints: each row is an inequality with probability `ineq_fraction`,
    with Sigma_s = 10^U(lo, hi); the other rows are equality rows, marked +inf.
    Draw order: the row kinds, then the values of all rows."""
    rng = np.random.default_rng(seed)
    ineq = rng.uniform(size=m) < ineq_fraction
    vals = 10.0 ** rng.uniform(lo, hi, size=m)
    return np.where(ineq, vals, np.inf)


def qp_family(n_side: int = 12, m: int = 40, seed: int = 12, bounded: float = 0.5, loose: bool = False):
    """A convex QP of the problem family NCO with equality rows only:
    Q = 2-D Laplacian of an n_side x n_side grid + I (SPD), q ~ N(0,1), A with
    m rows of 4 N(0,1) entries in distinct random columns, b = A x_f for a
    strictly interior x_f ~ U(-0.5, 0.5); a fraction `bounded` of the
    variables has bounds [-1 - U, 1 + U] (the others are free), or bounds
    [-1e3, 1e3] on every variable when `loose` (then none is active).
    Returns (Q lower CSC parts, q, A CSR parts, b, l, u, x0 = 0).
    Draw order: q, A columns and values, x_f, the bounded mask, the bounds."""
    rng = np.random.default_rng(seed)
    n = n_side * n_side
    rows, cols, vals = [], [], []
    for r_ in range(n_side):
        for c_ in range(n_side):
            k = r_ * n_side + c_
            rows.append(k); cols.append(k); vals.append(5.0)
            if r_ + 1 < n_side:
                rows.append(k + n_side); cols.append(k); vals.append(-1.0)
            if c_ + 1 < n_side:
                rows.append(k + 1); cols.append(k); vals.append(-1.0)
    Qp, Qi, Qx = _lower_csc(n, rows, cols, vals)
    q = rng.standard_normal(n)
    Jr, Jc, Jv = [0], [], []
    for _ in range(m):
        cs = np.sort(rng.choice(n, 4, replace=False))
        Jc.extend(cs.tolist())
        Jv.extend(rng.standard_normal(4).tolist())
        Jr.append(len(Jc))
    x_f = rng.uniform(-0.5, 0.5, n)
    A_ptr, A_idx, A_val = np.asarray(Jr, np.int32), np.asarray(Jc, np.int32), np.asarray(Jv, np.float64)
    b = np.zeros(m)
    for r_ in range(m):
        b[r_] = float(np.dot(A_val[A_ptr[r_]:A_ptr[r_ + 1]], x_f[A_idx[A_ptr[r_]:A_ptr[r_ + 1]]]))
    mask = rng.uniform(size=n) < bounded
    lo, hi = -1.0 - rng.uniform(size=n), 1.0 + rng.uniform(size=n)
    if loose:
        l, u = np.full(n, -1e3), np.full(n, 1e3)
    else:
        l, u = np.where(mask, lo, -np.inf), np.where(mask, hi, np.inf)
    return dict(n=n, m=m, Q_colptr=Qp, Q_rowidx=Qi, Q_val=Qx, q=q, A_rowptr=A_ptr, A_colidx=A_idx, A_val=A_val,
                b=b, l=l, u=u, x0=np.zeros(n))
