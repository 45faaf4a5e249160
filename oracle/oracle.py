"""Python face of the FP64 CPU oracle (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It wraps `ncl_oracle.c` (assembly of both KKT forms, minimum-degree
ordering, up-looking LDL^T with static pivoting, solves, symmetric products)
and adds, in plain numpy, the iterative refinement loop, the backward error and
the adjoint gradient.  It never imports or calls the GPU library.

Paper references (MadNCL, arXiv 2510.05885):
  condensed K1 = W + Sigma + rho J^T J ............ Sec. 3.3, eq. K1
  stabilized K2r = [[W+Sigma, J^T], [J, -I/rho]] .. Sec. 3.2, eq. K2r
  static pivoting with block-dependent sign ....... Sec. 3.1 ("Sparse LDL^T")
  pivot epsilon, Richardson refinement ............ Sec. 4.3
  inertia (n,0,0) / (n,m,0) ....................... Sec. 3.4, Prop. "inertia"
  slack elimination K1s, Omega, Delta s ........... Sec. 3.3, Prop. "Condensed KKT system"
  Delta y, Delta r, Delta z_l, Delta z_u .......... Sec. 3.3 eq. K1-elimination, Sec. 3.2
                                                    eq. K2-elimination, Sec. 3.1 eq. K3
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ncl_oracle.c")
_LIB = os.path.join(_HERE, "libncl_oracle.so")
_lib = None

CONDENSED, STABILIZED = 0, 1
# Proposed pivot-epsilon defaults: the paper fixes 1e-10 for the stabilized
# form (Sec. 4.3) and leaves the condensed value unstated.
DEFAULT_EPS = {CONDENSED: 1e-12, STABILIZED: 1e-10}

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile ncl_oracle.c into a shared library next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        asm_args = [C.c_int, C.c_int, _i32p, _i32p, _f64p, _f64p, _i32p, _i32p, _f64p, C.c_double,
                    _i32p, C.c_void_p, C.c_void_p]
        for name in ("or_condensed_assemble", "or_stabilized_assemble"):
            f = getattr(lib, name)
            f.argtypes = asm_args
            f.restype = C.c_int64
        lib.or_symv.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_int, _f64p, C.c_int, _f64p, C.c_int]
        lib.or_symv.restype = None
        lib.or_norms.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        lib.or_norms.restype = None
        lib.or_mindeg.argtypes = [C.c_int, _i32p, _i32p, _i32p]
        lib.or_mindeg.restype = C.c_int
        lib.or_factor.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i8p, C.c_double, C.c_double,
                                  C.POINTER(C.c_int)]
        lib.or_factor.restype = C.c_void_p
        lib.or_free.argtypes = [C.c_void_p]
        lib.or_free.restype = None
        lib.or_nnz_L.argtypes = [C.c_void_p]
        lib.or_nnz_L.restype = C.c_int64
        lib.or_inertia.argtypes = [C.c_void_p, _i64p]
        lib.or_inertia.restype = None
        lib.or_get_factor.argtypes = [C.c_void_p, _i32p, _i32p, _f64p, _f64p, _i32p]
        lib.or_get_factor.restype = None
        lib.or_solve.argtypes = [C.c_void_p, C.c_int, _f64p, C.c_int, _f64p, C.c_int]
        lib.or_solve.restype = None
        _lib = lib
    return _lib


# ---------------------------------------------------------------------------
# Assembly
# ---------------------------------------------------------------------------

@dataclass
class LowerCSC:
    """Symmetric matrix stored as its lower triangle in CSC."""
    N: int
    p: np.ndarray
    i: np.ndarray
    x: np.ndarray

    def to_scipy_full(self) -> sp.csc_matrix:
        A = sp.csc_matrix((self.x, self.i, self.p), shape=(self.N, self.N))
        return (A + sp.tril(A, -1).T).tocsc()

    def dense(self) -> np.ndarray:
        return self.to_scipy_full().toarray()


def assemble(inp, form: int = CONDENSED) -> LowerCSC:
    """K1 (form 0) or K2r (form 1) of `inp`, lower CSC, FP64 (Sec. 3.3 / 3.2)."""
    lib = _L()
    n, m = inp.n, inp.m
    N = n if form == CONDENSED else n + m
    f = lib.or_condensed_assemble if form == CONDENSED else lib.or_stabilized_assemble
    args = (n, m, np.ascontiguousarray(inp.W_colptr, np.int32), np.ascontiguousarray(inp.W_rowidx, np.int32),
            np.ascontiguousarray(inp.W_val, np.float64), np.ascontiguousarray(inp.Sigma, np.float64),
            np.ascontiguousarray(inp.J_rowptr, np.int32), np.ascontiguousarray(inp.J_colidx, np.int32),
            np.ascontiguousarray(inp.J_val, np.float64), float(inp.rho))
    Kp = np.zeros(N + 1, np.int32)
    nnz = f(*args, Kp, None, None)
    if nnz < 0:
        raise MemoryError("oracle assembly failed")
    Ki = np.zeros(max(nnz, 1), np.int32)
    Kx = np.zeros(max(nnz, 1), np.float64)
    f(*args, Kp, Ki.ctypes.data_as(C.c_void_p), Kx.ctypes.data_as(C.c_void_p))
    return LowerCSC(N, Kp, Ki[:nnz], Kx[:nnz])


def symv(K: LowerCSC, X: np.ndarray) -> np.ndarray:
    """K X for symmetric K (lower CSC), X of shape (N,) or (N, k)."""
    X2 = np.asarray(X, np.float64).reshape(K.N, -1)
    Xc = np.ascontiguousarray(X2.T)          # each column contiguous
    Y = np.zeros_like(Xc)
    _L().or_symv(K.N, K.p, K.i, K.x, Xc.shape[0], Xc, K.N, Y, K.N)
    Y = Y.T
    return Y.reshape(np.shape(X))


def norms(K: LowerCSC):
    """(max_ij |K_ij|, ||K||_inf) of the symmetric matrix."""
    a, b = C.c_double(), C.c_double()
    _L().or_norms(K.N, K.p, K.i, K.x, C.byref(a), C.byref(b))
    return a.value, b.value


def primal_block_max(K: LowerCSC, n: int) -> float:
    """max |K_ij| over the primal block i, j < n (the whole matrix for the
    condensed form; W + Sigma for the stabilized one).  In lower CSC an entry
    with row i < n also has column j <= i < n."""
    sel = K.i < n
    return float(np.abs(K.x[sel]).max()) if np.any(sel) else 0.0


def pivot_thresholds(K: LowerCSC, n: int, m: int, form: int, rho: float, eps: float, scale: str = "global"):
    """(primal, dual) static-pivot thresholds (Sec. 3.1).  "global": both are
    eps * max_ij |K_ij| of the assembled matrix.  "block": each block of the
    stabilized matrix uses its own norm, eps * max |K_xx| for primal pivots and
    eps / rho (the -1/rho I block of Sec. 3.2, eq. K2r) for dual pivots; for
    the condensed form this is the global rule.  "absolute": the solver's
    pivot epsilon of Sec. 4.3 taken as an absolute bound, eps for every
    pivot, in both forms."""
    if scale == "absolute":
        return float(eps), float(eps)
    if scale == "global" or form == CONDENSED:
        t = eps * norms(K)[0]
        return t, t
    if scale != "block":
        raise ValueError(scale)
    return eps * primal_block_max(K, n), eps / rho


def block_signs(n: int, m: int, form: int) -> np.ndarray:
    """+1 for primal rows, -1 for dual rows, in the unpermuted ordering."""
    s = np.ones(n if form == CONDENSED else n + m, np.int8)
    if form == STABILIZED:
        s[n:] = -1
    return s


# ---------------------------------------------------------------------------
# Ordering and factorization
# ---------------------------------------------------------------------------

def mindeg(K: LowerCSC) -> np.ndarray:
    perm = np.zeros(K.N, np.int32)
    rc = _L().or_mindeg(K.N, K.p, K.i, perm)
    if rc != 0:
        raise MemoryError("oracle ordering failed")
    return perm


class OracleError(RuntimeError):
    pass


class LDL:
    """P K P^T = L D L^T with static pivoting (Sec. 3.1), K lower CSC."""

    def __init__(self, K: LowerCSC, perm=None, signs=None, pivot_thr=0.0):
        """pivot_thr: one threshold for every pivot, or a (primal, dual) pair."""
        lib = _L()
        self.N = K.N
        self.perm = np.ascontiguousarray(mindeg(K) if perm is None else perm, np.int32)
        sg = np.ones(K.N, np.int8) if signs is None else np.ascontiguousarray(signs, np.int8)
        tp, td = (pivot_thr, pivot_thr) if np.ndim(pivot_thr) == 0 else pivot_thr
        st = C.c_int(0)
        h = lib.or_factor(K.N, K.p, K.i, K.x, self.perm, sg, float(tp), float(td), C.byref(st))
        self.status = st.value
        if not h:
            raise OracleError(f"oracle factorization failed (status {st.value})")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _L().or_free(h)
            self._h = None

    def inertia(self):
        out = np.zeros(4, np.int64)
        _L().or_inertia(self._h, out)
        return tuple(int(v) for v in out)      # (npos, nneg, nzero, nperturbed)

    def factor(self):
        """(L as scipy CSC unit lower incl. diagonal, D, perm) in the permuted ordering."""
        lib = _L()
        nnz = lib.or_nnz_L(self._h)
        Lp = np.zeros(self.N + 1, np.int32); Li = np.zeros(max(nnz, 1), np.int32)
        Lx = np.zeros(max(nnz, 1)); D = np.zeros(self.N); perm = np.zeros(self.N, np.int32)
        lib.or_get_factor(self._h, Lp, Li, Lx, D, perm)
        L = sp.csc_matrix((Lx[:nnz], Li[:nnz], Lp), shape=(self.N, self.N)) + sp.eye(self.N, format="csc")
        return L.tocsc(), D, perm

    def nnz_L(self) -> int:
        return int(_L().or_nnz_L(self._h))

    def solve(self, B: np.ndarray) -> np.ndarray:
        B2 = np.asarray(B, np.float64).reshape(self.N, -1)
        Bc = np.ascontiguousarray(B2.T)
        Xc = np.zeros_like(Bc)
        _L().or_solve(self._h, Bc.shape[0], Bc, self.N, Xc, self.N)
        return Xc.T.reshape(np.shape(B))


# ---------------------------------------------------------------------------
# Refinement, backward error, full solve
# ---------------------------------------------------------------------------

def backward_error(K: LowerCSC, X, B, Kinf=None) -> np.ndarray:
    """Normwise backward error per column: ||b - Kx||_inf / (||K||_inf ||x||_inf + ||b||_inf)."""
    X2 = np.asarray(X).reshape(K.N, -1); B2 = np.asarray(B).reshape(K.N, -1)
    if Kinf is None:
        Kinf = norms(K)[1]
    R = B2 - symv(K, X2)
    den = Kinf * np.abs(X2).max(axis=0) + np.abs(B2).max(axis=0)
    return np.abs(R).max(axis=0) / np.where(den > 0, den, 1.0)


def componentwise_backward_error(K: LowerCSC, X, B) -> np.ndarray:
    """Componentwise (Oettli-Prager) backward error per column:
    max_i |b - Kx|_i / (|K| |x| + |b|)_i, rows with a zero denominator skipped
    when their residual is zero too (infinite otherwise)."""
    X2 = np.asarray(X).reshape(K.N, -1); B2 = np.asarray(B).reshape(K.N, -1)
    R = np.abs(B2 - symv(K, X2))
    Ka = LowerCSC(K.N, K.p, K.i, np.abs(K.x))
    den = symv(Ka, np.abs(X2)) + np.abs(B2)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(den > 0, R / np.where(den > 0, den, 1.0), np.where(R > 0, np.inf, 0.0))
    return q.max(axis=0)


def residual_rel2(K: LowerCSC, X, B) -> np.ndarray:
    """||b - Kx||_2 / ||b||_2 per column."""
    X2 = np.asarray(X).reshape(K.N, -1); B2 = np.asarray(B).reshape(K.N, -1)
    nb = np.linalg.norm(B2, axis=0)
    return np.linalg.norm(B2 - symv(K, X2), axis=0) / np.where(nb > 0, nb, 1.0)


@dataclass
class SolveInfo:
    inertia: tuple = ()
    ir_steps: int = 0
    omega_history: list = field(default_factory=list)
    backward_error: float = np.inf
    backward_error_cw: float = np.inf
    inertia_ok: bool = False
    nnz_L: int = 0


def expected_inertia(n: int, m: int, form: int):
    """Inertia of a correctly regularized system (Sec. 3.4): (n,0,0) or (n,m,0)."""
    return (n, 0, 0) if form == CONDENSED else (n, m, 0)


def refine(K: LowerCSC, F: LDL, B, ir_max: int = 10, ir_tol: float = 1e-12, ir_stall: float = 0.5,
           Kinf=None, ir_cw_tol: float = 0.0):
    """Richardson refinement x <- x + F^-1 (b - K x) against the unperturbed K
    (Sec. 3.1 and 4.3).  The target is omega <= ir_tol and, when ir_cw_tol > 0,
    the componentwise backward error <= ir_cw_tol too; the distance to it is
    g = max(omega / ir_tol, omega_cw / ir_cw_tol).  Stops at g <= 1, after
    ir_max corrections, or when one correction fails to bring g below
    ir_stall times its previous value; the best iterate (smallest g) is
    returned.  Returns (X, omega history, corrections applied)."""
    B2 = np.asarray(B, np.float64).reshape(K.N, -1)
    if Kinf is None:
        Kinf = norms(K)[1]

    def measure(X):
        om = float(backward_error(K, X, B2, Kinf).max())
        g = om / ir_tol if ir_tol > 0 else (np.inf if om > 0 else 0.0)
        if ir_cw_tol > 0:
            g = max(g, float(componentwise_backward_error(K, X, B2).max()) / ir_cw_tol)
        return om, g

    X = F.solve(B2)
    om, g = measure(X)
    hist = [om]
    best_X, best_g, best_om = X, g, om
    steps = 0
    while g > 1.0 and steps < ir_max:
        R = B2 - symv(K, X)
        Xn = X + F.solve(R)
        omn, gn = measure(Xn)
        steps += 1
        hist.append(omn)
        if gn < best_g:
            best_X, best_g, best_om = Xn, gn, omn
        if gn > ir_stall * g:
            break
        X, om, g = Xn, omn, gn
    return best_X.reshape(np.shape(B)), hist, steps


def solve(inp, form: int, B, eps=None, ir_max: int = 10, ir_tol: float = 1e-12, ir_stall: float = 0.5,
          perm=None, K: LowerCSC | None = None, pivot_scale: str = "global", ir_cw_tol: float = 0.0):
    """Assemble, order, factor with static pivoting and refine: the whole path
    in FP64 on the CPU.  eps is relative to max_ij |K_ij| (pivot rule
    |d| < eps*||K||_max -> d = sign*eps*||K||_max), to each block's own norm
    with pivot_scale="block", or an absolute bound with pivot_scale="absolute"
    (see pivot_thresholds).  Refinement runs only when
    the inertia is the expected one (Sec. 4.3)."""
    if K is None:
        K = assemble(inp, form)
    if eps is None:
        eps = DEFAULT_EPS[form]
    kmax, kinf = norms(K)
    thr = pivot_thresholds(K, inp.n, inp.m, form, inp.rho, eps, pivot_scale)
    F = LDL(K, perm=perm, signs=block_signs(inp.n, inp.m, form), pivot_thr=thr)
    if F.status not in (0,):
        raise OracleError(f"factorization status {F.status}")
    info = SolveInfo(inertia=F.inertia(), nnz_L=F.nnz_L())
    info.inertia_ok = info.inertia[:3] == expected_inertia(inp.n, inp.m, form)
    if info.inertia_ok:
        X, hist, steps = refine(K, F, B, ir_max, ir_tol, ir_stall, kinf, ir_cw_tol)
    else:
        X = F.solve(B)
        hist, steps = [float(backward_error(K, X, B, kinf).max())], 0
    info.omega_history, info.ir_steps = hist, steps
    info.backward_error = float(backward_error(K, X, B, kinf).max())
    info.backward_error_cw = float(componentwise_backward_error(K, X, B).max())
    return X, info, F, K


# ---------------------------------------------------------------------------
# Adjoint of x = K^-1 b (condensed form)
# ---------------------------------------------------------------------------

def adjoint_condensed(inp, F: LDL, X, Xbar):
    """Gradients of a loss with dL/dX = Xbar through X = K^-1 B, K = W + Sigma + rho J^T J.

    lambda = K^-1 Xbar (K symmetric, so the transpose solve is a solve);
    dL/dB = lambda;  dL/dK = -lambda X^T summed over columns, which on the
    symmetric storage gives, for a stored lower W entry (i,j), i != j,
    -(lambda_i x_j + lambda_j x_i) and on the diagonal -lambda_i x_i;
    dL/dSigma_i = -lambda_i x_i;
    dL/dJ_ri = -rho [lambda_i (J x)_r + x_i (J lambda)_r];
    dL/drho = -(J lambda) . (J x).  All sums run over right-hand-side columns.
    Returns (gB, gW (per stored W entry), gSigma, gJ (per stored J entry), grho)."""
    X2 = np.asarray(X).reshape(inp.n, -1)
    Lam = F.solve(np.asarray(Xbar).reshape(inp.n, -1))
    Wrows = inp.W_rowidx.astype(np.int64)
    Wcols = np.repeat(np.arange(inp.n), np.diff(inp.W_colptr))
    off = Wrows != Wcols
    gW = -np.einsum("ec,ec->e", Lam[Wrows], X2[Wcols])
    gW = gW - off * np.einsum("ec,ec->e", Lam[Wcols], X2[Wrows])
    gS = -np.einsum("ic,ic->i", Lam, X2)
    J = sp.csr_matrix((inp.J_val, inp.J_colidx, inp.J_rowptr), shape=(inp.m, inp.n))
    JX = J @ X2
    JL = J @ Lam
    Jrows = np.repeat(np.arange(inp.m), np.diff(inp.J_rowptr))
    Jcols = inp.J_colidx.astype(np.int64)
    gJ = -inp.rho * (np.einsum("ec,ec->e", Lam[Jcols], JX[Jrows]) + np.einsum("ec,ec->e", X2[Jcols], JL[Jrows]))
    grho = -float(np.sum(JL * JX))
    return Lam.reshape(np.shape(Xbar)), gW, gS, gJ, grho


# ---------------------------------------------------------------------------
# Slack elimination (K1s) and the recovery of the rest of the Newton step
# ---------------------------------------------------------------------------
# Problem NCO (Sec. 3): the rows of J are the equality constraints c_E and the
# inequality constraints c_I, each inequality row with its slack s_r.  Here
# every row of J carries a slack barrier value Sigma_s[r]; +inf marks an
# equality row (the limit of the remark after the proposition: an active
# inequality, Sigma_s -> inf, is treated as an equality, Omega -> 1).
# Throughout, `inp.rho` is rho-hat = rho + delta.

def _J(inp) -> sp.csr_matrix:
    return sp.csr_matrix((inp.J_val, inp.J_colidx, inp.J_rowptr), shape=(inp.m, inp.n))


def _W_full(inp) -> sp.csc_matrix:
    Wl = sp.csc_matrix((inp.W_val, inp.W_rowidx, inp.W_colptr), shape=(inp.n, inp.n))
    return (Wl + sp.tril(Wl, -1).T).tocsc()


def k1s_omega(Sigma_s, rho: float) -> np.ndarray:
    """Omega_rr = Sigma_s,r / (rho + Sigma_s,r) (Sec. 3.3, Proposition
    "Condensed KKT system"); 1 on equality rows (Sigma_s = +inf)."""
    S = np.asarray(Sigma_s, np.float64)
    om = np.ones_like(S)
    fin = np.isfinite(S)
    om[fin] = S[fin] / (rho + S[fin])
    return om


def assemble_k1s(inp, Sigma_s) -> LowerCSC:
    """K1s = W_t + Sigma_t + rho J_E^T J_E + rho J_I^T Omega J_I (eq. K1s), as
    W + Sigma + rho J^T diag(omega) J over all rows of J, lower CSC, FP64."""
    J = _J(inp)
    K = _W_full(inp) + sp.diags(np.asarray(inp.Sigma, np.float64)) \
        + inp.rho * (J.T @ sp.diags(k1s_omega(Sigma_s, inp.rho)) @ J)
    low = sp.tril(K).tocsc()
    low.sort_indices()
    return LowerCSC(inp.n, low.indptr.astype(np.int32), low.indices.astype(np.int32), low.data.astype(np.float64))


def k1s_rhs(inp, Sigma_s, r_t, r_s) -> np.ndarray:
    """Right-hand side of eq. K1s as the elimination in the proof produces it:
    r_t + rho J_I^T (Sigma_s + rho I)^-1 r_s.  (The printed eq. K1s and the
    proof's intermediate equation omit the factor (Sigma_s + rho I)^-1; the
    substitution of Delta s into the first block row of K1' gives it.)  r_s
    is not read on equality rows."""
    S = np.asarray(Sigma_s, np.float64)
    ineq = np.isfinite(S)
    w = np.zeros(inp.m)
    w[ineq] = np.asarray(r_s, np.float64)[ineq] / (S[ineq] + inp.rho)
    return np.asarray(r_t, np.float64) + inp.rho * (_J(inp).T @ w)


def k1s_recover_ds(inp, Sigma_s, dt, r_s) -> np.ndarray:
    """Delta s = (Sigma_s + rho I)^-1 (rho J_I Delta t + r_s), the elimination
    in the proof of the proposition; 0 on equality rows (no slack)."""
    S = np.asarray(Sigma_s, np.float64)
    ineq = np.isfinite(S)
    Jdt = _J(inp) @ np.asarray(dt, np.float64)
    ds = np.zeros(inp.m)
    ds[ineq] = (inp.rho * Jdt[ineq] + np.asarray(r_s, np.float64)[ineq]) / (S[ineq] + inp.rho)
    return ds


def barrier_sigma(x, l, u, z_l, z_u) -> np.ndarray:
    """Sigma = (X - L)^-1 Z_l + (U - X)^-1 Z_u (Sec. 3.1, below eq. K2unreg);
    an infinite bound gives a zero term."""
    x, l, u = (np.asarray(a, np.float64) for a in (x, l, u))
    return z_l / (x - l) + z_u / (u - x)


def recover_dy(inp, dx, c, y_k, y) -> np.ndarray:
    """Delta y = -rho (J Delta x + c) + y_k - y (Sec. 3.3, eq. K1-elimination)."""
    return -inp.rho * (_J(inp) @ np.asarray(dx, np.float64) + c) + y_k - y


def recover_dr(rho: float, dy, y_k, y, r) -> np.ndarray:
    """Delta r = theta (Delta y - y_k + y) - r with theta = 1 / rho (Sec. 3.2,
    eq. K2-elimination)."""
    return (1.0 / rho) * (np.asarray(dy, np.float64) - y_k + y) - r


def recover_dz(x, l, u, z_l, z_u, dx, mu: float):
    """Delta z_l = -(X - L)^-1 (Z_l Delta x - mu e) - z_l and
    Delta z_u = (U - X)^-1 (Z_u Delta x + mu e) - z_u (Sec. 3.1, the blocks
    eliminated from eq. K3); with an infinite bound the first term vanishes."""
    x, l, u, dx = (np.asarray(a, np.float64) for a in (x, l, u, dx))
    dzl = -(z_l * dx - mu) / (x - l) - z_l
    dzu = (z_u * dx + mu) / (u - x) - z_u
    return dzl, dzu


# ---------------------------------------------------------------------------
# Inertia correction (Sec. 3.1: delta is raised until the inertia is right)
# ---------------------------------------------------------------------------

def inertia_correction(inp, form: int, delta_init: float, growth: float, delta_max: float, eps=None,
                       pivot_scale: str = "global", Sigma_s=None):
    """Factor with delta = 0, then delta_init, delta_init * growth, ... (the
    regularization of eq. K2: delta on the primal diagonal and rho-hat =
    rho + delta) until the inertia is the expected one or delta would exceed
    delta_max.  Sigma_s given: the K1s form (condensed only).  Returns
    (delta, attempts, inertia_ok, F, K)."""
    if eps is None:
        eps = DEFAULT_EPS[form]
    delta, attempts = 0.0, 0
    while True:
        case = inp.with_values(Sigma=np.asarray(inp.Sigma, np.float64) + delta, rho=inp.rho + delta)
        K = assemble_k1s(case, Sigma_s) if Sigma_s is not None else assemble(case, form)
        thr = pivot_thresholds(K, inp.n, inp.m, form, case.rho, eps, pivot_scale)
        F = LDL(K, signs=block_signs(inp.n, inp.m, form), pivot_thr=thr)
        attempts += 1
        ok = F.status == 0 and F.inertia()[:3] == expected_inertia(inp.n, inp.m, form)
        nxt = delta_init if delta == 0.0 else delta * growth
        if ok or nxt > delta_max:
            return delta, attempts, ok, F, K
        delta = nxt
