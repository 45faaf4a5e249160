"""Pins of the FP64 CPU oracle against facts fixed by the paper and by linear algebra.

Each test checks the oracle against something other than itself: hand-worked
values (tests/golden), matrix-vector identities computed with scipy, numpy's
dense solve and eigenvalues, the closed-form block factor of the stabilized
system (Sec. 3.2, eq. ldlk2r), the condensed/stabilized equivalence
(Sec. 3.3, eqs. K1 and K1-elimination), the inertia proposition (Sec. 3.4),
the static-pivot semantics (Sec. 3.1) and central finite differences.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dense
from oracle import oracle as O
from paper_2510_05885_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _tiny_input():
    g = json.load(open(os.path.join(GOLD, "assembly_tiny.json")))
    a = np.asarray
    inp = synth.KKTInput(g["n"], g["m"], a(g["W_colptr"], np.int32), a(g["W_rowidx"], np.int32),
                         a(g["W_val"], float), a(g["Sigma"], float), a(g["J_rowptr"], np.int32),
                         a(g["J_colidx"], np.int32), a(g["J_val"], float), g["rho"])
    return inp, g


def _full(inp):
    W = sp.csc_matrix((inp.W_val, inp.W_rowidx, inp.W_colptr), shape=(inp.n, inp.n))
    Wf = W + sp.tril(W, -1).T
    J = sp.csr_matrix((inp.J_val, inp.J_colidx, inp.J_rowptr), shape=(inp.m, inp.n))
    return Wf.tocsr(), J


def test_assembly_golden():
    inp, g = _tiny_input()
    for form, key in ((O.CONDENSED, "condensed_lower"), (O.STABILIZED, "stabilized_lower")):
        K = O.assemble(inp, form)
        assert K.p.tolist() == g[key]["colptr"]
        assert K.i.tolist() == g[key]["rowidx"]
        assert K.x.tolist() == g[key]["val"]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_assembly_matvec_identity(seed):
    inp = synth.random_system(40, 17, seed=seed, rho=1e3)
    W, J = _full(inp)
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((inp.n, 3))
    K = O.assemble(inp, O.CONDENSED)
    ref = W @ V + inp.Sigma[:, None] * V + inp.rho * (J.T @ (J @ V))
    scale = (abs(W) @ abs(V) + inp.Sigma[:, None] * abs(V) + inp.rho * (abs(J).T @ (abs(J) @ abs(V))))
    assert np.all(np.abs(O.symv(K, V) - ref) <= 1e-14 * scale + 1e-300)
    # pattern = pattern(W) U diag U pattern(J^T J), lower part
    P = (abs(W) + sp.eye(inp.n) + abs(J).T @ abs(J)).tocsc()
    P = sp.tril(P).tocsc(); P.sort_indices()
    assert np.array_equal(P.indptr, K.p) and np.array_equal(P.indices, K.i)
    # stabilized
    K2 = O.assemble(inp, O.STABILIZED)
    U = rng.standard_normal((inp.n + inp.m, 2))
    u, v = U[:inp.n], U[inp.n:]
    ref2 = np.vstack([W @ u + inp.Sigma[:, None] * u + J.T @ v, J @ u - v / inp.rho])
    assert np.allclose(O.symv(K2, U), ref2, rtol=1e-14, atol=1e-14 * np.abs(ref2).max())


def test_ldl_golden():
    inp, _ = _tiny_input()
    g = json.load(open(os.path.join(GOLD, "ldl_tiny.json")))
    K = O.assemble(inp, O.CONDENSED)
    F = O.LDL(K, perm=np.arange(3, dtype=np.int32))
    L, D, _ = F.factor()
    assert np.allclose(D, g["D"], rtol=1e-14, atol=0)
    for key, val in g["L_strict_lower"].items():
        i, j = (int(t) for t in key.strip("()").split(","))
        assert abs(L[i, j] - val) <= 1e-14 * abs(val)
    assert F.inertia() == (3, 0, 0, 0)


def _systems():
    out = []
    for seed in range(4):
        out.append((synth.random_system(30, 12, seed=seed, rho=50.0), O.CONDENSED))
        out.append((synth.random_system(30, 12, seed=10 + seed, rho=50.0), O.STABILIZED))
    return out


@pytest.mark.parametrize("case", range(8))
@pytest.mark.parametrize("ordering", ["natural", "mindeg"])
def test_factor_reconstructs_and_matches_dense(case, ordering):
    inp, form = _systems()[case]
    K = O.assemble(inp, form)
    perm = np.arange(K.N, dtype=np.int32) if ordering == "natural" else None
    F = O.LDL(K, perm=perm)
    L, D, p = F.factor()
    Kd = K.dense()
    PKP = Kd[np.ix_(p, p)]
    Ld = L.toarray()
    assert np.allclose(np.diag(Ld), 1.0) and np.allclose(np.triu(Ld, 1), 0.0)
    R = Ld @ np.diag(D) @ Ld.T
    assert np.abs(R - PKP).max() <= 1e-12 * np.abs(PKP).max()
    Ld2, D2, npert = dense.ldl(PKP)
    assert npert == 0
    assert np.allclose(D, D2, rtol=1e-10, atol=1e-12 * np.abs(D2).max())
    assert np.allclose(Ld, Ld2, rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("case", range(8))
def test_solve_matches_numpy(case):
    inp, form = _systems()[case]
    K = O.assemble(inp, form)
    B = synth.rhs(K.N, 3, seed=case)
    X, info, F, _ = O.solve(inp, form, B, K=K)
    Xr = np.linalg.solve(K.dense(), B)
    assert np.abs(X - Xr).max() <= 1e-10 * np.abs(Xr).max()
    assert info.backward_error <= 1e-14


@pytest.mark.parametrize("seed", range(6))
def test_inertia_matches_eigenvalues_indefinite(seed):
    """Sylvester: the signs of D equal the eigenvalue signs (Sec. 3.4)."""
    inp = synth.random_system(25, 9, seed=100 + seed, rho=3.0, spd=False)
    for form in (O.CONDENSED, O.STABILIZED):
        K = O.assemble(inp, form)
        F = O.LDL(K)
        npos, nneg, nzero, npert = F.inertia()
        assert npert == 0
        ev = np.linalg.eigvalsh(K.dense())
        assert (npos, nneg) == (int((ev > 0).sum()), int((ev < 0).sum()))


def test_inertia_invariants_workload():
    """Prop. 'inertia': In(K1) = (n,0,0) and In(K2r) = (n,m,0) when W + Sigma is SPD."""
    inp = synth.grid_banded()
    for form, exp in ((O.CONDENSED, (2000, 0, 0)), (O.STABILIZED, (2000, 1000, 0))):
        _, info, _, K = O.solve(inp, form, synth.rhs(inp.n if form == 0 else 3000, 1, seed=3))
        assert info.inertia[:3] == exp
        if form == O.STABILIZED:
            ev = np.linalg.eigvalsh(K.dense())
            assert (int((ev > 0).sum()), int((ev < 0).sum())) == (2000, 1000)


@pytest.mark.parametrize("seed", [0, 1])
def test_stabilized_y_first_closed_form(seed):
    """Sec. 3.2, eq. ldlk2r: with the dual block ordered first, D11 = -1/rho,
    L21 = -rho J^T and the trailing factor is that of the condensed matrix."""
    inp = synth.random_system(20, 8, seed=seed, rho=100.0)
    n, m = inp.n, inp.m
    q = O.mindeg(O.assemble(inp, O.CONDENSED))
    perm = np.concatenate([n + np.arange(m), q]).astype(np.int32)
    F2 = O.LDL(O.assemble(inp, O.STABILIZED), perm=perm)
    L2, D2, _ = F2.factor()
    L2 = L2.toarray()
    assert np.all(D2[:m] == -1.0 / inp.rho)
    _, J = _full(inp)
    L21 = L2[m:, :m]
    assert np.allclose(L21, -inp.rho * J.toarray().T[q, :], rtol=1e-15, atol=0)
    assert np.allclose(L2[:m, :m], np.eye(m))
    F1 = O.LDL(O.assemble(inp, O.CONDENSED), perm=q)
    L1, D1, _ = F1.factor()
    assert np.allclose(D2[m:], D1, rtol=1e-11)
    assert np.allclose(L2[m:, m:], L1.toarray(), rtol=1e-9, atol=1e-11)
    assert F2.inertia()[:3] == (n, m, 0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_condensed_equals_stabilized(seed):
    """K2r [u; v] = [b1; b2]  <=>  K1 u = b1 + rho J^T b2, v = rho (J u - b2) (Sec. 3.3)."""
    inp = synth.grid_banded(seed=seed) if seed == 0 else synth.random_system(50, 20, seed=seed, rho=1e3)
    n, m = inp.n, inp.m
    rng = np.random.default_rng(seed)
    b1 = rng.standard_normal(n); b2 = rng.standard_normal(m)
    _, J = _full(inp)
    xs, _, _, _ = O.solve(inp, O.STABILIZED, np.concatenate([b1, b2]))
    xc, _, _, _ = O.solve(inp, O.CONDENSED, b1 + inp.rho * (J.T @ b2))
    assert np.abs(xs[:n] - xc).max() <= 1e-9 * np.abs(xc).max()
    assert np.abs(xs[n:] - inp.rho * (J @ xc - b2)).max() <= 1e-7 * np.abs(xs[n:]).max()


def test_static_pivot_primal_zero_recovered_by_refinement():
    """An exact zero primal pivot is replaced by +eps*||K|| (Sec. 3.1) and
    refinement against the unperturbed matrix recovers the solution (Sec. 4.3)."""
    inp = synth.random_system(30, 10, seed=7, rho=10.0, empty_w_rows=[0], zero_sigma=[0])
    K = O.assemble(inp, O.STABILIZED)
    assert K.x[K.p[0]] == 0.0 and K.i[K.p[0]] == 0
    perm = np.arange(K.N, dtype=np.int32)
    B = synth.rhs(K.N, 2, seed=1)
    X, info, F, _ = O.solve(inp, O.STABILIZED, B, perm=perm)
    kmax = O.norms(K)[0]
    _, D, _ = F.factor()
    assert info.inertia == (30, 10, 0, 1)
    assert D[0] == 1e-10 * kmax
    assert info.ir_steps >= 1 and info.backward_error <= 1e-12
    Xr = np.linalg.solve(K.dense(), B)
    assert np.abs(X - Xr).max() <= 1e-8 * np.abs(Xr).max()


def test_static_pivot_dual_sign():
    """Dual pivots below the threshold take the negative sign (Sec. 3.1):
    y-first ordering at rho = 1e14 turns every -1/rho pivot into -eps*||K||."""
    inp = synth.random_system(20, 6, seed=3, rho=1e14)
    K = O.assemble(inp, O.STABILIZED)
    perm = np.concatenate([inp.n + np.arange(inp.m), np.arange(inp.n)]).astype(np.int32)
    kmax = O.norms(K)[0]
    F = O.LDL(K, perm=perm, signs=O.block_signs(inp.n, inp.m, O.STABILIZED), pivot_thr=1e-10 * kmax)
    _, D, _ = F.factor()
    assert np.all(D[:inp.m] == -1e-10 * kmax)
    assert F.inertia() == (20, 6, 0, 6)


def test_static_pivot_condensed_singular_and_zero_status():
    inp = synth.random_system(15, 5, seed=4, empty_w_rows=[3], empty_j_cols=[3], zero_sigma=[3])
    K = O.assemble(inp, O.CONDENSED)
    kmax = O.norms(K)[0]
    F = O.LDL(K, perm=np.arange(15, dtype=np.int32), pivot_thr=1e-12 * kmax)
    _, D, _ = F.factor()
    assert F.inertia() == (15, 0, 0, 1) and D[3] == 1e-12 * kmax
    F0 = O.LDL(K, perm=np.arange(15, dtype=np.int32), pivot_thr=0.0)
    assert F0.status == -7 and F0.inertia()[2] == 1


def test_nonfinite_rejected():
    inp = synth.random_system(10, 3, seed=1)
    bad = inp.W_val.copy(); bad[2] = np.nan
    with pytest.raises(O.OracleError):
        O.LDL(O.assemble(inp.with_values(W_val=bad), O.CONDENSED))


def _pattern_K(n, edges):
    r = [max(a, b) for a, b in edges] + list(range(n))
    c = [min(a, b) for a, b in edges] + list(range(n))
    A = sp.csc_matrix((np.ones(len(r)), (r, c)), shape=(n, n)); A.sum_duplicates(); A.sort_indices()
    return O.LowerCSC(n, A.indptr.astype(np.int32), A.indices.astype(np.int32), np.arange(1.0, A.nnz + 1))


def test_mindeg_closed_form_fill():
    n = 40
    # a path (tridiagonal, scrambled labels): minimum degree gives no fill
    lab = np.random.default_rng(0).permutation(n)
    K = _pattern_K(n, [(lab[i], lab[i + 1]) for i in range(n - 1)])
    p = O.mindeg(K)
    assert sorted(p.tolist()) == list(range(n))
    Kd = K.dense(); Kd = Kd + np.diag(10.0 * np.abs(Kd).sum(1))
    K2 = O.LowerCSC(n, K.p, K.i, np.array([Kd[i, j] for j in range(n) for i in K.i[K.p[j]:K.p[j + 1]]]))
    assert O.LDL(K2, perm=p).nnz_L() == n - 1
    # an arrow (hub 7 joined to all): the hub goes last, no fill
    K = _pattern_K(n, [(7, i) for i in range(n) if i != 7])
    p = O.mindeg(K)
    assert p[-1] == 7 or p[-2] == 7   # the last two form a clique; either order is fill-free
    Kd = K.dense(); Kd = Kd + np.diag(10.0 * np.abs(Kd).sum(1))
    K2 = O.LowerCSC(n, K.p, K.i, np.array([Kd[i, j] for j in range(n) for i in K.i[K.p[j]:K.p[j + 1]]]))
    assert O.LDL(K2, perm=p).nnz_L() == n - 1


def test_mindeg_beats_natural_on_grid():
    inp = synth.grid_banded()
    K = O.assemble(inp, O.CONDENSED)
    nat = O.LDL(K, perm=np.arange(K.N, dtype=np.int32)).nnz_L()
    md = O.LDL(K).nnz_L()
    assert md < nat


def test_refinement_recovers_heavily_perturbed_factor():
    """With a large pivot epsilon many pivots are perturbed; refinement against
    the unperturbed K still drives the backward error down (Sec. 3.1, 4.3)."""
    inp = synth.grid_banded(rho=1e4)
    K = O.assemble(inp, O.CONDENSED)
    B = synth.rhs(K.N, 1, seed=9)
    X, info, _, _ = O.solve(inp, O.CONDENSED, B, eps=3e-5, ir_max=30)
    assert info.inertia[3] > 100 and info.ir_steps >= 3
    assert info.backward_error <= 1e-12
    Kd = K.dense()
    Xr = np.linalg.solve(Kd, B)
    kappa = np.abs(Kd).sum(1).max() * np.abs(np.linalg.inv(Kd)).sum(1).max()
    # forward error <= 2 kappa_inf * omega (first-order perturbation bound)
    assert np.abs(X - Xr).max() <= 2 * kappa * info.backward_error * np.abs(Xr).max()


def test_adjoint_against_finite_differences():
    inp = synth.random_system(24, 8, seed=5, rho=20.0)
    n = inp.n
    rng = np.random.default_rng(0)
    B = rng.standard_normal((n, 3)); Wt = rng.standard_normal((n, 3))

    def loss(i):
        X, _, _, _ = O.solve(i, O.CONDENSED, B, ir_tol=0.0, ir_max=3)
        return float(np.sum(Wt * X))

    X, _, F, K = O.solve(inp, O.CONDENSED, B, ir_tol=0.0, ir_max=3)
    gB, gW, gS, gJ, grho = O.adjoint_condensed(inp, F, X, Wt)
    assert np.allclose(gB, np.linalg.solve(K.dense(), Wt), rtol=1e-10)
    h = 1e-6

    def fd(field, k):
        v = getattr(inp, field).copy(); v0 = v[k]
        v[k] = v0 + h; lp = loss(inp.with_values(**{field if field != "W_val" else "W_val": v}))
        v[k] = v0 - h; lm = loss(inp.with_values(**{field: v}))
        return (lp - lm) / (2 * h)

    for k in range(0, len(inp.W_val), 7):
        assert abs(fd("W_val", k) - gW[k]) <= 1e-6 * abs(gW[k]) + 1e-8
    for k in range(0, n, 5):
        assert abs(fd("Sigma", k) - gS[k]) <= 1e-6 * abs(gS[k]) + 1e-8
    for k in range(0, len(inp.J_val), 3):
        assert abs(fd("J_val", k) - gJ[k]) <= 1e-6 * abs(gJ[k]) + 1e-8
    lp = loss(inp.with_values(rho=inp.rho + h)); lm = loss(inp.with_values(rho=inp.rho - h))
    assert abs((lp - lm) / (2 * h) - grho) <= 1e-6 * abs(grho) + 1e-9


# ---------------------------------------------------------------------------
# Norms, backward errors and block-scaled pivot thresholds, against dense numpy
# ---------------------------------------------------------------------------

def _norm_cases():
    inp, _ = _tiny_input()
    out = [(inp, O.CONDENSED), (inp, O.STABILIZED)]
    for seed in range(3):
        r = synth.random_system(35, 14, seed=20 + seed, rho=1e3, spd=seed != 1)
        out += [(r, O.CONDENSED), (r, O.STABILIZED)]
    g = synth.grid_banded(nr=10, nc=12, m=50, band=20, rho=1e4, seed=2)
    out += [(g, O.CONDENSED), (g, O.STABILIZED)]
    return out


@pytest.mark.parametrize("case", range(10))
def test_norms_match_dense(case):
    """max_ij |K_ij| (the static-pivot scale, Sec. 3.1) and ||K||_inf (the
    backward-error scale) equal the dense matrix's, both forms."""
    inp, form = _norm_cases()[case]
    K = O.assemble(inp, form)
    Kd = K.dense()
    kmax, kinf = O.norms(K)
    assert kmax == np.abs(Kd).max()
    assert abs(kinf - np.abs(Kd).sum(axis=1).max()) <= 1e-15 * kinf
    n = inp.n
    assert O.primal_block_max(K, n) == np.abs(Kd[:n, :n]).max()


def _mutant_norms_lib(tmp_path, drop):
    """The oracle's C source with one statement removed, compiled on the side
    (a planted mistake: the suite must notice it)."""
    import ctypes
    import subprocess
    src = open(os.path.join(os.path.dirname(O.__file__), "ncl_oracle.c")).read()
    assert drop in src
    p = tmp_path / "mutant.c"
    p.write_text(src.replace(drop, ";"))
    so = tmp_path / "mutant.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(p), "-lm"])
    return ctypes.CDLL(str(so))


def test_norms_pin_catches_dropped_mirror(tmp_path):
    """A plausible slip in the row sums (the mirrored off-diagonal entry not
    counted) changes ||K||_inf and is caught by the dense comparison above."""
    import ctypes
    lib = _mutant_norms_lib(tmp_path, "if (Ki[p] != j) rs[j] += a;")
    inp = synth.random_system(35, 14, seed=21, rho=1e3)
    K = O.assemble(inp, O.CONDENSED)
    a, b = ctypes.c_double(), ctypes.c_double()
    ip = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    lib.or_norms(ctypes.c_int(K.N), ip(K.p), ip(K.i), ip(K.x), ctypes.byref(a), ctypes.byref(b))
    assert abs(b.value - np.abs(K.dense()).sum(axis=1).max()) > 1e-6 * b.value


@pytest.mark.parametrize("case", range(10))
def test_backward_errors_match_dense(case):
    """Normwise omega = ||b-Kx||_inf / (||K||_inf ||x||_inf + ||b||_inf),
    componentwise max_i |b-Kx|_i / (|K||x|+|b|)_i and ||b-Kx||_2/||b||_2,
    each against its dense definition, on a perturbed solution."""
    inp, form = _norm_cases()[case]
    K = O.assemble(inp, form)
    Kd = K.dense()
    rng = np.random.default_rng(case)
    B = rng.standard_normal((K.N, 3))
    # relative perturbation 1e-6: residuals far above the rounding of either product
    X = np.linalg.solve(Kd, B) * (1.0 + 1e-6 * rng.standard_normal((K.N, 3)))
    R = B - Kd @ X
    om = np.abs(R).max(0) / (np.abs(Kd).sum(1).max() * np.abs(X).max(0) + np.abs(B).max(0))
    assert np.allclose(O.backward_error(K, X, B), om, rtol=1e-8, atol=0)
    cw = (np.abs(R) / (np.abs(Kd) @ np.abs(X) + np.abs(B))).max(0)
    assert np.allclose(O.componentwise_backward_error(K, X, B), cw, rtol=1e-8, atol=0)
    r2 = np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)
    assert np.allclose(O.residual_rel2(K, X, B), r2, rtol=1e-8, atol=0)
    # the exact solution of a tiny system has a residual at rounding level
    assert O.componentwise_backward_error(K, np.linalg.solve(Kd, B), B).max() <= 1e-13


def test_componentwise_error_sees_what_normwise_misses():
    """A wrong entry in a row of small |K||x| leaves the normwise omega tiny
    (||K||_inf is set by other rows) but not the componentwise one."""
    n = 4
    Kd = np.diag([1e12, 1.0, 1.0, 1.0])
    K = O.LowerCSC(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.diag(Kd).copy())
    b = np.ones(n)
    x = np.linalg.solve(Kd, b)
    x[3] *= 1.5
    assert O.backward_error(K, x, b)[0] < 1e-12
    assert O.componentwise_backward_error(K, x, b)[0] == pytest.approx(0.5 / 2.5)


@pytest.mark.parametrize("seed", [0, 1])
def test_block_pivot_scale_dual_block(seed):
    """Block-scaled thresholds (the -1/rho I block of Sec. 3.2, eq. K2r,
    against its own norm 1/rho): with the dual block ordered first at
    rho = 1e14 the global rule replaces every -1/rho pivot by -eps*||K||_max,
    the block rule keeps -1/rho exactly (eq. ldlk2r: D11 = -1/rho).  Dense
    brute force under the same thresholds gives the same D."""
    inp = synth.random_system(20, 6, seed=30 + seed, rho=1e14)
    n, m = inp.n, inp.m
    K = O.assemble(inp, O.STABILIZED)
    Kd = K.dense()
    perm = np.concatenate([n + np.arange(m), np.arange(n)]).astype(np.int32)
    sg = O.block_signs(n, m, O.STABILIZED)
    tg = O.pivot_thresholds(K, n, m, O.STABILIZED, inp.rho, 1e-10, "global")
    tb = O.pivot_thresholds(K, n, m, O.STABILIZED, inp.rho, 1e-10, "block")
    assert tg == (1e-10 * np.abs(Kd).max(),) * 2
    assert tb == (1e-10 * np.abs(Kd[:n, :n]).max(), 1e-10 / inp.rho)
    Fg = O.LDL(K, perm=perm, signs=sg, pivot_thr=tg)
    Fb = O.LDL(K, perm=perm, signs=sg, pivot_thr=tb)
    _, Dg, _ = Fg.factor()
    _, Db, _ = Fb.factor()
    assert Fg.inertia() == (n, m, 0, m) and np.all(Dg[:m] == -tg[1])
    assert Fb.inertia() == (n, m, 0, 0) and np.all(Db[:m] == -1.0 / inp.rho)
    for thr, D, npert in ((tg, Dg, m), (tb, Db, 0)):
        _, Dd, npd = dense.ldl(Kd[np.ix_(perm, perm)], signs=sg[perm], pivot_thr=thr)
        # the dual pivots exactly; the primal ones carry rho * J^T J at rho = 1e14
        # and differ by rounding between the two elimination orders
        assert npd == npert and np.array_equal(D[:m], Dd[:m])
        assert np.allclose(D[m:], Dd[m:], rtol=1e-6, atol=1e-14 * np.abs(Dd).max())
    # condensed form: the block rule is the global rule
    Kc = O.assemble(inp, O.CONDENSED)
    assert O.pivot_thresholds(Kc, n, m, O.CONDENSED, inp.rho, 1e-12, "block") == \
        O.pivot_thresholds(Kc, n, m, O.CONDENSED, inp.rho, 1e-12, "global")


def test_block_pivot_scale_primal_threshold_uses_primal_block():
    """A primal zero pivot met first is replaced by +eps*max|K_xx| under the
    block rule (and by +eps*max|K| under the global rule)."""
    inp = synth.random_system(30, 10, seed=7, rho=1e-3, empty_w_rows=[0], zero_sigma=[0])
    K = O.assemble(inp, O.STABILIZED)
    perm = np.arange(K.N, dtype=np.int32)
    tp, td = O.pivot_thresholds(K, inp.n, inp.m, O.STABILIZED, inp.rho, 1e-10, "block")
    assert td == 1e-10 / inp.rho and tp < td   # rho < 1: the dual block has the larger norm
    F = O.LDL(K, perm=perm, signs=O.block_signs(inp.n, inp.m, O.STABILIZED), pivot_thr=(tp, td))
    _, D, _ = F.factor()
    assert D[0] == tp and F.inertia()[:3] == (30, 10, 0)


def test_norms_golden():
    """Hand-derived norms of the tiny fixture (tests/golden/assembly_tiny.json)."""
    inp, g = _tiny_input()
    K1 = O.assemble(inp, O.CONDENSED)
    K2 = O.assemble(inp, O.STABILIZED)
    assert O.norms(K1) == (g["norms"]["condensed"]["max_abs"], g["norms"]["condensed"]["inf"])
    assert O.norms(K2) == (g["norms"]["stabilized"]["max_abs"], g["norms"]["stabilized"]["inf"])
    assert O.primal_block_max(K2, inp.n) == g["norms"]["stabilized"]["primal_block_max"]


def test_absolute_pivot_scale():
    """The pivot epsilon of Sec. 4.3 read as an absolute bound: every pivot
    with |d| < eps is replaced by +-eps, whatever the norm of K.  With the dual
    block first at rho = 1e14, -1/rho = -1e-14 is replaced by -eps for
    eps = 1e-10 and kept for eps = 1e-16; a primal pivot of order 1e-8 (an
    empty W row with Sigma = 1e-8, eliminated first) is kept for eps = 1e-10
    although the global and block rules, relative to max |K| >= 1e4,
    replace it.  Dense brute force under the same thresholds gives the same D."""
    inp = synth.random_system(20, 6, seed=31, rho=1e14, empty_w_rows=[0], empty_j_cols=[0])
    inp.Sigma[0] = 1e-8
    inp.Sigma[1] = 1e4          # max |K| = max |K_xx| >= 1e4: the relative thresholds exceed 1e-8
    n, m = inp.n, inp.m
    K = O.assemble(inp, O.STABILIZED)
    Kd = K.dense()
    assert Kd[0, 0] == 1e-8 and np.count_nonzero(Kd[0]) == 1
    sg = O.block_signs(n, m, O.STABILIZED)
    perm = np.concatenate([[0], n + np.arange(m), np.arange(1, n)]).astype(np.int32)
    for form in (O.CONDENSED, O.STABILIZED):
        assert O.pivot_thresholds(K, n, m, form, inp.rho, 1e-10, "absolute") == (1e-10, 1e-10)
    for eps, dual_pert in ((1e-10, True), (1e-16, False)):
        thr = O.pivot_thresholds(K, n, m, O.STABILIZED, inp.rho, eps, "absolute")
        F = O.LDL(K, perm=perm, signs=sg, pivot_thr=thr)
        _, D, _ = F.factor()
        assert D[0] == 1e-8                                   # the primal 1e-8 pivot is kept
        assert np.all(D[1:m + 1] == (-eps if dual_pert else -1.0 / inp.rho))
        assert F.inertia() == (n, m, 0, m if dual_pert else 0)
        _, Dd, npd = dense.ldl(Kd[np.ix_(perm, perm)], signs=sg[perm], pivot_thr=thr)
        assert npd == F.inertia()[3] and np.array_equal(D[:m + 1], Dd[:m + 1])
    for scale in ("global", "block"):   # both relative rules replace the 1e-8 pivot
        thr = O.pivot_thresholds(K, n, m, O.STABILIZED, inp.rho, 1e-10, scale)
        F = O.LDL(K, perm=perm, signs=sg, pivot_thr=thr)
        assert F.factor()[1][0] == thr[0] > 1e-8


@pytest.mark.slow
def test_adjoint_config5_finite_differences():
    from fd_util import config5_fd_cases, fd_tolerance
    """Config 5: the condensed grid system at rho = 1e6, 16 right-hand sides,
    loss = sum(w * X); the oracle's adjoint gradient against central
    differences (h = 1e-6) of the oracle's own solves on 200 entries, 50 each
    of B, W, Sigma and J (tolerance: fd_tolerance)."""
    inp = synth.grid_banded(rho=1e6)
    rng = np.random.default_rng(5)
    B = rng.standard_normal((inp.n, 16)); Wt = rng.standard_normal((inp.n, 16))
    perm = O.mindeg(O.assemble(inp, O.CONDENSED))
    X, info, F, K = O.solve(inp, O.CONDENSED, B, perm=perm)
    gB, gW, gS, gJ, _ = O.adjoint_condensed(inp, F, X, Wt)
    h = 1e-6

    def loss(i, Bm):
        return float(np.sum(Wt * O.solve(i, O.CONDENSED, Bm, perm=perm)[0]))

    cases = config5_fd_cases(inp, rng)
    for field, g in (("W_val", gW), ("Sigma", gS), ("J_val", gJ)):
        tol = fd_tolerance(g, Wt, X, h)
        for k in cases[field]:
            v = getattr(inp, field).copy(); v0 = v[k]
            v[k] = v0 + h; lp = loss(inp.with_values(**{field: v}), B)
            v[k] = v0 - h; lm = loss(inp.with_values(**{field: v}), B)
            assert abs((lp - lm) / (2 * h) - g[k]) <= tol[k], (field, k)
    tol = fd_tolerance(gB, Wt, X, h)
    for i, c in cases["B"]:
        Bp = B.copy(); Bp[i, c] += h; lp = loss(inp, Bp)
        Bp[i, c] -= 2 * h; lm = loss(inp, Bp)
        assert abs((lp - lm) / (2 * h) - gB[i, c]) <= tol[i, c]


def test_refine_componentwise_criterion():
    """Stabilized OPF-shaped system with Sigma over 16 decades (absolute
    pivot bound, nothing perturbed): the first solve already has a normwise
    backward error far below u, so the normwise rule stops with no
    correction, while the componentwise error (Oettli-Prager, checked against
    dense numpy) is ~1e-9.  With ir_cw_tol = 1e-14 one correction brings it
    below the bound, and the returned iterate is the refined one."""
    inp = synth.opf_network(N=200, seed=3, rho=1e3)
    B = synth.rhs(inp.n + inp.m, 1, seed=11)
    x0, i0, _, K = O.solve(inp, O.STABILIZED, B, eps=1e-10, pivot_scale="absolute")
    x1, i1, _, _ = O.solve(inp, O.STABILIZED, B, eps=1e-10, pivot_scale="absolute", ir_cw_tol=1e-14)
    Kd = K.dense()
    cw = lambda x: float(np.max(np.abs(B - Kd @ x) / (np.abs(Kd) @ np.abs(x) + np.abs(B))))
    assert i0.inertia == i1.inertia == (inp.n, inp.m, 0, 0)
    assert i0.ir_steps == 0 and i0.backward_error < 1e-18
    assert cw(x0) > 1e-10 and cw(x0) == pytest.approx(i0.backward_error_cw, rel=1e-6)
    assert i1.ir_steps >= 1 and cw(x1) <= 1e-14
    assert i1.backward_error_cw == pytest.approx(cw(x1), rel=0.5)
