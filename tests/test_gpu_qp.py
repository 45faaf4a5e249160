"""GPU parity of Algorithm 1 (MadNCL, Sec. 2.3) on convex QPs: the library's
driver (ncl_qp_solve: every Newton direction a K1 factor + solve and the
recoveries of eqs. K1-elimination, K2-elimination and K3, all on the GPU)
against the oracle's Algorithm 1 with the same readings.

Both follow the same iterates up to rounding, so the status and the
iteration counts (outer, inner, extrapolation steps taken) are equal and the
returned points agree to the stopping tolerances.  This needs every K1 solve
accurate row by row: near the solution Sigma spans ~1e-9..1e13, where a
normwise backward error of 1e-12 still allows O(1) relative errors in the
rows of the free variables, and the trajectories then part.

Cases: bounds inactive (also against the dense KKT solve of the
equality-constrained QP), bounds active, an inconsistent A x = b
(infeasible), no constraint rows (m = 0), the FP32-factor path, a larger
grid (n = 1600, m = 400) that spans many blocks of every vector kernel, and
an x_0 outside its bounds (refused)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import ncl_algorithm as NA
from paper_2510_05885_amd import ncl_kkt as nk
from paper_2510_05885_amd import synth

from gpu_util import dev

pytestmark = pytest.mark.gpu


def _qp(d, q_scale=1.0):
    Ql = sp.csc_matrix((d["Q_val"], d["Q_rowidx"], d["Q_colptr"]), shape=(d["n"], d["n"]))
    Q = (Ql + sp.tril(Ql, -1).T).tocsc()
    A = sp.csr_matrix((d["A_val"], d["A_colidx"], d["A_rowptr"]), shape=(d["m"], d["n"]))
    return NA.QP(Q, q_scale * d["q"], A, d["b"], d["l"], d["u"])


def _gpu(d, q_scale=1.0, **kw):
    return nk.qp_solve(d["n"], d["m"], d["Q_colptr"], d["Q_rowidx"], dev(d["Q_val"]), dev(q_scale * d["q"]),
                       d["A_rowptr"], d["A_colidx"], dev(d["A_val"]), dev(d["b"]), dev(d["l"]), dev(d["u"]),
                       dev(d["x0"]), **kw)


def _close(a, b, tol):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max(initial=0.0)) <= tol * max(1.0, float(np.abs(b).max(initial=0.0)))


def _compare(name, d, q_scale=1.0, x_tol=1e-6, y_tol=1e-5, oracle_kw=None, **kw):
    print(f"[gpu] qp {name}: n={d['n']} m={d['m']}", flush=True)
    ref = NA.solve(_qp(d, q_scale), d["x0"], **(oracle_kw or {}))
    got = _gpu(d, q_scale, **kw)
    x, y = got.x.cpu().numpy(), got.y.cpu().numpy()
    print(f"[gpu]   status {got.status}/{ref.status} outer {got.outer}/{ref.outer} inner {got.inner}/{ref.inner} "
          f"extrapolated {got.extrapolated}/{ref.extrapolated} primal {got.primal_inf:.2e} dual {got.dual_inf:.2e}",
          flush=True)
    assert got.status == ref.status
    assert (got.outer, got.inner, got.extrapolated) == (ref.outer, ref.inner, ref.extrapolated)
    if ref.status == 0:
        assert _close(x, ref.x, x_tol)
        assert _close(y, ref.y, y_tol)
        assert _close(got.z_l.cpu().numpy(), ref.z_l, y_tol)
        assert _close(got.z_u.cpu().numpy(), ref.z_u, y_tol)
        assert got.primal_inf <= 1e-8 and got.dual_inf <= 1e-8
    return got, ref


@pytest.mark.parametrize("seed", [12, 13])
def test_qp_inactive_bounds(seed):
    d = synth.qp_family(seed=seed, loose=True)
    got, _ = _compare(f"loose seed {seed}", d)
    qp = _qp(d)
    n, m = d["n"], d["m"]
    K = np.block([[qp.Q.toarray(), -qp.A.T.toarray()], [qp.A.toarray(), np.zeros((m, m))]])
    sol = np.linalg.solve(K, np.r_[-qp.q, qp.b])
    assert _close(got.x.cpu().numpy(), sol[:n], 1e-7)
    assert got.extrapolated >= 1


def test_qp_active_bounds():
    d = synth.qp_family(seed=14, bounded=0.6)
    got, ref = _compare("active bounds", d, q_scale=6.0)
    x = got.x.cpu().numpy()
    act = (np.isfinite(d["l"]) & (x - d["l"] < 1e-6)) | (np.isfinite(d["u"]) & (d["u"] - x < 1e-6))
    assert act.sum() >= 3
    assert np.all(got.z_l.cpu().numpy() >= 0) and np.all(got.z_u.cpu().numpy() >= 0)


def test_qp_infeasible():
    d = synth.qp_family(seed=15, m=10, loose=True)
    Ap, Ai, Av = d["A_rowptr"], d["A_colidx"], d["A_val"]
    d["A_rowptr"] = np.r_[Ap, Ap[-1] + (Ap[1] - Ap[0])].astype(np.int32)
    d["A_colidx"] = np.r_[Ai, Ai[Ap[0]:Ap[1]]].astype(np.int32)
    d["A_val"] = np.r_[Av, Av[Ap[0]:Ap[1]]]
    d["b"] = np.r_[d["b"], d["b"][0] + 1.0]
    d["m"] = 11
    got, _ = _compare("infeasible", d)
    assert got.status == 1


def test_qp_no_constraint_rows():
    d = synth.qp_family(seed=16, m=0, bounded=0.7)
    _compare("m=0", d, q_scale=4.0)


def test_qp_fp32_factor():
    d = synth.qp_family(seed=14, bounded=0.6)
    _compare("fp32_ir", d, q_scale=6.0, precision="fp32_ir")


def test_qp_larger_grid():
    d = synth.qp_family(n_side=40, m=400, seed=17, bounded=0.5)
    _compare("grid 40x40", d, q_scale=3.0)


def test_qp_outer_iteration_limit():
    """Stopped after 3 outer iterations: status 2 (limit) with the oracle's
    iterate at that point."""
    d = synth.qp_family(seed=14, bounded=0.6)
    got, ref = _compare("outer limit 3", d, q_scale=6.0, oracle_kw=dict(max_outer=3), max_outer=3)
    assert got.status == ref.status == 2 and got.outer == 3
    assert _close(got.x.cpu().numpy(), ref.x, 1e-6)


def test_qp_refuses_x0_outside_bounds():
    print("[gpu] qp x0 outside bounds", flush=True)
    d = synth.qp_family(seed=14, bounded=0.6)
    k = int(np.flatnonzero(np.isfinite(d["l"]))[0])
    d["x0"] = d["x0"].copy()
    d["x0"][k] = d["l"][k]
    with pytest.raises(nk.NCLError) as e:
        _gpu(d)
    assert e.value.code == nk.NCL_ERR_ARG
