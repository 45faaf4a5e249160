"""Pins of the oracle's Algorithm 1 (MadNCL, Sec. 2.3) on convex QPs, against
facts that do not come from the algorithm:

* inactive bounds: the solution of the equality-constrained QP is one dense
  KKT solve, [[Q, -A^T], [A, 0]] [x; y] = [-q; b];
* active bounds: the result satisfies the QP's KKT conditions (feasibility,
  stationarity, z >= 0, complementarity), and re-solving the
  equality-constrained QP with the active bounds fixed gives the same x;
* an inconsistent A x = b drives rho to rho_max: status "infeasible".
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import ncl_algorithm as NA
from paper_2510_05885_amd import synth


def _qp(d, q_scale=1.0):
    Ql = sp.csc_matrix((d["Q_val"], d["Q_rowidx"], d["Q_colptr"]), shape=(d["n"], d["n"]))
    Q = (Ql + sp.tril(Ql, -1).T).tocsc()
    A = sp.csr_matrix((d["A_val"], d["A_colidx"], d["A_rowptr"]), shape=(d["m"], d["n"]))
    return NA.QP(Q, q_scale * d["q"], A, d["b"], d["l"], d["u"])


@pytest.mark.parametrize("seed", [12, 13])
def test_inactive_bounds_equal_kkt_solve(seed):
    d = synth.qp_family(seed=seed, loose=True)
    qp = _qp(d)
    res = NA.solve(qp, d["x0"])
    n, m = d["n"], d["m"]
    K = np.block([[qp.Q.toarray(), -qp.A.T.toarray()], [qp.A.toarray(), np.zeros((m, m))]])
    sol = np.linalg.solve(K, np.r_[-qp.q, qp.b])
    assert res.status == 0
    assert np.abs(res.x - sol[:n]).max() <= 1e-7 * max(1.0, np.abs(sol[:n]).max())
    assert np.abs(res.y - sol[n:]).max() <= 1e-6 * max(1.0, np.abs(sol[n:]).max())
    assert res.extrapolated >= 1          # the superlinear phase is reached


def test_active_bounds_satisfy_kkt_and_active_set_resolve():
    d = synth.qp_family(seed=14, bounded=0.6)
    qp = _qp(d, q_scale=6.0)              # a large linear term pushes variables onto their bounds
    res = NA.solve(qp, d["x0"])
    x, y, zl, zu = res.x, res.y, res.z_l, res.z_u
    assert res.status == 0
    assert res.primal_inf <= 1e-8 and res.dual_inf <= 1e-8
    assert np.all(x >= qp.l - 1e-12) and np.all(x <= qp.u + 1e-12)
    assert np.all(zl >= 0) and np.all(zu >= 0)
    fl, fu = np.isfinite(qp.l), np.isfinite(qp.u)
    assert np.max(zl[fl] * (x[fl] - qp.l[fl])) <= 1e-8 and np.max(zu[fu] * (qp.u[fu] - x[fu])) <= 1e-8
    act_l = fl & (x - qp.l < 1e-6)
    act_u = fu & (qp.u - x < 1e-6)
    act = act_l | act_u
    assert act.sum() >= 3                 # the test exercises active bounds
    # equality-constrained QP with the active bounds as equalities
    n, m = d["n"], d["m"]
    E = np.eye(n)[act]
    fixed = np.where(act_l, qp.l, qp.u)[act]
    Qd, Ad = qp.Q.toarray(), qp.A.toarray()
    C = np.vstack([Ad, E])
    K = np.block([[Qd, -C.T], [C, np.zeros((C.shape[0], C.shape[0]))]])
    sol = np.linalg.solve(K, np.r_[-qp.q, qp.b, fixed])
    assert np.abs(x - sol[:n]).max() <= 1e-6 * max(1.0, np.abs(sol[:n]).max())


def test_inconsistent_constraints_are_reported_infeasible():
    d = synth.qp_family(seed=15, m=10, loose=True)
    Ap, Ai, Av = d["A_rowptr"], d["A_colidx"], d["A_val"]
    # row 10 repeats row 0 with a different right-hand side
    d["A_rowptr"] = np.r_[Ap, Ap[-1] + (Ap[1] - Ap[0])].astype(np.int32)
    d["A_colidx"] = np.r_[Ai, Ai[Ap[0]:Ap[1]]].astype(np.int32)
    d["A_val"] = np.r_[Av, Av[Ap[0]:Ap[1]]]
    d["b"] = np.r_[d["b"], d["b"][0] + 1.0]
    d["m"] = 11
    res = NA.solve(_qp(d), d["x0"])
    assert res.status == 1
