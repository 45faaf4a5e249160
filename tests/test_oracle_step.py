"""Pins of the oracle's slack elimination (eq. K1s) and Newton-step recovery
(eqs. K1-elimination, K2-elimination and the eliminated blocks of K3) against
the unreduced Newton systems of Sec. 3, assembled and solved densely.

* K1s: for a problem with equality and inequality rows, K1 of the same
  problem with the slacks as explicit variables (x = (t, s), inequality rows
  of J extended by -I on the slack columns, the form used in the proof of the
  proposition "Condensed KKT system") is assembled by the oracle's own
  (pinned) condensed assembly and solved densely; eliminating the slacks must
  give the same Delta t, and the recovered Delta s the same slack step.
* Recovery: for a small NLP with finite bounds, the full system K3 (Delta x,
  Delta r, Delta y, Delta z_l, Delta z_u) is solved densely; the reduced
  chain -- Sigma, the K1 solve, then Delta y, Delta r, Delta z_l, Delta z_u --
  must reproduce it.  With a regularization delta > 0, the regularized K2 is
  the reference.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import oracle as O
from paper_2510_05885_amd import synth


def _nco(seed, nt=14, mE=3, mI=5, rho=37.0):
    """Random problem NCO data: W_t SPD (lower CSC), Sigma_t > 0, J_h = [J_E;
    J_I] with the inequality rows interleaved, Sigma_s (finite on inequality
    rows, +inf on equality rows)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((nt, nt))
    Wt = A @ A.T / nt + 0.5 * np.eye(nt)
    Wt[np.abs(Wt) < 0.3] = 0.0
    Wt = Wt + np.diag(np.abs(Wt).sum(1))           # diagonally dominant -> SPD
    m = mE + mI
    Jd = np.zeros((m, nt))
    for r in range(m):
        cols = rng.choice(nt, size=4, replace=False)
        Jd[r, cols] = rng.standard_normal(4)
    kinds = rng.permutation(np.r_[np.zeros(mE, bool), np.ones(mI, bool)])   # True = inequality
    Sigma_s = np.where(kinds, 10.0 ** rng.uniform(-3, 3, m), np.inf)
    Sigma_t = 10.0 ** rng.uniform(-2, 1, nt)
    low = sp.csc_matrix(np.tril(Wt))
    Jc = sp.csr_matrix(Jd)
    inp = synth.KKTInput(nt, m, low.indptr.astype(np.int32), low.indices.astype(np.int32), low.data.copy(),
                         Sigma_t, Jc.indptr.astype(np.int32), Jc.indices.astype(np.int32), Jc.data.copy(), rho)
    return inp, Wt, Jd, kinds, Sigma_s


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_k1s_equals_k1_with_explicit_slacks(seed):
    inp, Wt, Jd, kinds, Sigma_s = _nco(seed)
    nt, m, rho = inp.n, inp.m, inp.rho
    ineq = np.flatnonzero(kinds)
    mI = ineq.size
    # K1 over x = (t, s): J rows of inequality constraints get -1 on their slack
    n = nt + mI
    Jx = np.zeros((m, n))
    Jx[:, :nt] = Jd
    Jx[ineq, nt + np.arange(mI)] = -1.0
    Wx = np.zeros((n, n))
    Wx[:nt, :nt] = Wt
    low = sp.csc_matrix(np.tril(Wx))
    Jc = sp.csr_matrix(Jx)
    big = synth.KKTInput(n, m, low.indptr.astype(np.int32), low.indices.astype(np.int32), low.data.copy(),
                         np.r_[inp.Sigma, Sigma_s[ineq]], Jc.indptr.astype(np.int32), Jc.indices.astype(np.int32),
                         Jc.data.copy(), rho)
    K1 = O.assemble(big, O.CONDENSED).dense()
    rng = np.random.default_rng(100 + seed)
    r_t = rng.standard_normal(nt)
    r_s_rows = rng.standard_normal(m)          # entries on equality rows must not matter
    sol = np.linalg.solve(K1, np.r_[r_t, r_s_rows[ineq]])
    # eliminated form
    K1s = O.assemble_k1s(inp, Sigma_s).dense()
    b = O.k1s_rhs(inp, Sigma_s, r_t, r_s_rows)
    dt = np.linalg.solve(K1s, b)
    ds = O.k1s_recover_ds(inp, Sigma_s, dt, r_s_rows)
    scale = np.abs(sol).max()
    assert np.abs(dt - sol[:nt]).max() <= 1e-11 * scale
    assert np.abs(ds[ineq] - sol[nt:]).max() <= 1e-11 * scale
    assert np.all(ds[~kinds] == 0.0)
    # K1s is the Schur complement of the slack block of K1 (the proof's first step)
    K_tt, K_ts, K_ss = K1[:nt, :nt], K1[:nt, nt:], K1[nt:, nt:]
    schur = K_tt - K_ts @ np.linalg.solve(K_ss, K_ts.T)
    assert np.abs(K1s - schur).max() <= 1e-12 * np.abs(K1s).max()


def test_k1s_omega_limits_and_identity():
    rho = 50.0
    S = np.array([0.0, 1e-300, 1e-3, 50.0, 1e6, 1e300, np.inf])
    om = O.k1s_omega(S, rho)
    assert om[0] == 0.0 and om[-1] == 1.0 and om[3] == 0.5
    assert om[1] < 1e-300 and abs(om[-2] - 1.0) < 1e-15
    fin = np.isfinite(S)
    # I - rho (rho I + Sigma_s)^-1 = Sigma_s (rho I + Sigma_s)^-1
    assert np.allclose(1.0 - rho / (rho + S[fin]), om[fin], rtol=0, atol=4e-16)   # cancellation: absolute
    # all rows equality -> K1s is K1; a row with Sigma_s = 0 drops out of K1s
    inp, *_ = _nco(4)
    eq_all = np.full(inp.m, np.inf)
    assert np.abs(O.assemble_k1s(inp, eq_all).dense() - O.assemble(inp, O.CONDENSED).dense()).max() \
        <= 1e-13 * np.abs(O.assemble(inp, O.CONDENSED).dense()).max()
    S0 = eq_all.copy()
    S0[2] = 0.0
    J = sp.csr_matrix((inp.J_val, inp.J_colidx, inp.J_rowptr), shape=(inp.m, inp.n)).toarray()
    drop = inp.rho * np.outer(J[2], J[2])
    diff = O.assemble(inp, O.CONDENSED).dense() - O.assemble_k1s(inp, S0).dense()
    assert np.abs(diff - drop).max() <= 1e-12 * np.abs(drop).max()


def _nlp(seed, n=9, m=5):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    H = A @ A.T / n + np.eye(n)
    J = rng.standard_normal((m, n))
    l = -1.0 - rng.uniform(size=n)
    u = 1.0 + rng.uniform(size=n)
    x = rng.uniform(-0.5, 0.5, n)
    z_l, z_u = rng.uniform(0.1, 2.0, n), rng.uniform(0.1, 2.0, n)
    y, y_k, r, c, g = (rng.standard_normal(k) for k in (m, m, m, m, n))
    return H, J, l, u, x, z_l, z_u, y, y_k, r, c, g


def _reduced_chain(H, J, l, u, x, z_l, z_u, y, y_k, r, c, g, mu, rho, delta):
    """Sigma, K1 solve for Delta x (Sec. 3.3, eq. K1), then the recoveries."""
    n, m = H.shape[0], J.shape[0]
    rho_hat = rho + delta
    Sigma = O.barrier_sigma(x, l, u, z_l, z_u)
    K1 = H + np.diag(Sigma) + delta * np.eye(n) + rho_hat * J.T @ J
    rhs = J.T @ (y_k - rho_hat * c) - (g - mu / (x - l) + mu / (u - x))
    dx = np.linalg.solve(K1, rhs)
    low = sp.csc_matrix(np.tril(np.eye(n)))
    Jc = sp.csr_matrix(J)
    inp = synth.KKTInput(n, m, low.indptr.astype(np.int32), low.indices.astype(np.int32), low.data.copy(),
                         np.zeros(n), Jc.indptr.astype(np.int32), Jc.indices.astype(np.int32), Jc.data.copy(),
                         rho_hat)
    dy = O.recover_dy(inp, dx, c, y_k, y)
    dr = O.recover_dr(rho_hat, dy, y_k, y, r)
    dzl, dzu = O.recover_dz(x, l, u, z_l, z_u, dx, mu)
    return dx, dr, dy, dzl, dzu


@pytest.mark.parametrize("seed", [0, 1])
def test_recovery_reproduces_K3(seed):
    H, J, l, u, x, z_l, z_u, y, y_k, r, c, g = _nlp(seed)
    n, m = H.shape[0], J.shape[0]
    mu, rho = 0.07, 25.0
    I_n, I_m = np.eye(n), np.eye(m)
    Z = np.zeros
    K3 = np.block([
        [H, Z((n, m)), -J.T, -I_n, I_n],
        [Z((m, n)), rho * I_m, -I_m, Z((m, n)), Z((m, n))],
        [J, I_m, Z((m, m)), Z((m, n)), Z((m, n))],
        [np.diag(z_l), Z((n, m)), Z((n, m)), np.diag(x - l), Z((n, n))],
        [-np.diag(z_u), Z((n, m)), Z((n, m)), Z((n, n)), np.diag(u - x)],
    ])
    F = np.r_[g - J.T @ y - z_l + z_u, y_k + rho * r - y, c + r, z_l * (x - l) - mu, z_u * (u - x) - mu]
    sol = np.linalg.solve(K3, -F)
    ref = np.split(sol, np.cumsum([n, m, m, n]))
    got = _reduced_chain(H, J, l, u, x, z_l, z_u, y, y_k, r, c, g, mu, rho, 0.0)
    for a, b in zip(got, ref):
        assert np.abs(a - b).max() <= 1e-10 * max(np.abs(b).max(), 1.0)


def test_recovery_reproduces_regularized_K2():
    """delta > 0: the reduced chain with rho-hat = rho + delta against the
    regularized K2 (eq. K2) with the right-hand side of eq. K2unreg."""
    H, J, l, u, x, z_l, z_u, y, y_k, r, c, g = _nlp(7)
    n, m = H.shape[0], J.shape[0]
    mu, rho, delta = 0.01, 12.0, 0.3
    Sigma = O.barrier_sigma(x, l, u, z_l, z_u)
    Z = np.zeros
    K2 = np.block([
        [H + np.diag(Sigma) + delta * np.eye(n), Z((n, m)), J.T],
        [Z((m, n)), (rho + delta) * np.eye(m), np.eye(m)],
        [J, np.eye(m), Z((m, m))],
    ])
    rhs = -np.r_[g - J.T @ y - mu / (x - l) + mu / (u - x), y_k + (rho + delta) * r - y, c + r]
    sol = np.linalg.solve(K2, rhs)
    dx_ref, dr_ref, dy_ref = sol[:n], sol[n:n + m], -sol[n + m:]
    dx, dr, dy, _, _ = _reduced_chain(H, J, l, u, x, z_l, z_u, y, y_k, r, c, g, mu, rho, delta)
    for a, b in ((dx, dx_ref), (dr, dr_ref), (dy, dy_ref)):
        assert np.abs(a - b).max() <= 1e-10 * max(np.abs(b).max(), 1.0)


def test_barrier_terms_with_infinite_bounds():
    """An infinite bound contributes nothing to Sigma and leaves Delta z = -z
    (its multiplier is zero); a bound far away gives the same up to rounding."""
    x = np.array([0.2, -0.3])
    l = np.array([-np.inf, -1.0])
    u = np.array([1.0, np.inf])
    z_l, z_u = np.array([0.0, 0.5]), np.array([0.7, 0.0])
    S = O.barrier_sigma(x, l, u, z_l, z_u)
    assert S[0] == 0.7 / 0.8 and S[1] == 0.5 / 0.7
    dzl, dzu = O.recover_dz(x, l, u, z_l, z_u, np.array([0.1, 0.2]), 0.01)
    assert dzl[0] == 0.0 and dzu[1] == 0.0
    far = O.recover_dz(x, np.array([-1e300, -1.0]), np.array([1.0, 1e300]), z_l, z_u, np.array([0.1, 0.2]), 0.01)
    assert np.allclose(far[0], dzl) and np.allclose(far[1], dzu)


def _nonconvex(seed, n=40, m=12, rho=3.0):
    """Small system whose W has clearly negative eigenvalues, so delta = 0
    gives the wrong inertia; eigenvalue margins keep the PD test unambiguous."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.r_[-rng.uniform(2.0, 30.0, 5), rng.uniform(1.0, 10.0, n - 5)]
    W = (Q * ev) @ Q.T
    W[np.abs(W) < 0.2] = 0.0
    W = (W + W.T) / 2
    J = np.zeros((m, n))
    for r in range(m):
        J[r, rng.choice(n, 3, replace=False)] = rng.standard_normal(3)
    low = sp.csc_matrix(np.tril(W))
    Jc = sp.csr_matrix(J)
    inp = synth.KKTInput(n, m, low.indptr.astype(np.int32), low.indices.astype(np.int32), low.data.copy(),
                         10.0 ** rng.uniform(-2, 0, n), Jc.indptr.astype(np.int32), Jc.indices.astype(np.int32),
                         Jc.data.copy(), rho)
    return inp, W, J


@pytest.mark.parametrize("form", [O.CONDENSED, O.STABILIZED])
def test_inertia_correction_stops_at_first_definite_delta(form):
    """Brute force with eigvalsh over the same delta sequence: the loop stops
    at the first delta for which M = W + Sigma + delta I + (rho + delta) J^T J
    is positive definite -- the condition for inertia (n, 0, 0) of K1 and
    (n, m, 0) of K2r (Sec. 3.4; eq. ldlk2r)."""
    inp, W, J = _nonconvex(3)
    d0, g, dmax = 1e-2, 8.0, 1e6
    delta, attempts, ok, F, K = O.inertia_correction(inp, form, d0, g, dmax)
    cands = [0.0] + [d0 * g ** k for k in range(20)]
    def mineig(dl):
        M = W + np.diag(inp.Sigma + dl) + (inp.rho + dl) * J.T @ J
        return np.linalg.eigvalsh(M).min()
    first = next(k for k, dl in enumerate(cands) if mineig(dl) > 0)
    assert ok and attempts == first + 1 and delta == cands[first]
    assert mineig(cands[first]) > 1e-3 and mineig(cands[first - 1]) < -1e-3   # margins: unambiguous
    ev = np.linalg.eigvalsh(K.dense())
    expect = O.expected_inertia(inp.n, inp.m, form)
    assert (int((ev > 0).sum()), int((ev < 0).sum())) == expect[:2]


def test_inertia_correction_gives_up_at_delta_max():
    inp, W, J = _nonconvex(3)
    delta, attempts, ok, F, K = O.inertia_correction(inp, O.CONDENSED, 1e-6, 2.0, 1e-4)
    assert not ok and delta <= 1e-4 and delta * 2.0 > 1e-4 and attempts == 1 + 7
