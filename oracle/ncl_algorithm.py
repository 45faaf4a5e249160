"""Algorithm 1 (MadNCL, Sec. 2.3) on a convex quadratic program, FP64 on the
CPU -- test infrastructure only: the reference for the library's driver
(ncl_qp_solve).  It never imports or calls the GPU library.

Problem (the NCO form of Sec. 3 with equality rows only):
    min 1/2 x^T Q x + q^T x   s.t.  A x = b,  l <= x <= u
(entries of l, u may be infinite).  The NCL subproblem NC_k adds the free
variables r (c(x) + r = 0) and the term y_k^T r + rho/2 ||r||^2 (Sec. 2.2).
Every Newton step solves the condensed system K1 = Q + Sigma + rho A^T A
(Sec. 3.3, eq. K1) and recovers Delta y, Delta r (eqs. K1-elimination,
K2-elimination) and Delta z_l, Delta z_u (Sec. 3.1, eq. K3).

Readings where the paper is silent (the library's driver takes the same):
  * y_0 = 0 (the paper computes y_0 by least squares); r_0 = -c(x_0), so the
    third block of F starts at zero; z_0 = mu_0 / distance to each finite
    bound; eta_0 = min(mu_0^1.1, 0.1 mu_0), omega_0 = 100 mu_0^(1+gamma) (the
    update formulas of Algorithm 1 applied at k = 0).
  * Step length: one alpha for primal and dual variables, the largest alpha
    <= 1 keeping x strictly inside its bounds and z positive with the
    fraction-to-boundary factor tau = max(0.99, 1 - mu); then halved (at most
    30 times) until ||F_k||_inf does not increase.
  * Inner iterations ("using MadNLP" in Algorithm 1) are these Newton steps
    from w_k until ||F_k||_inf <= omega_k (at most max_inner).
  * The optimality test uses the full stationarity Q x + q - A^T y - z_l + z_u
    (the paper's test omits the bound multipliers) and also asks the
    complementarity max(z_l (x - l), z_u (u - x)) <= omega_star: without it
    the test can pass at a point that is only mu-optimal.
  * mu is kept at or above mu_min = min(eta_star, omega_star) / 10 (the
    usual floor of interior-point codes): Algorithm 1's update
    min(mu^tau, mu_fac mu) is superlinear, and near 1e-16 the distance of an
    iterate to an active bound rounds to zero.
  * Complementarity rows of F for infinite bounds are 0 (z is 0 there).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

GAMMA, TAU, MU_FAC, RHO_MAX, THETA = 0.05, 1.99, 0.2, 1e14, 0.5   # Algorithm 1's constants
RHO0, MU0 = 100.0, 0.1


@dataclass
class QP:
    Q: sp.csc_matrix        # symmetric (full)
    q: np.ndarray
    A: sp.csr_matrix
    b: np.ndarray
    l: np.ndarray
    u: np.ndarray


@dataclass
class Result:
    x: np.ndarray
    y: np.ndarray
    z_l: np.ndarray
    z_u: np.ndarray
    r: np.ndarray
    status: int             # 0 optimal, 1 infeasible, 2 iteration limit
    outer: int
    inner: int              # Newton steps in inner loops
    extrapolated: int       # outer iterations that accepted the extrapolation step
    primal_inf: float
    dual_inf: float


def _inv_dist(x, l, u):
    fl, fu = np.isfinite(l), np.isfinite(u)
    il = np.zeros_like(x)
    iu = np.zeros_like(x)
    il[fl] = 1.0 / (x[fl] - l[fl])
    iu[fu] = 1.0 / (u[fu] - x[fu])
    return il, iu, fl, fu


def F(qp: QP, w, yk, rho, mu):
    """The five blocks of F_k(w) (Sec. 2.3, eq. kktnclipm)."""
    x, r, y, zl, zu = w
    fl, fu = np.isfinite(qp.l), np.isfinite(qp.u)
    g = qp.Q @ x + qp.q
    c = qp.A @ x - qp.b
    cl = np.where(fl, zl * np.where(fl, x - qp.l, 0.0) - mu, 0.0)
    cu = np.where(fu, zu * np.where(fu, qp.u - x, 0.0) - mu, 0.0)
    return [g - qp.A.T @ y - zl + zu, yk + rho * r - y, c + r, cl, cu]


def fnorm(blocks):
    return max(float(np.abs(b).max()) if b.size else 0.0 for b in blocks)


def newton_direction(qp: QP, w, yk, rho, mu):
    """d = (Delta x, Delta r, Delta y, Delta z_l, Delta z_u) from the condensed
    system: Sigma, K1 = Q + Sigma + rho A^T A and its right-hand side
    A^T (y_k - rho c) - (grad phi - mu/(x - l) + mu/(u - x)) (Sec. 3.3, eq. K1),
    then the recoveries."""
    x, r, y, zl, zu = w
    il, iu, fl, fu = _inv_dist(x, qp.l, qp.u)
    Sigma = zl * il + zu * iu
    g = qp.Q @ x + qp.q
    c = qp.A @ x - qp.b
    K = (qp.Q + sp.diags(Sigma) + rho * (qp.A.T @ qp.A)).tocsc()
    rhs = qp.A.T @ (yk - rho * c) - (g - mu * il + mu * iu)
    dx = spla.spsolve(K, rhs)
    dy = -rho * (qp.A @ dx + c) + yk - y
    dr = (1.0 / rho) * (dy - yk + y) - r
    dzl = np.where(fl, -(zl * dx - mu) * il - zl, 0.0)
    dzu = np.where(fu, (zu * dx + mu) * iu - zu, 0.0)
    return [dx, dr, dy, dzl, dzu]


def max_step(qp: QP, w, d, mu):
    """Largest alpha <= 1 with x strictly inside and z positive, scaled by the
    fraction-to-boundary factor tau = max(0.99, 1 - mu)."""
    x, _, _, zl, zu = w
    dx, _, _, dzl, dzu = d
    tau = max(0.99, 1.0 - mu)
    a = 1.0
    fl, fu = np.isfinite(qp.l), np.isfinite(qp.u)
    for mask, num, den in ((fl & (dx < 0), x - qp.l, -dx), (fu & (dx > 0), qp.u - x, dx),
                           (fl & (dzl < 0), zl, -dzl), (fu & (dzu < 0), zu, -dzu)):
        if mask.any():
            a = min(a, float(tau * (num[mask] / den[mask]).min()))
    return a


def _step(w, d, a):
    return [wi + a * di for wi, di in zip(w, d)]


def newton_step(qp: QP, w, yk, rho, mu):
    """One inner Newton step with the fraction-to-boundary rule and halving on
    ||F_k||_inf."""
    f0 = fnorm(F(qp, w, yk, rho, mu))
    d = newton_direction(qp, w, yk, rho, mu)
    a = max_step(qp, w, d, mu)
    for _ in range(30):
        wn = _step(w, d, a)
        if fnorm(F(qp, wn, yk, rho, mu)) <= f0:
            return wn
        a *= 0.5
    return _step(w, d, a)


def solve(qp: QP, x0, eta_star=1e-8, omega_star=1e-8, max_outer=100, max_inner=100, log=None) -> Result:
    """Algorithm 1 (MadNCL), with the readings listed in the module header.
    With a list as `log`, appends per outer iteration (k, rho, mu after the
    update, ||F|| before and after the extrapolation step, its alpha, accepted,
    inner steps, ||r||, dual, complementarity)."""
    n, m = qp.Q.shape[0], qp.A.shape[0]
    x = np.asarray(x0, np.float64).copy()
    fl, fu = np.isfinite(qp.l), np.isfinite(qp.u)
    rho, mu = RHO0, MU0
    mu_min = min(eta_star, omega_star) / 10.0
    r = -(qp.A @ x - qp.b)
    y = np.zeros(m)
    yk = y.copy()
    zl = np.where(fl, mu / np.where(fl, x - qp.l, 1.0), 0.0)
    zu = np.where(fu, mu / np.where(fu, qp.u - x, 1.0), 0.0)
    eta, omega = min(mu ** 1.1, 0.1 * mu), 100.0 * mu ** (1.0 + GAMMA)
    w = [x, r, y, zl, zu]
    inner = extrap = 0
    status = 2
    k = 0
    for k in range(1, max_outer + 1):
        # extrapolation step (eq. ncl:extrapolation)
        f0 = fnorm(F(qp, w, yk, rho, mu))
        d = newton_direction(qp, w, yk, rho, mu)
        a = max_step(qp, w, d, mu)
        wp = _step(w, d, a)
        fp = fnorm(F(qp, wp, yk, rho, mu))
        accept = fp <= THETA * f0 + 10.0 * a ** 0.2 * mu
        steps = 0
        if accept:
            w = wp
            extrap += 1
        else:
            while fnorm(F(qp, w, yk, rho, mu)) > omega and steps < max_inner:
                w = newton_step(qp, w, yk, rho, mu)
                steps += 1
            inner += steps
        x, r, y, zl, zu = w
        rn = float(np.abs(r).max()) if m else 0.0
        if rn <= eta:
            yk = yk + rho * r
            mu_new = max(min(mu ** TAU, MU_FAC * mu), mu_min)
            eta = min(mu_new ** 1.1, 0.1 * mu)
            omega = 100.0 * mu_new ** (1.0 + GAMMA)
            mu = mu_new
        else:
            rho = min(RHO_MAX, 10.0 * rho)
        dual = float(np.abs(qp.Q @ x + qp.q - qp.A.T @ y - zl + zu).max())
        comp = max(float(np.max(zl[fl] * (x[fl] - qp.l[fl]), initial=0.0)),
                   float(np.max(zu[fu] * (qp.u[fu] - x[fu]), initial=0.0)))
        if log is not None:
            log.append((k, rho, mu, f0, a, fp, accept, steps, rn, dual, comp))
        if rn <= eta_star and dual <= omega_star and comp <= omega_star:
            status = 0
            break
        if rho >= RHO_MAX and rn > eta_star:
            status = 1
            break
    x, r, y, zl, zu = w
    return Result(x, y, zl, zu, r, status, k, inner, extrap, float(np.abs(qp.A @ x - qp.b).max(initial=0.0)),
                  float(np.abs(qp.Q @ x + qp.q - qp.A.T @ y - zl + zu).max()))
