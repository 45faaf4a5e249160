"""GPU parity of the slack elimination (eq. K1s) and of the Newton-step
recovery kernels against the oracle (Sec. 3.1-3.3).

* K1s factor + solve on an OPF-shaped system of 2000 nodes (n = 10k, rows of
  J inequalities with probability 1/3, Sigma_s log-uniform in [1e-4, 1e4]):
  inertia, backward error against the oracle's K1s, and the solution against
  the oracle's; the K1s right-hand side and the Delta s recovery elementwise.
* Edge cases: every row an equality (+inf) gives bitwise the K1 factor; every
  row Sigma_s = 0 drops J out of K1s; a negative Sigma_s is refused as a
  non-finite input; the adjoint refuses a K1s factor; a batch of three systems
  with their own rho.
* Delta y, Delta r, Delta z_l, Delta z_u and Sigma elementwise against the
  oracle (bounds partly infinite).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_05885_amd import ncl_kkt as nk
from paper_2510_05885_amd import synth

from gpu_util import dev

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def _setup(N=2000, seed=3, rho=1e4):
    inp = synth.opf_network(N=N, seed=seed, rho=rho, sigma_lo=-4, sigma_hi=4)
    Ss = synth.slack_sigma(inp.m, seed=seed + 10)
    return inp, Ss


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_k1s_factor_solve_matches_oracle(precision):
    print(f"[gpu] K1s factor + solve, {precision}", flush=True)
    inp, Ss = _setup()
    rng = np.random.default_rng(4)
    r_t, r_s = rng.standard_normal(inp.n), rng.standard_normal(inp.m)
    kkt = nk.KKT.from_input(inp, precision=precision, ir_cw_tol=1e-14)
    J, Ssd = dev(inp.J_val), dev(Ss)
    rc = kkt.factor_k1s(dev(inp.W_val), dev(inp.Sigma), J, Ssd, inp.rho)
    assert rc in (0, nk.NCL_WARN_FELL_BACK_FP64)
    assert kkt.inertia()[:3] == (inp.n, 0, 0)
    b = kkt.k1s_rhs(J, dev(r_t), dev(r_s), Ssd).cpu().numpy()
    b_or = O.k1s_rhs(inp, Ss, r_t, r_s)
    print(f"[gpu]   rhs rel err {_rel(b, b_or):.1e}", flush=True)
    assert _rel(b, b_or) <= 1e-13
    K = O.assemble_k1s(inp, Ss)
    X, info = kkt.solve(dev(b_or))
    x = X.cpu().numpy()
    xo, io, _, _ = O.solve(inp, O.CONDENSED, b_or, K=K, ir_cw_tol=1e-14)
    cw = float(O.componentwise_backward_error(K, x, b_or).max())
    print(f"[gpu]   cw {cw:.2e} (lib {info.backward_error_cw:.2e}) fwd {_rel(x, xo):.2e} "
          f"oracle inertia {io.inertia}", flush=True)
    assert io.inertia[:3] == (inp.n, 0, 0)
    assert cw <= 2e-14 and info.backward_error_cw <= 1e-14
    assert _rel(x, xo) <= 1e-8
    ds = kkt.k1s_recover(J, X, dev(r_s), Ssd).cpu().numpy()
    ds_or = O.k1s_recover_ds(inp, Ss, x, r_s)
    assert _rel(ds, ds_or) <= 1e-13
    assert np.all(ds[np.isinf(Ss)] == 0.0)
    kkt.close()


def test_k1s_edge_cases():
    print("[gpu] K1s edge cases", flush=True)
    inp = synth.random_system(300, 120, seed=5, rho=50.0)
    W, S, J = dev(inp.W_val), dev(inp.Sigma), dev(inp.J_val)
    b = dev(synth.rhs(inp.n, 1, seed=1)[:, 0])
    # all equality rows: exactly K1
    k1 = nk.KKT.from_input(inp)
    k1.factor(W, S, J, inp.rho)
    x1, _ = k1.solve(b)
    ks = nk.KKT.from_input(inp)
    ks.factor_k1s(W, S, J, dev(np.full(inp.m, np.inf)), inp.rho)
    xs, _ = ks.solve(b)
    assert np.array_equal(x1.cpu().numpy(), xs.cpu().numpy())
    assert ks.inertia() == k1.inertia()
    # Sigma_s = 0 on every row: J drops out, K1s = W + Sigma
    zero = np.zeros(inp.m)
    ks.factor_k1s(W, S, J, dev(zero), inp.rho)
    xz, _ = ks.solve(b)
    K = O.assemble_k1s(inp, zero)
    xo, _, _, _ = O.solve(inp, O.CONDENSED, b.cpu().numpy(), K=K)
    assert _rel(xz.cpu().numpy(), xo) <= 1e-10
    # a negative Sigma_s is a non-finite input
    bad = np.full(inp.m, np.inf)
    bad[7] = -1.0
    with pytest.raises(nk.NCLError) as e:
        ks.factor_k1s(W, S, J, dev(bad), inp.rho)
    assert e.value.code == nk.NCL_ERR_NONFINITE
    # the adjoint is of K1: refused after a K1s factor
    import torch
    ks.factor_k1s(W, S, J, dev(np.full(inp.m, 1.0)), inp.rho)
    X, _ = ks.solve(b)
    with pytest.raises(nk.NCLError) as e:
        ks.backward(J, X, X, gSigma=torch.empty_like(X))
    assert e.value.code == nk.NCL_ERR_STATE
    k1.close()
    ks.close()


def test_k1s_batched_per_system_rho():
    print("[gpu] K1s batched", flush=True)
    inps = [synth.batched_system(k, N) for k, N in enumerate([150, 400, 90])]
    Ss = [synth.slack_sigma(i.m, seed=20 + k) for k, i in enumerate(inps)]
    kkt = nk.KKT.analyze_batched(inps, ir_cw_tol=1e-14)
    cat = lambda f: dev(np.concatenate([getattr(i, f) for i in inps]))
    J = cat("J_val")
    Ssd = dev(np.concatenate(Ss))
    rho = np.array([i.rho for i in inps])
    kkt.factor_k1s(cat("W_val"), cat("Sigma"), J, Ssd, rho)
    rng = np.random.default_rng(8)
    r_t = [rng.standard_normal(i.n) for i in inps]
    r_s = [rng.standard_normal(i.m) for i in inps]
    b = kkt.k1s_rhs(J, dev(np.concatenate(r_t)), dev(np.concatenate(r_s)), Ssd)
    X, _ = kkt.solve(b)
    x = X.cpu().numpy()
    inert = kkt.inertia_batched()
    off = 0
    for k, i in enumerate(inps):
        bk = O.k1s_rhs(i, Ss[k], r_t[k], r_s[k])
        assert _rel(b.cpu().numpy()[off:off + i.n], bk) <= 1e-13
        K = O.assemble_k1s(i, Ss[k])
        xo, io, _, _ = O.solve(i, O.CONDENSED, bk, K=K, ir_cw_tol=1e-14)
        assert tuple(inert[k][:3]) == io.inertia[:3] == (i.n, 0, 0)
        assert float(O.componentwise_backward_error(K, x[off:off + i.n], bk).max()) <= 2e-14
        assert _rel(x[off:off + i.n], xo) <= 1e-8
        off += i.n
    kkt.close()


def test_step_recovery_matches_oracle():
    print("[gpu] step recovery kernels", flush=True)
    inp, _ = _setup(N=1500, seed=6, rho=3e3)
    n, m = inp.n, inp.m
    rng = np.random.default_rng(11)
    kkt = nk.KKT.from_input(inp)
    J = dev(inp.J_val)
    kkt.factor(dev(inp.W_val), dev(inp.Sigma), J, inp.rho)
    dx, c, y_k, y, r = (rng.standard_normal(k) for k in (n, m, m, m, m))
    dy = kkt.recover_dy(J, dev(dx), dev(c), dev(y_k), dev(y)).cpu().numpy()
    assert _rel(dy, O.recover_dy(inp, dx, c, y_k, y)) <= 1e-13
    dr = kkt.recover_dr(dev(dy), dev(y_k), dev(y), dev(r)).cpu().numpy()
    assert _rel(dr, O.recover_dr(inp.rho, dy, y_k, y, r)) <= 1e-14
    x = rng.uniform(-0.5, 0.5, n)
    l = np.where(rng.uniform(size=n) < 0.3, -np.inf, -1.0 - rng.uniform(size=n))
    u = np.where(rng.uniform(size=n) < 0.3, np.inf, 1.0 + rng.uniform(size=n))
    z_l = np.where(np.isinf(l), 0.0, rng.uniform(0.1, 2.0, n))
    z_u = np.where(np.isinf(u), 0.0, rng.uniform(0.1, 2.0, n))
    sig = kkt.barrier_sigma(*(dev(a) for a in (x, l, u, z_l, z_u))).cpu().numpy()
    assert _rel(sig, O.barrier_sigma(x, l, u, z_l, z_u)) <= 1e-15
    dzl, dzu = kkt.recover_dz(*(dev(a) for a in (x, l, u, z_l, z_u, dx)), 0.03)
    ozl, ozu = O.recover_dz(x, l, u, z_l, z_u, dx, 0.03)
    assert _rel(dzl.cpu().numpy(), ozl) <= 1e-15 and _rel(dzu.cpu().numpy(), ozu) <= 1e-15
    kkt.close()


def _indefinite(shift, form_rho=5.0):
    """Config-1 grid system with W shifted by -shift I: W indefinite, so
    delta = 0 gives the wrong inertia."""
    inp = synth.grid_banded(rho=form_rho)
    Wl = inp.W_val.copy()
    cols = np.repeat(np.arange(inp.n), np.diff(inp.W_colptr))
    diag = inp.W_rowidx == cols
    Wl[diag] -= shift
    return inp.with_values(W_val=Wl)


@pytest.mark.parametrize("form", ["condensed", "stabilized"])
def test_inertia_correction_matches_oracle(form):
    """Same delta sequence as the oracle's loop: the same delta, number of
    factorizations and inertia, and the regularized solve against the
    oracle's."""
    print(f"[gpu] inertia correction, {form}", flush=True)
    inp = _indefinite(4.5)
    f = O.CONDENSED if form == "condensed" else O.STABILIZED
    d0, g, dmax = 1e-3, 8.0, 1e6
    dl_o, att_o, ok_o, F, K = O.inertia_correction(inp, f, d0, g, dmax)
    kkt = nk.KKT.from_input(inp, form=form, ir_cw_tol=1e-14)
    rc, dl, att = kkt.factor_regularized(dev(inp.W_val), dev(inp.Sigma), dev(inp.J_val), inp.rho, d0, g, dmax)
    print(f"[gpu]   delta {dl} ({att} factorizations) oracle {dl_o} ({att_o}); inertia {kkt.inertia()}", flush=True)
    assert ok_o and att_o > 1
    assert rc == 0 and dl == dl_o and att == att_o
    assert kkt.inertia()[:3] == F.inertia()[:3] == O.expected_inertia(inp.n, inp.m, f)
    b = synth.rhs(K.N, 1, seed=3)[:, 0]
    X, info = kkt.solve(dev(b))
    case = inp.with_values(Sigma=inp.Sigma + dl, rho=inp.rho + dl)
    xo, io, _, _ = O.solve(case, f, b, K=K, ir_cw_tol=1e-14)
    x = X.cpu().numpy()
    assert float(O.componentwise_backward_error(K, x, b).max()) <= 2e-14
    assert _rel(x, xo) <= 1e-8
    # delta_max too small: gives up with the wrong inertia after the same count
    rc2, dl2, att2 = kkt.factor_regularized(dev(inp.W_val), dev(inp.Sigma), dev(inp.J_val), inp.rho, d0, g, d0)
    assert rc2 == nk.NCL_WARN_INERTIA and dl2 == d0 and att2 == 2
    kkt.close()
