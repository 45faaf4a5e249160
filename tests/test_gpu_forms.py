"""GPU checks of the three forms beside the plain FP64 path, against the oracle:
FP32 factor + FP64 refinement (with the FP64 refactor fallback), batched
independent systems in one handle, and the adjoint (autograd) of x = K^-1 b."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_05885_amd import ncl_kkt as nk
from paper_2510_05885_amd import synth

from gpu_util import colmajor, dev, factor_solve, kappa_inf, omega_cpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rho", [1e2, 1e4, 1e6, 1e8])
@pytest.mark.parametrize("nrhs", [1, 16])
def test_fp32_ir_matches_oracle(rho, nrhs):
    """FP32 fronts on MFMA, pivot test / residual / refinement in FP64 (config-3
    shape).  Either refinement reaches 1e-12 or the FP64 refactor does."""
    print(f"[gpu] fp32_ir rho={rho:g} nrhs={nrhs}", flush=True)
    inp = synth.grid_banded(rho=rho, seed=3)
    B = synth.rhs(inp.n, nrhs, seed=5)
    kkt = nk.KKT.from_input(inp, precision="fp32_ir")
    rc, X, info = factor_solve(kkt, inp, B)
    Xo, io, _, _ = O.solve(inp, O.CONDENSED, B)
    om = omega_cpu(inp, "condensed", X, B)
    assert om <= 1e-12, (om, info)
    assert kkt.inertia()[:3] == (inp.n, 0, 0)
    tol = 2 * kappa_inf(inp, "condensed") * (om + io.backward_error) + 1e-15
    assert np.abs(X - Xo).max() <= tol * np.abs(Xo).max()
    if rho <= 1e4:
        assert not info.fell_back_fp64 and info.ir_steps >= 1
    if rho >= 1e8:
        assert info.fell_back_fp64


@pytest.mark.parametrize("sticky", [True, False])
def test_fp32_sticky_policy(sticky):
    """One handle through an increasing-rho sequence (as in an NCL outer loop):
    after an FP32 factor had to be replaced at rho = r, later factors with
    rho >= r go to FP64 directly (one frontal pass instead of two) and a factor
    at a smaller rho tries FP32 again.  Every solve meets the tolerance."""
    print(f"[gpu] fp32 sticky={sticky}", flush=True)
    base = synth.grid_banded(rho=1e2, seed=3)
    kkt = nk.KKT.from_input(base, precision="fp32_ir", fp32_sticky=sticky)
    B = synth.rhs(base.n, 1, seed=5)
    passes = []
    for rho in (1e2, 1e8, 1e9, 1e3):
        inp = base.with_values(rho=rho)
        kkt.set_timing(True)
        rc, X, info = factor_solve(kkt, inp, B)
        tm = kkt.timing()
        kkt.set_timing(False)
        assert omega_cpu(inp, "condensed", X, B) <= 1e-12, (rho, info)
        passes.append((info.fell_back_fp64, tm["launches"]["small_fronts"]))
    one = passes[0][1]                        # launches of one frontal pass (FP32 kept at 1e2)
    assert not passes[0][0]
    assert passes[1][0] and passes[1][1] == 2 * one      # FP32 tried, replaced by FP64
    assert passes[2][0]
    assert passes[2][1] == (one if sticky else 2 * one)  # sticky: FP64 directly
    assert not passes[3][0] and passes[3][1] == one       # smaller rho: FP32 again


def test_fp32_ir_stabilized():
    print("[gpu] fp32_ir stabilized", flush=True)
    inp = synth.grid_banded(rho=1e3, seed=4)
    B = synth.rhs(inp.n + inp.m, 2, seed=6)
    kkt = nk.KKT.from_input(inp, form="stabilized", precision="fp32_ir")
    rc, X, info = factor_solve(kkt, inp, B)
    assert omega_cpu(inp, "stabilized", X, B) <= 1e-12
    assert kkt.inertia()[:3] == (inp.n, inp.m, 0)


def test_batched_matches_per_system_oracle():
    """Independent condensed systems of uneven size in one handle (the
    block-diagonal union), per-system rho; each system against the oracle."""
    print("[gpu] batched 8 systems", flush=True)
    sizes = [40, 75, 120, 33, 260, 90, 150, 61]
    inps = [synth.batched_system(k, N) for k, N in enumerate(sizes)]
    kkt = nk.KKT.analyze_batched(inps)
    W = np.concatenate([i.W_val for i in inps])
    S = np.concatenate([i.Sigma for i in inps])
    J = np.concatenate([i.J_val for i in inps])
    rho = np.array([i.rho for i in inps])
    B = [synth.rhs(i.n, 2, seed=k) for k, i in enumerate(inps)]
    rc = kkt.factor(dev(W), dev(S), dev(J), rho)
    X, info = kkt.solve(colmajor(np.vstack(B)))
    X = X.cpu().numpy()
    assert info.backward_error <= 1e-12
    inert = kkt.inertia_batched()
    off = 0
    for k, i in enumerate(inps):
        Xk = X[off:off + i.n]
        off += i.n
        Xo, io, _, K = O.solve(i, O.CONDENSED, B[k])
        assert tuple(inert[k][:3]) == io.inertia[:3] == (i.n, 0, 0)
        assert float(O.backward_error(K, Xk, B[k]).max()) <= 1e-12
        assert np.abs(Xk - Xo).max() <= 1e-6 * np.abs(Xo).max()


def test_batched_equals_one_at_a_time():
    print("[gpu] batched vs single", flush=True)
    inps = [synth.batched_system(k, N) for k, N in enumerate([50, 140, 80])]
    kb = nk.KKT.analyze_batched(inps)
    rc = kb.factor(dev(np.concatenate([i.W_val for i in inps])), dev(np.concatenate([i.Sigma for i in inps])),
                   dev(np.concatenate([i.J_val for i in inps])), np.array([i.rho for i in inps]))
    B = [synth.rhs(i.n, 1, seed=k) for k, i in enumerate(inps)]
    Xb, _ = kb.solve(colmajor(np.vstack(B)))
    Xb = Xb.cpu().numpy()
    off = 0
    for k, i in enumerate(inps):
        ks = nk.KKT.from_input(i)
        _, Xs, _ = factor_solve(ks, i, B[k])
        assert np.abs(Xb[off:off + i.n] - Xs).max() <= 1e-9 * np.abs(Xs).max()
        off += i.n


@pytest.mark.timeout(900)
def test_batched_workload_256_systems():
    """The batched workload at its stated size: 256 OPF-shaped systems of
    125..5000 nodes (n 625..25k, log-uniform), per-system rho and Sigma, in
    one handle.  Every system: inertia (n, 0, 0) and backward error against
    its own K on the CPU; 16 of them (the largest, the smallest and 14 spread
    between) against the oracle's solution."""
    print("[gpu] 256-system batch", flush=True)
    sizes = synth.batched_sizes(256)
    inps = [synth.batched_system(k, int(N)) for k, N in enumerate(sizes)]
    kkt = nk.KKT.analyze_batched(inps, ir_tol=1e-10, ir_cw_tol=1e-14)
    B = [synth.rhs(i.n, 1, seed=k) for k, i in enumerate(inps)]
    rc = kkt.factor(dev(np.concatenate([i.W_val for i in inps])), dev(np.concatenate([i.Sigma for i in inps])),
                    dev(np.concatenate([i.J_val for i in inps])), np.array([i.rho for i in inps]))
    X, info = kkt.solve(colmajor(np.vstack(B)))
    X = X.cpu().numpy()
    print(f"[gpu]   rc={rc} omega={info.backward_error:.2e} cw={info.backward_error_cw:.2e} "
          f"ir_steps={info.ir_steps}", flush=True)
    assert rc == 0 and info.backward_error_cw <= 1e-14
    inert = kkt.inertia_batched()
    order = np.argsort([i.n for i in inps])
    sample = set(order[np.linspace(0, len(order) - 1, 16).astype(int)].tolist())
    off = 0
    worst_cw = worst_fwd = 0.0
    for k, i in enumerate(inps):
        Xk = X[off:off + i.n]
        off += i.n
        assert tuple(inert[k][:3]) == (i.n, 0, 0), k
        K = O.assemble(i, O.CONDENSED)
        worst_cw = max(worst_cw, float(O.componentwise_backward_error(K, Xk, B[k]).max()))
        if k % 64 == 63:
            print(f"[gpu]   checked {k + 1} systems", flush=True)
        if k in sample:
            Xo, io, _, _ = O.solve(i, O.CONDENSED, B[k], ir_cw_tol=1e-14, K=K)
            assert io.inertia[:3] == (i.n, 0, 0)
            worst_fwd = max(worst_fwd, float(np.abs(Xk - Xo).max() / np.abs(Xo).max()))
    print(f"[gpu]   max cw backward error {worst_cw:.2e}; max forward error vs oracle (16 systems) "
          f"{worst_fwd:.2e}", flush=True)
    assert worst_cw <= 2e-14
    assert worst_fwd <= 1e-6


def test_adjoint_matches_oracle_gradient():
    """Reverse mode of x = K(W, Sigma, J, rho)^-1 b through torch.autograd
    (config-5 shape, reduced): gradients w.r.t. b and every stored W, Sigma,
    J entry and rho agree with the oracle's adjoint formulas."""
    import torch
    print("[gpu] adjoint", flush=True)
    inp = synth.grid_banded(nr=10, nc=12, m=50, band=20, rho=1e3, seed=5)
    n = inp.n
    rng = np.random.default_rng(0)
    B = rng.standard_normal((n, 4))
    Wt = rng.standard_normal((n, 4))
    kkt = nk.KKT.from_input(inp)
    Wv = dev(inp.W_val).requires_grad_()
    Sv = dev(inp.Sigma).requires_grad_()
    Jv = dev(inp.J_val).requires_grad_()
    rv = torch.tensor(inp.rho, dtype=torch.float64, device="cuda", requires_grad=True)
    Bleaf = torch.tensor(np.ascontiguousarray(B.T), dtype=torch.float64, device="cuda", requires_grad=True)
    X = nk.kkt_solve(kkt, Wv, Sv, Jv, rv, Bleaf.t())
    loss = (X * dev(Wt)).sum()
    loss.backward()
    Xo, _, F, K = O.solve(inp, O.CONDENSED, B)
    gB, gW, gS, gJ, gr = O.adjoint_condensed(inp, F, Xo, Wt)
    rel = lambda a, b: np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
    assert rel(Bleaf.grad.cpu().numpy().T, gB) <= 1e-8
    assert rel(Wv.grad.cpu().numpy(), gW) <= 1e-8
    assert rel(Sv.grad.cpu().numpy(), gS) <= 1e-8
    assert rel(Jv.grad.cpu().numpy(), gJ) <= 1e-8
    assert abs(rv.grad.item() - gr) <= 1e-8 * abs(gr)
