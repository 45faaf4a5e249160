"""GPU edge cases through the C ABI, each against the oracle: static pivots of
the dual sign under the three threshold rules (Sec. 3.1, Sec. 3.2 eq. K2r,
Sec. 4.3), an exact zero pivot of the condensed form, the stabilized form on a
primal block whose Sigma spans 16 decades, a front too large for the
LDS-staged assembly, an FP32 factor that overflows, the solve's three
backward-error measures, the componentwise refinement criterion, and the
binding's argument checks.  Each case prints its name before the GPU work."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_05885_amd import ncl_kkt as nk
from paper_2510_05885_amd import synth

from gpu_util import colmajor, dev, factor_solve, form_id, omega_cpu

pytestmark = pytest.mark.gpu


def _yfirst(inp):
    n, m = inp.n, inp.m
    return np.concatenate([np.arange(n, n + m), np.arange(n)]).astype(np.int32)


@pytest.mark.parametrize("scale", ["global", "block", "absolute"])
def test_dual_static_pivot_yfirst(scale):
    """Dual block ordered first at rho = 1e14: each dual pivot is a leaf of the
    elimination tree, so it is -1/rho = -1e-14 exactly (eq. ldlk2r) in any
    topological reordering.  The global rule (eps ||K||_max >= 1e-10) and the
    absolute one (eps = 1e-10) replace all m of them by a negative pivot; the
    block rule (eps / rho = 1e-24) keeps them.  Inertia (n, m, 0) and the
    perturbed count equal the oracle's under the same order."""
    print(f"[gpu] y-first rho=1e14 pivot_scale={scale}", flush=True)
    inp = synth.grid_banded(rho=1e14)
    n, m = inp.n, inp.m
    B = synth.rhs(n + m, 1, seed=2)
    perm = _yfirst(inp)
    kkt = nk.KKT.from_input(inp, form="stabilized", user_perm=perm, pivot_scale=scale)
    rc, X, info = factor_solve(kkt, inp, B)
    Xo, io, _, K = O.solve(inp, O.STABILIZED, B, perm=perm, pivot_scale=scale)
    npert = m if scale != "block" else 0
    assert kkt.inertia() == io.inertia == (n, m, 0, npert)
    om = float(O.backward_error(K, X, B).max())
    assert om <= max(1e-12, 10 * io.backward_error), (om, io.backward_error, info)
    kkt.close()


def test_condensed_exact_zero_pivot():
    """Condensed form with row i of K empty (no W entry, no J entry, Sigma_i =
    0): its pivot is exactly 0 in any ordering and becomes +eps ||K||_max
    (Sec. 3.1), one perturbed pivot, inertia (n, 0, 0), in both
    implementations.  With b_i = 0 the system is consistent; x_i = 0 and the
    rest of x matches the oracle."""
    print("[gpu] condensed zero pivot", flush=True)
    i0 = 5
    inp = synth.random_system(60, 20, seed=9, rho=1e3, empty_w_rows=[i0], empty_j_cols=[i0], zero_sigma=[i0])
    B = synth.rhs(inp.n, 2, seed=4)
    B[i0] = 0.0
    kkt = nk.KKT.from_input(inp)
    rc, X, info = factor_solve(kkt, inp, B)
    Xo, io, _, K = O.solve(inp, O.CONDENSED, B)
    assert np.count_nonzero(K.dense()[i0]) == 0
    assert kkt.inertia() == io.inertia == (inp.n, 0, 0, 1)
    assert rc == 0 and info.backward_error <= 1e-12
    assert omega_cpu(inp, "condensed", X, B) <= 1e-12
    assert np.all(X[i0] == 0.0)
    assert np.abs(X - Xo).max() <= 1e-9 * np.abs(Xo).max()


@pytest.mark.parametrize("scale", ["global", "block", "absolute"])
def test_stabilized_wide_sigma(scale):
    """Stabilized OPF-shaped system (2000 nodes, rho = 1e3) with Sigma over
    [1e-8, 1e8].  The relative rules replace legitimate primal pivots (edge
    variables with no W entry and Sigma ~1e-8, below eps max|K_xx| ~ 1e-2),
    and refinement cannot recover them: the library, like the oracle (which
    stops at omega ~1e-11 with componentwise errors ~1), may stop short of
    1e-12 (status NCL_WARN_IR_NOT_CONVERGED allowed); the inertia is the
    oracle's.  With the absolute bound nothing is perturbed (every
    primal pivot >= min Sigma, every dual one <= -1/rho, in any order) and
    refinement with the componentwise criterion reaches omega <= 1e-12 and
    omega_cw <= 1e-14; x then matches the oracle refined the same way."""
    print(f"[gpu] stabilized wide Sigma pivot_scale={scale}", flush=True)
    inp = synth.opf_network(N=2000, seed=3, rho=1e3)
    B = synth.rhs(inp.n + inp.m, 1, seed=11)
    kkt = nk.KKT.from_input(inp, form="stabilized", pivot_scale=scale, ir_cw_tol=1e-14)
    rc, X, info = factor_solve(kkt, inp, B)
    Xo, io, _, K = O.solve(inp, O.STABILIZED, B, pivot_scale=scale, ir_cw_tol=1e-14)
    inert = kkt.inertia()
    assert inert[:3] == io.inertia[:3] == (inp.n, inp.m, 0)
    om = float(O.backward_error(K, X, B).max())
    cw = float(O.componentwise_backward_error(K, X, B).max())
    print(f"[gpu]   rc={rc} npert={inert[3]} (oracle {io.inertia[3]}) omega={om:.2e} cw={cw:.2e} "
          f"oracle omega={io.backward_error:.2e} cw={io.backward_error_cw:.2e}", flush=True)
    if scale == "absolute":
        assert rc == 0 and inert[3] == io.inertia[3] == 0
        assert om <= 1e-12 and cw <= 1e-14 and info.backward_error_cw <= 1e-14
        assert np.abs(X - Xo).max() <= 1e-10 * np.abs(Xo).max()
    else:
        assert rc in (0, nk.NCL_WARN_IR_NOT_CONVERGED)
        assert om <= 1e-9
    kkt.close()


def test_front_beyond_lds_assembly():
    """One dense front of order 3200 (a full J row couples every variable):
    in FP64 its columns (4 x 3200 x 8 bytes per workgroup) do not fit the LDS
    slice and are assembled in place in global memory."""
    print("[gpu] dense front f=3200 (in-place column assembly)", flush=True)
    inp = synth.random_system(3200, 2, seed=21, rho=1.0, w_density=0.0005, j_per_row=3200)
    B = synth.rhs(inp.n, 1, seed=3)
    kkt = nk.KKT.from_input(inp)
    assert kkt.stats()["max_front"] > 3072
    rc, X, info = factor_solve(kkt, inp, B)
    Xo, io, _, K = O.solve(inp, O.CONDENSED, B, perm=np.arange(inp.n, dtype=np.int32))
    assert rc == 0 and kkt.inertia()[:3] == io.inertia[:3] == (inp.n, 0, 0)
    assert float(O.backward_error(K, X, B).max()) <= 1e-12
    assert np.abs(X - Xo).max() <= 1e-8 * np.abs(Xo).max()
    kkt.close()


@pytest.mark.parametrize("n", [950, 1000, 1024])
def test_dense_front_panel_layouts(n):
    """One dense front with p = n pivots: 15 panels with the last one 54 wide
    (n = 950: the forward sweep takes pairs and then the last panel alone), 16
    panels with the last one 40 wide (n = 1000: the last pair's second panel
    is narrow) and 16 full panels (n = 1024).  Every backward panel below the
    last two has several row tasks, so each is finished by the next launch's
    first task, and the first panel by a finish-only record.  The solution
    matches the oracle's."""
    print(f"[gpu] dense front n={n} (sweep panel layouts)", flush=True)
    inp = synth.random_system(n, 2, seed=21, rho=1.0, w_density=0.0005, j_per_row=n)
    B = synth.rhs(inp.n, 1, seed=3)
    kkt = nk.KKT.from_input(inp, ir_cw_tol=1e-14)
    assert kkt.stats()["max_front"] == n
    rc, X, info = factor_solve(kkt, inp, B)
    Xo, io, _, K = O.solve(inp, O.CONDENSED, B, perm=np.arange(inp.n, dtype=np.int32))
    assert rc == 0 and kkt.inertia()[:3] == io.inertia[:3] == (inp.n, 0, 0)
    assert float(O.backward_error(K, X, B).max()) <= 1e-12
    assert info.backward_error_cw <= 1e-14
    assert np.abs(X - Xo).max() <= 1e-8 * np.abs(Xo).max()
    kkt.close()


def test_fp32_overflow_falls_back_to_fp64():
    """K finite in FP64 but not in FP32 (Sigma_3 = 1e39 > FLT_MAX): the FP32
    factor meets an infinite pivot, the library refactors in FP64 instead of
    failing (status NCL_WARN_FELL_BACK_FP64), and the solve matches the
    oracle.  pivot_eps 1e-45 keeps eps ||K||_max = 1e-6 below every pivot."""
    print("[gpu] fp32 overflow -> fp64", flush=True)
    inp = synth.grid_banded(nr=10, nc=12, m=50, band=20, rho=1e4, seed=5)
    inp.Sigma[3] = 1e39
    B = synth.rhs(inp.n, 1, seed=1)
    kkt = nk.KKT.from_input(inp, precision="fp32_ir", pivot_eps=1e-45)
    rc = kkt.factor(dev(inp.W_val), dev(inp.Sigma), dev(inp.J_val), inp.rho)
    assert rc == nk.NCL_WARN_FELL_BACK_FP64
    assert kkt.inertia() == (inp.n, 0, 0, 0)
    X, info = kkt.solve(colmajor(B))
    X = X.cpu().numpy()
    Xo, io, _, K = O.solve(inp, O.CONDENSED, B, eps=1e-45)
    assert info.fell_back_fp64 and info.backward_error <= 1e-12
    assert float(O.backward_error(K, X, B).max()) <= 1e-12
    assert np.abs(X - Xo).max() <= 1e-8 * np.abs(Xo).max()
    # NaN in the input is still an error, in either precision
    bad = inp.Sigma.copy(); bad[0] = np.nan
    with pytest.raises(nk.NCLError) as e:
        kkt.factor(dev(inp.W_val), dev(bad), dev(inp.J_val), inp.rho)
    assert e.value.code == -6
    kkt.close()


def test_solve_info_measures_match_cpu():
    """The solve's omega, componentwise error and ||b - Kx||_2 / ||b||_2, on
    an unrefined solve whose residual is far above rounding (stabilized
    wide-Sigma system under the global relative pivot rule, which replaces
    legitimate pivots), equal the values computed on the CPU from the
    returned x against the oracle's K."""
    print("[gpu] solve info measures", flush=True)
    inp = synth.opf_network(N=500, seed=3, rho=1e3)
    B = synth.rhs(inp.n + inp.m, 3, seed=8)
    kkt = nk.KKT.from_input(inp, form="stabilized", pivot_scale="global", ir_max_steps=0)
    rc, X, info = factor_solve(kkt, inp, B)
    K = O.assemble(inp, O.STABILIZED)
    om = float(O.backward_error(K, X, B).max())
    cw = float(O.componentwise_backward_error(K, X, B).max())
    r2 = float(O.residual_rel2(K, X, B).max())
    print(f"[gpu]   omega {om:.3e} / {info.backward_error:.3e}  cw {cw:.3e} / {info.backward_error_cw:.3e}  "
          f"rel2 {r2:.3e} / {info.resid_rel2:.3e}", flush=True)
    assert kkt.inertia()[3] > 0 and cw > 1e-6 and r2 > 1e-12
    assert info.backward_error == pytest.approx(om, rel=1e-6)
    assert info.backward_error_cw == pytest.approx(cw, rel=1e-6)
    assert info.resid_rel2 == pytest.approx(r2, rel=1e-6)
    kkt.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_componentwise_refinement_target(precision):
    """With ir_cw_tol = 1e-14 the solve refines until the componentwise
    backward error (measured on the CPU) is at most 1e-14, at every rho of
    the config-3 sweep; the FP32 factor needs at least one correction."""
    for rho in (1e2, 1e4, 1e6):
        print(f"[gpu] componentwise target {precision} rho={rho:g}", flush=True)
        inp = synth.grid_banded(rho=rho, seed=3)
        B = synth.rhs(inp.n, 2, seed=5)
        kkt = nk.KKT.from_input(inp, precision=precision, ir_tol=1e-10, ir_cw_tol=1e-14, fp32_sticky=False)
        rc, X, info = factor_solve(kkt, inp, B)
        K = O.assemble(inp, O.CONDENSED)
        cw = float(O.componentwise_backward_error(K, X, B).max())
        assert rc in (0, nk.NCL_WARN_FELL_BACK_FP64), (rc, info)
        assert info.backward_error_cw <= 1e-14 and cw <= 2e-14, (cw, info)
        if precision == "fp32_ir" and not info.fell_back_fp64:
            assert info.ir_steps >= 1
        kkt.close()


def test_binding_argument_checks():
    """The binding checks sizes, dtypes and devices before calling the library."""
    print("[gpu] binding checks", flush=True)
    import torch
    inp = synth.random_system(20, 5, seed=3)
    kkt = nk.KKT.from_input(inp)
    W, S, J = dev(inp.W_val), dev(inp.Sigma), dev(inp.J_val)
    with pytest.raises(ValueError):
        kkt.factor(W[:-1], S, J, inp.rho)
    with pytest.raises(TypeError):
        kkt.factor(W, S.float(), J, inp.rho)
    with pytest.raises(TypeError):
        kkt.factor(W, S.cpu(), J, inp.rho)
    kkt.factor(W, S, J, inp.rho)
    with pytest.raises(TypeError):
        kkt.solve(torch.ones(20, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        kkt.solve(dev(np.ones((20, 2))), X=dev(np.ones((20, 3))).t().contiguous().t())
    inps = [synth.batched_system(k, N) for k, N in enumerate([30, 40])]
    kb = nk.KKT.analyze_batched(inps)
    with pytest.raises(ValueError):   # one rho per system
        kb.factor(dev(np.concatenate([i.W_val for i in inps])), dev(np.concatenate([i.Sigma for i in inps])),
                  dev(np.concatenate([i.J_val for i in inps])), 1e3)
    kkt.close()
    kb.close()


def test_adjoint_refuses_a_refactored_handle():
    """kkt_solve's backward uses the handle's current factor and rho: after a
    second forward pass on the same handle, backward of the first raises
    instead of returning gradients of the wrong matrix.  Backward of the
    second still works."""
    print("[gpu] adjoint generation guard", flush=True)
    import torch
    inp = synth.grid_banded(nr=8, nc=10, m=30, band=20, rho=1e3, seed=5)
    kkt = nk.KKT.from_input(inp)
    B = dev(synth.rhs(inp.n, 1, seed=1)[:, 0])
    W1 = dev(inp.W_val).requires_grad_()
    X1 = nk.kkt_solve(kkt, W1, dev(inp.Sigma), dev(inp.J_val), inp.rho, B)
    W2 = dev(inp.W_val).requires_grad_()
    X2 = nk.kkt_solve(kkt, W2, dev(inp.Sigma), dev(inp.J_val), 2 * inp.rho, B)
    with pytest.raises(RuntimeError, match="refactored"):
        X1.sum().backward()
    X2.sum().backward()
    assert torch.isfinite(W2.grad).all()
    kkt.close()
