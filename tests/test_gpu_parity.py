"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Each case prints its name before touching the GPU.  The solution x and the
inertia are unique (Sec. 3.4); L, D and the set of perturbed pivots depend on
the ordering and are not compared.  Bar: backward error <= 1e-12 measured on
the CPU against the oracle's K, inertia counts equal to the oracle's, and
|x - x_oracle|_inf <= 2 kappa_inf (omega_gpu + omega_oracle) |x_oracle|_inf
(first-order perturbation bound) where kappa is computable, else 1e-6.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_05885_amd import ncl_kkt as nk
from paper_2510_05885_amd import synth

from gpu_util import colmajor, dev, factor_solve, form_id, kappa_inf, omega_cpu

pytestmark = pytest.mark.gpu


def _case(name, make, form, nrhs=1, ordering="nd", check_kappa=True, **opts):
    print(f"[gpu] {name} form={form} nrhs={nrhs} ordering={ordering}", flush=True)
    inp = make()
    N = inp.n if form == "condensed" else inp.n + inp.m
    B = synth.rhs(N, nrhs, seed=11)
    kkt = nk.KKT.from_input(inp, form=form, ordering=ordering, **opts)
    rc, X, info = factor_solve(kkt, inp, B)
    Xo, io, _, _ = O.solve(inp, form_id(form), B)
    om = omega_cpu(inp, form, X, B)
    inert = kkt.inertia()
    assert inert[:3] == io.inertia[:3], (inert, io.inertia)
    assert rc in (0,), rc
    assert om <= 1e-12, om
    assert info.backward_error <= 1e-12
    scale = np.abs(Xo).max()
    if check_kappa and N <= 3000:
        tol = 2 * kappa_inf(inp, form) * (om + io.backward_error) + 1e-15
    else:
        tol = 1e-6
    err = np.abs(X - Xo).max() / scale
    assert err <= tol, (err, tol)
    kkt.close()
    return X, info


SMALL = [
    ("random30", lambda: synth.random_system(30, 12, seed=1, rho=50.0)),
    ("random97", lambda: synth.random_system(97, 41, seed=2, rho=1e3, w_density=0.05)),
    ("grid-banded-2000", lambda: synth.grid_banded()),
    ("opf-N500", lambda: synth.opf_network(N=500, seed=3, rho=1e4, sigma_lo=-4, sigma_hi=4)),
]


@pytest.mark.parametrize("idx", range(len(SMALL)))
@pytest.mark.parametrize("form", ["condensed", "stabilized"])
def test_parity_small(idx, form):
    name, make = SMALL[idx]
    _case(name, make, form)


@pytest.mark.parametrize("form", ["condensed", "stabilized"])
def test_parity_natural_ordering(form):
    _case("grid-natural", lambda: synth.grid_banded(nr=20, nc=25, m=250), form, ordering="natural")


@pytest.mark.parametrize("nrhs", [3, 16, 21])
def test_parity_multi_rhs(nrhs):
    _case("grid-banded-multi", lambda: synth.grid_banded(), "condensed", nrhs=nrhs)


def test_parity_opf_large_fronts():
    """Delaunay network with fronts above the LDS bound (global-memory MFMA
    path)."""
    _case("opf-N5000", lambda: synth.opf_network(N=5000, seed=7, rho=1e4), "condensed", check_kappa=False)


@pytest.mark.parametrize("form", ["condensed", "stabilized"])
def test_parity_many_large_fronts(form):
    """LDS bound lowered to 64: most fronts take the large-front path, with
    partial last panels and multi-panel fronts."""
    _case("opf-N2000 fm64", lambda: synth.opf_network(N=2000, seed=3, rho=1e4, sigma_lo=-4, sigma_hi=4), form,
          small_front_max=64)


@pytest.mark.parametrize("rho", [1e2, 1e6, 1e8])
def test_parity_rho_sweep(rho):
    _case(f"grid-rho{rho:g}", lambda: synth.grid_banded(rho=rho), "condensed")
    _case(f"grid-rho{rho:g}", lambda: synth.grid_banded(rho=rho), "stabilized")


def test_static_pivot_zero_primal_pivot_natural_order():
    """An exact zero primal pivot (empty W row, Sigma = 0) met first in natural
    order is perturbed to +eps||K|| (Sec. 3.1); refinement recovers x."""
    print("[gpu] zero-pivot stabilized natural", flush=True)
    inp = synth.random_system(30, 10, seed=7, rho=10.0, empty_w_rows=[0], zero_sigma=[0])
    B = synth.rhs(40, 2, seed=1)
    kkt = nk.KKT.from_input(inp, form="stabilized", ordering="natural")
    rc, X, info = factor_solve(kkt, inp, B)
    npos, nneg, nzero, npert = kkt.inertia()
    assert (npos, nneg, nzero) == (30, 10, 0) and npert >= 1
    assert omega_cpu(inp, "stabilized", X, B) <= 1e-12
    assert info.ir_steps >= 1


def test_determinism_bitwise():
    print("[gpu] determinism", flush=True)
    inp = synth.opf_network(N=2000, seed=4, rho=1e5)
    B = synth.rhs(inp.n, 2, seed=2)
    kkt = nk.KKT.from_input(inp)
    _, X1, _ = factor_solve(kkt, inp, B)
    _, X2, _ = factor_solve(kkt, inp, B)
    assert np.array_equal(X1, X2)


def test_error_paths():
    print("[gpu] error paths", flush=True)
    import torch
    inp = synth.random_system(20, 5, seed=3)
    kkt = nk.KKT.from_input(inp)
    with pytest.raises(nk.NCLError) as e:
        kkt.solve(dev(np.ones(20)))
    assert e.value.code == -5
    with pytest.raises(nk.NCLError) as e:
        kkt.factor(dev(inp.W_val), dev(inp.Sigma), dev(inp.J_val), 0.0)
    assert e.value.code == -1
    bad = inp.W_val.copy(); bad[0] = np.nan
    with pytest.raises(nk.NCLError) as e:
        kkt.factor(dev(bad), dev(inp.Sigma), dev(inp.J_val), inp.rho)
    assert e.value.code == -6
    # a valid factorization afterwards still works
    rc, X, info = factor_solve(kkt, inp, synth.rhs(20, 1, seed=0))
    assert rc == 0 and info.backward_error <= 1e-12
    torch.cuda.synchronize()


def test_wrong_inertia_reported():
    """An indefinite W (large negative eigenvalue) gives the wrong inertia:
    status NCL_WARN_INERTIA, counts equal to the oracle's (Sec. 3.4)."""
    print("[gpu] wrong inertia", flush=True)
    inp = synth.random_system(25, 5, seed=12, rho=1.0, spd=False)
    kkt = nk.KKT.from_input(inp)
    rc = kkt.factor(dev(inp.W_val), dev(inp.Sigma), dev(inp.J_val), inp.rho)
    _, io, _, _ = O.solve(inp, O.CONDENSED, synth.rhs(25, 1))
    assert io.inertia[:3] != (25, 0, 0)
    assert rc == nk.NCL_WARN_INERTIA
    assert kkt.inertia()[:3] == io.inertia[:3]


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_graph_replays_match_eager(precision):
    """The factorization and the sweeps replayed from HIP graphs give bitwise
    the same results as eager launches, over several refactorizations with
    different values and eager work in between."""
    print(f"[gpu] graph vs eager {precision}", flush=True)
    import torch
    inp0 = synth.opf_network(N=3000, seed=9, rho=1e3)
    kg = nk.KKT.from_input(inp0, precision=precision, use_graphs=True)
    ke = nk.KKT.from_input(inp0, precision=precision, use_graphs=False)
    for k in range(3):
        Sigma, rho = synth.opf_sequence_values(inp0, 5 * k)
        inp = inp0.with_values(Sigma=Sigma, rho=rho)
        B = synth.rhs(inp.n, 2, seed=k)
        rcg, Xg, ig = factor_solve(kg, inp, B)
        torch.cuda.synchronize()
        rce, Xe, ie = factor_solve(ke, inp, B)
        assert rcg == rce and kg.inertia() == ke.inertia()
        assert np.array_equal(Xg, Xe), k
        assert omega_cpu(inp, "condensed", Xg, B) <= 1e-12
