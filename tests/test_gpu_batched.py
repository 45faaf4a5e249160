"""The batched form in one persistent launch per phase (options.persistent):
every front of every system factored by one launch whose workgroups take
fronts from a ticket counter in topological order and wait on their
children's completion counters, and both triangular sweeps in a second
launch.  Each system against the oracle; repeats and graph replays bitwise
equal; per-system device times; the full 256-system batch of the batched
workload (OPF-shaped systems of 125..5000 nodes)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_05885_amd import ncl_kkt as nk
from paper_2510_05885_amd import synth

from gpu_util import colmajor, dev

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="persistent launches disabled: the first run of "
                     "test_persistent_batch_matches_oracle[fp64] stopped making progress (no output for "
                     "180 s after the factor + solve began) and its cause has not been found; the library "
                     "refuses options.persistent = 1 until it is"),
]


def _batch(inps, nrhs, **opts):
    kkt = nk.KKT.analyze_batched(inps, **opts)
    W = dev(np.concatenate([i.W_val for i in inps]))
    S = dev(np.concatenate([i.Sigma for i in inps]))
    J = dev(np.concatenate([i.J_val for i in inps]))
    rho = np.array([i.rho for i in inps])
    B = [synth.rhs(i.n, nrhs, seed=k) for k, i in enumerate(inps)]
    rc = kkt.factor(W, S, J, rho)
    X, info = kkt.solve(colmajor(np.vstack(B)))
    return kkt, rc, X.cpu().numpy(), info, B


def _check_against_oracle(kkt, inps, X, B, cw_tol=1e-14):
    inert = kkt.inertia_batched()
    off = 0
    worst = 0.0
    for k, i in enumerate(inps):
        Xk = X[off:off + i.n]
        off += i.n
        Xo, io, _, K = O.solve(i, O.CONDENSED, B[k], ir_cw_tol=cw_tol)
        assert tuple(inert[k][:3]) == io.inertia[:3] == (i.n, 0, 0), k
        assert float(O.backward_error(K, Xk, B[k]).max()) <= 1e-12, k
        cw = float(O.componentwise_backward_error(K, Xk, B[k]).max())
        assert cw <= 2 * cw_tol, (k, cw)
        worst = max(worst, float(np.abs(Xk - Xo).max() / np.abs(Xo).max()))
    return worst


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_persistent_batch_matches_oracle(precision):
    print(f"[gpu] persistent batch of 8, {precision}", flush=True)
    sizes = [40, 75, 120, 33, 260, 90, 150, 61]
    inps = [synth.batched_system(k, N) for k, N in enumerate(sizes)]
    kkt, rc, X, info, B = _batch(inps, 2, persistent=1, precision=precision, ir_cw_tol=1e-14)
    assert rc in (0, nk.NCL_WARN_FELL_BACK_FP64) and info.backward_error_cw <= 1e-14
    fwd = _check_against_oracle(kkt, inps, X, B)
    print(f"[gpu]   max forward error vs oracle {fwd:.2e}", flush=True)
    assert fwd <= 1e-8
    f_ms, s_ms = kkt.system_times()
    print(f"[gpu]   per-system factor ms {np.round(f_ms, 3)} solve ms {np.round(s_ms, 3)}", flush=True)
    assert np.all(f_ms > 0) and np.all(s_ms >= f_ms)
    kkt.close()


def test_persistent_repeatable_and_graph_equals_eager():
    """Fronts are factored in whatever order the workgroups take them, but each
    one does the same arithmetic on the same inputs: bitwise equal results over
    repeats, with graph replays or eager launches, and after another matrix."""
    print("[gpu] persistent determinism", flush=True)
    inps = [synth.batched_system(k, N) for k, N in enumerate([300, 1200, 80, 700])]
    out = []
    for graphs in (True, False):
        kkt = nk.KKT.analyze_batched(inps, persistent=1, use_graphs=graphs)
        W = dev(np.concatenate([i.W_val for i in inps]))
        J = dev(np.concatenate([i.J_val for i in inps]))
        rho = np.array([i.rho for i in inps])
        S0 = np.concatenate([i.Sigma for i in inps])
        B = colmajor(np.vstack([synth.rhs(i.n, 1, seed=k) for k, i in enumerate(inps)]))
        for rep in range(3):
            kkt.factor(W, dev(S0 * (1.0 + rep)), J, rho)   # a different matrix in between
            kkt.factor(W, dev(S0), J, rho)
            X, _ = kkt.solve(B)
            out.append(X.cpu().numpy())
        kkt.close()
    assert all(np.array_equal(out[0], x) for x in out[1:])


def test_persistent_single_system():
    """The persistent launches on one (non-batched) system with fronts above the
    LDS bound, against the oracle."""
    print("[gpu] persistent single system", flush=True)
    inp = synth.opf_network(N=2000, seed=3, rho=1e4, sigma_lo=-4, sigma_hi=4)
    B = synth.rhs(inp.n, 3, seed=2)
    kkt = nk.KKT.from_input(inp, persistent=1, small_front_max=64, ir_cw_tol=1e-14)
    rc = kkt.factor(dev(inp.W_val), dev(inp.Sigma), dev(inp.J_val), inp.rho)
    X, info = kkt.solve(colmajor(B))
    X = X.cpu().numpy()
    Xo, io, _, K = O.solve(inp, O.CONDENSED, B, ir_cw_tol=1e-14)
    assert rc == 0 and kkt.inertia()[:3] == io.inertia[:3]
    assert float(O.componentwise_backward_error(K, X, B).max()) <= 2e-14
    assert np.abs(X - Xo).max() <= 1e-8 * np.abs(Xo).max()
    kkt.close()


@pytest.mark.timeout(900)
def test_batched_workload_256_systems():
    """The batched workload itself: 256 OPF-shaped systems of 125..5000 nodes
    (n 625..25k), per-system rho and Sigma, factored and solved by the two
    persistent launches; every system against the oracle."""
    print("[gpu] 256-system batch", flush=True)
    sizes = synth.batched_sizes(256)
    inps = [synth.batched_system(k, int(N)) for k, N in enumerate(sizes)]
    kkt, rc, X, info, B = _batch(inps, 1, persistent=1, ir_tol=1e-10, ir_cw_tol=1e-14)
    print(f"[gpu]   rc={rc} omega={info.backward_error:.2e} cw={info.backward_error_cw:.2e} "
          f"ir_steps={info.ir_steps}", flush=True)
    assert rc == 0
    fwd = _check_against_oracle(kkt, inps, X, B)
    f_ms, s_ms = kkt.system_times()
    print(f"[gpu]   max forward error vs oracle {fwd:.2e}; latency p50/p99 {np.percentile(s_ms, 50):.2f}/"
          f"{np.percentile(s_ms, 99):.2f} ms", flush=True)
    assert fwd <= 1e-6
    kkt.close()
