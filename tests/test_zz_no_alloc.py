"""ncl_kkt_backward_noalloc (staging in the library's fixed device scratch)
against ncl_kkt_backward (staging in the handle's workspace), through the C
ABI: bitwise equal gradients on two calls in a row, the second on a smaller
system, plus a call at the capacity limit and one beyond it (NCL_ERR_SCRATCH)."""
import numpy as np
import pytest

from paper_2510_05885_amd import ncl_kkt as nk
from paper_2510_05885_amd import synth

from gpu_util import dev

pytestmark = pytest.mark.gpu


def _grads(kkt, inp, X, Lam, noalloc):
    import torch
    g = [torch.full((k,), np.nan, dtype=torch.float64, device="cuda")
         for k in (kkt.nnzW, kkt.order, kkt.nnzJ, kkt.S)]
    kkt.backward(dev(inp.J_val), X, Lam, *g, noalloc=noalloc)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in g]


def _colmajor(rng, n, q):
    import torch
    return torch.as_tensor(np.ascontiguousarray(rng.standard_normal((q, n))), device="cuda").t()


def _check(inp, nrhs, seed):
    print(f"[gpu] backward_noalloc n={inp.n} m={inp.m} nrhs={nrhs}", flush=True)
    kkt = nk.KKT.from_input(inp)
    kkt.factor(dev(inp.W_val), dev(inp.Sigma), dev(inp.J_val), inp.rho)
    rng = np.random.default_rng(seed)
    X, Lam = _colmajor(rng, inp.n, nrhs), _colmajor(rng, inp.n, nrhs)
    ref = _grads(kkt, inp, X, Lam, noalloc=False)
    got = _grads(kkt, inp, X, Lam, noalloc=True)
    for a, b in zip(ref, got):
        assert np.all(np.isfinite(a)) and np.array_equal(a, b)
    return kkt


def test_backward_noalloc_matches_allocating_entry_point():
    big = synth.grid_banded(rho=1e6)                                     # n = 2000, m = 1000
    small = synth.grid_banded(nr=10, nc=12, m=50, band=20, rho=1e3, seed=5)
    _check(big, 16, 1).close()
    _check(small, 3, 2).close()


def test_backward_noalloc_capacity():
    # 70000 Jacobian rows: 2 x 70000 x 14 <= 2^21 < 2 x 70000 x 16
    inp = synth.random_system(1000, 70000, seed=4, rho=10.0, j_per_row=1, w_density=0.002)
    kkt = _check(inp, 14, 3)
    import torch
    X = torch.zeros((16, inp.n), dtype=torch.float64, device="cuda").t()
    with pytest.raises(nk.NCLError) as e:
        kkt.backward(dev(inp.J_val), X, X, noalloc=True)
    assert e.value.code == nk.NCL_ERR_SCRATCH
    kkt.close()
