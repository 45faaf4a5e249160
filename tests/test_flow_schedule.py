"""Host checks of the dataflow schedule of the large fronts (no GPU).

The dataflow launch runs a level's diagonal-block, panel-solve and tile-update
tasks in ticket order, each waiting on device counters.  These tests take the
schedule from ncl_kkt_get_flow and check, on the CPU:
  * deadlock freedom: executed one by one in ticket order, every task finds
    its counters already at their targets;
  * coverage: the task set is exactly the blocked right-looking LDL^T of each
    front (every diagonal block, 32-row panel block and lower 64x64 tile of
    every step, nothing twice);
  * race freedom: whenever two tasks of a front touch the same entries and one
    of them writes, the one that comes first in the sequential algorithm is
    guaranteed complete before the other starts (happens-before through the
    counters, with counters that count a chain of tasks taken in chain order).
"""
import numpy as np
import pytest

from paper_2510_05885_amd import synth
from paper_2510_05885_amd.ncl_kkt import KKT

W = 64
DIAG, PANEL, UPD = 0, 1, 2


def _schedule(inp, form, **opts):
    k = KKT.from_input(inp, form=form, host_only=True, **opts)
    first, parent, rp, rows = k.supernodes()
    tasks, deps, nctr, launches = k.flow_schedule()
    k.close()
    p = np.diff(first)
    f = np.diff(rp)
    return tasks, deps, nctr, launches, p, f


def _waits(tasks, deps, t):
    d0, nd = tasks[t, 5], tasks[t, 6]
    return [(int(c), int(v)) for c, v in deps[d0:d0 + nd]]


def _cases():
    return [(synth.opf_network(N=300, seed=2), "condensed", {}),
            (synth.opf_network(N=300, seed=2), "stabilized", {}),
            (synth.opf_network(N=1000, seed=3), "condensed", {"small_front_max": 64}),
            (synth.random_system(400, 150, seed=5, w_density=0.05), "stabilized", {"small_front_max": 64})]


@pytest.fixture(scope="module", params=range(4), ids=["opf300-cond", "opf300-stab", "opf1000-cond-fm64",
                                                      "random-stab-fm64"])
def sched(request):
    inp, form, opts = _cases()[request.param]
    return _schedule(inp, form, **opts)


def test_ticket_order_is_deadlock_free(sched):
    tasks, deps, nctr, launches, p, f = sched
    assert len(launches) > 0 and len(tasks) > 0
    ctr = np.zeros(nctr, np.int64)
    for first, count, ticket, grid in launches:
        assert 1 <= grid <= count
        for t in range(first, first + count):
            for c, v in _waits(tasks, deps, t):
                assert c != ticket
                assert ctr[c] >= v, f"task {t} waits on counter {c} >= {v}, reached {ctr[c]}"
            if tasks[t, 7] >= 0:
                ctr[tasks[t, 7]] += 1


def _expected_tasks(s, p, f):
    out = set()
    for k0 in range(0, p, W):
        k1 = min(k0 + W, p)
        out.add((DIAG, s, k0, 0, 0))
        for r0 in range(k1, f, 32):
            out.add((PANEL, s, k0, r0, 0))
        for j0 in range(k1, f, W):
            for i0 in range(j0, f, W):
                if not (i0 == k1 and j0 == k1 and k1 < p):
                    out.add((UPD, s, k0, i0, j0))
    return out


def test_task_set_is_the_blocked_factorization(sched):
    tasks, deps, nctr, launches, p, f = sched
    got = [tuple(int(x) for x in t[:5]) for t in tasks]
    assert len(got) == len(set(got)), "a task appears twice"
    fronts = sorted(set(t[1] for t in got))
    want = set()
    for s in fronts:
        want |= _expected_tasks(s, int(p[s]), int(f[s]))
    assert set(got) == want
    # every large front of the plan is factored by exactly one launch
    for first, count, _, _ in launches:
        lv = set(int(s) for s in tasks[first:first + count, 1])
        for first2, count2, _, _ in launches:
            if first2 != first:
                assert not lv & set(int(s) for s in tasks[first2:first2 + count2, 1])


def _footprint(t, p, f):
    """(lower-storage rectangles, upper-storage rectangles, D ranges, Z panels),
    each split into reads and writes; rectangles are (r0, r1, c0, c1)."""
    typ, s, k0 = int(t[0]), int(t[1]), int(t[2])
    w = min(W, p - k0)
    k1 = k0 + w
    R, Wr, UR, UW, DR, DW, ZR, ZW = [], [], [], [], [], [], [], []
    if typ == DIAG:
        nr = min(W, f - k0)
        R.append((k0, k0 + nr, k0, k0 + nr))
        Wr.append((k0, k0 + nr, k0, k0 + nr))
        if k0 > 0:
            R.append((k0, k0 + nr, k0 - W, k0))
            DR.append((k0 - W, k0))
        DW.append((k0, k1))
        ZW.append(k0)
    elif typ == PANEL:
        r0 = int(t[3])
        r1 = min(r0 + 32, f)
        R.append((r0, r1, k0, k1))
        Wr.append((r0, r1, k0, k1))
        UW.append((k0, k1, r0, r1))
        DR.append((k0, k1))
        ZR.append(k0)
    else:
        i0, j0 = int(t[3]), int(t[4])
        i1, j1 = min(i0 + W, f), min(j0 + W, f)
        R += [(i0, i1, k0, k1), (j0, j1, k0, k1), (i0, i1, j0, j1)]
        Wr.append((i0, i1, j0, j1))
        DR.append((k0, k1))
    return R, Wr, UR, UW, DR, DW, ZR, ZW


def _lower_overlap(a, b):
    r0, r1 = max(a[0], b[0]), min(a[1], b[1])
    c0, c1 = max(a[2], b[2]), min(a[3], b[3])
    return r0 < r1 and c0 < c1 and r1 - 1 >= c0       # some entry with row >= column


def _rect_overlap(a, b):
    return max(a[0], b[0]) < min(a[1], b[1]) and max(a[2], b[2]) < min(a[3], b[3])


def _range_overlap(a, b):
    return max(a[0], b[0]) < min(a[1], b[1])


def _conflict(fa, fb):
    Ra, Wa, URa, UWa, DRa, DWa, ZRa, ZWa = fa
    Rb, Wb, URb, UWb, DRb, DWb, ZRb, ZWb = fb
    for x in Wa:
        if any(_lower_overlap(x, y) for y in Rb + Wb):
            return True
    for x in Wb:
        if any(_lower_overlap(x, y) for y in Ra):
            return True
    for x in UWa:
        if any(_rect_overlap(x, y) for y in URb + UWb):
            return True
    for x in UWb:
        if any(_rect_overlap(x, y) for y in URa):
            return True
    if any(_range_overlap(x, y) for x in DWa for y in DRb + DWb) or any(_range_overlap(x, y) for x in DWb
                                                                         for y in DRa):
        return True
    return bool(set(ZWa) & set(ZRb + ZWb) or set(ZWb) & set(ZRa))


def _seq_key(t):
    typ, k0 = int(t[0]), int(t[2])
    return (k0, typ, int(t[3]), int(t[4]))


def _race_violations(tasks, deps, launches, p, f):
    """Conflicting pairs of one front not ordered by happens-before, plus
    counters with partial targets that are not chains."""
    bad = []
    for first, count, ticket, grid in launches:
        ids = list(range(first, first + count))
        signalers = {}
        for t in ids:
            if tasks[t, 7] >= 0:
                signalers.setdefault(int(tasks[t, 7]), []).append(t)
        # happens-before, reading a wait (c >= v) as "the first v signalers of
        # c in ticket order are complete" ...
        hb = {}
        partial = set()
        for t in ids:                           # ticket order: predecessors come first
            req = set()
            for c, v in _waits(tasks, deps, t):
                sig = signalers[c]
                assert v <= len(sig)
                if v < len(sig):
                    partial.add(c)
                for q in sig[:v]:
                    req.add(q)
                    req |= hb[q]
            hb[t] = req
        # ... which holds when such a counter's signalers form a chain (each
        # waits for the one before it), so they complete in ticket order
        for c in partial:
            sig = signalers[c]
            for m in range(1, len(sig)):
                if sig[m - 1] not in hb[sig[m]]:
                    bad.append(("chain", c))
        by_front = {}
        for t in ids:
            by_front.setdefault(int(tasks[t, 1]), []).append(t)
        for s, ts in by_front.items():
            fp = {t: _footprint(tasks[t], int(p[s]), int(f[s])) for t in ts}
            ts = sorted(ts, key=lambda t: _seq_key(tasks[t]))
            for i, a in enumerate(ts):
                for b in ts[i + 1:]:
                    if _conflict(fp[a], fp[b]) and a not in hb[b]:
                        bad.append((tuple(tasks[a][:5]), tuple(tasks[b][:5])))
    return bad


def test_schedule_is_race_free(sched):
    tasks, deps, nctr, launches, p, f = sched
    assert _race_violations(tasks, deps, launches, p, f) == []


def test_race_check_catches_a_dropped_dependency(sched):
    # plant a mistake in a copy of the schedule: the first update of a later
    # panel step forgets its waits
    tasks, deps, nctr, launches, p, f = sched
    t = tasks.copy()
    cand = [i for i in range(len(t)) if t[i, 0] == UPD and t[i, 2] > 0 and t[i, 6] > 0]
    if not cand:
        pytest.skip("no multi-panel front in this case")
    t[cand[0], 6] = 0
    assert _race_violations(t, deps, launches, p, f) != []


def test_schedule_does_not_depend_on_the_option():
    inp = synth.opf_network(N=300, seed=2)
    a = _schedule(inp, "condensed", large_flow=True)
    b = _schedule(inp, "condensed", large_flow=False)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
