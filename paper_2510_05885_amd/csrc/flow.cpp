// flow.cpp — task graph of one level's large-front factorization for the
// single dataflow launch (k_large_flow).
//
// Per large front (p pivots, order f) and 64-column panel k (k0 = 64k,
// k1 = min(k0 + 64, p)) the tasks are those of the right-looking blocked
// LDL^T with static pivoting:
//   DIAG(k)        the diagonal block: for k > 0 its own update by panel k-1,
//                  LDL^T, inverse Z_k = L_kk^-1, publish L, D, Z;
//   PANEL(k, r0)   rows r0..r0+31 below it: L = A Z_k^T D_k^-1;
//   UPD(k, i0, j0) the 64x64 tile at (i0, j0), i0 >= j0 >= k1:
//                  C -= L_i D_k L_j^T (the tile (k1, k1) is left to DIAG(k+1)).
// Dependencies are expressed through counters that the kernel polls:
//   dc            DIAG tasks done for the front (DIAG(k) done <=> dc >= k+1);
//   pc[k][rb]     PANEL(k) tasks done among the 64-row block rb (relative to
//                 k1) — a task reads two such blocks;
//   tv[I][J]      updates applied to the 64-aligned tile (I, J) — the write
//                 order of every tile.
// The order of the task list comes from a list-scheduling simulation with the
// launch's number of workgroups and rough task durations, highest upward rank
// (longest path to the end) first; each task starts in the simulation only
// after its predecessors finished, so the list is a topological order, which
// is what the ticket scheme of the kernel needs to be free of deadlock.
#include <algorithm>
#include <cstdint>
#include <functional>
#include <queue>
#include <stdexcept>
#include <utility>
#include <vector>

#include "plan.hpp"

namespace ncl {

namespace {

struct FTask {
    int type, s, k0, a, b;
    int sig = -1;
    std::vector<std::pair<int, int>> waits;   // (counter, target)
    std::vector<int> pred;                    // task ids (simulation)
    double dur = 0.0;
    double flops = 0.0;
};

}  // namespace

void build_flow(Plan& P, LargeStep& st, const std::vector<int>& large, int workers) {
    constexpr int W = 64;
    const int64_t ctr0 = P.flow_nctr;
    int64_t next = ctr0;
    st.flow_ticket = next++;
    std::vector<FTask> T;
    for (int s : large) {
        const int f = (int)(P.sn_rowptr[s + 1] - P.sn_rowptr[s]);
        const int p = P.sn_first[s + 1] - P.sn_first[s];
        const int np = (p + W - 1) / W;
        const int nT = (f + W - 1) / W;
        const int dc = (int)next++;
        // pc[k][rb]
        std::vector<int64_t> pc_base(np);
        std::vector<std::vector<int>> pc_target(np);
        std::vector<std::vector<std::vector<int>>> pc_tasks(np);
        for (int k = 0; k < np; ++k) {
            const int k1 = std::min(W * k + W, p);
            const int nrb = k1 < f ? (f - k1 + W - 1) / W : 0;
            pc_base[k] = next;
            next += nrb;
            pc_target[k].assign(nrb, 0);
            pc_tasks[k].assign(nrb, {});
        }
        const int64_t tv_base = next;
        next += (int64_t)nT * (nT + 1) / 2;
        auto tv = [&](int I, int J) { return (int)(tv_base + (int64_t)I * (I + 1) / 2 + J); };
        std::vector<int> cntU((size_t)nT * (nT + 1) / 2, 0), lastU((size_t)nT * (nT + 1) / 2, -1);
        auto tix = [&](int I, int J) { return (size_t)I * (I + 1) / 2 + J; };
        // waits and predecessors on the aligned tiles overlapping rows [r0, r1) x cols [c0, c1)
        auto tile_deps = [&](FTask& t, int r0, int r1, int c0, int c1) {
            for (int J = c0 / W; J <= (c1 - 1) / W; ++J)
                for (int I = std::max(J, r0 / W); I <= (r1 - 1) / W; ++I) {
                    const size_t q = tix(I, J);
                    if (cntU[q] == 0) continue;
                    t.waits.push_back({tv(I, J), cntU[q]});
                    t.pred.push_back(lastU[q]);
                }
        };
        int prev_diag = -1;
        for (int k = 0; k < np; ++k) {
            const int k0 = W * k, w = std::min(W, p - k0), k1 = k0 + w;
            // DIAG(k)
            {
                FTask t{kFlowDiag, s, k0, 0, 0};
                if (k > 0) {
                    t.waits.push_back({(int)pc_base[k - 1], pc_target[k - 1][0]});
                    for (int q : pc_tasks[k - 1][0]) t.pred.push_back(q);
                    tile_deps(t, k0, std::min(k0 + W, f), k0, std::min(k0 + W, f));
                }
                t.sig = dc;
                t.dur = k == 0 ? 22.0 : 35.0;
                t.flops = 2.0 * w * w * w / 3.0 + (k > 0 ? (double)W * w * w : 0.0);
                prev_diag = (int)T.size();
                T.push_back(std::move(t));
            }
            // PANEL(k, r0)
            for (int r0 = k1; r0 < f; r0 += 32) {
                const int r1 = std::min(r0 + 32, f);
                const int rb = (r0 - k1) / W;
                FTask t{kFlowPanel, s, k0, r0, 0};
                t.waits.push_back({dc, k + 1});
                t.pred.push_back(prev_diag);
                tile_deps(t, r0, r1, k0, k1);
                t.sig = (int)(pc_base[k] + rb);
                t.dur = 8.0;
                t.flops = (double)(r1 - r0) * w * w;
                pc_target[k][rb] += 1;
                pc_tasks[k][rb].push_back((int)T.size());
                T.push_back(std::move(t));
            }
            // UPD(k, i0, j0)
            std::vector<std::pair<size_t, int>> done;   // tiles written this step
            for (int j0 = k1; j0 < f; j0 += W)
                for (int i0 = j0; i0 < f; i0 += W) {
                    if (i0 == k1 && j0 == k1 && k1 < p) continue;   // DIAG(k+1) updates it
                    const int i1 = std::min(i0 + W, f), j1 = std::min(j0 + W, f);
                    const int rbi = (i0 - k1) / W, rbj = (j0 - k1) / W;
                    FTask t{kFlowUpd, s, k0, i0, j0};
                    t.waits.push_back({(int)(pc_base[k] + rbi), pc_target[k][rbi]});
                    for (int q : pc_tasks[k][rbi]) t.pred.push_back(q);
                    if (rbj != rbi) {
                        t.waits.push_back({(int)(pc_base[k] + rbj), pc_target[k][rbj]});
                        for (int q : pc_tasks[k][rbj]) t.pred.push_back(q);
                    }
                    tile_deps(t, i0, i1, j0, j1);
                    const bool aligned = i0 % W == 0 && j0 % W == 0;
                    if (aligned) {
                        t.sig = tv(i0 / W, j0 / W);
                        done.push_back({tix(i0 / W, j0 / W), (int)T.size()});
                    } else if (k != np - 1) {
                        throw std::logic_error("flow: unaligned update tile before the last panel");
                    }
                    const double ri = i1 - i0, rj = j1 - j0;
                    t.flops = 2.0 * ((i0 == j0) ? ri * (ri + 1) / 2 : ri * rj) * w;
                    t.dur = 12.0;
                    T.push_back(std::move(t));
                }
            for (auto& q : done) {
                cntU[q.first] += 1;
                lastU[q.first] = q.second;
            }
        }
    }
    // ---- upward ranks (task ids are a topological order: preds have smaller ids)
    const int n = (int)T.size();
    std::vector<std::vector<int>> succ(n);
    std::vector<int> npred(n, 0);
    for (int i = 0; i < n; ++i) {
        std::sort(T[i].pred.begin(), T[i].pred.end());
        T[i].pred.erase(std::unique(T[i].pred.begin(), T[i].pred.end()), T[i].pred.end());
        for (int q : T[i].pred) {
            if (q < 0 || q >= i) throw std::logic_error("flow: predecessor out of order");
            succ[q].push_back(i);
        }
        npred[i] = (int)T[i].pred.size();
    }
    std::vector<double> rank(n, 0.0);
    for (int i = n - 1; i >= 0; --i) {
        double m = 0.0;
        for (int q : succ[i]) m = std::max(m, rank[q]);
        rank[i] = T[i].dur + m;
    }
    // ---- list scheduling with `workers` slots
    auto worse = [&](int a, int b) { return rank[a] != rank[b] ? rank[a] < rank[b] : a > b; };
    std::priority_queue<int, std::vector<int>, decltype(worse)> ready(worse);
    typedef std::pair<double, int> Ev;
    std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> running;
    for (int i = 0; i < n; ++i)
        if (npred[i] == 0) ready.push(i);
    std::vector<int> order;
    order.reserve(n);
    double now = 0.0;
    const int nw = std::max(1, std::min(workers, n));
    while ((int)order.size() < n) {
        while ((int)running.size() < nw && !ready.empty()) {
            const int i = ready.top();
            ready.pop();
            order.push_back(i);
            running.push({now + T[i].dur, i});
        }
        if (running.empty()) throw std::logic_error("flow: dependency cycle");
        const Ev e = running.top();
        running.pop();
        now = e.first;
        for (int q : succ[e.second])
            if (--npred[q] == 0) ready.push(q);
    }
    // ---- emit
    st.flow_first = (int64_t)P.flow_task.size() / 8;
    st.flow_count = n;
    st.flow_grid = nw;
    st.flow_flops = 0.0;
    for (int i : order) {
        const FTask& t = T[i];
        P.flow_task.insert(P.flow_task.end(), {t.type, t.s, t.k0, t.a, t.b, (int)(P.flow_dep.size() / 2),
                                               (int)t.waits.size(), t.sig});
        for (auto& wt : t.waits) {
            P.flow_dep.push_back(wt.first);
            P.flow_dep.push_back(wt.second);
        }
        st.flow_flops += t.flops;
    }
    P.flow_nctr = next;
    if (next > INT32_MAX) throw std::length_error("flow: too many counters");
}

}  // namespace ncl
