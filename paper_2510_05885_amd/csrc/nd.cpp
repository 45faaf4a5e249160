// nd.cpp — fill-reducing ordering for the symbolic analysis: multilevel
// nested dissection on the graph of K, leaves ordered by minimum degree.
//
// Any symmetric permutation is admissible for both KKT forms (the condensed
// matrix is SPD; the stabilized one is symmetric quasi-definite and hence
// strongly factorizable, Sec. 3.2), so the ordering is chosen purely for fill
// and for a wide, shallow elimination tree: the frontal factorization is
// scheduled level by level on the GPU.
//
// Outline (all deterministic, seeded):
//   1. merge indistinguishable vertices (equal closed neighbourhoods) into
//      weighted supervariables;
//   2. recursive bisection: coarsen by heavy-edge matching, grow an initial
//      2-way partition by BFS from several seeds, refine with FM passes while
//      projecting back, turn the edge cut into a vertex separator with a
//      minimum vertex cover of the cut (Koenig), number the separator last;
//   3. subgraphs below the leaf size are ordered by weighted minimum degree.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <queue>
#include <vector>

#include "nd.hpp"

namespace ncl {

namespace {

struct Rng {
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed * 0x9E3779B97F4A7C15ULL + 0x1234567ULL) {}
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
    int below(int n) { return (int)(next() % (uint64_t)n); }
};

struct G {
    int n = 0;
    std::vector<int> xadj, adj, vw, ew;
    int64_t total_w() const { return std::accumulate(vw.begin(), vw.end(), (int64_t)0); }
};

// ---------------------------------------------------------------------------
// coarsening
// ---------------------------------------------------------------------------
G coarsen(const G& g, std::vector<int>& cmap, Rng& rng, int maxvw) {
    std::vector<int> order(g.n);
    std::iota(order.begin(), order.end(), 0);
    for (int i = g.n - 1; i > 0; --i) std::swap(order[i], order[rng.below(i + 1)]);
    std::vector<int> match(g.n, -1);
    cmap.assign(g.n, -1);
    int nc = 0;
    for (int u : order) {
        if (match[u] != -1) continue;
        int best = -1, bw = -1;
        for (int e = g.xadj[u]; e < g.xadj[u + 1]; ++e) {
            int v = g.adj[e];
            if (match[v] != -1 || v == u || g.vw[u] + g.vw[v] > maxvw) continue;
            if (g.ew[e] > bw || (g.ew[e] == bw && g.vw[v] < g.vw[best])) { bw = g.ew[e]; best = v; }
        }
        if (best >= 0) {
            match[u] = best; match[best] = u;
            cmap[u] = cmap[best] = nc++;
        } else {
            match[u] = u;
            cmap[u] = nc++;
        }
    }
    G c;
    c.n = nc;
    c.vw.assign(nc, 0);
    std::vector<int> first(nc, -1);
    for (int u = 0; u < g.n; ++u) {
        c.vw[cmap[u]] += g.vw[u];
        if (first[cmap[u]] == -1) first[cmap[u]] = u;
    }
    c.xadj.assign(nc + 1, 0);
    std::vector<int> pos(nc, -1);
    for (int C = 0; C < nc; ++C) {
        int u = first[C];
        int v = match[u];
        int start = (int)c.adj.size();
        for (int t = 0; t < (u == v ? 1 : 2); ++t) {
            const int w = t == 0 ? u : v;
            for (int e = g.xadj[w]; e < g.xadj[w + 1]; ++e) {
                int D = cmap[g.adj[e]];
                if (D == C) continue;
                if (pos[D] < start) {
                    pos[D] = (int)c.adj.size();
                    c.adj.push_back(D);
                    c.ew.push_back(g.ew[e]);
                } else {
                    c.ew[pos[D]] += g.ew[e];
                }
            }
        }
        c.xadj[C + 1] = (int)c.adj.size();
    }
    return c;
}

// ---------------------------------------------------------------------------
// 2-way FM refinement of an edge cut with a balance window on part 0
// ---------------------------------------------------------------------------
int64_t cut_of(const G& g, const std::vector<int>& part) {
    int64_t cut = 0;
    for (int u = 0; u < g.n; ++u)
        for (int e = g.xadj[u]; e < g.xadj[u + 1]; ++e)
            if (part[u] != part[g.adj[e]]) cut += g.ew[e];
    return cut / 2;
}

void fm_refine(const G& g, std::vector<int>& part, int64_t lo0, int64_t hi0, int passes) {
    const int n = g.n;
    std::vector<int> gain(n), locked(n);
    std::vector<int> moved;
    for (int pass = 0; pass < passes; ++pass) {
        int64_t w0 = 0;
        for (int u = 0; u < n; ++u) if (part[u] == 0) w0 += g.vw[u];
        int64_t cut = 0;
        using Item = std::pair<int, int>;  // (gain, -vertex) max-heap
        std::priority_queue<Item> heap[2];
        for (int u = 0; u < n; ++u) {
            int id = 0, ed = 0;
            for (int e = g.xadj[u]; e < g.xadj[u + 1]; ++e) {
                if (part[g.adj[e]] == part[u]) id += g.ew[e]; else ed += g.ew[e];
            }
            gain[u] = ed - id;
            cut += ed;
            locked[u] = 0;
            if (ed > 0) heap[part[u]].push({gain[u], -u});
        }
        cut /= 2;
        int64_t best_cut = cut, start_cut = cut;
        int64_t best_imb = std::max<int64_t>(0, std::max(lo0 - w0, w0 - hi0));
        moved.clear();
        size_t best_len = 0;
        int since_best = 0;
        while (since_best < 64) {
            // pick the side to move from: the one that keeps (or restores) balance
            int from = -1;
            int cand[2] = {-1, -1};
            for (int sd = 0; sd < 2; ++sd) {
                while (!heap[sd].empty()) {
                    auto [gn, nv] = heap[sd].top();
                    int v = -nv;
                    if (locked[v] || part[v] != sd || gain[v] != gn) { heap[sd].pop(); continue; }
                    cand[sd] = v;
                    break;
                }
            }
            auto ok = [&](int v) {
                if (v < 0) return false;
                int64_t nw0 = part[v] == 0 ? w0 - g.vw[v] : w0 + g.vw[v];
                int64_t imb = std::max<int64_t>(0, std::max(lo0 - nw0, nw0 - hi0));
                int64_t cur = std::max<int64_t>(0, std::max(lo0 - w0, w0 - hi0));
                return imb <= cur || imb == 0;
            };
            bool ok0 = ok(cand[0]), ok1 = ok(cand[1]);
            if (ok0 && ok1) from = gain[cand[0]] >= gain[cand[1]] ? 0 : 1;
            else if (ok0) from = 0;
            else if (ok1) from = 1;
            if (from < 0) break;
            int v = cand[from];
            heap[from].pop();
            cut -= gain[v];
            w0 += part[v] == 0 ? -g.vw[v] : g.vw[v];
            part[v] ^= 1;
            locked[v] = 1;
            gain[v] = -gain[v];
            moved.push_back(v);
            for (int e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
                int u = g.adj[e];
                int d = 2 * g.ew[e];
                gain[u] += (part[u] == part[v]) ? -d : d;
                if (!locked[u]) heap[part[u]].push({gain[u], -u});
            }
            int64_t imb = std::max<int64_t>(0, std::max(lo0 - w0, w0 - hi0));
            if (imb < best_imb || (imb == best_imb && cut < best_cut)) {
                best_imb = imb; best_cut = cut; best_len = moved.size(); since_best = 0;
            } else {
                ++since_best;
            }
        }
        for (size_t k = moved.size(); k > best_len; --k) part[moved[k - 1]] ^= 1;
        if (best_cut >= start_cut && best_len == 0) break;
    }
}

// BFS-grown initial bisection on a small graph, best of several seeds.
void initial_bisect(const G& g, std::vector<int>& part, Rng& rng, int64_t lo0, int64_t hi0) {
    int64_t W = g.total_w();
    int64_t target = (lo0 + hi0) / 2;
    std::vector<int> trial(g.n), bestp;
    int64_t best = -1, best_imb = -1;
    std::vector<int> q;
    std::vector<char> seen(g.n);
    const int tries = 8;
    for (int t = 0; t < tries; ++t) {
        std::fill(trial.begin(), trial.end(), 1);
        std::fill(seen.begin(), seen.end(), 0);
        int64_t w0 = 0;
        q.clear();
        size_t qh = 0;
        int seed = rng.below(g.n);
        q.push_back(seed); seen[seed] = 1;
        while (w0 < target) {
            if (qh == q.size()) {            // disconnected: restart from an unseen vertex
                int s = -1;
                for (int u = 0; u < g.n; ++u) if (!seen[u]) { s = u; break; }
                if (s < 0) break;
                q.push_back(s); seen[s] = 1;
            }
            int u = q[qh++];
            if (w0 + g.vw[u] > hi0 && w0 >= lo0) continue;
            trial[u] = 0;
            w0 += g.vw[u];
            for (int e = g.xadj[u]; e < g.xadj[u + 1]; ++e) {
                int v = g.adj[e];
                if (!seen[v]) { seen[v] = 1; q.push_back(v); }
            }
        }
        fm_refine(g, trial, lo0, hi0, 4);
        int64_t c = cut_of(g, trial);
        int64_t x0 = 0;
        for (int u = 0; u < g.n; ++u) if (trial[u] == 0) x0 += g.vw[u];
        int64_t imb = std::max<int64_t>(0, std::max(lo0 - x0, x0 - hi0));
        if (best < 0 || imb < best_imb || (imb == best_imb && c < best)) {
            best = c; best_imb = imb; bestp = trial;
        }
    }
    part = bestp;
    (void)W;
}

// Multilevel edge bisection; part[u] in {0,1}.
void bisect(const G& g0, std::vector<int>& part, Rng& rng) {
    int64_t W = g0.total_w();
    int64_t lo0 = (int64_t)(0.45 * (double)W), hi0 = (int64_t)(0.55 * (double)W);
    std::vector<G> levels;
    std::vector<std::vector<int>> maps;
    const G* cur = &g0;
    int maxvw = (int)std::max<int64_t>(1, (int64_t)(1.5 * (double)W / 64.0));
    while (cur->n > 96) {
        std::vector<int> cmap;
        G c = coarsen(*cur, cmap, rng, maxvw);
        if (c.n > 0.92 * cur->n) break;
        maps.push_back(std::move(cmap));
        levels.push_back(std::move(c));
        cur = &levels.back();
    }
    std::vector<int> p;
    // the balance window must admit at least one vertex at coarse levels
    int64_t maxw = 0;
    for (int u = 0; u < cur->n; ++u) maxw = std::max<int64_t>(maxw, cur->vw[u]);
    initial_bisect(*cur, p, rng, std::min(lo0, W / 2 - maxw / 2), std::max(hi0, W / 2 + maxw / 2));
    for (int l = (int)levels.size() - 1; l >= 0; --l) {
        const G& fine = (l == 0) ? g0 : levels[l - 1];
        std::vector<int> pf(fine.n);
        for (int u = 0; u < fine.n; ++u) pf[u] = p[maps[l][u]];
        p.swap(pf);
        int64_t mw = 0;
        for (int u = 0; u < fine.n; ++u) mw = std::max<int64_t>(mw, fine.vw[u]);
        fm_refine(fine, p, std::min(lo0, W / 2 - mw / 2), std::max(hi0, W / 2 + mw / 2), 6);
    }
    part.swap(p);
}

// Vertex separator from an edge cut: minimum vertex cover of the bipartite
// graph of cut edges (Koenig's theorem via maximum matching).  Returns sep[u] = 1.
void cut_to_separator(const G& g, const std::vector<int>& part, std::vector<char>& sep) {
    sep.assign(g.n, 0);
    std::vector<int> lid(g.n, -1), left, right;
    for (int u = 0; u < g.n; ++u) {
        bool b = false;
        for (int e = g.xadj[u]; e < g.xadj[u + 1] && !b; ++e) b = part[g.adj[e]] != part[u];
        if (!b) continue;
        if (part[u] == 0) { lid[u] = (int)left.size(); left.push_back(u); }
        else { lid[u] = (int)right.size(); right.push_back(u); }
    }
    const int nl = (int)left.size(), nr = (int)right.size();
    std::vector<int> matchL(nl, -1), matchR(nr, -1);
    for (int s = 0; s < nl; ++s) {              // greedy start
        int u = left[s];
        for (int e = g.xadj[u]; e < g.xadj[u + 1]; ++e) {
            int v = g.adj[e];
            if (part[v] == 1 && matchR[lid[v]] < 0) { matchL[s] = lid[v]; matchR[lid[v]] = s; break; }
        }
    }
    // augmenting paths by BFS over alternating paths from each free left vertex
    std::vector<int> visR(nr, -1), parR(nr, -1), bq;
    for (int s = 0; s < nl; ++s) {
        if (matchL[s] >= 0) continue;
        bq.assign(1, s);
        int found = -1;
        for (size_t h = 0; h < bq.size() && found < 0; ++h) {
            int a = bq[h], ua = left[a];
            for (int e = g.xadj[ua]; e < g.xadj[ua + 1]; ++e) {
                int v = g.adj[e];
                if (part[v] != 1) continue;
                int r = lid[v];
                if (visR[r] == s) continue;
                visR[r] = s;
                parR[r] = a;
                if (matchR[r] < 0) { found = r; break; }
                bq.push_back(matchR[r]);
            }
        }
        for (int r = found; r >= 0;) {
            int a = parR[r];
            int prev = matchL[a];
            matchL[a] = r;
            matchR[r] = a;
            r = prev;
        }
    }
    // Koenig: Z = vertices reachable from unmatched left vertices by alternating paths
    std::vector<char> zl(nl, 0), zr(nr, 0);
    std::vector<int> q;
    for (int s = 0; s < nl; ++s) if (matchL[s] < 0) { zl[s] = 1; q.push_back(s); }
    for (size_t h = 0; h < q.size(); ++h) {
        int a = q[h], ua = left[a];
        for (int e = g.xadj[ua]; e < g.xadj[ua + 1]; ++e) {
            int v = g.adj[e];
            if (part[v] != 1) continue;
            int r = lid[v];
            if (zr[r]) continue;
            zr[r] = 1;
            int a2 = matchR[r];
            if (a2 >= 0 && !zl[a2]) { zl[a2] = 1; q.push_back(a2); }
        }
    }
    for (int s = 0; s < nl; ++s) if (!zl[s]) sep[left[s]] = 1;
    for (int r = 0; r < nr; ++r) if (zr[r]) sep[right[r]] = 1;
}

// Weighted minimum degree on a small graph (dense bitsets); returns local order.
void small_mindeg(const G& g, std::vector<int>& order) {
    const int n = g.n;
    const int words = (n + 63) / 64;
    std::vector<uint64_t> A((size_t)n * words, 0);
    for (int u = 0; u < n; ++u)
        for (int e = g.xadj[u]; e < g.xadj[u + 1]; ++e) {
            int v = g.adj[e];
            A[(size_t)u * words + v / 64] |= 1ULL << (v % 64);
        }
    std::vector<char> done(n, 0);
    order.clear();
    for (int step = 0; step < n; ++step) {
        int best = -1;
        int64_t bd = -1;
        for (int u = 0; u < n; ++u) {
            if (done[u]) continue;
            int64_t d = 0;
            const uint64_t* row = &A[(size_t)u * words];
            for (int w = 0; w < words; ++w) {
                uint64_t bits = row[w];
                while (bits) {
                    int b = __builtin_ctzll(bits);
                    bits &= bits - 1;
                    d += g.vw[w * 64 + b];
                }
            }
            if (best < 0 || d < bd) { best = u; bd = d; }
        }
        done[best] = 1;
        order.push_back(best);
        const uint64_t* rb = &A[(size_t)best * words];
        std::vector<int> nb;
        for (int w = 0; w < words; ++w) {
            uint64_t bits = rb[w];
            while (bits) { int b = __builtin_ctzll(bits); bits &= bits - 1; nb.push_back(w * 64 + b); }
        }
        for (int u : nb) {
            uint64_t* ru = &A[(size_t)u * words];
            for (int w = 0; w < words; ++w) ru[w] |= rb[w];
            ru[u / 64] &= ~(1ULL << (u % 64));
            ru[best / 64] &= ~(1ULL << (best % 64));
        }
    }
}

// Induced subgraph of `verts` (global ids in `big`); gl is a scratch global->local map (-1).
G induced(const G& big, const std::vector<int>& verts, std::vector<int>& gl) {
    G s;
    s.n = (int)verts.size();
    for (int k = 0; k < s.n; ++k) gl[verts[k]] = k;
    s.xadj.assign(s.n + 1, 0);
    s.vw.resize(s.n);
    for (int k = 0; k < s.n; ++k) {
        int u = verts[k];
        s.vw[k] = big.vw[u];
        for (int e = big.xadj[u]; e < big.xadj[u + 1]; ++e) {
            int l = gl[big.adj[e]];
            if (l >= 0) { s.adj.push_back(l); s.ew.push_back(big.ew[e]); }
        }
        s.xadj[k + 1] = (int)s.adj.size();
    }
    for (int k = 0; k < s.n; ++k) gl[verts[k]] = -1;
    return s;
}

}  // namespace

// Nested-dissection order of a compressed graph.  Returns vertices in
// elimination order.
std::vector<int> nd_order_graph(int n, const std::vector<int>& xadj, const std::vector<int>& adj,
                                const std::vector<int>& vw, int leaf, uint64_t seed) {
    G g;
    g.n = n;
    g.xadj = xadj;
    g.adj = adj;
    g.vw = vw;
    g.ew.assign(adj.size(), 1);
    for (int u = 0; u < n; ++u)
        for (int e = xadj[u]; e < xadj[u + 1]; ++e) g.ew[e] = vw[u] * vw[adj[e]];
    std::vector<int> out(n, -1);
    std::vector<int> gl(n, -1);
    Rng rng(seed);
    struct Task { std::vector<int> verts; int lo, hi; };
    std::vector<Task> stack;
    {
        Task t;
        t.verts.resize(n);
        std::iota(t.verts.begin(), t.verts.end(), 0);
        t.lo = 0; t.hi = n;
        stack.push_back(std::move(t));
    }
    std::vector<int> comp, q;
    while (!stack.empty()) {
        Task t = std::move(stack.back());
        stack.pop_back();
        const int k = (int)t.verts.size();
        if (k == 0) continue;
        G s = induced(g, t.verts, gl);
        if (k <= leaf) {
            std::vector<int> ord;
            small_mindeg(s, ord);
            for (int a = 0; a < k; ++a) out[t.lo + a] = t.verts[ord[a]];
            continue;
        }
        // connected components
        comp.assign(k, -1);
        int nc = 0;
        for (int r = 0; r < k; ++r) {
            if (comp[r] >= 0) continue;
            q.assign(1, r);
            comp[r] = nc;
            for (size_t h = 0; h < q.size(); ++h) {
                int u = q[h];
                for (int e = s.xadj[u]; e < s.xadj[u + 1]; ++e)
                    if (comp[s.adj[e]] < 0) { comp[s.adj[e]] = nc; q.push_back(s.adj[e]); }
            }
            ++nc;
        }
        if (nc > 1) {
            std::vector<std::vector<int>> parts(nc);
            for (int a = 0; a < k; ++a) parts[comp[a]].push_back(t.verts[a]);
            int pos = t.lo;
            for (int c = 0; c < nc; ++c) {
                Task u;
                u.lo = pos; u.hi = pos + (int)parts[c].size();
                pos = u.hi;
                u.verts = std::move(parts[c]);
                stack.push_back(std::move(u));
            }
            continue;
        }
        std::vector<int> part;
        bisect(s, part, rng);
        std::vector<char> sep;
        cut_to_separator(s, part, sep);
        Task A, B;
        std::vector<int> S;
        for (int a = 0; a < k; ++a) {
            if (sep[a]) S.push_back(t.verts[a]);
            else if (part[a] == 0) A.verts.push_back(t.verts[a]);
            else B.verts.push_back(t.verts[a]);
        }
        if (A.verts.empty() || B.verts.empty()) {
            // bisection failed to split: order this piece by minimum degree
            std::vector<int> ord;
            small_mindeg(s, ord);
            for (int a = 0; a < k; ++a) out[t.lo + a] = t.verts[ord[a]];
            continue;
        }
        // separator last, ordered by minimum degree within it
        {
            G ss = induced(g, S, gl);
            std::vector<int> ord;
            if (ss.n <= 2048) small_mindeg(ss, ord);
            else { ord.resize(ss.n); std::iota(ord.begin(), ord.end(), 0); }
            int base = t.hi - (int)S.size();
            for (int a = 0; a < (int)S.size(); ++a) out[base + a] = S[ord[a]];
        }
        A.lo = t.lo; A.hi = t.lo + (int)A.verts.size();
        B.lo = A.hi; B.hi = B.lo + (int)B.verts.size();
        stack.push_back(std::move(A));
        stack.push_back(std::move(B));
    }
    return out;
}

// Indistinguishable-vertex compression, then nested dissection, then
// expansion.  Input: symmetric adjacency (CSR, no self loops) of N vertices.
// Output perm[k] = vertex eliminated k-th.
std::vector<int> nd_order(int N, const std::vector<int64_t>& xadj, const std::vector<int>& adj,
                          int leaf, uint64_t seed) {
    // closed-neighbourhood hash
    std::vector<uint64_t> h(N);
    auto mix = [](uint64_t x) {
        x += 0x9E3779B97F4A7C15ULL;
        x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
        x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
        return x ^ (x >> 31);
    };
    for (int u = 0; u < N; ++u) {
        uint64_t s = mix((uint64_t)u);
        for (int64_t e = xadj[u]; e < xadj[u + 1]; ++e) s += mix((uint64_t)adj[e]);
        h[u] = s ^ (uint64_t)(xadj[u + 1] - xadj[u]) * 0xD6E8FEB86659FD93ULL;
    }
    std::vector<int> idx(N);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return h[a] != h[b] ? h[a] < h[b] : a < b; });
    std::vector<int> rep(N);
    std::iota(rep.begin(), rep.end(), 0);
    std::vector<int> mark(N, -1);
    for (int a = 0; a < N;) {
        int b = a;
        while (b < N && h[idx[b]] == h[idx[a]]) ++b;
        for (int x = a; x < b; ++x) {
            int u = idx[x];
            if (rep[u] != u) continue;
            mark[u] = u;
            for (int64_t e = xadj[u]; e < xadj[u + 1]; ++e) mark[adj[e]] = u;
            for (int y = x + 1; y < b; ++y) {
                int v = idx[y];
                if (rep[v] != v || xadj[v + 1] - xadj[v] != xadj[u + 1] - xadj[u] || mark[v] != u) continue;
                bool same = true;
                for (int64_t e = xadj[v]; e < xadj[v + 1] && same; ++e) same = mark[adj[e]] == u;
                if (same) rep[v] = u;
            }
        }
        a = b;
    }
    std::vector<int> cid(N, -1), members_ptr, members;
    int nc = 0;
    for (int u = 0; u < N; ++u) if (rep[u] == u) cid[u] = nc++;
    for (int u = 0; u < N; ++u) cid[u] = cid[rep[u]];
    std::vector<int> vw(nc, 0);
    for (int u = 0; u < N; ++u) vw[cid[u]]++;
    members_ptr.assign(nc + 1, 0);
    for (int u = 0; u < N; ++u) members_ptr[cid[u] + 1]++;
    for (int c = 0; c < nc; ++c) members_ptr[c + 1] += members_ptr[c];
    members.resize(N);
    {
        std::vector<int> fill(members_ptr.begin(), members_ptr.end() - 1);
        for (int u = 0; u < N; ++u) members[fill[cid[u]]++] = u;
    }
    std::vector<int> cx(nc + 1, 0), ca;
    std::vector<int> seen(nc, -1);
    for (int c = 0; c < nc; ++c) {
        int u = members[members_ptr[c]];
        seen[c] = c;
        for (int64_t e = xadj[u]; e < xadj[u + 1]; ++e) {
            int d = cid[adj[e]];
            if (seen[d] != c) { seen[d] = c; ca.push_back(d); }
        }
        cx[c + 1] = (int)ca.size();
    }
    std::vector<int> cord = nd_order_graph(nc, cx, ca, vw, leaf, seed);
    std::vector<int> perm;
    perm.reserve(N);
    for (int c : cord)
        for (int k = members_ptr[c]; k < members_ptr[c + 1]; ++k) perm.push_back(members[k]);
    return perm;
}

}  // namespace ncl
