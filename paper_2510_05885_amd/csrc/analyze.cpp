// analyze.cpp — symbolic analysis of the KKT matrix (host, once per pattern).
//
// Produces the Plan used by every numeric factorization and solve:
//   * the full symmetric CSR of K in unpermuted numbering, with the source of
//     every entry: W entry, Sigma (diagonal), J entry (stabilized off-diagonal
//     blocks), -1/rho (stabilized dual diagonal) and, for the condensed form,
//     the list of J-entry pairs whose products make up (J^T J)_ij
//     (condensed: Sec. 3.3 eq. K1; stabilized: Sec. 3.2 eq. K2r);
//   * a fill-reducing ordering (nested dissection, natural or user);
//   * the elimination tree, its postorder, column counts, fundamental
//     supernodes and relaxed amalgamation into fronts;
//   * every front's row list, the K-entry -> front-slot map and the
//     child-contribution -> parent-row maps (extend-add);
//   * the level schedule (leaves first) and the device storage layout.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <stdexcept>

#include "analyze.hpp"
#include "nd.hpp"

namespace ncl {

namespace {

struct AnalyzeError : std::runtime_error {
    int code;
    AnalyzeError(int c, const char* m) : std::runtime_error(m), code(c) {}
};

void check_W(int n, const int32_t* Wp, const int32_t* Wi) {
    if (Wp[0] != 0) throw AnalyzeError(-2, "W_colptr[0] != 0");
    for (int j = 0; j < n; ++j) {
        if (Wp[j + 1] < Wp[j]) throw AnalyzeError(-2, "W_colptr not monotone");
        for (int p = Wp[j]; p < Wp[j + 1]; ++p) {
            int i = Wi[p];
            if (i < j || i >= n) throw AnalyzeError(-2, "W entry outside the lower triangle");
            if (p > Wp[j] && Wi[p - 1] >= i) throw AnalyzeError(-2, "W rows unsorted or duplicate");
        }
    }
}

void check_J(int n, int m, const int32_t* Jp, const int32_t* Jj) {
    if (m > 0 && Jp[0] != 0) throw AnalyzeError(-2, "J_rowptr[0] != 0");
    for (int r = 0; r < m; ++r) {
        if (Jp[r + 1] < Jp[r]) throw AnalyzeError(-2, "J_rowptr not monotone");
        for (int p = Jp[r]; p < Jp[r + 1]; ++p) {
            int j = Jj[p];
            if (j < 0 || j >= n) throw AnalyzeError(-2, "J column out of range");
            if (p > Jp[r] && Jj[p - 1] >= j) throw AnalyzeError(-2, "J columns unsorted or duplicate");
        }
    }
}

// Rows of the full symmetric CSR of one system, appended to P (global numbering).
void build_system_rows(Plan& P, const SysInput& in, int64_t vo, int64_t wo, int64_t jo) {
    const int n = in.n, m = in.m;
    const bool stab = P.form == 1;
    const int Ns = stab ? n + m : n;
    // transpose of W (lower CSC) -> per row i: (col j <= i, W index)
    std::vector<int> Tp(n + 1, 0), Tj, Tw;
    for (int j = 0; j < n; ++j)
        for (int p = in.Wp[j]; p < in.Wp[j + 1]; ++p) Tp[in.Wi[p] + 1]++;
    for (int i = 0; i < n; ++i) Tp[i + 1] += Tp[i];
    Tj.resize(Tp[n]); Tw.resize(Tp[n]);
    {
        std::vector<int> f(Tp.begin(), Tp.end() - 1);
        for (int j = 0; j < n; ++j)
            for (int p = in.Wp[j]; p < in.Wp[j + 1]; ++p) { int q = f[in.Wi[p]]++; Tj[q] = j; Tw[q] = p; }
    }
    // J transpose (columns -> rows r increasing)
    std::vector<int> Cp(n + 1, 0), Cr, Ck;
    const int nJ = m > 0 ? in.Jp[m] : 0;
    for (int k = 0; k < nJ; ++k) Cp[in.Jj[k] + 1]++;
    for (int j = 0; j < n; ++j) Cp[j + 1] += Cp[j];
    Cr.resize(nJ); Ck.resize(nJ);
    {
        std::vector<int> f(Cp.begin(), Cp.end() - 1);
        for (int r = 0; r < m; ++r)
            for (int k = in.Jp[r]; k < in.Jp[r + 1]; ++k) { int q = f[in.Jj[k]]++; Cr[q] = r; Ck[q] = k; }
    }
    std::vector<int> mark(Ns, -1), wsrc(Ns, -1), jsrc(Ns, -1);
    std::vector<int> cols;
    const int64_t base_nnz = (int64_t)P.Kj.size();
    const int64_t base_row = vo;
    for (int i = 0; i < Ns; ++i) {
        cols.clear();
        auto add = [&](int c) { if (mark[c] != i) { mark[c] = i; cols.push_back(c); wsrc[c] = -1; jsrc[c] = -1; } };
        add(i);
        uint8_t diag_flag = 0;
        if (i < n) {
            for (int q = Tp[i]; q < Tp[i + 1]; ++q) { add(Tj[q]); wsrc[Tj[q]] = (int)(wo + Tw[q]); }
            for (int p = in.Wp[i]; p < in.Wp[i + 1]; ++p) { add(in.Wi[p]); wsrc[in.Wi[p]] = (int)(wo + p); }
            diag_flag = 1;
            if (stab) {
                for (int q = Cp[i]; q < Cp[i + 1]; ++q) { add(n + Cr[q]); jsrc[n + Cr[q]] = (int)(jo + Ck[q]); }
            } else {
                for (int q = Cp[i]; q < Cp[i + 1]; ++q) {
                    int r = Cr[q];
                    for (int k = in.Jp[r]; k < in.Jp[r + 1]; ++k) add(in.Jj[k]);
                }
            }
        } else {
            int r = i - n;
            for (int k = in.Jp[r]; k < in.Jp[r + 1]; ++k) { add(in.Jj[k]); jsrc[in.Jj[k]] = (int)(jo + k); }
            diag_flag = 2;
        }
        std::sort(cols.begin(), cols.end());
        for (int c : cols) {
            P.Kj.push_back((int)(vo + c));
            P.src_w.push_back(wsrc[c]);
            P.src_j.push_back(jsrc[c]);
            P.src_flag.push_back(c == i ? diag_flag : 0);
        }
        P.Kp.push_back((int64_t)P.Kj.size());
    }
    P.prod_ptr.resize(P.Kj.size() + 1);
    // product pairs for the condensed form: entry (a_col, b_col) gets (a, b)
    // for every J row r holding both, r increasing.
    if (!stab) {
        const int64_t nz0 = base_nnz, nz1 = (int64_t)P.Kj.size();
        std::vector<int64_t> cnt(nz1 - nz0 + 1, 0);
        auto find = [&](int row, int col) -> int64_t {
            const int64_t lo = P.Kp[base_row + row], hi = P.Kp[base_row + row + 1];
            const int* b = P.Kj.data();
            int64_t pos = std::lower_bound(b + lo, b + hi, (int)(vo + col)) - b;
            return pos;
        };
        for (int pass = 0; pass < 2; ++pass) {
            std::vector<int64_t> fill;
            if (pass == 1) {
                for (size_t e = 1; e < cnt.size(); ++e) cnt[e] += cnt[e - 1];
                fill.assign(cnt.begin(), cnt.end() - 1);
                const int64_t pb = (int64_t)P.prod_a.size();
                P.prod_a.resize(pb + cnt.back());
                P.prod_b.resize(pb + cnt.back());
                for (int64_t e = nz0; e < nz1; ++e) P.prod_ptr[e + 1] = pb + cnt[e - nz0 + 1];
                for (int r = 0; r < m; ++r)
                    for (int ka = in.Jp[r]; ka < in.Jp[r + 1]; ++ka)
                        for (int kb = in.Jp[r]; kb < in.Jp[r + 1]; ++kb) {
                            int64_t e = find(in.Jj[ka], in.Jj[kb]);
                            int64_t q = pb + fill[e - nz0]++;
                            P.prod_a[q] = (int)(jo + ka);
                            P.prod_b[q] = (int)(jo + kb);
                        }
            } else {
                for (int r = 0; r < m; ++r)
                    for (int ka = in.Jp[r]; ka < in.Jp[r + 1]; ++ka)
                        for (int kb = in.Jp[r]; kb < in.Jp[r + 1]; ++kb)
                            cnt[find(in.Jj[ka], in.Jj[kb]) - nz0 + 1]++;
            }
        }
    } else {
        for (int64_t e = base_nnz; e < (int64_t)P.Kj.size(); ++e) P.prod_ptr[e + 1] = P.prod_ptr[e];
    }
}

// Liu's elimination tree of the permuted matrix, using the full CSR and iperm.
void etree_of(const Plan& P, const std::vector<int>& perm, const std::vector<int>& iperm,
              std::vector<int>& parent) {
    const int N = (int)P.N;
    parent.assign(N, -1);
    std::vector<int> anc(N, -1);
    for (int k = 0; k < N; ++k) {
        const int r = perm[k];
        for (int64_t q = P.Kp[r]; q < P.Kp[r + 1]; ++q) {
            int i = iperm[P.Kj[q]];
            while (i != -1 && i < k) {
                int nx = anc[i];
                anc[i] = k;
                if (nx == -1) parent[i] = k;
                i = nx;
            }
        }
    }
}

// Postorder of a forest given by parent[] (children visited in increasing index).
std::vector<int> postorder(const std::vector<int>& parent) {
    const int N = (int)parent.size();
    std::vector<int> head(N, -1), next(N, -1), out;
    out.reserve(N);
    for (int j = N - 1; j >= 0; --j)
        if (parent[j] >= 0) { next[j] = head[parent[j]]; head[parent[j]] = j; }
    std::vector<int> stack;
    for (int r = 0; r < N; ++r) {
        if (parent[r] >= 0) continue;
        stack.push_back(r);
        while (!stack.empty()) {
            int v = stack.back();
            if (head[v] >= 0) {
                int c = head[v];
                head[v] = next[c];
                stack.push_back(c);
            } else {
                stack.pop_back();
                out.push_back(v);
            }
        }
    }
    return out;
}

// Column counts (incl. diagonal) of L via row subtrees, permuted numbering.
std::vector<int> column_counts(const Plan& P, const std::vector<int>& perm, const std::vector<int>& iperm,
                               const std::vector<int>& parent) {
    const int N = (int)P.N;
    std::vector<int> cc(N, 1), flag(N, -1);
    for (int k = 0; k < N; ++k) {
        flag[k] = k;
        const int r = perm[k];
        for (int64_t q = P.Kp[r]; q < P.Kp[r + 1]; ++q) {
            int i = iperm[P.Kj[q]];
            if (i >= k) continue;
            while (flag[i] != k) { flag[i] = k; cc[i]++; i = parent[i]; }
        }
    }
    return cc;
}

inline double stor(double p, double f) { return p * f - p * (p - 1.0) / 2.0; }

}  // namespace

int build_plan(Plan& P, int form, const std::vector<SysInput>& sys, int ordering, const int32_t* user_perm,
               const PlanConfig& cfg, std::string& err) {
    auto t0 = std::chrono::steady_clock::now();
    try {
        P = Plan();
        P.cfg = cfg;
        P.form = form;
        P.S = (int)sys.size();
        // ---------------- sizes and validation -----------------------------
        P.sys_voff.assign(P.S + 1, 0);
        P.sys_woff.assign(P.S + 1, 0);
        P.sys_joff.assign(P.S + 1, 0);
        std::vector<int64_t> sys_roff(P.S + 1, 0);
        for (int s = 0; s < P.S; ++s) {
            const SysInput& in = sys[s];
            if (in.n < 1 || in.m < 0) throw AnalyzeError(-1, "n must be >= 1 and m >= 0");
            if (!in.Wp || !in.Wi || (in.m > 0 && (!in.Jp || !in.Jj))) throw AnalyzeError(-1, "null pattern pointer");
            check_W(in.n, in.Wp, in.Wi);
            check_J(in.n, in.m, in.Jp, in.Jj);
            P.sys_n.push_back(in.n);
            P.sys_m.push_back(in.m);
            const int64_t Ns = form == 1 ? (int64_t)in.n + in.m : in.n;
            P.sys_voff[s + 1] = P.sys_voff[s] + Ns;
            P.sys_woff[s + 1] = P.sys_woff[s] + in.Wp[in.n];
            P.sys_joff[s + 1] = P.sys_joff[s] + (in.m > 0 ? in.Jp[in.m] : 0);
            sys_roff[s + 1] = sys_roff[s] + in.m;
        }
        P.N = P.sys_voff[P.S];
        P.nnzW = P.sys_woff[P.S];
        P.nnzJ = P.sys_joff[P.S];
        P.nJrows = sys_roff[P.S];
        if (P.N > (int64_t)INT32_MAX / 2 || P.nnzW > INT32_MAX || P.nnzJ > INT32_MAX)
            throw AnalyzeError(-1, "problem too large for 32-bit indices");
        const int N = (int)P.N;
        P.row_sys.resize(N);
        P.row_sign.resize(N);
        for (int s = 0; s < P.S; ++s)
            for (int64_t i = P.sys_voff[s]; i < P.sys_voff[s + 1]; ++i) {
                P.row_sys[i] = s;
                P.row_sign[i] = (form == 1 && i - P.sys_voff[s] >= P.sys_n[s]) ? -1 : 1;
            }
        // W / J coordinates for the adjoint
        P.Jp.assign(1, 0);
        for (int s = 0; s < P.S; ++s) {
            const SysInput& in = sys[s];
            for (int r = 0; r < in.m; ++r) {
                for (int k = in.Jp[r]; k < in.Jp[r + 1]; ++k) P.Jj.push_back((int)(P.sys_voff[s] + in.Jj[k]));
                P.Jp.push_back((int64_t)P.Jj.size());
                P.Jrow_sys.push_back(s);
            }
            for (int j = 0; j < in.n; ++j)
                for (int p = in.Wp[j]; p < in.Wp[j + 1]; ++p) {
                    P.Wrow_of.push_back((int)(P.sys_voff[s] + in.Wi[p]));
                    P.Wcol_of32.push_back((int)(P.sys_voff[s] + j));
                }
        }
        // ---------------- full CSR of K with sources ----------------------
        P.Kp.assign(1, 0);
        P.prod_ptr.assign(1, 0);
        for (int s = 0; s < P.S; ++s)
            build_system_rows(P, sys[s], P.sys_voff[s], P.sys_woff[s], P.sys_joff[s]);
        P.nnz_lower = 0;
        for (int i = 0; i < N; ++i)
            for (int64_t q = P.Kp[i]; q < P.Kp[i + 1]; ++q) if (P.Kj[q] <= i) P.nnz_lower++;

        // ---------------- ordering ------------------------------------------
        std::vector<int> perm(N);
        if (ordering == 2) {
            if (!user_perm) throw AnalyzeError(-1, "user ordering without a permutation");
            std::vector<char> seen(N, 0);
            for (int k = 0; k < N; ++k) {
                int v = user_perm[k];
                if (v < 0 || v >= N || seen[v]) throw AnalyzeError(-1, "user_perm is not a permutation");
                seen[v] = 1;
                perm[k] = v;
            }
        } else if (ordering == 1) {
            std::iota(perm.begin(), perm.end(), 0);
        } else {
            std::vector<int64_t> xadj(N + 1, 0);
            std::vector<int> adj;
            adj.reserve(P.Kj.size());
            for (int i = 0; i < N; ++i) {
                for (int64_t q = P.Kp[i]; q < P.Kp[i + 1]; ++q) if (P.Kj[q] != i) adj.push_back(P.Kj[q]);
                xadj[i + 1] = (int64_t)adj.size();
            }
            perm = nd_order(N, xadj, adj, cfg.nd_leaf, 12345);
        }
        std::vector<int> iperm(N);
        for (int k = 0; k < N; ++k) iperm[perm[k]] = k;

        // ---------------- etree, postorder, column counts -------------------
        std::vector<int> parent;
        etree_of(P, perm, iperm, parent);
        {
            std::vector<int> post = postorder(parent);
            std::vector<int> p1(N);
            for (int k = 0; k < N; ++k) p1[k] = perm[post[k]];
            perm.swap(p1);
            for (int k = 0; k < N; ++k) iperm[perm[k]] = k;
            etree_of(P, perm, iperm, parent);
        }
        std::vector<int> cc = column_counts(P, perm, iperm, parent);
        std::vector<int> nchild(N, 0);
        for (int j = 0; j < N; ++j) if (parent[j] >= 0) nchild[parent[j]]++;

        // ---------------- fundamental supernodes ----------------------------
        std::vector<int> fs_first;           // first column of each fundamental supernode
        for (int j = 0; j < N; ++j) {
            bool cont = j > 0 && parent[j - 1] == j && nchild[j] == 1 && cc[j - 1] == cc[j] + 1;
            if (!cont) fs_first.push_back(j);
        }
        const int nfs = (int)fs_first.size();
        fs_first.push_back(N);
        std::vector<int> col_fs(N);
        for (int s = 0; s < nfs; ++s)
            for (int j = fs_first[s]; j < fs_first[s + 1]; ++j) col_fs[j] = s;
        std::vector<int> fs_parent(nfs, -1);
        for (int s = 0; s < nfs; ++s) {
            int last = fs_first[s + 1] - 1;
            if (parent[last] >= 0) fs_parent[s] = col_fs[parent[last]];
        }
        // ---------------- relaxed amalgamation ------------------------------
        // group[s] = representative fundamental supernode; merged children are
        // absorbed into their parent when few explicit zeros are added.
        std::vector<double> g_p(nfs), g_f(nfs), g_z(nfs, 0.0);
        for (int s = 0; s < nfs; ++s) {
            g_p[s] = fs_first[s + 1] - fs_first[s];
            g_f[s] = cc[fs_first[s]];
        }
        std::vector<int> grp(nfs);
        std::iota(grp.begin(), grp.end(), 0);
        std::vector<int> ch_ptr(nfs + 1, 0), ch_list;
        for (int s = 0; s < nfs; ++s) if (fs_parent[s] >= 0) ch_ptr[fs_parent[s] + 1]++;
        for (int s = 0; s < nfs; ++s) ch_ptr[s + 1] += ch_ptr[s];
        ch_list.resize(ch_ptr[nfs]);
        {
            std::vector<int> f(ch_ptr.begin(), ch_ptr.end() - 1);
            for (int s = 0; s < nfs; ++s) if (fs_parent[s] >= 0) ch_list[f[fs_parent[s]]++] = s;
        }
        for (int P0 = 0; P0 < nfs; ++P0) {          // increasing = children first
            // candidate children, largest pivot count first
            std::vector<int> kids(ch_list.begin() + ch_ptr[P0], ch_list.begin() + ch_ptr[P0 + 1]);
            std::sort(kids.begin(), kids.end(), [&](int a, int b) { return g_p[a] != g_p[b] ? g_p[a] > g_p[b] : a < b; });
            for (int c : kids) {
                double pm = g_p[c] + g_p[P0];
                double fm = g_p[c] + g_f[P0];
                double sm = stor(pm, fm);
                double zm = g_z[c] + g_z[P0] + (sm - stor(g_p[c], g_f[c]) - stor(g_p[P0], g_f[P0]));
                double zf = zm / sm;
                bool ok = (pm <= 8 && zf <= 0.8) || (pm <= 24 && zf <= 0.35) || (pm <= 64 && zf <= 0.12) ||
                          zf <= 0.04 || (fm > cfg.relax_big_front && zf <= cfg.relax_big_zeros);
                if (fm > 4000) ok = false;
                if (!ok) continue;
                grp[c] = P0;
                g_p[P0] = pm; g_f[P0] = fm; g_z[P0] = zm;
            }
        }
        // resolve representatives (a merged child's group is its parent's group)
        for (int s = nfs - 1; s >= 0; --s) {
            if (grp[s] != s) grp[s] = grp[grp[s]];
        }
        // group tree: parent of a group = group of fs_parent of its representative
        std::vector<int> gparent(nfs, -2);
        for (int s = 0; s < nfs; ++s) if (grp[s] == s) gparent[s] = fs_parent[s] >= 0 ? grp[fs_parent[s]] : -1;
        // final column order: postorder of the group tree, member columns in
        // increasing (postordered) index
        std::vector<std::vector<int>> gcols(nfs);
        for (int j = 0; j < N; ++j) gcols[grp[col_fs[j]]].push_back(j);
        std::vector<int> gp_full(nfs, -1);
        for (int s = 0; s < nfs; ++s) gp_full[s] = (grp[s] == s) ? gparent[s] : -3;
        // postorder over groups only
        std::vector<int> gids;
        for (int s = 0; s < nfs; ++s) if (grp[s] == s) gids.push_back(s);
        std::vector<int> gidx(nfs, -1);
        for (size_t k = 0; k < gids.size(); ++k) gidx[gids[k]] = (int)k;
        std::vector<int> gpar(gids.size());
        for (size_t k = 0; k < gids.size(); ++k) gpar[k] = gparent[gids[k]] >= 0 ? gidx[gparent[gids[k]]] : -1;
        std::vector<int> gpost = postorder(gpar);
        std::vector<int> perm2;
        perm2.reserve(N);
        P.nsn = (int)gids.size();
        P.sn_first.assign(1, 0);
        for (int k : gpost) {
            for (int j : gcols[gids[k]]) perm2.push_back(perm[j]);
            P.sn_first.push_back((int)perm2.size());
        }
        // algorithmic size of the factor for this ordering: the column counts of
        // the elimination tree, before amalgamation padding (the group order
        // above is a topological order of the same tree, so each column keeps
        // its count); per final supernode for the timing classes
        std::vector<double> col_exact(N), col_cnt(N);
        P.nnzL_exact = 0;
        P.flops_exact = 0.0;
        {
            std::vector<int> old_pos(N);
            for (int j = 0; j < N; ++j) old_pos[perm[j]] = j;
            for (int k = 0; k < N; ++k) {
                const double c = (double)cc[old_pos[perm2[k]]] - 1.0;
                col_exact[k] = c * (c + 2.0);
                col_cnt[k] = c + 1.0;
                P.nnzL_exact += (int64_t)c + 1;
                P.flops_exact += col_exact[k];
            }
        }
        perm.swap(perm2);
        for (int k = 0; k < N; ++k) iperm[perm[k]] = k;
        P.perm = perm;
        P.iperm = iperm;
        const int nsn = P.nsn;
        std::vector<int> col_sn(N);
        for (int s = 0; s < nsn; ++s)
            for (int j = P.sn_first[s]; j < P.sn_first[s + 1]; ++j) col_sn[j] = s;

        // ---------------- front row structure (union rule) -----------------
        // lower pattern of the permuted matrix by columns
        std::vector<int64_t> Ap(N + 1, 0);
        std::vector<int> Ai;
        for (int r = 0; r < N; ++r)
            for (int64_t q = P.Kp[r]; q < P.Kp[r + 1]; ++q) {
                int a = iperm[r], b = iperm[P.Kj[q]];
                if (a > b) Ap[b + 1]++;
            }
        for (int j = 0; j < N; ++j) Ap[j + 1] += Ap[j];
        Ai.resize(Ap[N]);
        {
            std::vector<int64_t> f(Ap.begin(), Ap.end() - 1);
            for (int r = 0; r < N; ++r)
                for (int64_t q = P.Kp[r]; q < P.Kp[r + 1]; ++q) {
                    int a = iperm[r], b = iperm[P.Kj[q]];
                    if (a > b) Ai[f[b]++] = a;
                }
        }
        P.sn_parent.assign(nsn, -1);
        P.sn_rowptr.assign(nsn + 1, 0);
        std::vector<int> mark(N, -1), list;
        std::vector<std::vector<int>> kids(nsn);
        for (int s = 0; s < nsn; ++s) {
            const int first = P.sn_first[s], last = P.sn_first[s + 1] - 1;
            list.clear();
            for (int j = first; j <= last; ++j) { list.push_back(j); mark[j] = s; }
            size_t npiv = list.size();
            for (int j = first; j <= last; ++j)
                for (int64_t q = Ap[j]; q < Ap[j + 1]; ++q) {
                    int i = Ai[q];
                    if (i > last && mark[i] != s) { mark[i] = s; list.push_back(i); }
                }
            for (int c : kids[s]) {
                for (int64_t q = P.sn_rowptr[c] + (P.sn_first[c + 1] - P.sn_first[c]); q < P.sn_rowptr[c + 1]; ++q) {
                    int i = P.sn_rows[q];
                    if (i < first) throw AnalyzeError(-4, "internal: child contribution below its parent");
                    if (i > last && mark[i] != s) { mark[i] = s; list.push_back(i); }
                }
            }
            std::sort(list.begin() + npiv, list.end());
            P.sn_rows.insert(P.sn_rows.end(), list.begin(), list.end());
            P.sn_rowptr[s + 1] = (int64_t)P.sn_rows.size();
            if (list.size() > npiv) {
                int par = col_sn[list[npiv]];
                P.sn_parent[s] = par;
                kids[par].push_back(s);
            }
        }
        P.child_ptr.assign(nsn + 1, 0);
        for (int s = 0; s < nsn; ++s) {
            P.child_ptr[s + 1] = P.child_ptr[s] + (int)kids[s].size();
            P.child_list.insert(P.child_list.end(), kids[s].begin(), kids[s].end());
        }
        P.sn_sys.resize(nsn);
        for (int s = 0; s < nsn; ++s) P.sn_sys[s] = P.row_sys[perm[P.sn_first[s]]];

        // ---------------- sizes, flops, large/small -------------------------
        P.nnzL = 0;
        P.flops = P.small_flops = P.large_flops = 0.0;
        P.max_front = 0;
        P.sn_large.assign(nsn, 0);
        P.sn_flop_ratio.assign(nsn, 1.0);
        P.sn_nnz_ratio.assign(nsn, 1.0);
        P.n_large = 0;
        for (int s = 0; s < nsn; ++s) {
            const int64_t f = P.sn_rowptr[s + 1] - P.sn_rowptr[s];
            const int64_t p = P.sn_first[s + 1] - P.sn_first[s];
            P.nnzL += p * f - p * (p - 1) / 2;
            double fl = 0.0;
            for (int64_t k = 0; k < p; ++k) {
                double r = (double)(f - k - 1);
                fl += r + r * (r + 1.0);     // column scaling + lower rank-1 update
            }
            P.flops += fl;
            double ex = 0.0;
            for (int j = P.sn_first[s]; j < P.sn_first[s + 1]; ++j) ex += col_exact[j];
            P.sn_flop_ratio[s] = fl > 0.0 ? ex / fl : 1.0;
            double nz = 0.0;
            for (int j = P.sn_first[s]; j < P.sn_first[s + 1]; ++j) nz += col_cnt[j];
            P.sn_nnz_ratio[s] = nz / (double)(p * f - p * (p - 1) / 2);
            P.max_front = std::max<int>(P.max_front, (int)f);
            if (f > cfg.small_front_max) { P.sn_large[s] = 1; P.n_large++; P.large_flops += fl; }
            else P.small_flops += fl;
        }

        // ---------------- K-entry -> front slot -----------------------------
        {
            std::vector<int64_t> cnt(nsn + 1, 0);
            for (int r = 0; r < N; ++r)
                for (int64_t q = P.Kp[r]; q < P.Kp[r + 1]; ++q) {
                    int a = iperm[r], b = iperm[P.Kj[q]];
                    if (a >= b) cnt[col_sn[b] + 1]++;
                }
            for (int s = 0; s < nsn; ++s) cnt[s + 1] += cnt[s];
            P.kent_ptr = cnt;
            const int64_t total = cnt[nsn];
            P.kent_csr.resize(total);
            P.kent_pos.resize(total);
            P.kent_col.resize(total);
            std::vector<int64_t> f(cnt.begin(), cnt.end() - 1);
            for (int r = 0; r < N; ++r)
                for (int64_t q = P.Kp[r]; q < P.Kp[r + 1]; ++q) {
                    int a = iperm[r], b = iperm[P.Kj[q]];
                    if (a < b) continue;
                    int s = col_sn[b];
                    const int* rb = P.sn_rows.data() + P.sn_rowptr[s];
                    const int* re = P.sn_rows.data() + P.sn_rowptr[s + 1];
                    const int np = P.sn_first[s + 1] - P.sn_first[s];
                    int lr;
                    if (a <= P.sn_first[s + 1] - 1) lr = a - P.sn_first[s];
                    else {
                        const int* it = std::lower_bound(rb + np, re, a);
                        if (it == re || *it != a) throw AnalyzeError(-4, "internal: K entry outside its front");
                        lr = (int)(it - rb);
                    }
                    int lc = b - P.sn_first[s];
                    int fsz = (int)(re - rb);
                    int64_t k = f[s]++;
                    P.kent_csr[k] = q;
                    P.kent_pos[k] = lr + lc * fsz;
                    P.kent_col[k] = lc;
                }
            // sort each front's entries by (local column, position) for the
            // column-wise large-front assembly (and locality everywhere)
            P.kcol_base.assign(nsn + 1, 0);
            std::vector<int64_t> idx;
            for (int s = 0; s < nsn; ++s) {
                const int64_t b0 = P.kent_ptr[s], b1 = P.kent_ptr[s + 1];
                idx.resize(b1 - b0);
                std::iota(idx.begin(), idx.end(), b0);
                std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return P.kent_pos[x] < P.kent_pos[y]; });
                std::vector<int64_t> c2(idx.size());
                std::vector<int> p2(idx.size()), l2(idx.size());
                for (size_t t = 0; t < idx.size(); ++t) {
                    c2[t] = P.kent_csr[idx[t]]; p2[t] = P.kent_pos[idx[t]]; l2[t] = P.kent_col[idx[t]];
                }
                std::copy(c2.begin(), c2.end(), P.kent_csr.begin() + b0);
                std::copy(p2.begin(), p2.end(), P.kent_pos.begin() + b0);
                std::copy(l2.begin(), l2.end(), P.kent_col.begin() + b0);
                const int np = P.sn_first[s + 1] - P.sn_first[s];
                P.kcol_base[s] = (int64_t)P.kcol_ptr.size();
                if (P.sn_large[s]) {
                    // column segments (pos sorted => column sorted since pos = row + col*f)
                    int64_t t = b0;
                    for (int j = 0; j <= np; ++j) {
                        while (t < b1 && P.kent_col[t] < j) ++t;
                        P.kcol_ptr.push_back(t);
                    }
                }
            }
            P.kcol_base[nsn] = (int64_t)P.kcol_ptr.size();
        }

        // ---------------- extend-add maps -----------------------------------
        P.rel_ptr.assign(nsn + 1, 0);
        P.inv_ptr.assign(nsn + 1, 0);
        for (int s = 0; s < nsn; ++s) {
            const int np = P.sn_first[s + 1] - P.sn_first[s];
            const int64_t f = P.sn_rowptr[s + 1] - P.sn_rowptr[s];
            const int64_t c = f - np;
            P.rel_ptr[s + 1] = P.rel_ptr[s] + c;
            const int par = P.sn_parent[s];
            if (par >= 0 && P.sn_large[par])
                P.inv_ptr[s + 1] = P.inv_ptr[s] + (P.sn_rowptr[par + 1] - P.sn_rowptr[par]);
            else
                P.inv_ptr[s + 1] = P.inv_ptr[s];
        }
        P.rel.resize(P.rel_ptr[nsn]);
        P.inv.assign(P.inv_ptr[nsn], -1);
        for (int s = 0; s < nsn; ++s) {
            const int par = P.sn_parent[s];
            if (par < 0) continue;
            const int np = P.sn_first[s + 1] - P.sn_first[s];
            const int* pb = P.sn_rows.data() + P.sn_rowptr[par];
            const int* pe = P.sn_rows.data() + P.sn_rowptr[par + 1];
            const int pnp = P.sn_first[par + 1] - P.sn_first[par];
            for (int64_t q = P.sn_rowptr[s] + np, a = 0; q < P.sn_rowptr[s + 1]; ++q, ++a) {
                int i = P.sn_rows[q];
                int lr;
                if (i <= P.sn_first[par + 1] - 1) lr = i - P.sn_first[par];
                else {
                    const int* it = std::lower_bound(pb + pnp, pe, i);
                    if (it == pe || *it != i) throw AnalyzeError(-4, "internal: contribution row missing in parent");
                    lr = (int)(it - pb);
                }
                P.rel[P.rel_ptr[s] + a] = lr;
                if (P.sn_large[par]) P.inv[P.inv_ptr[s] + lr] = (int)a;
            }
        }

        // ---------------- levels -------------------------------------------
        P.sn_level.assign(nsn, 0);
        P.nlevels = 0;
        for (int s = 0; s < nsn; ++s) {
            int lv = 0;
            for (int k = P.child_ptr[s]; k < P.child_ptr[s + 1]; ++k) lv = std::max(lv, P.sn_level[P.child_list[k]] + 1);
            P.sn_level[s] = lv;
            P.nlevels = std::max(P.nlevels, lv + 1);
        }
        P.level_ptr.assign(P.nlevels + 1, 0);
        for (int s = 0; s < nsn; ++s) P.level_ptr[P.sn_level[s] + 1]++;
        for (int l = 0; l < P.nlevels; ++l) P.level_ptr[l + 1] += P.level_ptr[l];
        P.level_list.resize(nsn);
        P.level_fmax.assign(P.nlevels, 0);
        {
            std::vector<int> f(P.level_ptr.begin(), P.level_ptr.end() - 1);
            for (int s = 0; s < nsn; ++s) {
                P.level_list[f[P.sn_level[s]]++] = s;
                P.level_fmax[P.sn_level[s]] =
                    std::max<int>(P.level_fmax[P.sn_level[s]], (int)(P.sn_rowptr[s + 1] - P.sn_rowptr[s]));
            }
        }

        // ---------------- storage -------------------------------------------
        auto align = [](int64_t x) { return (x + 31) & ~(int64_t)31; };
        P.L_off.assign(nsn, 0);
        P.CB_off.assign(nsn, 0);
        P.CB_ld.assign(nsn, 0);
        P.U_off.assign(nsn, 0);
        int64_t off = 0;
        for (int s = 0; s < nsn; ++s) {
            const int64_t f = P.sn_rowptr[s + 1] - P.sn_rowptr[s];
            const int64_t p = P.sn_first[s + 1] - P.sn_first[s];
            P.L_off[s] = off;
            off = align(off + (P.sn_large[s] ? f * f : f * p));
        }
        for (int s = 0; s < nsn; ++s) {
            const int64_t f = P.sn_rowptr[s + 1] - P.sn_rowptr[s];
            const int64_t p = P.sn_first[s + 1] - P.sn_first[s];
            const int64_t c = f - p;
            if (P.sn_large[s]) {
                P.CB_off[s] = P.L_off[s] + p + p * f;
                P.CB_ld[s] = (int)f;
            } else {
                P.CB_off[s] = off;
                P.CB_ld[s] = (int)std::max<int64_t>(c, 1);
                off = align(off + c * c);
            }
        }
        P.factor_elems = std::max<int64_t>(off, 32);
        int64_t uoff = 0;
        for (int s = 0; s < nsn; ++s) {
            const int64_t f = P.sn_rowptr[s + 1] - P.sn_rowptr[s];
            const int64_t p = P.sn_first[s + 1] - P.sn_first[s];
            P.U_off[s] = uoff;
            uoff = align(uoff + (f - p));
        }
        P.U_elems = std::max<int64_t>(uoff, 32);
        P.M_off.assign(nsn, -1);   // -1: small front (no panel inverses)
        int64_t moff = 0;
        for (int s = 0; s < nsn; ++s) {
            if (!P.sn_large[s]) continue;
            const int64_t p = P.sn_first[s + 1] - P.sn_first[s];
            P.M_off[s] = moff;
            moff += ((p + cfg.panel - 1) / cfg.panel) * (int64_t)cfg.panel * cfg.panel;
        }
        P.M_elems = std::max<int64_t>(moff, 32);

        // ---------------- schedule ------------------------------------------
        const int nb = cfg.panel, T = cfg.tile;
        for (int l = 0; l < P.nlevels; ++l) {
            std::vector<int> small, large;
            for (int k = P.level_ptr[l]; k < P.level_ptr[l + 1]; ++k) {
                int s = P.level_list[k];
                (P.sn_large[s] ? large : small).push_back(s);
            }
            std::sort(small.begin(), small.end(), [&](int a, int b) {
                int64_t fa = P.sn_rowptr[a + 1] - P.sn_rowptr[a], fb = P.sn_rowptr[b + 1] - P.sn_rowptr[b];
                return fa != fb ? fa > fb : a < b;
            });
            // batches by front-size class (32-wide), each launch sized for its largest front
            size_t k = 0;
            while (k < small.size()) {
                LevelBatch b;
                b.level = l;
                b.first = (int64_t)P.small_list.size();
                int f0 = (int)(P.sn_rowptr[small[k] + 1] - P.sn_rowptr[small[k]]);
                int cls = (f0 + 31) / 32;
                b.fmax = f0;
                while (k < small.size()) {
                    int fk = (int)(P.sn_rowptr[small[k] + 1] - P.sn_rowptr[small[k]]);
                    if ((fk + 31) / 32 != cls) break;
                    P.small_list.push_back(small[k]);
                    ++k;
                }
                b.count = (int64_t)P.small_list.size() - b.first;
                P.small_batches.push_back(b);
            }
            if (large.empty()) continue;
            LargeStep st;
            st.level = l;
            st.asm_first = (int64_t)P.large_asm.size() / 2;
            for (int s : large) {
                const int f = (int)(P.sn_rowptr[s + 1] - P.sn_rowptr[s]);
                const int np = P.sn_first[s + 1] - P.sn_first[s];
                st.asm_fmax = std::max(st.asm_fmax, f);
                for (int j = 0; j < f; ++j) {
                    P.large_asm.push_back(s); P.large_asm.push_back(j);
                    if (P.asm_seg_ptr.empty()) P.asm_seg_ptr.push_back(0);
                    P.asm_col.push_back(P.L_off[s] + (int64_t)j * f);
                    P.asm_fj.push_back(f); P.asm_fj.push_back(j);
                    if (j < np) {
                        P.asm_kr.push_back(P.kcol_ptr[P.kcol_base[s] + j]);
                        P.asm_kr.push_back(P.kcol_ptr[P.kcol_base[s] + j + 1]);
                    } else {
                        P.asm_kr.push_back(0); P.asm_kr.push_back(0);
                    }
                    for (int k = P.child_ptr[s]; k < P.child_ptr[s + 1]; ++k) {
                        const int ch = P.child_list[k];
                        const int b = P.inv[P.inv_ptr[ch] + j];
                        if (b < 0) continue;
                        const int cc = (int)(P.sn_rowptr[ch + 1] - P.sn_rowptr[ch]) - (P.sn_first[ch + 1] - P.sn_first[ch]);
                        P.asm_seg_cb.push_back(P.CB_off[ch] + (int64_t)b * P.CB_ld[ch]);
                        P.asm_seg_rel.push_back(P.rel_ptr[ch]);
                        P.asm_seg_bc.push_back(b); P.asm_seg_bc.push_back(cc);
                    }
                    P.asm_seg_ptr.push_back((int64_t)P.asm_seg_cb.size());
                }
            }
            st.asm_count = (int64_t)P.large_asm.size() / 2 - st.asm_first;
            int maxp = 0;
            for (int s : large) maxp = std::max(maxp, P.sn_first[s + 1] - P.sn_first[s]);
            for (int k0 = 0; k0 < maxp; k0 += nb) {
                st.diag_first.push_back((int64_t)P.large_diag.size() / 2);
                st.panel_first.push_back((int64_t)P.large_panel.size() / 3);
                st.upd_first.push_back((int64_t)P.large_upd.size() / 4);
                double fl = 0.0;
                for (int s : large) {
                    const int f = (int)(P.sn_rowptr[s + 1] - P.sn_rowptr[s]);
                    const int p = P.sn_first[s + 1] - P.sn_first[s];
                    if (k0 >= p) continue;
                    const int k1 = std::min(k0 + nb, p);
                    P.large_diag.push_back(s); P.large_diag.push_back(k0);
                    for (int r0 = k1; r0 < f; r0 += 32) {
                        P.large_panel.push_back(s); P.large_panel.push_back(k0); P.large_panel.push_back(r0);
                    }
                    for (int j0 = k1; j0 < f; j0 += T)
                        for (int i0 = j0; i0 < f; i0 += T) {
                            if (i0 == k1 && j0 == k1 && k1 < p) continue;   // the next diagonal block
                            P.large_upd.push_back(s); P.large_upd.push_back(k0);
                            P.large_upd.push_back(i0); P.large_upd.push_back(j0);
                            double ri = std::min(T, f - i0), rj = std::min(T, f - j0);
                            double ent = (i0 == j0) ? ri * (ri + 1) / 2 : ri * rj;
                            fl += 2.0 * ent * (k1 - k0) * P.sn_flop_ratio[s];
                        }
                }
                st.diag_count.push_back((int64_t)P.large_diag.size() / 2 - st.diag_first.back());
                st.panel_count.push_back((int64_t)P.large_panel.size() / 3 - st.panel_first.back());
                st.upd_count.push_back((int64_t)P.large_upd.size() / 4 - st.upd_first.back());
                st.upd_flops.push_back(fl);
            }
            P.large_steps.push_back(std::move(st));
        }
        // ---------------- persistent launches ------------------------------
        {
            P.pers_order.resize(nsn);
            std::iota(P.pers_order.begin(), P.pers_order.end(), 0);
            std::stable_sort(P.pers_order.begin(), P.pers_order.end(), [&](int a, int b) {
                if (P.sn_level[a] != P.sn_level[b]) return P.sn_level[a] < P.sn_level[b];
                return P.sn_rowptr[a + 1] - P.sn_rowptr[a] > P.sn_rowptr[b + 1] - P.sn_rowptr[b];
            });
            P.pers_asm.assign(2 * (size_t)nsn, 0);
            for (size_t t = 0; t < P.large_asm.size() / 2; ++t) {
                const int s = P.large_asm[2 * t];
                if (P.pers_asm[2 * s + 1] == 0) P.pers_asm[2 * s] = (int64_t)t;
                P.pers_asm[2 * s + 1]++;
            }
            P.sys_nfronts.assign(P.S, 0);
            for (int s = 0; s < nsn; ++s) {
                P.sys_nfronts[P.sn_sys[s]]++;
                const int f = (int)(P.sn_rowptr[s + 1] - P.sn_rowptr[s]);
                P.pers_fmax = std::max(P.pers_fmax, f);
                if (P.sn_large[s]) P.pers_fmax_large = std::max(P.pers_fmax_large, f);
                else P.pers_fmax_small = std::max(P.pers_fmax_small, f);
            }
        }
        // ---------------- solve schedule -----------------------------------
        {
            const int PW = 64;   // kPanel
            // rows per task: the panel's columns are taken 16 at a time by the
            // four waves, the rest of the workgroup takes more rows
            auto task_rows = [](int w) { return 64 * (4 / ((w + 15) / 16)); };
            // entries [a0, a1) of child ch's update vector landing in parent rows [lo, hi)
            auto child_range = [&](int ch, int lo, int hi, int& a0, int& a1) {
                const int* r = P.rel.data() + P.rel_ptr[ch];
                const int cc = (int)(P.rel_ptr[ch + 1] - P.rel_ptr[ch]);
                a0 = (int)(std::lower_bound(r, r + cc, lo) - r);
                a1 = (int)(std::lower_bound(r, r + cc, hi) - r);
            };
            for (int s = 0; s < nsn; ++s)
                for (int64_t q = P.rel_ptr[s] + 1; q < P.rel_ptr[s + 1]; ++q)
                    if (P.rel[q] <= P.rel[q - 1]) throw AnalyzeError(-4, "internal: update-vector map not increasing");
            std::vector<std::vector<int>> sn_pids(nsn);   // panels of each front, in column order
            std::vector<int64_t> pan_task0;               // first task of each panel
            for (int l = 0; l < P.nlevels; ++l) {
                int maxj = 0;
                for (int k = P.level_ptr[l]; k < P.level_ptr[l + 1]; ++k) {
                    int s = P.level_list[k];
                    int p = P.sn_first[s + 1] - P.sn_first[s];
                    maxj = std::max(maxj, (p + PW - 1) / PW);
                }
                for (int j = 0; j < maxj; ++j) {
                    SolveStep st;
                    st.level = l; st.j = j;
                    st.p_first = (int64_t)P.solve_p.size() / 6;
                    st.s_first = (int64_t)P.solve_s.size();
                    int slot = 0;
                    for (int k = P.level_ptr[l]; k < P.level_ptr[l + 1]; ++k) {
                        int s = P.level_list[k];
                        const int p = P.sn_first[s + 1] - P.sn_first[s];
                        const int f = (int)(P.sn_rowptr[s + 1] - P.sn_rowptr[s]);
                        const int c0 = j * PW;
                        if (c0 >= p) continue;
                        const int w = std::min(PW, p - c0);
                        const int below = f - c0 - w;
                        st.fwd_bytes += 8.0 * ((double)w * (w + 1) / 2.0 + (double)below * w) * P.sn_nnz_ratio[s];
                        if (!P.sn_large[s] && p <= 64 && f <= 128) {
                            P.solve_s.push_back(s);
                            continue;
                        }
                        const int pid = (int)(P.solve_pan.size() / 7);
                        sn_pids[s].push_back(pid);
                        pan_task0.push_back((int64_t)P.solve_p.size() / 6);
                        const int GR = task_rows(w);
                        if (!P.sn_large[s] && below > 64)
                            throw AnalyzeError(-4, "internal: LDS-path front with more than 64 rows below a panel");
                        const int ntask = std::max(1, (below + GR - 1) / GR);
                        const int seg0 = (int)(P.solve_seg.size() / 3);
                        if (c0 == 0)
                            for (int q = P.child_ptr[s]; q < P.child_ptr[s + 1]; ++q) {
                                int a0, a1;
                                child_range(P.child_list[q], 0, w, a0, a1);
                                if (a1 > a0) { P.solve_seg.push_back(P.child_list[q]); P.solve_seg.push_back(a0); P.solve_seg.push_back(a1); }
                            }
                        const int nseg = (int)(P.solve_seg.size() / 3) - seg0;
                        for (int v : {s, c0, w, slot, ntask, seg0, nseg}) P.solve_pan.push_back(v);
                        for (int t = 0; t < ntask; ++t) {
                            const int r0 = below > 0 ? c0 + w + t * GR : f;
                            const int r1 = below > 0 ? std::min(f, r0 + GR) : f;
                            const int tseg0 = (int)(P.solve_seg.size() / 3);
                            if (c0 == 0 && r1 > r0)
                                for (int q = P.child_ptr[s]; q < P.child_ptr[s + 1]; ++q) {
                                    int a0, a1;
                                    child_range(P.child_list[q], r0, r1, a0, a1);
                                    if (a1 > a0) { P.solve_seg.push_back(P.child_list[q]); P.solve_seg.push_back(a0); P.solve_seg.push_back(a1); }
                                }
                            const int tnseg = (int)(P.solve_seg.size() / 3) - tseg0;
                            for (int v : {pid, r0, r1, t, tseg0, tnseg}) P.solve_p.push_back(v);
                        }
                        slot += ntask;
                    }
                    st.p_count = (int64_t)P.solve_p.size() / 6 - st.p_first;
                    st.s_count = (int64_t)P.solve_s.size() - st.s_first;
                    P.solve_max_slots = std::max<int64_t>(P.solve_max_slots, slot);
                    P.solve_steps.push_back(st);
                }
            }
            // Backward: a panel swept by several tasks is finished (its x from
            // the tasks' sums) by the first task of the front's previous panel,
            // whose rows start with it; a front's first panel by a finish-only
            // record launched after its level's last step.
            const int64_t nreg = (int64_t)P.solve_p.size() / 6;
            P.solve_fin.assign(4 * (size_t)nreg, 0);
            auto fin_fields = [&](int pid, int* out) {
                const int* pn = P.solve_pan.data() + 7 * (size_t)pid;
                out[0] = pn[1]; out[1] = pn[2]; out[2] = pn[3]; out[3] = pn[4];
            };
            for (int s = 0; s < nsn; ++s) {
                const std::vector<int>& pids = sn_pids[s];
                for (size_t j = 0; j + 1 < pids.size(); ++j) {
                    if (P.solve_pan[7 * (size_t)pids[j + 1] + 4] <= 1) continue;
                    if (!P.sn_large[s]) throw AnalyzeError(-4, "internal: multi-task panel in an LDS-path front");
                    const int64_t t0 = pan_task0[pids[j]];
                    if (P.solve_p[6 * t0 + 3] != 0 || P.solve_p[6 * t0 + 1] != P.solve_pan[7 * (size_t)pids[j + 1] + 1] ||
                        P.solve_pan[7 * (size_t)pids[j] + 4] <= 1)
                        throw AnalyzeError(-4, "internal: first task of a panel does not start at the next panel");
                    fin_fields(pids[j + 1], P.solve_fin.data() + 4 * t0);
                }
            }
            for (SolveStep& st : P.solve_steps) {
                if (st.j != 0) continue;
                st.f_first = (int64_t)P.solve_p.size() / 6;
                for (int k = P.level_ptr[st.level]; k < P.level_ptr[st.level + 1]; ++k) {
                    const int s = P.level_list[k];
                    if (sn_pids[s].empty()) continue;
                    const int pid = sn_pids[s][0];
                    if (P.solve_pan[7 * (size_t)pid + 4] <= 1) continue;
                    const int f = (int)(P.sn_rowptr[s + 1] - P.sn_rowptr[s]);
                    for (int v : {pid, f, f, -1, 0, 0}) P.solve_p.push_back(v);
                    int fin[4];
                    fin_fields(pid, fin);
                    for (int v : fin) P.solve_fin.push_back(v);
                }
                st.f_count = (int64_t)P.solve_p.size() / 6 - st.f_first;
            }
            // Forward: a large front's panels are taken two at a time (2k and
            // 2k + 1 in step k of its level): its tasks own the rows below the
            // second panel, 64 each, and form both panels' y themselves.  Other
            // fronts keep one panel per step.  Tasks refer to the first
            // panel's record; solve_fx holds (w of the second panel or 0, its
            // pivot rows' contribution segments (first, count), 0).
            {
                std::vector<int64_t> s_first_of(P.nlevels, 0), s_count_of(P.nlevels, 0);
                for (const SolveStep& st : P.solve_steps)
                    if (st.j == 0) { s_first_of[st.level] = st.s_first; s_count_of[st.level] = st.s_count; }
                for (int l = 0; l < P.nlevels; ++l) {
                    int maxk = 0;
                    for (int k = P.level_ptr[l]; k < P.level_ptr[l + 1]; ++k) {
                        const int s = P.level_list[k];
                        const int np = (int)sn_pids[s].size();
                        maxk = std::max(maxk, P.sn_large[s] ? (np + 1) / 2 : np);
                    }
                    if (s_count_of[l] > 0) maxk = std::max(maxk, 1);
                    for (int kk = 0; kk < maxk; ++kk) {
                        SolveStep st;
                        st.level = l; st.j = kk;
                        st.p_first = (int64_t)P.fsolve_p.size() / 6;
                        if (kk == 0) { st.s_first = s_first_of[l]; st.s_count = s_count_of[l]; }
                        for (int k = P.level_ptr[l]; k < P.level_ptr[l + 1]; ++k) {
                            const int s = P.level_list[k];
                            const std::vector<int>& pids = sn_pids[s];
                            const bool lg = P.sn_large[s] != 0;
                            const size_t j = lg ? 2 * (size_t)kk : (size_t)kk;
                            if (j >= pids.size()) continue;
                            const int pid = pids[j];
                            const int* pn = P.solve_pan.data() + 7 * (size_t)pid;
                            const int c0 = pn[1], w = pn[2];
                            const int f = (int)(P.sn_rowptr[s + 1] - P.sn_rowptr[s]);
                            const int w2 = (lg && j + 1 < pids.size()) ? P.solve_pan[7 * (size_t)pids[j + 1] + 2] : 0;
                            if (w2 > 0 && w != PW) throw AnalyzeError(-4, "internal: paired panel narrower than 64");
                            auto bytes = [&](int cc, int ww) {
                                const int below = f - cc - ww;
                                return 8.0 * ((double)ww * (ww + 1) / 2.0 + (double)below * ww) * P.sn_nnz_ratio[s];
                            };
                            st.fwd_bytes += bytes(c0, w) + (w2 > 0 ? bytes(c0 + w, w2) : 0.0);
                            const int rs = c0 + w + w2;                 // first row below the step's panels
                            const int below = f - rs;
                            const int GR = w2 > 0 ? 64 : task_rows(w);
                            const int ntask = std::max(1, (below + GR - 1) / GR);
                            int s2seg0 = (int)(P.solve_seg.size() / 3), s2nseg = 0;
                            if (w2 > 0 && c0 == 0) {
                                for (int q = P.child_ptr[s]; q < P.child_ptr[s + 1]; ++q) {
                                    int a0, a1;
                                    child_range(P.child_list[q], w, w + w2, a0, a1);
                                    if (a1 > a0) { P.solve_seg.push_back(P.child_list[q]); P.solve_seg.push_back(a0); P.solve_seg.push_back(a1); }
                                }
                                s2nseg = (int)(P.solve_seg.size() / 3) - s2seg0;
                            }
                            for (int t = 0; t < ntask; ++t) {
                                const int r0 = below > 0 ? rs + t * GR : f;
                                const int r1 = below > 0 ? std::min(f, r0 + GR) : f;
                                const int tseg0 = (int)(P.solve_seg.size() / 3);
                                if (c0 == 0 && r1 > r0)
                                    for (int q = P.child_ptr[s]; q < P.child_ptr[s + 1]; ++q) {
                                        int a0, a1;
                                        child_range(P.child_list[q], r0, r1, a0, a1);
                                        if (a1 > a0) { P.solve_seg.push_back(P.child_list[q]); P.solve_seg.push_back(a0); P.solve_seg.push_back(a1); }
                                    }
                                const int tnseg = (int)(P.solve_seg.size() / 3) - tseg0;
                                for (int v : {pid, r0, r1, t, tseg0, tnseg}) P.fsolve_p.push_back(v);
                                for (int v : {w2, s2seg0, s2nseg, 0}) P.fsolve_x.push_back(v);
                            }
                        }
                        st.p_count = (int64_t)P.fsolve_p.size() / 6 - st.p_first;
                        P.fsolve_steps.push_back(st);
                    }
                }
            }
        }
    } catch (const AnalyzeError& e) {
        err = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        err = "host allocation failed";
        return -3;
    }
    P.analyze_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return 0;
}

}  // namespace ncl
