/*
 * ncl_oracle.c — plain, slow, FP64 reference for the NCL KKT hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark call into this file.  It shares no code,
 * header, table or helper with the GPU library and never calls it.
 *
 * What it computes (paper: "MadNCL", Sec. 3):
 *   - the condensed matrix K1 = W + Sigma + rho J^T J (Sec. 3.3, eq. K1), SPD
 *     when W + Sigma is;
 *   - the stabilized matrix K2r = [[W + Sigma, J^T], [J, -(1/rho) I]]
 *     (Sec. 3.2, eq. K2r), symmetric quasi-definite;
 *   - a fill-reducing minimum-degree ordering (any symmetric permutation is
 *     admissible for both matrices, Sec. 3.2: SQD matrices are strongly
 *     factorizable);
 *   - an LDL^T factorization without pivoting, row by row ("up-looking"),
 *     with static pivoting (Sec. 3.1, "Sparse LDL^T factorization"): a pivot
 *     with |d| below the threshold is replaced by the threshold with the sign
 *     of the block (before reordering) the pivot belongs to;
 *   - the inertia read off D (Sylvester's law, Sec. 3.4, Prop. "inertia");
 *   - solves x = P^T L^-T D^-1 L^-1 P b and the product y = K x.
 *
 * All indices are 0-based int32, all values double.  Matrices in "lower CSC"
 * store, for each column j, the rows i >= j in increasing order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_ALLOC -3
#define OR_ERR_NONFINITE -6
#define OR_ERR_ZERO_PIVOT -7

/* ------------------------------------------------------------------------- */
/* Assembly                                                                   */
/* ------------------------------------------------------------------------- */

/* Column-wise transpose of J (CSR m x n) -> CSC arrays (Tp[n+1], Tr[nnz], Tv[nnz]);
 * within each column the row indices r come out increasing.  Tv stores the
 * position of each entry in J's value array. */
static int transpose_J(int n, int m, const int *Jp, const int *Jj, int **Tp_, int **Tr_, int **Tv_)
{
    int nnz = Jp[m];
    int *Tp = calloc((size_t)n + 1, sizeof(int));
    int *Tr = malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    int *Tv = malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    int *w = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!Tp || !Tr || !Tv || !w) { free(Tp); free(Tr); free(Tv); free(w); return OR_ERR_ALLOC; }
    for (int k = 0; k < nnz; ++k) Tp[Jj[k] + 1]++;
    for (int j = 0; j < n; ++j) Tp[j + 1] += Tp[j];
    memcpy(w, Tp, sizeof(int) * (size_t)n);
    for (int r = 0; r < m; ++r)
        for (int k = Jp[r]; k < Jp[r + 1]; ++k) {
            int q = w[Jj[k]]++;
            Tr[q] = r;
            Tv[q] = k;
        }
    free(w);
    *Tp_ = Tp; *Tr_ = Tr; *Tv_ = Tv;
    return OR_OK;
}

/* Condensed matrix K = W + diag(Sigma) + rho * J^T J, lower CSC (Sec. 3.3, eq. K1).
 * Pattern = pattern(W) U diagonal U {(i,j): some row r of J has J_ri, J_rj != 0}.
 * If Ki == NULL only Kp is filled (pattern count pass).  Entry values:
 *   K_ij = (W_ij + [i==j] Sigma_i) + rho * s_ij,  s_ij = sum over r (increasing) of J_ri J_rj.
 * Returns nnz(K lower) or a negative error. */
int64_t or_condensed_assemble(int n, int m, const int *Wp, const int *Wi, const double *Wx,
                              const double *Sigma, const int *Jp, const int *Jj, const double *Jx,
                              double rho, int *Kp, int *Ki, double *Kx)
{
    int *Tp, *Tr, *Tv;
    if (transpose_J(n, m, Jp, Jj, &Tp, &Tr, &Tv)) return OR_ERR_ALLOC;
    int *mark = malloc(sizeof(int) * (size_t)n);
    int *list = malloc(sizeof(int) * (size_t)n);
    double *acc = calloc((size_t)n, sizeof(double));
    double *wv = calloc((size_t)n, sizeof(double));
    if (!mark || !list || !acc || !wv) { free(Tp); free(Tr); free(Tv); free(mark); free(list); free(acc); free(wv); return OR_ERR_ALLOC; }
    for (int i = 0; i < n; ++i) mark[i] = -1;
    int64_t nz = 0;
    for (int j = 0; j < n; ++j) {
        int cnt = 0;
        mark[j] = j; list[cnt++] = j;
        for (int p = Wp[j]; p < Wp[j + 1]; ++p) {
            int i = Wi[p];
            if (mark[i] != j) { mark[i] = j; list[cnt++] = i; }
        }
        for (int q = Tp[j]; q < Tp[j + 1]; ++q) {
            int r = Tr[q];
            for (int k = Jp[r]; k < Jp[r + 1]; ++k) {
                int i = Jj[k];
                if (i >= j && mark[i] != j) { mark[i] = j; list[cnt++] = i; }
            }
        }
        if (Ki) {
            /* sort the row list (insertion sort: columns are short) */
            for (int a = 1; a < cnt; ++a) {
                int v = list[a], b = a - 1;
                while (b >= 0 && list[b] > v) { list[b + 1] = list[b]; --b; }
                list[b + 1] = v;
            }
            for (int a = 0; a < cnt; ++a) { acc[list[a]] = 0.0; wv[list[a]] = 0.0; }
            for (int p = Wp[j]; p < Wp[j + 1]; ++p) wv[Wi[p]] += Wx[p];
            wv[j] += Sigma[j];
            for (int q = Tp[j]; q < Tp[j + 1]; ++q) {       /* increasing r */
                int r = Tr[q];
                double jrj = Jx[Tv[q]];
                for (int k = Jp[r]; k < Jp[r + 1]; ++k) {
                    int i = Jj[k];
                    if (i >= j) acc[i] += Jx[k] * jrj;
                }
            }
            for (int a = 0; a < cnt; ++a) {
                int i = list[a];
                Ki[nz + a] = i;
                Kx[nz + a] = wv[i] + rho * acc[i];
            }
        }
        Kp[j] = (int)nz;
        nz += cnt;
    }
    Kp[n] = (int)nz;
    free(Tp); free(Tr); free(Tv); free(mark); free(list); free(acc); free(wv);
    return nz;
}

/* Stabilized matrix K2r = [[W + Sigma, J^T], [J, -(1/rho) I]] of order n + m,
 * lower CSC (Sec. 3.2, eq. K2r).  Column j < n holds W's column j (with Sigma_j
 * added on the diagonal, which is always stored) followed by rows n + r for
 * every J_rj != 0; column n + r holds only the diagonal -1/rho.
 * If Ki == NULL only Kp is filled.  Returns nnz or a negative error. */
int64_t or_stabilized_assemble(int n, int m, const int *Wp, const int *Wi, const double *Wx,
                               const double *Sigma, const int *Jp, const int *Jj, const double *Jx,
                               double rho, int *Kp, int *Ki, double *Kx)
{
    int *Tp, *Tr, *Tv;
    if (transpose_J(n, m, Jp, Jj, &Tp, &Tr, &Tv)) return OR_ERR_ALLOC;
    int64_t nz = 0;
    for (int j = 0; j < n; ++j) {
        Kp[j] = (int)nz;
        int has_diag = (Wp[j] < Wp[j + 1] && Wi[Wp[j]] == j);
        if (!has_diag) {
            if (Ki) { Ki[nz] = j; Kx[nz] = Sigma[j]; }
            ++nz;
        }
        for (int p = Wp[j]; p < Wp[j + 1]; ++p) {
            if (Ki) { Ki[nz] = Wi[p]; Kx[nz] = Wx[p] + (Wi[p] == j ? Sigma[j] : 0.0); }
            ++nz;
        }
        for (int q = Tp[j]; q < Tp[j + 1]; ++q) {
            if (Ki) { Ki[nz] = n + Tr[q]; Kx[nz] = Jx[Tv[q]]; }
            ++nz;
        }
    }
    for (int r = 0; r < m; ++r) {
        Kp[n + r] = (int)nz;
        if (Ki) { Ki[nz] = n + r; Kx[nz] = -1.0 / rho; }
        ++nz;
    }
    Kp[n + m] = (int)nz;
    free(Tp); free(Tr); free(Tv);
    return nz;
}

/* y = K x for a symmetric K given by its lower CSC; nrhs columns, column-major. */
void or_symv(int N, const int *Kp, const int *Ki, const double *Kx, int nrhs,
             const double *X, int ldx, double *Y, int ldy)
{
    for (int c = 0; c < nrhs; ++c) {
        const double *x = X + (size_t)c * ldx;
        double *y = Y + (size_t)c * ldy;
        for (int i = 0; i < N; ++i) y[i] = 0.0;
        for (int j = 0; j < N; ++j)
            for (int p = Kp[j]; p < Kp[j + 1]; ++p) {
                int i = Ki[p];
                y[i] += Kx[p] * x[j];
                if (i != j) y[j] += Kx[p] * x[i];
            }
    }
}

/* max_ij |K_ij| and max_i sum_j |K_ij| of a symmetric K in lower CSC. */
void or_norms(int N, const int *Kp, const int *Ki, const double *Kx, double *maxabs, double *infnorm)
{
    double *rs = calloc((size_t)N, sizeof(double));
    double mx = 0.0;
    for (int j = 0; j < N; ++j)
        for (int p = Kp[j]; p < Kp[j + 1]; ++p) {
            double a = fabs(Kx[p]);
            if (a > mx) mx = a;
            rs[Ki[p]] += a;
            if (Ki[p] != j) rs[j] += a;
        }
    double inf = 0.0;
    for (int i = 0; i < N; ++i) if (rs[i] > inf) inf = rs[i];
    free(rs);
    *maxabs = mx;
    *infnorm = inf;
}

/* ------------------------------------------------------------------------- */
/* Minimum-degree ordering on the quotient graph                              */
/* ------------------------------------------------------------------------- */

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

typedef struct { int *a; int len, cap; } ivec;

static int iv_push(ivec *v, int x)
{
    if (v->len == v->cap) {
        int nc = v->cap ? 2 * v->cap : 4;
        int *na = realloc(v->a, sizeof(int) * (size_t)nc);
        if (!na) return OR_ERR_ALLOC;
        v->a = na; v->cap = nc;
    }
    v->a[v->len++] = x;
    return OR_OK;
}

static void iv_free(ivec *v) { free(v->a); v->a = NULL; v->len = v->cap = 0; }

/* Plain minimum-degree ordering on a quotient graph.
 *
 * 1. Vertices with identical closed neighbourhoods (indistinguishable
 *    vertices) are merged once, up front, into weighted supervariables.
 * 2. Repeatedly the supervariable p of least weighted degree (sum of the
 *    weights of the distinct supervariables reachable from it) is
 *    eliminated: it becomes an element whose variable list is its reach, and
 *    the elements adjacent to p are absorbed into it.  Degrees are recomputed
 *    exactly for every supervariable in the new element.  Ties go to the most
 *    recently inserted supervariable of the lowest degree bucket.
 * 3. When p is adjacent to every remaining supervariable the rest is a clique
 *    and is appended as is (any order gives the same fill).
 * Members of a supervariable are numbered consecutively, in increasing index.
 * perm[k] = original index of the k-th pivot. */
static uint64_t mix64(uint64_t x)
{
    x ^= x >> 33; x *= 0xff51afd7ed558ccdULL; x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL; x ^= x >> 33;
    return x;
}

static const uint64_t *g_hash_key;
static int cmp_by_hash(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    if (g_hash_key[x] != g_hash_key[y]) return g_hash_key[x] < g_hash_key[y] ? -1 : 1;
    return (x > y) - (x < y);
}

int or_mindeg(int N, const int *Ap, const int *Ai, int *perm)
{
    int rc = OR_OK;
    int *Gp = calloc((size_t)N + 1, sizeof(int)), *Gi = NULL;
    int *rep = malloc(sizeof(int) * (size_t)N), *wgt = calloc((size_t)N, sizeof(int));
    int *order = malloc(sizeof(int) * (size_t)N), *fill = malloc(sizeof(int) * (size_t)N);
    uint64_t *hv = malloc(sizeof(uint64_t) * (size_t)N);
    ivec *V = calloc((size_t)N, sizeof(ivec));   /* variable neighbours */
    ivec *E = calloc((size_t)N, sizeof(ivec));   /* element neighbours */
    ivec *L = calloc((size_t)N, sizeof(ivec));   /* element variable lists */
    ivec *members = calloc((size_t)N, sizeof(ivec));
    int *status = calloc((size_t)N, sizeof(int)); /* 0 var, 1 element, 2 absorbed, 3 merged away */
    int *deg = malloc(sizeof(int) * (size_t)N);
    int *head = malloc(sizeof(int) * ((size_t)N + 1));
    int *next = malloc(sizeof(int) * (size_t)N);
    int *prev = malloc(sizeof(int) * (size_t)N);
    int64_t *mark = calloc((size_t)N, sizeof(int64_t));
    int64_t stamp = 0;
    if (!Gp || !rep || !wgt || !order || !fill || !hv || !V || !E || !L || !members || !status || !deg ||
        !head || !next || !prev || !mark) { rc = OR_ERR_ALLOC; goto done; }

    /* full adjacency, diagonal dropped, rows sorted (filled in column order) */
    for (int j = 0; j < N; ++j)
        for (int p = Ap[j]; p < Ap[j + 1]; ++p)
            if (Ai[p] != j) { Gp[Ai[p] + 1]++; Gp[j + 1]++; }
    for (int v = 0; v < N; ++v) Gp[v + 1] += Gp[v];
    Gi = malloc(sizeof(int) * (size_t)(Gp[N] > 0 ? Gp[N] : 1));
    if (!Gi) { rc = OR_ERR_ALLOC; goto done; }
    memcpy(fill, Gp, sizeof(int) * (size_t)N);
    for (int j = 0; j < N; ++j)
        for (int p = Ap[j]; p < Ap[j + 1]; ++p) {
            int i = Ai[p];
            if (i == j) continue;
            Gi[fill[i]++] = j;
            Gi[fill[j]++] = i;
        }
    for (int v = 0; v < N; ++v)
        qsort(Gi + Gp[v], (size_t)(Gp[v + 1] - Gp[v]), sizeof(int), cmp_int);

    /* indistinguishable vertices: equal closed neighbourhoods */
    for (int v = 0; v < N; ++v) {
        uint64_t h = mix64((uint64_t)v + 1);
        for (int p = Gp[v]; p < Gp[v + 1]; ++p) h += mix64((uint64_t)Gi[p] + 1);
        hv[v] = h ^ mix64((uint64_t)(Gp[v + 1] - Gp[v]) * 0x9e3779b97f4a7c15ULL);
        order[v] = v;
        rep[v] = v;
    }
    g_hash_key = hv;
    qsort(order, (size_t)N, sizeof(int), cmp_by_hash);
    for (int a = 0; a < N;) {
        int b = a;
        while (b < N && hv[order[b]] == hv[order[a]]) ++b;
        for (int x = a; x < b; ++x) {
            int u = order[x];
            if (rep[u] != u) continue;
            for (int y = x + 1; y < b; ++y) {
                int v = order[y];
                if (rep[v] != v || Gp[u + 1] - Gp[u] != Gp[v + 1] - Gp[v]) continue;
                /* compare N[u] and N[v] (closed) */
                ++stamp;
                mark[u] = stamp;
                for (int p = Gp[u]; p < Gp[u + 1]; ++p) mark[Gi[p]] = stamp;
                int same = (mark[v] == stamp);
                for (int p = Gp[v]; same && p < Gp[v + 1]; ++p)
                    if (mark[Gi[p]] != stamp) same = 0;
                if (same) rep[v] = u;
            }
        }
        a = b;
    }
    for (int v = 0; v < N; ++v) {
        if (iv_push(&members[rep[v]], v)) { rc = OR_ERR_ALLOC; goto done; }
        wgt[rep[v]]++;
        if (rep[v] != v) status[v] = 3;
    }
    /* quotient graph on the supervariables */
    for (int v = 0; v < N; ++v) {
        if (status[v] == 3) continue;
        ++stamp;
        mark[v] = stamp;
        for (int p = Gp[v]; p < Gp[v + 1]; ++p) {
            int r = rep[Gi[p]];
            if (mark[r] != stamp) { mark[r] = stamp; if (iv_push(&V[v], r)) { rc = OR_ERR_ALLOC; goto done; } }
        }
    }
    free(Gi); Gi = NULL;

    for (int d = 0; d <= N; ++d) head[d] = -1;
    int nleft = 0;
    for (int v = 0; v < N; ++v) {
        if (status[v] == 3) continue;
        int d = 0;
        for (int a = 0; a < V[v].len; ++a) d += wgt[V[v].a[a]];
        deg[v] = d;
        next[v] = head[d]; prev[v] = -1;
        if (head[d] >= 0) prev[head[d]] = v;
        head[d] = v;
        nleft += wgt[v];
    }
    int mindeg = 0, k = 0;
    while (k < N) {
        while (head[mindeg] < 0) ++mindeg;
        int p = head[mindeg];
        if (mindeg == nleft - wgt[p]) {
            /* p sees every remaining supervariable: the remainder is a clique */
            for (int d = mindeg; d <= N; ++d)
                for (int v = head[d]; v >= 0; v = next[v])
                    for (int a = 0; a < members[v].len; ++a) perm[k++] = members[v].a[a];
            break;
        }
        head[mindeg] = next[p];
        if (next[p] >= 0) prev[next[p]] = -1;
        for (int a = 0; a < members[p].len; ++a) perm[k++] = members[p].a[a];
        nleft -= wgt[p];

        /* new element p: reach of p through variables and elements */
        ++stamp;
        mark[p] = stamp;
        ivec Lp = {0};
        for (int a = 0; a < V[p].len; ++a) {
            int u = V[p].a[a];
            if (status[u] == 0 && mark[u] != stamp) { mark[u] = stamp; if (iv_push(&Lp, u)) { rc = OR_ERR_ALLOC; goto done; } }
        }
        for (int a = 0; a < E[p].len; ++a) {
            int e = E[p].a[a];
            if (status[e] != 1) continue;
            for (int b = 0; b < L[e].len; ++b) {
                int u = L[e].a[b];
                if (status[u] == 0 && mark[u] != stamp) { mark[u] = stamp; if (iv_push(&Lp, u)) { rc = OR_ERR_ALLOC; goto done; } }
            }
            status[e] = 2;
            iv_free(&L[e]);
        }
        status[p] = 1;
        iv_free(&V[p]);
        iv_free(&E[p]);
        L[p] = Lp;
        int64_t in_lp = stamp;

        for (int a = 0; a < Lp.len; ++a) {
            int u = Lp.a[a];
            int w = 0;
            for (int b = 0; b < E[u].len; ++b)
                if (status[E[u].a[b]] == 1) E[u].a[w++] = E[u].a[b];
            E[u].len = w;
            if (iv_push(&E[u], p)) { rc = OR_ERR_ALLOC; goto done; }
            w = 0;
            for (int b = 0; b < V[u].len; ++b) {
                int x = V[u].a[b];
                if (status[x] == 0 && mark[x] != in_lp) V[u].a[w++] = x;
            }
            V[u].len = w;
        }
        for (int a = 0; a < Lp.len; ++a) {
            int u = Lp.a[a];
            ++stamp;
            mark[u] = stamp;
            int d = 0;
            for (int b = 0; b < V[u].len; ++b) {
                int x = V[u].a[b];
                if (mark[x] != stamp) { mark[x] = stamp; d += wgt[x]; }
            }
            for (int b = 0; b < E[u].len; ++b) {
                const ivec *le = &L[E[u].a[b]];
                for (int c = 0; c < le->len; ++c) {
                    int x = le->a[c];
                    if (status[x] == 0 && mark[x] != stamp) { mark[x] = stamp; d += wgt[x]; }
                }
            }
            if (prev[u] >= 0) next[prev[u]] = next[u]; else head[deg[u]] = next[u];
            if (next[u] >= 0) prev[next[u]] = prev[u];
            deg[u] = d;
            prev[u] = -1; next[u] = head[d];
            if (head[d] >= 0) prev[head[d]] = u;
            head[d] = u;
            if (d < mindeg) mindeg = d;
        }
    }
done:
    if (V) for (int v = 0; v < N; ++v) iv_free(&V[v]);
    if (E) for (int v = 0; v < N; ++v) iv_free(&E[v]);
    if (L) for (int v = 0; v < N; ++v) iv_free(&L[v]);
    if (members) for (int v = 0; v < N; ++v) iv_free(&members[v]);
    free(Gp); free(Gi); free(rep); free(wgt); free(order); free(fill); free(hv);
    free(V); free(E); free(L); free(members); free(status); free(deg); free(head); free(next); free(prev);
    free(mark);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Up-looking LDL^T with static pivoting                                      */
/* ------------------------------------------------------------------------- */

typedef struct or_ldl {
    int N;
    int *perm;      /* perm[k] = original index of pivot k */
    int *Lp;        /* strictly lower L, CSC in the permuted ordering */
    int *Li;
    double *Lx;
    double *D;
    int64_t npos, nneg, nzero, nperturbed;
} or_ldl;

void or_free(or_ldl *F)
{
    if (!F) return;
    free(F->perm); free(F->Lp); free(F->Li); free(F->Lx); free(F->D); free(F);
}

/* Nodes of row k's pattern in L: all etree ancestors of the columns j < k of
 * row k of the permuted matrix, up to (excluding) k.  Written to out[], count
 * returned; flag[] marks visited nodes with k. */
static int row_reach(int k, const int *Rp, const int *Rj, const int *parent, int *flag, int *out)
{
    int cnt = 0;
    flag[k] = k;
    for (int q = Rp[k]; q < Rp[k + 1]; ++q) {
        int i = Rj[q];
        while (flag[i] != k) {
            flag[i] = k;
            out[cnt++] = i;
            i = parent[i];
        }
    }
    return cnt;
}


/* Factor P K P^T = L D L^T, K symmetric in lower CSC (original ordering),
 * perm[k] = original index of pivot k.  Static pivot (Sec. 3.1): pivot k
 * belongs to the primal block when sign[perm[k]] > 0 and to the dual block
 * otherwise (blocks of the unpermuted matrix); its threshold t is thr_primal
 * or thr_dual accordingly.  When |d_k| < t (strict), d_k is replaced by t for
 * a primal pivot and by -t for a dual pivot.  A threshold <= 0 disables the
 * rule for its block.  With one global threshold both are equal; with
 * block-scaled thresholds each block uses its own norm (the -1/rho block of
 * Sec. 3.2, eq. K2r, is then measured against 1/rho, not against W + Sigma).
 * On NaN/Inf: status -6; on an exact zero pivot that the rule did not
 * replace: status -7. */
or_ldl *or_factor(int N, const int *Kp, const int *Ki, const double *Kx, const int *perm,
                  const signed char *sign, double thr_primal, double thr_dual, int *status)
{
    *status = OR_OK;
    or_ldl *F = calloc(1, sizeof(or_ldl));
    int *iperm = malloc(sizeof(int) * (size_t)N);
    int *Rp = calloc((size_t)N + 1, sizeof(int));
    int *parent = malloc(sizeof(int) * (size_t)N);
    int *anc = malloc(sizeof(int) * (size_t)N);
    int *flag = malloc(sizeof(int) * (size_t)N);
    int *pat = malloc(sizeof(int) * (size_t)N);
    int *len = calloc((size_t)N, sizeof(int));
    double *x = calloc((size_t)N, sizeof(double));
    double *Cd = calloc((size_t)N, sizeof(double));
    int *Rj = NULL; double *Rx = NULL;
    if (!F || !iperm || !Rp || !parent || !anc || !flag || !pat || !len || !x || !Cd) { *status = OR_ERR_ALLOC; goto fail; }
    F->N = N;
    F->perm = malloc(sizeof(int) * (size_t)N);
    F->D = malloc(sizeof(double) * (size_t)N);
    F->Lp = calloc((size_t)N + 1, sizeof(int));
    if (!F->perm || !F->D || !F->Lp) { *status = OR_ERR_ALLOC; goto fail; }
    for (int k = 0; k < N; ++k) { F->perm[k] = perm[k]; iperm[perm[k]] = k; }

    /* rows of the strictly lower part of C = P K P^T, plus its diagonal */
    for (int j = 0; j < N; ++j)
        for (int p = Kp[j]; p < Kp[j + 1]; ++p) {
            if (!isfinite(Kx[p])) { *status = OR_ERR_NONFINITE; goto fail; }
            int a = iperm[Ki[p]], b = iperm[j];
            if (a == b) continue;
            Rp[(a > b ? a : b) + 1]++;
        }
    for (int k = 0; k < N; ++k) Rp[k + 1] += Rp[k];
    Rj = malloc(sizeof(int) * (size_t)(Rp[N] > 0 ? Rp[N] : 1));
    Rx = malloc(sizeof(double) * (size_t)(Rp[N] > 0 ? Rp[N] : 1));
    if (!Rj || !Rx) { *status = OR_ERR_ALLOC; goto fail; }
    {
        int *w = malloc(sizeof(int) * (size_t)N);
        memcpy(w, Rp, sizeof(int) * (size_t)N);
        for (int j = 0; j < N; ++j)
            for (int p = Kp[j]; p < Kp[j + 1]; ++p) {
                int a = iperm[Ki[p]], b = iperm[j];
                if (a == b) { Cd[a] += Kx[p]; continue; }
                int r = a > b ? a : b, c = a > b ? b : a;
                Rj[w[r]] = c; Rx[w[r]] = Kx[p]; w[r]++;
            }
        free(w);
    }

    /* elimination tree (Liu): ancestor links with path compression */
    for (int k = 0; k < N; ++k) {
        parent[k] = -1; anc[k] = -1;
        for (int q = Rp[k]; q < Rp[k + 1]; ++q) {
            int i = Rj[q];
            while (i != -1 && i < k) {
                int nx = anc[i];
                anc[i] = k;
                if (nx == -1) parent[i] = k;
                i = nx;
            }
        }
    }

    /* column counts from the row patterns */
    for (int k = 0; k < N; ++k) flag[k] = -1;
    for (int k = 0; k < N; ++k) {
        int cnt = row_reach(k, Rp, Rj, parent, flag, pat);
        for (int a = 0; a < cnt; ++a) F->Lp[pat[a] + 1]++;
    }
    for (int k = 0; k < N; ++k) F->Lp[k + 1] += F->Lp[k];
    F->Li = malloc(sizeof(int) * (size_t)(F->Lp[N] > 0 ? F->Lp[N] : 1));
    F->Lx = malloc(sizeof(double) * (size_t)(F->Lp[N] > 0 ? F->Lp[N] : 1));
    if (!F->Li || !F->Lx) { *status = OR_ERR_ALLOC; goto fail; }

    /* numeric: row k of L from a sparse triangular solve with rows < k */
    for (int k = 0; k < N; ++k) flag[k] = -1;
    for (int k = 0; k < N; ++k) {
        int cnt = row_reach(k, Rp, Rj, parent, flag, pat);
        qsort(pat, (size_t)cnt, sizeof(int), cmp_int);   /* increasing = topological */
        for (int q = Rp[k]; q < Rp[k + 1]; ++q) x[Rj[q]] += Rx[q];
        double d = Cd[k];
        for (int a = 0; a < cnt; ++a) {
            int i = pat[a];
            double yi = x[i];
            x[i] = 0.0;
            for (int p = F->Lp[i]; p < F->Lp[i] + len[i]; ++p) x[F->Li[p]] -= F->Lx[p] * yi;
            double lki = yi / F->D[i];
            d -= lki * yi;
            int p = F->Lp[i] + len[i]++;
            F->Li[p] = k;
            F->Lx[p] = lki;
        }
        if (!isfinite(d)) { *status = OR_ERR_NONFINITE; goto fail; }
        {
            int dual = sign[perm[k]] < 0;
            double t = dual ? thr_dual : thr_primal;
            if (t > 0.0 && fabs(d) < t) {
                d = dual ? -t : t;
                F->nperturbed++;
            }
        }
        if (d > 0.0) F->npos++;
        else if (d < 0.0) F->nneg++;
        else F->nzero++;
        F->D[k] = d;
    }
    if (F->nzero > 0) *status = OR_ERR_ZERO_PIVOT;
    free(iperm); free(Rp); free(parent); free(anc); free(flag); free(pat); free(len); free(x); free(Cd);
    free(Rj); free(Rx);
    return F;
fail:
    free(iperm); free(Rp); free(parent); free(anc); free(flag); free(pat); free(len); free(x); free(Cd);
    free(Rj); free(Rx);
    or_free(F);
    return NULL;
}

int64_t or_nnz_L(const or_ldl *F) { return F->Lp[F->N]; }

void or_inertia(const or_ldl *F, int64_t *out4)
{
    out4[0] = F->npos; out4[1] = F->nneg; out4[2] = F->nzero; out4[3] = F->nperturbed;
}

/* Copy out L (strictly lower, CSC, permuted ordering), D and perm. */
void or_get_factor(const or_ldl *F, int *Lp, int *Li, double *Lx, double *D, int *perm)
{
    memcpy(Lp, F->Lp, sizeof(int) * (size_t)(F->N + 1));
    memcpy(Li, F->Li, sizeof(int) * (size_t)F->Lp[F->N]);
    memcpy(Lx, F->Lx, sizeof(double) * (size_t)F->Lp[F->N]);
    memcpy(D, F->D, sizeof(double) * (size_t)F->N);
    memcpy(perm, F->perm, sizeof(int) * (size_t)F->N);
}

/* X = P^T L^-T D^-1 L^-1 P B, nrhs columns, column-major. */
void or_solve(const or_ldl *F, int nrhs, const double *B, int ldb, double *X, int ldx)
{
    int N = F->N;
    double *w = malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    for (int c = 0; c < nrhs; ++c) {
        const double *b = B + (size_t)c * ldb;
        double *xo = X + (size_t)c * ldx;
        for (int k = 0; k < N; ++k) w[k] = b[F->perm[k]];
        for (int j = 0; j < N; ++j)
            for (int p = F->Lp[j]; p < F->Lp[j + 1]; ++p) w[F->Li[p]] -= F->Lx[p] * w[j];
        for (int j = 0; j < N; ++j) w[j] /= F->D[j];
        for (int j = N - 1; j >= 0; --j)
            for (int p = F->Lp[j]; p < F->Lp[j + 1]; ++p) w[j] -= F->Lx[p] * w[F->Li[p]];
        for (int k = 0; k < N; ++k) xo[F->perm[k]] = w[k];
    }
    free(w);
}
