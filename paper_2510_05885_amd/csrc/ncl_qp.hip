// ncl_qp.hip — Algorithm 1 (MadNCL, Sec. 2.3) on a convex quadratic program,
// driven from the host through the library's own entry points: every Newton
// step assembles and factors K1 = Q + Sigma + rho A^T A (Sec. 3.3, eq. K1),
// solves it with refinement, and recovers Delta y, Delta r (eqs.
// K1-elimination, K2-elimination) and Delta z_l, Delta z_u (Sec. 3.1, eq. K3).
// The vector arithmetic of the outer and inner loops runs in the kernels
// below; only scalars (norms, step lengths) come back to the host.
//
// Readings where the paper is silent (listed with the header declaration):
// y_0 = 0; r_0 = -c(x_0); z_0 central; one step length for all variables from
// the fraction-to-boundary rule, halved until ||F_k|| does not increase;
// complementarity in the optimality test; mu kept >= min(eta*, omega*) / 10.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/ncl_kkt.h"

namespace {

constexpr int kBlk = 256;
constexpr double kGamma = 0.05, kTau = 1.99, kMuFac = 0.2, kRhoMax = 1e14, kTheta = 0.5;   // Algorithm 1
constexpr double kRho0 = 100.0, kMu0 = 0.1;

struct QpHipError {
    hipError_t e;
};
#define QPCHK(x)                                         \
    do {                                                 \
        hipError_t e_ = (x);                             \
        if (e_ != hipSuccess) throw QpHipError{e_};      \
    } while (0)

struct QpLibError {
    int code;
};
inline void lib_ok(int rc) {
    if (rc < 0) throw QpLibError{rc};
}

unsigned int blocks(int64_t n) { return (unsigned int)((n + kBlk - 1) / kBlk); }

// Block-wide max (or min) of one value per thread into partial[blockIdx.x].
__device__ void block_reduce(double v, bool is_min, double* partial) {
    __shared__ double sm[kBlk];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int o = kBlk / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            sm[threadIdx.x] = is_min ? fmin(sm[threadIdx.x], sm[threadIdx.x + o]) : fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

// out[0] = max (or min) of partial[0, cnt) -- one block, fixed order.
__global__ void k_reduce(const double* __restrict__ partial, int cnt, int is_min, double* __restrict__ out) {
    double v = is_min ? INFINITY : 0.0;
    for (int i = threadIdx.x; i < cnt; i += kBlk) v = is_min ? fmin(v, partial[i]) : fmax(v, partial[i]);
    block_reduce(v, is_min != 0, out);
}

// g = Q x + q with Q as full symmetric CSR (value index per entry).
__global__ void k_grad(int n, const int64_t* __restrict__ Qp, const int* __restrict__ Qj, const int* __restrict__ Qk,
                       const double* __restrict__ Qv, const double* __restrict__ x, const double* __restrict__ q,
                       double* __restrict__ g) {
    const int i = blockIdx.x * kBlk + threadIdx.x;
    if (i >= n) return;
    double a = 0.0;
    for (int64_t e = Qp[i]; e < Qp[i + 1]; ++e) a += Qv[Qk[e]] * x[Qj[e]];
    g[i] = a + q[i];
}

// c = A x - b.
__global__ void k_cons(int m, const int64_t* __restrict__ Ap, const int* __restrict__ Aj, const double* __restrict__ Av,
                       const double* __restrict__ x, const double* __restrict__ b, double* __restrict__ c) {
    const int r = blockIdx.x * kBlk + threadIdx.x;
    if (r >= m) return;
    double a = 0.0;
    for (int64_t k = Ap[r]; k < Ap[r + 1]; ++k) a += Av[k] * x[Aj[k]];
    c[r] = a - b[r];
}

// out = A^T v, A^T in CSC (rows increasing per column, value index per entry).
__global__ void k_atv(int n, const int64_t* __restrict__ Tp, const int* __restrict__ Tr, const int* __restrict__ Tk,
                      const double* __restrict__ Av, const double* __restrict__ v, double* __restrict__ out) {
    const int i = blockIdx.x * kBlk + threadIdx.x;
    if (i >= n) return;
    double a = 0.0;
    for (int64_t q = Tp[i]; q < Tp[i + 1]; ++q) a += Av[Tk[q]] * v[Tr[q]];
    out[i] = a;
}

// t = y_k - rho c.
__global__ void k_t(int m, const double* __restrict__ yk, const double* __restrict__ c, double rho, double* __restrict__ t) {
    const int r = blockIdx.x * kBlk + threadIdx.x;
    if (r < m) t[r] = yk[r] - rho * c[r];
}

// Right-hand side of K1: A^T (y_k - rho c) - (g - mu / (x - l) + mu / (u - x));
// an infinite bound gives mu / inf = 0.
// (rhs may be atv.)
__global__ void k_rhs(int n, const double* atv, const double* __restrict__ g, const double* __restrict__ x,
                      const double* __restrict__ l, const double* __restrict__ u, double mu, double* rhs) {
    const int i = blockIdx.x * kBlk + threadIdx.x;
    if (i < n) rhs[i] = atv[i] - (g[i] - mu / (x[i] - l[i]) + mu / (u[i] - x[i]));
}

// max over the n-sized blocks of F at one point: with stat, the stationarity
// rows g - A^T y - z_l + z_u; with comp, the complementarity rows
// z_l (x - l) - mu and z_u (u - x) - mu of the finite bounds (0 for an
// infinite bound, whose multiplier is 0).
__global__ void k_fmax_n(int n, const double* __restrict__ g, const double* __restrict__ aty,
                         const double* __restrict__ zl, const double* __restrict__ zu, const double* __restrict__ x,
                         const double* __restrict__ l, const double* __restrict__ u, double mu, int stat, int comp,
                         double* __restrict__ partial) {
    const int i = blockIdx.x * kBlk + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        if (stat) v = fabs(g[i] - aty[i] - zl[i] + zu[i]);
        if (comp) {
            if (!isinf(l[i])) v = fmax(v, fabs(zl[i] * (x[i] - l[i]) - mu));
            if (!isinf(u[i])) v = fmax(v, fabs(zu[i] * (u[i] - x[i]) - mu));
        }
    }
    block_reduce(v, false, partial);
}

enum { kRowsF = 0, kRowsR = 1, kRowsC = 2 };

// max over the m-sized rows: kRowsF the two blocks of F, |y_k + rho r - y| and
// |c + r|; kRowsR |r| (the subproblem's infeasibility); kRowsC |c|.
__global__ void k_fmax_m(int m, const double* __restrict__ yk, const double* __restrict__ r,
                         const double* __restrict__ y, const double* __restrict__ c, double rho, int mode,
                         double* __restrict__ partial) {
    const int i = blockIdx.x * kBlk + threadIdx.x;
    double v = 0.0;
    if (i < m) {
        if (mode == kRowsR) v = fabs(r[i]);
        else if (mode == kRowsC) v = fabs(c[i]);
        else v = fmax(fabs(yk[i] + rho * r[i] - y[i]), fabs(c[i] + r[i]));
    }
    block_reduce(v, false, partial);
}

// min over the finite bounds of the distances x - l and u - x (1 if none).
__global__ void k_interior(int n, const double* __restrict__ x, const double* __restrict__ l,
                           const double* __restrict__ u, double* __restrict__ partial) {
    const int i = blockIdx.x * kBlk + threadIdx.x;
    double v = 1.0;
    if (i < n) {
        if (!isinf(l[i])) v = fmin(v, x[i] - l[i]);
        if (!isinf(u[i])) v = fmin(v, u[i] - x[i]);
        if (isnan(x[i]) || isnan(l[i]) || isnan(u[i])) v = -1.0;
    }
    block_reduce(v, true, partial);
}

// min over the step bounds: tau (x - l) / -dx, tau (u - x) / dx, tau z / -dz
// (finite bounds, moving toward them); 1 if none.
__global__ void k_step(int n, const double* __restrict__ x, const double* __restrict__ dx,
                       const double* __restrict__ zl, const double* __restrict__ dzl, const double* __restrict__ zu,
                       const double* __restrict__ dzu, const double* __restrict__ l, const double* __restrict__ u,
                       double tau, double* __restrict__ partial) {
    const int i = blockIdx.x * kBlk + threadIdx.x;
    double a = 1.0;
    if (i < n) {
        if (!isinf(l[i])) {
            if (dx[i] < 0.0) a = fmin(a, tau * ((x[i] - l[i]) / -dx[i]));
            if (dzl[i] < 0.0) a = fmin(a, tau * (zl[i] / -dzl[i]));
        }
        if (!isinf(u[i])) {
            if (dx[i] > 0.0) a = fmin(a, tau * ((u[i] - x[i]) / dx[i]));
            if (dzu[i] < 0.0) a = fmin(a, tau * (zu[i] / -dzu[i]));
        }
    }
    block_reduce(a, true, partial);
}

// out = v + a dv (out may be v).
__global__ void k_axpy(int64_t n, double a, const double* v, const double* __restrict__ dv, double* out) {
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (i < n) out[i] = v[i] + a * dv[i];
}

// z_l = mu / (x - l), z_u = mu / (u - x) on finite bounds, 0 otherwise.
__global__ void k_init_z(int n, const double* __restrict__ x, const double* __restrict__ l, const double* __restrict__ u,
                         double mu, double* __restrict__ zl, double* __restrict__ zu) {
    const int i = blockIdx.x * kBlk + threadIdx.x;
    if (i >= n) return;
    zl[i] = isinf(l[i]) ? 0.0 : mu / (x[i] - l[i]);
    zu[i] = isinf(u[i]) ? 0.0 : mu / (u[i] - x[i]);
}

__global__ void k_scale(int64_t n, double a, const double* __restrict__ v, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (i < n) out[i] = a * v[i];
}

// The primal-dual point w = (x, r, y, z_l, z_u) in one allocation.
struct Point {
    double *x, *r, *y, *zl, *zu;
};

struct QpSolver {
    int n = 0, m = 0;
    hipStream_t st = nullptr;
    ncl_kkt_t h = nullptr;
    const double *Qv = nullptr, *q = nullptr, *Av = nullptr, *b = nullptr, *l = nullptr, *u = nullptr;
    std::vector<void*> allocs;
    int64_t *Qp = nullptr, *Ap = nullptr, *Tp = nullptr;
    int *Qj = nullptr, *Qk = nullptr, *Aj = nullptr, *Tr = nullptr, *Tk = nullptr;
    double *g = nullptr, *c = nullptr, *aty = nullptr, *t = nullptr, *rhs = nullptr, *sigma = nullptr;
    double *yk = nullptr, *partial = nullptr, *scal = nullptr, *host = nullptr;
    Point w[2]{}, d{};   // w[0] / w[1]: current and trial points (swapped), d: the direction

    ~QpSolver() {
        (void)hipStreamSynchronize(st);
        if (h) ncl_kkt_destroy(h);
        for (void* p : allocs) (void)hipFree(p);
        if (host) (void)hipHostFree(host);
    }
    template <typename T>
    T* alloc(int64_t cnt) {
        void* p = nullptr;
        QPCHK(hipMalloc(&p, sizeof(T) * (size_t)std::max<int64_t>(cnt, 1)));
        allocs.push_back(p);
        return static_cast<T*>(p);
    }
    template <typename T>
    T* upload(const std::vector<T>& v) {
        T* p = alloc<T>((int64_t)v.size());
        if (!v.empty()) QPCHK(hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
        return p;
    }
    Point point() {
        double* base = alloc<double>(3 * (int64_t)n + 2 * (int64_t)m);
        return Point{base, base + n, base + n + m, base + n + 2 * m, base + 2 * n + 2 * m};
    }
    double fetch(double* dptr) {
        QPCHK(hipGetLastError());
        QPCHK(hipMemcpyAsync(host, dptr, sizeof(double), hipMemcpyDeviceToHost, st));
        QPCHK(hipStreamSynchronize(st));
        return host[0];
    }
    double reduce(int cnt, bool is_min) {
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlk), 0, st, partial, cnt, is_min ? 1 : 0, scal);
        return fetch(scal);
    }

    // g, c and A^T y at x, y
    void eval(const Point& p) {
        hipLaunchKernelGGL(k_grad, dim3(blocks(n)), dim3(kBlk), 0, st, n, Qp, Qj, Qk, Qv, p.x, q, g);
        if (m > 0) {
            hipLaunchKernelGGL(k_cons, dim3(blocks(m)), dim3(kBlk), 0, st, m, Ap, Aj, Av, p.x, b, c);
            hipLaunchKernelGGL(k_atv, dim3(blocks(n)), dim3(kBlk), 0, st, n, Tp, Tr, Tk, Av, p.y, aty);
        } else {
            QPCHK(hipMemsetAsync(aty, 0, sizeof(double) * n, st));
        }
    }
    // ||F_k(w)||_inf (Sec. 2.3, eq. kktnclipm)
    double fnorm(const Point& p, double rho, double mu) {
        eval(p);
        const int bn = (int)blocks(n), bm = (int)blocks(std::max(m, 1));
        hipLaunchKernelGGL(k_fmax_n, dim3(bn), dim3(kBlk), 0, st, n, g, aty, p.zl, p.zu, p.x, l, u, mu, 1, 1, partial);
        hipLaunchKernelGGL(k_fmax_m, dim3(bm), dim3(kBlk), 0, st, m, yk, p.r, p.y, c, rho, (int)kRowsF, partial + bn);
        return reduce(bn + bm, false);
    }
    // Newton direction d at w: Sigma, K1 factor and solve, recoveries
    void direction(const Point& p, double rho, double mu) {
        eval(p);
        lib_ok(ncl_kkt_barrier_sigma(h, p.x, l, u, p.zl, p.zu, sigma, st));
        lib_ok(ncl_kkt_factor(h, Qv, sigma, Av, rho, st));
        if (m > 0) {
            hipLaunchKernelGGL(k_t, dim3(blocks(m)), dim3(kBlk), 0, st, m, yk, c, rho, t);
            hipLaunchKernelGGL(k_atv, dim3(blocks(n)), dim3(kBlk), 0, st, n, Tp, Tr, Tk, Av, t, rhs);
        } else {
            QPCHK(hipMemsetAsync(rhs, 0, sizeof(double) * n, st));
        }
        hipLaunchKernelGGL(k_rhs, dim3(blocks(n)), dim3(kBlk), 0, st, n, rhs, g, p.x, l, u, mu, rhs);
        ncl_kkt_solve_info info;
        lib_ok(ncl_kkt_solve(h, rhs, n, d.x, n, 1, st, &info));
        if (m > 0) {
            lib_ok(ncl_kkt_recover_dy(h, Av, d.x, c, yk, p.y, d.y, st));
            lib_ok(ncl_kkt_recover_dr(h, d.y, yk, p.y, p.r, d.r, st));
        }
        lib_ok(ncl_kkt_recover_dz(h, p.x, l, u, p.zl, p.zu, d.x, mu, d.zl, d.zu, st));
    }
    double max_step(const Point& p, double mu) {
        const double tau = std::max(0.99, 1.0 - mu);
        const int bn = (int)blocks(n);
        hipLaunchKernelGGL(k_step, dim3(bn), dim3(kBlk), 0, st, n, p.x, d.x, p.zl, d.zl, p.zu, d.zu, l, u, tau,
                           partial);
        return reduce(bn, true);
    }
    void step(const Point& p, double a, const Point& out) {
        const int64_t len = 3 * (int64_t)n + 2 * (int64_t)m;   // the five vectors are contiguous
        hipLaunchKernelGGL(k_axpy, dim3(blocks(len)), dim3(kBlk), 0, st, len, a, p.x, d.x, out.x);
    }
};

}  // namespace

extern "C" {

void ncl_qp_default_options(ncl_qp_options* o) {
    if (!o) return;
    o->eta_star = 1e-8;
    o->omega_star = 1e-8;
    o->max_outer = 100;
    o->max_inner = 100;
    o->precision = NCL_FP64;
    o->print_level = 0;
}

int ncl_qp_solve(const ncl_qp_options* opt, int32_t n, int32_t m, const int32_t* Q_colptr, const int32_t* Q_rowidx,
                 const double* Q_val, const double* q, const int32_t* A_rowptr, const int32_t* A_colidx,
                 const double* A_val, const double* b, const double* l, const double* u, double* x, double* y,
                 double* z_l, double* z_u, ncl_qp_result* res, void* stream) {
    if (!opt || n < 1 || m < 0 || !Q_colptr || !Q_rowidx || !Q_val || !q || !x || !y || !z_l || !z_u || !l || !u ||
        !res)
        return NCL_ERR_ARG;
    if (m > 0 && (!A_rowptr || !A_colidx || !A_val || !b)) return NCL_ERR_ARG;
    if (!(opt->eta_star > 0.0) || !(opt->omega_star > 0.0) || opt->max_outer < 1 || opt->max_inner < 1)
        return NCL_ERR_ARG;
    std::memset(res, 0, sizeof(*res));
    QpSolver P;
    P.n = n;
    P.m = m;
    P.st = (hipStream_t)stream;
    P.Qv = Q_val; P.q = q; P.Av = A_val; P.b = b; P.l = l; P.u = u;
    try {
        // KKT handle on the patterns of Q (lower CSC) and A (CSR)
        ncl_kkt_options ko;
        ncl_kkt_default_options(&ko);
        ko.form = NCL_CONDENSED;
        ko.precision = opt->precision;
        // Sigma spans many decades near the end (z / (x - l) up to ~1e13 on active bounds), so a
        // pivot threshold relative to ||K||_max would exceed K1's legitimate pivots (>= the
        // smallest eigenvalue of Q): the absolute rule leaves them alone, and refinement must
        // reach a componentwise backward error, which a normwise one does not imply here.
        ko.pivot_scale = NCL_PIVOT_ABSOLUTE;
        ko.ir_cw_tol = 1e-14;
        std::vector<int32_t> emptyp(1, 0);
        int rc = ncl_kkt_analyze(&P.h, &ko, n, m, Q_colptr, Q_rowidx, m > 0 ? A_rowptr : emptyp.data(),
                                 m > 0 ? A_colidx : emptyp.data());
        if (rc) return rc;
        // Q as full symmetric CSR, A's CSR and its transpose (CSC), on the device
        std::vector<int64_t> qp(n + 1, 0);
        for (int j = 0; j < n; ++j)
            for (int64_t e = Q_colptr[j]; e < Q_colptr[j + 1]; ++e) {
                const int i = Q_rowidx[e];
                if (i < 0 || i >= n || i < j) return NCL_ERR_PATTERN;
                qp[i + 1]++;
                if (i != j) qp[j + 1]++;
            }
        for (int i = 0; i < n; ++i) qp[i + 1] += qp[i];
        std::vector<int> qj(qp[n]), qk(qp[n]);
        std::vector<int64_t> fill(qp.begin(), qp.end() - 1);
        for (int j = 0; j < n; ++j)
            for (int64_t e = Q_colptr[j]; e < Q_colptr[j + 1]; ++e) {
                const int i = Q_rowidx[e];
                qj[fill[i]] = j; qk[fill[i]++] = (int)e;
                if (i != j) { qj[fill[j]] = i; qk[fill[j]++] = (int)e; }
            }
        P.Qp = P.upload(qp); P.Qj = P.upload(qj); P.Qk = P.upload(qk);
        if (m > 0) {
            std::vector<int64_t> ap(A_rowptr, A_rowptr + m + 1);
            std::vector<int> aj(A_colidx, A_colidx + A_rowptr[m]);
            std::vector<int64_t> tp(n + 1, 0);
            for (int c : aj) tp[c + 1]++;
            for (int i = 0; i < n; ++i) tp[i + 1] += tp[i];
            std::vector<int> tr(aj.size()), tk(aj.size());
            std::vector<int64_t> tf(tp.begin(), tp.end() - 1);
            for (int r = 0; r < m; ++r)
                for (int64_t k = ap[r]; k < ap[r + 1]; ++k) { tr[tf[aj[k]]] = r; tk[tf[aj[k]]++] = (int)k; }
            P.Ap = P.upload(ap); P.Aj = P.upload(aj); P.Tp = P.upload(tp); P.Tr = P.upload(tr); P.Tk = P.upload(tk);
        }
        P.g = P.alloc<double>(n); P.c = P.alloc<double>(m); P.aty = P.alloc<double>(n); P.t = P.alloc<double>(m);
        P.rhs = P.alloc<double>(n); P.sigma = P.alloc<double>(n); P.yk = P.alloc<double>(m);
        P.partial = P.alloc<double>(blocks(n) + blocks(std::max(m, 1)) + 1);
        P.scal = P.alloc<double>(1);
        QPCHK(hipHostMalloc((void**)&P.host, sizeof(double), hipHostMallocDefault));
        for (auto& p : P.w) p = P.point();
        P.d = P.point();
        const int nb = (int)blocks(n), mb = (int)blocks(std::max(m, 1));
        const double mu_min = std::min(opt->eta_star, opt->omega_star) / 10.0;
        // initial point: x_0 (caller's, strictly inside), r_0 = -c(x_0), y_0 = 0, z_0 central
        double rho = kRho0, mu = kMu0;
        Point* W = &P.w[0];
        Point* Wt = &P.w[1];
        QPCHK(hipMemcpyAsync(W->x, x, sizeof(double) * n, hipMemcpyDeviceToDevice, P.st));
        hipLaunchKernelGGL(k_interior, dim3(nb), dim3(kBlk), 0, P.st, n, W->x, l, u, P.partial);
        if (!(P.reduce(nb, true) > 0.0)) return NCL_ERR_ARG;   // x_0 not strictly inside its bounds
        P.eval(*W);
        if (m > 0) hipLaunchKernelGGL(k_scale, dim3(blocks(m)), dim3(kBlk), 0, P.st, (int64_t)m, -1.0, P.c, W->r);
        if (m > 0) {
            QPCHK(hipMemsetAsync(W->y, 0, sizeof(double) * m, P.st));
            QPCHK(hipMemsetAsync(P.yk, 0, sizeof(double) * m, P.st));
        }
        hipLaunchKernelGGL(k_init_z, dim3(nb), dim3(kBlk), 0, P.st, n, W->x, l, u, mu, W->zl, W->zu);
        double eta = std::min(std::pow(mu, 1.1), 0.1 * mu), omega = 100.0 * std::pow(mu, 1.0 + kGamma);
        int status = 2, k = 0, inner = 0, extrap = 0;
        double rn = 0.0, dual = 0.0;
        for (k = 1; k <= opt->max_outer; ++k) {
            // extrapolation step (Sec. 2.3, eq. ncl:extrapolation)
            const double f0 = P.fnorm(*W, rho, mu);
            P.direction(*W, rho, mu);
            const double a = P.max_step(*W, mu);
            P.step(*W, a, *Wt);
            const double fp = P.fnorm(*Wt, rho, mu);
            const bool accept = fp <= kTheta * f0 + 10.0 * std::pow(a, 0.2) * mu;
            int steps = 0;
            if (accept) {
                std::swap(W, Wt);
                ++extrap;
            } else {
                for (double f = f0; f > omega && steps < opt->max_inner; ++steps) {
                    // one inner Newton step: fraction to the boundary, halved until ||F_k|| does not grow
                    P.direction(*W, rho, mu);
                    double al = P.max_step(*W, mu), fn = 0.0;
                    bool ok = false;
                    for (int h = 0; h < 30 && !ok; ++h) {
                        P.step(*W, al, *Wt);
                        fn = P.fnorm(*Wt, rho, mu);
                        ok = fn <= f;
                        if (!ok) al *= 0.5;
                    }
                    if (!ok) {   // 30 halvings without decrease: take the last, halved once more
                        P.step(*W, al, *Wt);
                        fn = P.fnorm(*Wt, rho, mu);
                    }
                    std::swap(W, Wt);
                    f = fn;
                }
                inner += steps;
            }
            // outer update (Algorithm 1)
            if (m > 0) {
                hipLaunchKernelGGL(k_fmax_m, dim3(mb), dim3(kBlk), 0, P.st, m, P.yk, W->r, W->y, P.c, rho,
                                   (int)kRowsR, P.partial);
                rn = P.reduce(mb, false);
            } else {
                rn = 0.0;
            }
            if (rn <= eta) {
                if (m > 0) hipLaunchKernelGGL(k_axpy, dim3(blocks(m)), dim3(kBlk), 0, P.st, (int64_t)m, rho, P.yk, W->r, P.yk);
                const double mu_new = std::max(std::min(std::pow(mu, kTau), kMuFac * mu), mu_min);
                eta = std::min(std::pow(mu_new, 1.1), 0.1 * mu);
                omega = 100.0 * std::pow(mu_new, 1.0 + kGamma);
                mu = mu_new;
            } else {
                rho = std::min(kRhoMax, 10.0 * rho);
            }
            // optimality: stationarity (with the bound multipliers) and complementarity
            P.eval(*W);
            hipLaunchKernelGGL(k_fmax_n, dim3(nb), dim3(kBlk), 0, P.st, n, P.g, P.aty, W->zl, W->zu, W->x, l, u, 0.0,
                               1, 0, P.partial);
            dual = P.reduce(nb, false);
            hipLaunchKernelGGL(k_fmax_n, dim3(nb), dim3(kBlk), 0, P.st, n, P.g, P.aty, W->zl, W->zu, W->x, l, u, 0.0,
                               0, 1, P.partial);
            const double comp = P.reduce(nb, false);
            if (opt->print_level > 0)
                std::fprintf(stderr,
                             "ncl_qp %3d  rho %.1e  mu %.3e  |F| %.6e  alpha %.6e  |F+| %.6e  %s  inner %3d  "
                             "|r| %.3e  dual %.3e  comp %.3e\n",
                             k, rho, mu, f0, a, fp, accept ? "extrap" : "newton", steps, rn, dual, comp);
            if (rn <= opt->eta_star && dual <= opt->omega_star && comp <= opt->omega_star) {
                status = 0;
                break;
            }
            if (rho >= kRhoMax && rn > opt->eta_star) {
                status = 1;
                break;
            }
        }
        // results: x, y, z; the primal infeasibility ||A x - b||
        QPCHK(hipMemcpyAsync(x, W->x, sizeof(double) * n, hipMemcpyDeviceToDevice, P.st));
        if (m > 0) QPCHK(hipMemcpyAsync(y, W->y, sizeof(double) * m, hipMemcpyDeviceToDevice, P.st));
        QPCHK(hipMemcpyAsync(z_l, W->zl, sizeof(double) * n, hipMemcpyDeviceToDevice, P.st));
        QPCHK(hipMemcpyAsync(z_u, W->zu, sizeof(double) * n, hipMemcpyDeviceToDevice, P.st));
        double pinf = 0.0;
        if (m > 0) {
            P.eval(*W);
            hipLaunchKernelGGL(k_fmax_m, dim3(mb), dim3(kBlk), 0, P.st, m, P.yk, W->r, W->y, P.c, rho, (int)kRowsC,
                               P.partial);
            pinf = P.reduce(mb, false);
        }
        res->status = status;
        res->outer = std::min(k, opt->max_outer);
        res->inner = inner;
        res->extrapolated = extrap;
        res->primal_inf = pinf;
        res->dual_inf = dual;
        QPCHK(hipStreamSynchronize(P.st));
    } catch (const QpHipError&) {
        return NCL_ERR_HIP;
    } catch (const QpLibError& e) {
        return e.code;
    }
    return NCL_OK;
}

}  // extern "C"
