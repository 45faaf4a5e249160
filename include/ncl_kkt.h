/*
 * ncl_kkt.h — C ABI of the MI355X KKT factor/solve library for the Newton
 * step of Algorithm NCL (MadNCL, arXiv 2510.05885).
 *
 * The library assembles and solves, by supernodal multifrontal LDL^T with
 * static pivoting, one of two symmetric KKT matrices built from the Hessian
 * block W (n x n), the barrier diagonal Sigma (n) and the Jacobian J (m x n):
 *
 *   condensed  (NCL_CONDENSED):  K = W + Sigma + rho J^T J            order n
 *              Sec. 3.3, eq. K1.  SPD when the system is correctly
 *              regularized; expected inertia (n, 0, 0) (Sec. 3.4).
 *   stabilized (NCL_STABILIZED): K = [[W + Sigma, J^T], [J, -(1/rho) I]]
 *              Sec. 3.2, eq. K2r.  Symmetric quasi-definite; expected
 *              inertia (n, m, 0) (Sec. 3.4, Prop. "inertia").
 *
 * rho is the effective penalty of the paper (rho-hat = rho + delta, Sec. 3.1);
 * a caller that regularizes with delta passes Sigma + delta and rho + delta.
 *
 * Static pivoting (Sec. 3.1 "Sparse LDL^T factorization", Sec. 4.3): a pivot d
 * with |d| < t (strict) is replaced by s * t, where s = +1 for a primal row and
 * -1 for a dual row of the unpermuted matrix, and t is the threshold of that
 * row's block: t = eps * ||K||_max for every pivot (NCL_PIVOT_GLOBAL, default;
 * ||K||_max = max_ij |K_ij| of the assembled, unpermuted K in FP64), or, with
 * NCL_PIVOT_BLOCK in the stabilized form, eps * max |(W + Sigma)_ij| for
 * primal pivots and eps / rho for dual pivots (the norm of the -1/rho I block
 * of Sec. 3.2, eq. K2r), or t = eps for every pivot (NCL_PIVOT_ABSOLUTE: the
 * solver's pivot epsilon of Sec. 4.3 as an absolute bound; it leaves alone
 * the small but legitimate pivots of a primal block whose Sigma spans many
 * decades).  A pivot of the wrong sign and magnitude above the
 * threshold is kept and shows in the inertia.  The factor is thus of a
 * slightly perturbed matrix; solves refine against the unperturbed K
 * (Richardson, Sec. 4.3).
 *
 * Memory: patterns are host arrays copied at analyze time.  Values,
 * right-hand sides, solutions and gradients are caller-owned DEVICE buffers
 * (double).  The handle owns all device workspace; it is allocated by
 * ncl_kkt_analyze and reused by every factor / solve (they allocate nothing).
 * All device work is ordered on the caller's stream (a hipStream_t passed as
 * void*; NULL = the null stream).
 *
 * Return codes: 0 success; negative = error (nothing usable produced);
 * positive = completed with a warning.
 */
#ifndef NCL_KKT_H
#define NCL_KKT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ncl_kkt_s *ncl_kkt_t;

enum { NCL_CONDENSED = 0, NCL_STABILIZED = 1 };
enum { NCL_FP64 = 0, NCL_FP32_IR = 1 };
enum { NCL_ORDER_ND = 0, NCL_ORDER_NATURAL = 1, NCL_ORDER_USER = 2 };
enum { NCL_PIVOT_GLOBAL = 0, NCL_PIVOT_BLOCK = 1, NCL_PIVOT_ABSOLUTE = 2 };

#define NCL_OK 0
#define NCL_ERR_ARG (-1)        /* bad argument (sizes, null pointers, rho <= 0, ...) */
#define NCL_ERR_PATTERN (-2)    /* unsorted / duplicate / out-of-range / upper-triangle index */
#define NCL_ERR_ALLOC (-3)      /* host or device allocation failed */
#define NCL_ERR_HIP (-4)        /* a HIP runtime call failed */
#define NCL_ERR_STATE (-5)      /* call out of order (solve before factor, ...) */
#define NCL_ERR_NONFINITE (-6)  /* NaN or Inf met in the assembled matrix, or in a pivot of an
                                   FP64 factorization (an FP32 factor that meets one is
                                   replaced by an FP64 refactorization instead) */
#define NCL_ERR_SCRATCH (-7)    /* ncl_kkt_backward_noalloc: 2 x m x nrhs exceeds its fixed
                                   scratch of 2^21 doubles */
#define NCL_WARN_INERTIA 1      /* factor done, inertia differs from (n,0,0) / (n,m,0) */
#define NCL_WARN_IR_NOT_CONVERGED 2  /* refinement stopped above ir_tol */
#define NCL_WARN_FELL_BACK_FP64 3    /* FP32 factor insufficient; refactored in FP64 */

/* Options.  Fill with ncl_kkt_default_options, then override. */
typedef struct {
    int32_t form;          /* NCL_CONDENSED or NCL_STABILIZED */
    int32_t precision;     /* NCL_FP64, or NCL_FP32_IR: FP32 factor + FP64 refinement */
    double pivot_eps;      /* relative static-pivot epsilon; <= 0: 1e-12 condensed,
                              1e-10 stabilized (the paper's value, Sec. 4.3) */
    int32_t ir_max_steps;  /* max refinement corrections per solve (default 10) */
    double ir_tol;         /* converged when the normwise backward error omega <= ir_tol
                              (default 1e-12) and, if ir_cw_tol > 0, the componentwise one
                              <= ir_cw_tol */
    double ir_stall;       /* stop when a correction does not reduce the distance to the
                              target, max(omega / ir_tol, omega_cw / ir_cw_tol), below
                              ir_stall * previous (default 0.5) */
    int32_t ordering;      /* NCL_ORDER_ND (default), NCL_ORDER_NATURAL, NCL_ORDER_USER */
    const int32_t *user_perm; /* host, used when ordering == NCL_ORDER_USER: user_perm[k] =
                                 unpermuted index of the k-th pivot (length n or n+m) */
    int32_t use_graphs;    /* 1 (default): replay the fixed launch sequences of the frontal
                              factorization and of the triangular sweeps as HIP graphs */
    int32_t small_front_max; /* fronts up to this order are factored in LDS; 0 = device limit */
    double relax_big_zeros;  /* supernode amalgamation: fraction of explicit zeros allowed in
                                fronts above 128 rows; < 0 selects the default (0.2) */
    int32_t fp32_sticky;     /* NCL_FP32_IR only.  1 (default): once an FP32 factor had to be
                                replaced by FP64 (wrong inertia, or refinement above ir_tol)
                                at rho = r, every later factor with max rho >= r is computed
                                in FP64 directly; a factor with max rho < r tries FP32 again
                                (rho grows along an NCL outer loop, Algorithm 1).  0: always
                                try FP32 first. */
    int32_t pivot_scale;     /* NCL_PIVOT_GLOBAL (default), NCL_PIVOT_BLOCK (stabilized form:
                                each block's own norm, see above; same as global for the
                                condensed form) or NCL_PIVOT_ABSOLUTE */
    double ir_cw_tol;        /* > 0: refinement must also bring the componentwise backward
                                error max_i |b - Kx|_i / (|K||x| + |b|)_i to <= ir_cw_tol;
                                0 (default): normwise criterion only */
    int32_t persistent;      /* disabled: the persistent launches (every front of every
                                system factored by one launch whose workgroups take fronts
                                from a ticket counter in topological order, both sweeps by a
                                second one) are switched off until a stall seen in them is
                                explained.  0 or -1 (default): level-scheduled launches;
                                1: NCL_ERR_ARG. */
    int32_t persistent_grid; /* workgroups of the persistent launches (unused while they are
                                disabled) */
} ncl_kkt_options;

/* Result of one solve, each figure the max over columns (and systems), all
 * measured against the unperturbed K in FP64:
 *   omega    = ||b - Kx||_inf / (||K||_inf ||x||_inf + ||b||_inf)  (normwise)
 *   omega_cw = max_i |b - Kx|_i / (|K| |x| + |b|)_i                (componentwise)
 *   rel2     = ||b - Kx||_2 / ||b||_2 */
typedef struct {
    int32_t ir_steps;        /* refinement corrections applied */
    int32_t fell_back_fp64;  /* 1 when an FP64 refactor was needed (FP32_IR only) */
    double backward_error;   /* final omega */
    double backward_error0;  /* omega of the unrefined solve */
    double backward_error_cw;  /* final omega_cw */
    double resid_rel2;       /* final rel2 */
} ncl_kkt_solve_info;

/* Sizes of the symbolic analysis. */
typedef struct {
    int64_t order;          /* n (condensed) or n + m (stabilized), summed over systems */
    int64_t nnz_K_lower;    /* stored lower entries of K (incl. diagonal) */
    int64_t nnz_L;          /* entries of L incl. diagonal, supernodal (with padding zeros) */
    double flops_factor;    /* flops of the partial frontal factorizations as executed
                               (amalgamation padding included) */
    int64_t n_supernodes;
    int64_t n_levels;       /* levels of the supernodal tree (leaves = level 0) */
    int64_t max_front;      /* largest front order */
    int64_t n_large_fronts; /* fronts handled by the global-memory MFMA path */
    int64_t device_bytes;   /* device workspace held by the handle */
    double analyze_seconds; /* host time of the symbolic analysis */
    int64_t nnz_L_exact;    /* entries of L incl. diagonal for the same ordering, without
                               amalgamation padding (column counts of the elimination tree) */
    double flops_exact;     /* sum over columns j of c_j (c_j + 2), c_j = entries of column j
                               of L below the diagonal: the factorization's algorithmic flops */
} ncl_kkt_stats;

void ncl_kkt_default_options(ncl_kkt_options *o);

/* Symbolic analysis on the fixed sparsity pattern (Sec. 4.1: the symbolic
 * factorization is computed once and reused).  W: lower-triangular CSC
 * (W_colptr[n+1], W_rowidx sorted, row >= column); J: CSR m x n (J_rowptr[m+1],
 * J_colidx sorted).  m may be 0.  Host arrays, copied.  Orders the matrix,
 * builds the supernodal elimination tree and every map, then allocates and
 * uploads the device workspace (current HIP device).  *h is NULL on error. */
int ncl_kkt_analyze(ncl_kkt_t *h, const ncl_kkt_options *o, int32_t n, int32_t m,
                    const int32_t *W_colptr, const int32_t *W_rowidx,
                    const int32_t *J_rowptr, const int32_t *J_colidx);

/* Same analysis without touching any GPU: the handle can only be inspected
 * (ncl_kkt_get_stats / ncl_kkt_get_perm / ncl_kkt_get_supernodes) and
 * destroyed.  factor/solve on it return NCL_ERR_STATE. */
int ncl_kkt_analyze_host(ncl_kkt_t *h, const ncl_kkt_options *o, int32_t n, int32_t m,
                         const int32_t *W_colptr, const int32_t *W_rowidx,
                         const int32_t *J_rowptr, const int32_t *J_colidx);

/* Batched condensed systems: `count` independent systems analyzed into one
 * handle (the block-diagonal union).  Arrays of per-system host pointers.
 * Values for factor/solve are the per-system arrays concatenated in system
 * order (W values, Sigma, J values, right-hand-side rows).  form must be
 * NCL_CONDENSED. */
int ncl_kkt_analyze_batched(ncl_kkt_t *h, const ncl_kkt_options *o, int32_t count,
                            const int32_t *n, const int32_t *m,
                            const int32_t *const *W_colptr, const int32_t *const *W_rowidx,
                            const int32_t *const *J_rowptr, const int32_t *const *J_colidx);

/* Numeric factorization on new values (device pointers, lengths nnz(W), n,
 * nnz(J)): assembles K of the chosen form on the GPU (Sec. 3.3 eq. K1 /
 * Sec. 3.2 eq. K2r), computes ||K||_max, and factors it with the static-pivot
 * rule.  rho > 0 (Sec. 3.4 assumes rho > 0).  Returns NCL_WARN_INERTIA when
 * the inertia differs from the expected one (the factor is still usable),
 * NCL_ERR_NONFINITE on NaN/Inf.  Synchronizes the stream to read the inertia. */
int ncl_kkt_factor(ncl_kkt_t h, const double *W_val, const double *Sigma,
                   const double *J_val, double rho, void *stream);

/* Batched factor: rho is a HOST array of `count` penalties. */
int ncl_kkt_factor_batched(ncl_kkt_t h, const double *W_val, const double *Sigma,
                           const double *J_val, const double *rho, void *stream);

/* ---- slack elimination and the rest of the Newton step -------------------
 * Problem NCO (Sec. 3): the rows of J are equality constraints c_E and
 * inequality constraints c_I; an inequality row r has a slack s_r whose
 * barrier diagonal is Sigma_s[r] (Sec. 3.3, the definition of Sigma_s).
 * Sigma_s is a DEVICE array with one entry per row of J (all systems
 * concatenated like J's rows): Sigma_s[r] >= 0 for an inequality row, +inf
 * for an equality row -- the limit in which an active inequality acts as an
 * equality (the remark after the proposition "Condensed KKT system").
 * Vectors are device arrays in the caller's (unpermuted) order: length n for
 * variables, m for rows of J (sums over the systems of a batched handle).
 * rho below is rho-hat = rho + delta of each system from the last factor
 * call.  Condensed handles only (NCL_ERR_ARG otherwise); NCL_ERR_STATE before
 * a factor or on a host-only handle.  Stream-ordered, nothing allocated. */

/* Factors K1s = W_t + Sigma_t + rho J_E^T J_E + rho J_I^T Omega J_I (Sec. 3.3,
 * eq. K1s) with Omega_rr = Sigma_s,r / (rho + Sigma_s,r): K1's assembly with
 * the products of row r weighted by Omega_rr (1 on equality rows).  Same
 * pattern, static pivoting and returns as ncl_kkt_factor; rho is a HOST array
 * of one penalty per system.  A negative or NaN Sigma_s gives
 * NCL_ERR_NONFINITE.  ncl_kkt_backward refuses such a factor (NCL_ERR_STATE):
 * its adjoint is of K1. */
int ncl_kkt_factor_k1s(ncl_kkt_t h, const double *W_val, const double *Sigma_t,
                       const double *J_val, const double *Sigma_s, const double *rho,
                       void *stream);

/* Inertia correction (Sec. 3.1: the regularization delta is raised until
 * the desired inertia is obtained).  Factors with delta = 0, then delta_init,
 * delta_init * growth, ... -- delta added to the primal diagonal (Sigma + delta)
 * and to the penalty (rho-hat = rho + delta, eq. K2) -- and stops at the
 * first factor with the expected inertia ((n,0,0) condensed, (n,m,0)
 * stabilized) or when the next delta would exceed delta_max (then the last
 * factor stays, NCL_WARN_INERTIA).  Sigma_s non-NULL: the K1s form
 * (condensed only, see ncl_kkt_factor_k1s).  Single-system handles.
 * delta_init > 0, growth > 1, delta_max >= 0, else NCL_ERR_ARG.  Writes the
 * delta used and the number of factorizations (host; either may be NULL).
 * Later solves are of the regularized matrix.  Allocates a Sigma-sized work
 * array on first use. */
int ncl_kkt_factor_regularized(ncl_kkt_t h, const double *W_val, const double *Sigma,
                               const double *J_val, const double *Sigma_s, double rho,
                               double delta_init, double growth, double delta_max,
                               double *delta_out, int32_t *attempts_out, void *stream);

/* b = r_t + rho J_I^T (Sigma_s + rho I)^-1 r_s, the right-hand side of K1s
 * that eliminating Delta s from eq. K1' produces (the proof of the
 * proposition; the printed eq. K1s omits the factor (Sigma_s + rho I)^-1).
 * r_t: n, r_s: m (entries of equality rows are not read), b: n. */
int ncl_kkt_k1s_rhs(ncl_kkt_t h, const double *J_val, const double *r_t, const double *r_s,
                    const double *Sigma_s, double *b, void *stream);

/* Delta s = (Sigma_s + rho I)^-1 (rho J_I Delta t + r_s) (the proof of the
 * proposition); ds[r] = 0 on equality rows.  dt: n, r_s and ds: m. */
int ncl_kkt_k1s_recover(ncl_kkt_t h, const double *J_val, const double *dt, const double *r_s,
                        const double *Sigma_s, double *ds, void *stream);

/* Delta y = -rho (J Delta x + c) + y_k - y (Sec. 3.3, eq. K1-elimination).
 * dx: n; c, y_k, y, dy: m. */
int ncl_kkt_recover_dy(ncl_kkt_t h, const double *J_val, const double *dx, const double *c,
                       const double *y_k, const double *y, double *dy, void *stream);

/* Delta r = theta (Delta y - y_k + y) - r, theta = 1 / rho (Sec. 3.2,
 * eq. K2-elimination).  All of length m. */
int ncl_kkt_recover_dr(ncl_kkt_t h, const double *dy, const double *y_k, const double *y,
                       const double *r, double *dr, void *stream);

/* Delta z_l = -(X - L)^-1 (Z_l Delta x - mu e) - z_l and
 * Delta z_u = (U - X)^-1 (Z_u Delta x + mu e) - z_u (Sec. 3.1, the blocks
 * eliminated from eq. K3).  All of length n; an infinite bound (l = -inf,
 * u = +inf) makes its quotient 0 (its multiplier should be 0).  Needs an
 * analyzed device handle, not a factor.  mu must be finite. */
int ncl_kkt_recover_dz(ncl_kkt_t h, const double *x, const double *l, const double *u,
                       const double *z_l, const double *z_u, const double *dx, double mu,
                       double *dz_l, double *dz_u, void *stream);

/* Sigma = (X - L)^-1 Z_l + (U - X)^-1 Z_u, the barrier diagonal (Sec. 3.1,
 * below eq. K2unreg; Sigma_t and Sigma_s are its t and s parts).  Length n;
 * infinite bounds give zero terms.  Needs an analyzed device handle. */
int ncl_kkt_barrier_sigma(ncl_kkt_t h, const double *x, const double *l, const double *u,
                          const double *z_l, const double *z_u, double *sigma, void *stream);

/* Solve K X = B for nrhs >= 1 columns (device, column-major, leading
 * dimensions >= order), with FP64 iterative refinement against the
 * unperturbed K (Sec. 4.3); refinement runs only when the inertia is the
 * expected one.  B and X must not overlap.  info may be NULL.  Returns
 * NCL_WARN_IR_NOT_CONVERGED when refinement stops short of its criterion
 * (ir_tol, ir_cw_tol), and NCL_WARN_FELL_BACK_FP64 when the FP32 factor had to
 * be replaced (then the solve refactors in FP64 from the assembled K). */
int ncl_kkt_solve(ncl_kkt_t h, const double *B, int64_t ldb, double *X, int64_t ldx,
                  int32_t nrhs, void *stream, ncl_kkt_solve_info *info);

/* Inertia of the last factorization (Sec. 3.4): counts of positive,
 * negative and zero pivots after the static-pivot rule, and how many pivots
 * the rule replaced.  Batched handles: totals over systems.  Host outputs. */
int ncl_kkt_inertia(ncl_kkt_t h, int64_t *npos, int64_t *nneg, int64_t *nzero,
                    int64_t *nperturbed);

/* Per-system inertia of a batched handle: out[4*s + {0,1,2,3}]. */
int ncl_kkt_inertia_batched(ncl_kkt_t h, int64_t *out);

/* Adjoint of X = K^-1 B for the condensed form K = W + Sigma + rho J^T J
 * (Sec. 3.3, eq. K1) in reverse mode.  Given the solution X and
 * Lambda = K^-1 Xbar (the adjoint solve: K is symmetric, so it is an ordinary
 * ncl_kkt_solve on the same factor), writes (device arrays, overwritten):
 *   gW[e]  = -sum_c (Lambda_ic X_jc + Lambda_jc X_ic) for a stored lower W
 *            entry e = (i, j), i != j;  -sum_c Lambda_ic X_ic when i == j;
 *   gSigma[i] = -sum_c Lambda_ic X_ic;
 *   gJ[k]  = -rho sum_c [Lambda_ic (J X_c)_r + X_ic (J Lambda_c)_r], k = (r, i);
 *   gRho[s] = -sum_c (J Lambda_c) . (J X_c)   (one value per system).
 * J_val are the Jacobian values of the last factorization (device).  X and
 * Lambda share the leading dimension ld; 1 <= nrhs <= 16.  Any of gW,
 * gSigma, gJ, gRho may be NULL.  Stream-ordered, no synchronization.
 * NCL_ERR_STATE after ncl_kkt_factor_k1s (the factor is then of K1s). */
int ncl_kkt_backward(ncl_kkt_t h, const double *J_val, const double *X, const double *Lambda, int64_t ld,
                     int32_t nrhs, double *gW, double *gSigma, double *gJ, double *gRho, void *stream);

/* ncl_kkt_backward for callers that cannot allocate device memory during the
 * call (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): same arguments, results and errors, but the staging of
 * J X and J Lambda (m x nrhs each) lives in the library's fixed device
 * scratch of 2^21 doubles (16 MiB, one copy per GPU, held until the process
 * ends) instead of the handle's workspace; it calls no allocator.  Returns
 * NCL_ERR_SCRATCH when 2 x m x nrhs > 2^21.  Calls that overlap on one GPU
 * share that scratch and race: order them on one stream.  Every value in it is
 * written by the call before it is read (nothing needs clearing). */
int ncl_kkt_backward_noalloc(ncl_kkt_t h, const double *J_val, const double *X, const double *Lambda, int64_t ld,
                             int32_t nrhs, double *gW, double *gSigma, double *gJ, double *gRho, void *stream);

int ncl_kkt_get_stats(ncl_kkt_t h, ncl_kkt_stats *st);

/* Fill-reducing permutation in use: perm[k] = unpermuted index of pivot k. */
int ncl_kkt_get_perm(ncl_kkt_t h, int32_t *perm);

/* Supernode partition (in pivot order): first[s] .. first[s+1]-1 are the
 * pivots of supernode s (first has n_supernodes+1 entries); parent[s] is the
 * parent supernode or -1; row_ptr (n_supernodes+1) / rows give each front's
 * row list in pivot numbering (pivots first, then the contribution rows).
 * Pass NULL for rows to query only row_ptr. */
int ncl_kkt_get_supernodes(ncl_kkt_t h, int32_t *first, int32_t *parent, int64_t *row_ptr,
                           int32_t *rows);

/* Kernel timing.  When enabled, factor and solve record HIP events around
 * every kernel class on the caller's stream and accumulate device time (ms)
 * and launch counts, readable with ncl_kkt_get_timing. */
typedef struct {
    double ms[8];          /* 0 assemble, 1 small fronts, 2 large-front assembly,
                              3 large-front panel solve, 4 large-front trailing update (MFMA)
                              with the next panel's diagonal blocks in the same launch,
                              5 forward/backward solve, 6 residual,
                              7 large-front first-panel diagonal blocks (LDL^T + inverse) */
    int64_t launches[8];
    /* Algorithmic work of the timed launches.  Flops of a front are scaled by
     * its exact / executed ratio and bytes of L by its exact / stored ratio
     * (amalgamation padding is not work); explicit inverses are not counted. */
    double update_flops;   /* update launches (tiles and the diagonal blocks launched with them) */
    double small_flops;    /* small-front launches */
    double assemble_bytes; /* assembly: 8 (nnz(W) + nnz(J) + n + nnz(lower K)) per launch */
    double solve_bytes;    /* solve sweeps: L read once per sweep (FP64 size: 8 bytes an entry) */
    double panel_flops;    /* panel-solve launches (rows x w^2) */
    double diag_flops;     /* first-panel diagonal-block launches: per block w^3/3 (LDL^T) */
} ncl_kkt_timing;

int ncl_kkt_set_timing(ncl_kkt_t h, int32_t enable);   /* enabling also clears totals */
int ncl_kkt_get_timing(ncl_kkt_t h, ncl_kkt_timing *t);

/* Per-system device times of the last factor and solve of a handle factored
 * by the persistent launch (options.persistent), in milliseconds from the start
 * of that factor launch: factor_ms[s] = when system s's factorization
 * finished, solve_ms[s] = when its last triangular sweep finished.  Host arrays
 * of `count` (= number of systems) entries; either may be NULL.  While the
 * persistent launches are disabled no handle has these: NCL_ERR_STATE. */
int ncl_kkt_get_system_times(ncl_kkt_t h, double *factor_ms, double *solve_ms);

void ncl_kkt_destroy(ncl_kkt_t h);
const char *ncl_kkt_strerror(int code);

/* ---- Algorithm 1 on a convex quadratic program ---------------------------
 *   min 1/2 x^T Q x + q^T x   s.t.  A x = b,  l <= x <= u
 * (the problem family NCO of Sec. 3 with equality rows only; entries of l, u
 * may be -inf / +inf).  Algorithm 1 (MadNCL, Sec. 2.3): outer iterations on
 * the NCL subproblem with multiplier estimate y_k, penalty rho and barrier mu;
 * each first tries the extrapolation step (eq. ncl:extrapolation, accepted
 * when ||F_k(w + alpha d)|| <= theta ||F_k(w)|| + 10 alpha^0.2 mu), else takes
 * Newton steps until ||F_k||_inf <= omega_k (F_k of eq. kktnclipm); then
 * y_k += rho r and mu, eta, omega shrink when ||r||_inf <= eta_k, else
 * rho *= 10 (at most 1e14).  Every Newton direction is one ncl_kkt_factor +
 * ncl_kkt_solve of K1 = Q + Sigma + rho A^T A (Sec. 3.3, eq. K1) on a
 * condensed handle analysed once (static pivots by the absolute rule, refinement
 * to a componentwise backward error of 1e-14: Sigma spans many decades near
 * the solution), then ncl_kkt_recover_dy, _dr, _dz.
 * Constants: gamma 0.05, tau 1.99, mu factor 0.2, theta 0.5, rho_0 100,
 * mu_0 0.1.  Where the paper leaves a choice open the driver takes:
 *   y_0 = 0, r_0 = -(A x_0 - b), z_0 = mu_0 / (distance to each finite bound);
 *   eta_0 and omega_0 from Algorithm 1's update formulas at mu_0;
 *   one step length for all variables, the largest <= 1 keeping x strictly
 *   inside and z positive, scaled by tau = max(0.99, 1 - mu), then halved (at
 *   most 30 times) until ||F_k||_inf does not increase;
 *   optimal when ||r||_inf <= eta_star, ||Q x + q - A^T y - z_l + z_u||_inf
 *   <= omega_star and max(z_l (x - l), z_u (u - x)) <= omega_star;
 *   infeasible when rho reached 1e14 and ||r||_inf > eta_star;
 *   mu >= min(eta_star, omega_star) / 10. */
typedef struct {
    double eta_star;      /* primal tolerance (default 1e-8) */
    double omega_star;    /* dual and complementarity tolerance (default 1e-8) */
    int32_t max_outer;    /* outer iterations (default 100) */
    int32_t max_inner;    /* Newton steps per inner loop (default 100) */
    int32_t precision;    /* of the KKT factor: NCL_FP64 (default) or NCL_FP32_IR */
    int32_t print_level;  /* 1: one line per outer iteration on stderr (rho, mu after the
                             update, ||F_k|| before and after the extrapolation step, its
                             alpha, accepted or not, inner steps, ||r||, dual and
                             complementarity measures); 0 (default): silent */
} ncl_qp_options;

typedef struct {
    int32_t status;       /* 0 optimal, 1 infeasible, 2 outer-iteration limit */
    int32_t outer;        /* outer iterations done */
    int32_t inner;        /* Newton steps taken in inner loops */
    int32_t extrapolated; /* outer iterations whose extrapolation step was accepted */
    double primal_inf;    /* ||A x - b||_inf at the returned x */
    double dual_inf;      /* ||Q x + q - A^T y - z_l + z_u||_inf at the returned point */
} ncl_qp_result;

void ncl_qp_default_options(ncl_qp_options *o);

/* Solves the QP above.  Patterns are host arrays: Q lower-triangular CSC
 * (Q_colptr[n+1], Q_rowidx sorted, row >= column, the diagonal stored), A CSR
 * m x n (A_rowptr[m+1], A_colidx sorted); m may be 0.  Values and vectors are
 * DEVICE arrays: Q_val (nnz of Q's lower part), q (n), A_val (nnz(A)), b (m),
 * l, u (n).  x (n) holds x_0 on entry, which must lie strictly inside every
 * finite bound (NCL_ERR_ARG otherwise), and the solution on return; y (m),
 * z_l, z_u (n) receive the multipliers (z 0 for infinite bounds).  res (host)
 * receives the status and counts.  Allocates its handle and work vectors on
 * the current device and frees them before returning; synchronizes the stream
 * several times per iteration (to read norms and step lengths).  Errors of the
 * KKT calls are returned as they are (NCL_ERR_NONFINITE for a non-finite
 * matrix, ...); x, y, z are then unspecified. */
int ncl_qp_solve(const ncl_qp_options *opt, int32_t n, int32_t m, const int32_t *Q_colptr,
                 const int32_t *Q_rowidx, const double *Q_val, const double *q,
                 const int32_t *A_rowptr, const int32_t *A_colidx, const double *A_val,
                 const double *b, const double *l, const double *u, double *x, double *y,
                 double *z_l, double *z_u, ncl_qp_result *res, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NCL_KKT_H */
