// kernels.hpp — device-side plan and launchers of the KKT factor/solve kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>


namespace ncl {

constexpr int kNrhsMax = 16;   // columns per solve sweep (wider solves are chunked)
constexpr int kPanel = 64;       // pivot block width of the large-front path
constexpr int kSmallMax = 128;   // largest front order of the LDS-resident path
constexpr int kTile = 64;        // tile order of the large-front MFMA update
constexpr int kSolveRowsMax = 256;  // rows below a solve panel per task (fewer for wide panels)
constexpr int kPanInts = 7;      // ints per solve panel: s, c0, w, slot0, tasks, seg0, nseg
constexpr int kPTaskInts = 6;    // ints per solve task: panel, r0, r1, index, seg0, nseg
// A sweep task as the kernels read it: the task, its panel and its front in
// one record, so that one round trip brings everything the task needs.
//   ints  0..5   the task (panel, r0, r1, index, seg0, nseg)
//   ints  6..12  the panel (s, c0, w, slot0, tasks, seg0, nseg)
//   ints 13..15  the front (first pivot, pivots p, order f)
//   int64 at ints 16, 18, 20, 22: L_off, U_off, M_off, first row-list entry
//   ints 24..27  backward: the panel this task finishes (c0, w, slot0, tasks; tasks 0: none)
//   ints 28..31  forward: the second panel's width (0: one panel), its pivot rows' segments
//                (first, count), 0
constexpr int kTaskRec = 32;
constexpr int kTaskRec64 = 16;
constexpr int kInertiaSlots = 64;  // partial inertia counters per system (spreads the atomics)
constexpr int kNonfiniteInput = 1;   // status bit: NaN/Inf in the assembled K (its norms)
constexpr int kNonfiniteFactor = 4;  // status bit: NaN/Inf pivot met by the factorization
constexpr int kResWidth = 6;         // residual figures per (row chunk, column), see launch_residual
constexpr size_t kAsmLdsMax = 96 * 1024;  // large-front column assembly staged in LDS (4 columns per
                                           // workgroup) up to this size

// Device copies of the plan (all device pointers), passed by value.
struct DevPlan {
    int64_t N;
    int64_t n_primal;          // rows [0, n_primal) form the primal block (N for the condensed form)
    int S;
    int form;
    int n_fronts;              // supernodes (fronts)
    // full CSR of K with value sources
    const int64_t* Kp;
    const int* Kj;
    const int* Krow;
    const int* src_w;
    const int* src_j;
    const uint8_t* src_flag;
    const int64_t* prod_ptr;
    const int* prod_a;
    const int* prod_b;
    const int* row_sys;
    const int8_t* row_sign;
    const int* perm;
    // supernodes
    const int* sn_first;
    const int64_t* sn_rowptr;
    const int* sn_rows;
    const int* child_ptr;
    const int* child_list;
    const int* sn_sys;
    const int* sn_parent;      // parent supernode or -1
    const int* jrow_of;        // row of J of each stored J entry (condensed form)
    const int64_t* kent_ptr;
    const int64_t* kent_csr;
    const int* kent_pos;
    const int64_t* kcol_ptr;
    const int64_t* kcol_base;
    const int64_t* rel_ptr;
    const int* rel;
    const int64_t* inv_ptr;
    const int* inv;
    const int64_t* L_off;
    const int64_t* CB_off;
    const int* CB_ld;
    const int64_t* U_off;      // in elements of one column block (times kNrhsMax applied)
    const int64_t* M_off;      // large fronts: offset of the per-panel inverses L_kk^-1 (64 x 64 each)
    // large-front column assembly tasks (see Plan::asm_*)
    const int64_t* asm_col;
    const int* asm_fj;
    const int64_t* asm_kr;
    const int64_t* asm_seg_ptr;
    const int64_t* asm_seg_cb;
    const int64_t* asm_seg_rel;
    const int* asm_seg_bc;
    // per system
    const double* sys_thr;     // static-pivot thresholds, 2 per system: primal, dual pivots
    unsigned long long* inertia;  // 4 per system: npos, nneg, nzero, nperturbed
    unsigned long long* inertia_part;  // kInertiaSlots x 4 per system, summed into inertia
    int* nonfinite;            // status bits kNonfiniteInput | kNonfiniteFactor
};

// ---- assembly (FP64) ------------------------------------------------------
// Optional per-launch timing.  While a LaunchTimer is installed on the
// calling thread, every kernel launch asks it for a start/stop event pair and,
// when given one, is launched with hipExtLaunchKernel, whose events carry the
// kernel's own begin and end timestamps (no launch gaps in the figure).
struct LaunchTimer {
    virtual bool take(hipEvent_t* start, hipEvent_t* stop) = 0;
    virtual ~LaunchTimer() = default;
};
LaunchTimer* set_launch_timer(LaunchTimer* t);   // returns the previous one

// omega: per row of J, the weight of its products (K1s), or nullptr (K1, K2r).
void launch_assemble(const DevPlan& d, int64_t nnzF, const double* W, const double* Sigma, const double* J,
                     const double* sys_rho, const double* omega, double* K, hipStream_t st);
// ---- slack elimination (K1s) and step recovery (vectors in the caller's
// order; rows of J of all systems concatenated; rho per system) -------------
void launch_k1s_omega(int64_t nrows, const double* Sigma_s, const int* Jrow_sys, const double* sys_rho, double* omega,
                      int* nonfinite, hipStream_t st);
void launch_k1s_rhs(int64_t n, const int64_t* Jt_ptr, const int* Jt_row, const int* Jt_k, const double* J,
                    const double* r_t, const double* r_s, const double* Sigma_s, const int* Jrow_sys,
                    const double* sys_rho, const int* row_sys, double* b, hipStream_t st);
void launch_k1s_ds(int64_t nrows, const int64_t* Jp, const int* Jj, const double* J, const double* dt,
                   const double* r_s, const double* Sigma_s, const int* Jrow_sys, const double* sys_rho, double* ds,
                   hipStream_t st);
void launch_recover_dy(int64_t nrows, const int64_t* Jp, const int* Jj, const double* J, const double* dx,
                       const double* c, const double* y_k, const double* y, const int* Jrow_sys, const double* sys_rho,
                       double* dy, hipStream_t st);
void launch_recover_dr(int64_t nrows, const double* dy, const double* y_k, const double* y, const double* r,
                       const int* Jrow_sys, const double* sys_rho, double* dr, hipStream_t st);
void launch_recover_dz(int64_t n, const double* x, const double* l, const double* u, const double* z_l,
                       const double* z_u, const double* dx, double mu, double* dz_l, double* dz_u, hipStream_t st);
void launch_add_scalar(int64_t n, const double* in, double delta, double* out, hipStream_t st);
void launch_barrier_sigma(int64_t n, const double* x, const double* l, const double* u, const double* z_l,
                          const double* z_u, double* sigma, hipStream_t st);
// Block per chunk of rows: partial[3c..3c+2] = max |K_ij|, max row sum of |K|,
// max |K_ij| over the primal block.
void launch_chunk_norms(const DevPlan& d, const double* K, const int* chunk_row0, const int* chunk_rows, int nchunks,
                        double* partial, hipStream_t st);
// out[s*width + k] = reduction over the chunks of system s of partial[c*width + k]:
// a sum where bit (k mod period) of sum_mask is set, else a max.  Fixed order
// (deterministic).  1 <= period <= 32.
void launch_reduce(const int* sys_chunk_ptr, int S, int width, int period, unsigned int sum_mask,
                   const double* partial, double* out, hipStream_t st);
// kmax, kinf and the two static-pivot thresholds per system (thr[2s] primal,
// thr[2s+1] dual) from the reduced norms.  mode 0: eps * max |K_ij| for both;
// 1, block rule: primal eps * max |K_xx|, dual eps / rho; 2: eps for both.
// Flags non-finite norms.
void launch_thresholds(int S, const double* norms3, double eps, int mode, const double* sys_rho, double* kmax,
                       double* kinf, double* thr, int* nonfinite, hipStream_t st);

// ---- numeric factorization (T = double or float) --------------------------
template <typename T>
void launch_small_fronts(const DevPlan& d, const int* list, int count, int fmax, const double* K, T* F, T* D,
                         hipStream_t st);
template <typename T>
void launch_large_asm(const DevPlan& d, int64_t first, int count, int fmax, const double* K, T* F, hipStream_t st);
template <typename T>
void launch_large_diag(const DevPlan& d, const int* tasks, int count, T* F, T* D, T* M, hipStream_t st);
template <typename T>
void launch_large_panel(const DevPlan& d, const int* tasks, int count, T* F, const T* D, const T* M, hipStream_t st);
// Panel k's trailing update (utasks) and panel k+1's diagonal blocks (dtasks)
// in one launch.
template <typename T>
void launch_large_dstep(const DevPlan& d, const int* dtasks, int nd, const int* utasks, int nu, T* F, T* D, T* M,
                        hipStream_t st);

// ---- persistent launches (batched systems) ----------------------------------
// One launch factors every front: workgroups take fronts from *ticket in
// topological order, wait until the front's children are done, factor the
// whole front themselves and signal the parent.  ctr holds nsn child-done
// counters; ctr and *ticket start at zero (the ticket on a cache line of its
// own).  A wait gives up after `timeout` wall_clock64 ticks and sets bit 1 of
// *status (the results are then invalid, but the launch ends).  tstamp[0] =
// launch start, tstamp[1 + sys] = completion of the system's last root front.
// asm_rng: per large front (first column task, count); lds_elems: dynamic LDS
// per workgroup (elements of T) >= max(small front f^2, 4 x largest large front).
template <typename T>
void launch_persist_factor(const DevPlan& d, const int* order, int ntask, const int64_t* asm_rng, int fcap,
                           int lds_elems, int grid, int* ctr, int* ticket, int* status, unsigned long long timeout,
                           unsigned long long* tstamp, const double* K, T* F, T* D, T* M, hipStream_t st);
// One launch for both sweeps: tickets [0, nsn) forward in topological order,
// [nsn, 2 nsn) backward in reverse.  ctr: 3 nsn + S ints (children forward
// done, forward done, backward done, per-system backward count), zero like
// *ticket.  tstamp[1 + S + sys] = completion of the system's backward sweep.
// fcap >= every front order; LDS = fcap x nrhs + 64 x 65 + 256 x nrhs of T.
template <typename T>
void launch_persist_solve(const DevPlan& d, const int* order, int nsn, const int* sys_nfronts, int fcap, int grid,
                          int* ctr, int* ticket, int* status, unsigned long long timeout, unsigned long long* tstamp,
                          const T* F, const T* Z, const T* D, const T* Y, T* Y2, T* U, int nrhs,
                          hipStream_t st);

// ---- solves -----------------------------------------------------------------
template <typename T>
void launch_permute_in(const DevPlan& d, const double* B, int64_t ldb, int nrhs, T* Y, hipStream_t st);
template <typename T>
void launch_permute_out(const DevPlan& d, const T* Y, int nrhs, double* X, int64_t ldx, hipStream_t st);
// Y: right-hand side in pivot order (updated in place by the forward sweep
// for rows that are not yet solved); Y2: the pivots' y after the forward sweep,
// their x after the backward sweep.  One-wave fronts (p <= 64, f <= 128):
template <typename T>
void launch_fwd_S(const DevPlan& d, const int* fronts, int count, const T* F, const T* Y, T* Y2, T* U, int nrhs,
                  hipStream_t st);
template <typename T>
void launch_bwd_S(const DevPlan& d, const int* fronts, int count, const T* F, const T* D, T* Y2, int nrhs,
                  hipStream_t st);
// The other fronts, one launch per panel step of a level (task records of
// kTaskRec ints, contribution segments: see the sweep kernels).  Backward:
// the step's task sums go to pw, the previous step's are read from pr (each
// slots x kPanel x kNrhsMax, two halves used in turn).
template <typename T>
void launch_fwd_P(const DevPlan& d, const int* tasks, int count, const int* segs, const T* F,
                  const T* Z, T* Y, T* Y2, T* U, int nrhs, hipStream_t st);
template <typename T>
void launch_bwd_P(const DevPlan& d, const int* tasks, int count, const T* F, const T* Z,
                  const T* D, T* Y2, T* pw, const T* pr, int nrhs, hipStream_t st);

// ---- refinement -------------------------------------------------------------
// R = B - K X; per chunk of rows (all of one system) and column, kResWidth figures:
// max |r|, max |x|, max |b|, sum r^2, sum b^2, max |r_i| / (|K||x| + |b|)_i.
void launch_residual(const DevPlan& d, const double* K, const double* B, int64_t ldb, const double* X,
                     int64_t ldx, double* R, int nrhs, const int* chunk_row0, const int* chunk_rows, int nchunks,
                     double* partial, hipStream_t st);
void launch_axpy_cols(double* X, int64_t ldx, const double* DX, int64_t N, int nrhs, hipStream_t st);
void launch_copy_cols(double* dst, int64_t ldd, const double* src, int64_t lds, int64_t N, int nrhs,
                      hipStream_t st);
void launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t st);
void launch_zero_i32(int* p, int64_t n, hipStream_t st);
void launch_reduce_inertia(const DevPlan& d, int S, hipStream_t st);   // inertia = sum of the partials

// Raises the dynamic-LDS limit of the LDS-resident kernels to the device maximum.
hipError_t configure_kernels(int max_dynamic_lds);
// Static LDS bytes of the persistent factorization kernel (FP64 or FP32), -1 on error.
int persist_factor_static_lds(int fp32);

// ---- adjoint (condensed) ----------------------------------------------------
void launch_adjoint(const DevPlan& d, int64_t nnzW, const int* W_row, const int* W_col, int64_t nJrows,
                    const int64_t* Jp, const int* Jj, const int* Jrow_sys, const double* Jval, const double* sys_rho,
                    const double* X, const double* Lam, int64_t ld, int nrhs, double* gW, double* gSigma,
                    double* gJ, double* gRho, double* JX, double* JL, const int64_t* sys_jrow, hipStream_t st);

}  // namespace ncl
