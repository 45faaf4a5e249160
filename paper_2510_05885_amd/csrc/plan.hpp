// plan.hpp — host-side symbolic plan of the supernodal multifrontal LDL^T.
//
// Everything here is computed once per sparsity pattern (the paper reuses the
// symbolic factorization across iterations, Sec. 4.1) and uploaded once.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ncl {

// Fronts of order above this bound use the global-memory path.  The LDS path
// stores a full front x front tile of T; the bound is set per plan from the
// device's LDS limit and the element size.
struct PlanConfig {
    int small_front_max = 90;   // fronts with f <= this run in one workgroup in LDS
    int panel = 64;             // pivot block width of the large-front path
    int tile = 64;              // tile order of the large-front update
    int nd_leaf = 64;           // nested-dissection leaf size (compressed vertices)
    int relax_big_front = 128;  // fronts above this order (the global-memory path, swept in
    double relax_big_zeros = 0.2;  // panels anyway) may carry up to this fraction of zeros
};

struct LevelBatch {            // one launch of the small-front kernel
    int level = 0;
    int fmax = 0;              // largest front in the batch (sets LDS size)
    int64_t first = 0, count = 0;  // range in Plan::small_list
};

struct LargeStep {             // launches of the large-front path for one level
    int level = 0;
    int64_t asm_first = 0, asm_count = 0;     // (front, column) tasks in large_asm
    int asm_fmax = 0;                         // largest front of the level (column buffer size)
    // per panel step k: diagonal-block, panel (TRSM) and update tasks
    std::vector<int64_t> diag_first, diag_count;
    std::vector<int64_t> panel_first, panel_count;
    std::vector<int64_t> upd_first, upd_count;
    std::vector<double> upd_flops;            // algorithmic flops of each update launch
};

// Solve schedule: a front with p <= 64 pivots and f <= 128 rows is swept by
// one wave; every other front in panels of up to 64 pivot columns, each panel
// split into tasks of up to 64 rows below it (one workgroup each).  Per level
// and panel index j, one launch of the one-wave fronts (j = 0) and one of the
// panel tasks.
struct SolveStep {
    int level = 0, j = 0;
    int64_t p_first = 0, p_count = 0;   // tasks in Plan::solve_p (kPTaskInts each)
    int64_t s_first = 0, s_count = 0;   // small fronts in Plan::solve_s (one wave each)
    int64_t f_first = 0, f_count = 0;   // j = 0 only: finish-only records in Plan::solve_p, run
                                        // after the level's backward steps
    double fwd_bytes = 0.0;             // algorithmic bytes of L read by the step (FP64; padding
                                        // zeros of amalgamated fronts not counted)
};

struct Plan {
    // ---- problem --------------------------------------------------------
    int form = 0;               // 0 condensed, 1 stabilized
    int S = 1;                  // number of independent systems (batched)
    int64_t N = 0;              // order of the (block-diagonal) matrix
    std::vector<int> sys_n, sys_m;
    std::vector<int64_t> sys_voff;   // S+1: first unpermuted index of each system
    std::vector<int64_t> sys_woff, sys_joff;  // offsets of each system's W / J values
    int64_t nnzW = 0, nnzJ = 0, nJrows = 0;
    std::vector<int> row_sys;        // N: system of each unpermuted index
    std::vector<int8_t> row_sign;    // N: +1 primal, -1 dual (unpermuted)

    // ---- full symmetric CSR of K (unpermuted), with value sources -------
    std::vector<int64_t> Kp;         // N+1
    std::vector<int> Kj;             // nnzF column indices
    std::vector<int> src_w;          // nnzF: W value index or -1
    std::vector<int> src_j;          // nnzF: J value index or -1 (stabilized J / J^T blocks)
    std::vector<uint8_t> src_flag;   // bit0: add Sigma[row]; bit1: add -1/rho
    std::vector<int64_t> prod_ptr;   // nnzF+1: pairs of J value indices (condensed)
    std::vector<int> prod_a, prod_b;
    int64_t nnz_lower = 0;

    // ---- J structure (for the adjoint) -----------------------------------
    std::vector<int64_t> Jp;          // rows of the concatenated J
    std::vector<int> Jj;              // unpermuted column indices (global)
    std::vector<int> Jrow_sys;
    std::vector<int64_t> Wcol_of;     // per stored W entry: global column; row in Wrow_of
    std::vector<int> Wrow_of, Wcol_of32;

    // ---- ordering --------------------------------------------------------
    std::vector<int> perm, iperm;    // perm[k] = unpermuted index of pivot k

    // ---- supernodes ------------------------------------------------------
    int nsn = 0;
    std::vector<int> sn_first;       // nsn+1
    std::vector<int> sn_parent;      // nsn
    std::vector<int64_t> sn_rowptr;  // nsn+1
    std::vector<int> sn_rows;        // pivot numbering; pivots first then CB rows
    std::vector<int> sn_level;
    std::vector<int> sn_sys;
    std::vector<int> child_ptr, child_list;
    std::vector<uint8_t> sn_large;

    // front assembly of K entries: per supernode (csr position, local position)
    std::vector<int64_t> kent_ptr;   // nsn+1
    std::vector<int64_t> kent_csr;
    std::vector<int> kent_pos;       // local row + local col * f
    std::vector<int> kent_col;       // local column (large fronts, sorted by it)
    std::vector<int64_t> kcol_ptr;   // large fronts: per (front, local col) segment, indexed by
    std::vector<int64_t> kcol_base;  //   kcol_base[s] + j, length p+1

    // extend-add maps: child CB row a -> local row in the parent front
    std::vector<int64_t> rel_ptr;    // nsn+1 (length c_s)
    std::vector<int> rel;
    // large parents: for each child, parent local row -> child CB index or -1
    std::vector<int64_t> inv_ptr;    // nsn+1 (length f_parent when the parent is large)
    std::vector<int> inv;

    // ---- storage ---------------------------------------------------------
    std::vector<int64_t> L_off;      // offset of front s's L (ld = f) in the factor buffer
    std::vector<int64_t> CB_off;     // offset of the contribution block
    std::vector<int> CB_ld;
    int64_t factor_elems = 0;        // factor buffer length (elements of T)
    std::vector<int64_t> U_off;      // solve: update vector of each front (c_s * nrhs_max)
    std::vector<int64_t> M_off;      // large fronts: per-panel inverses L_kk^-1 (panel^2 each)
    int64_t M_elems = 0;
    int64_t U_elems = 0;

    // ---- schedule --------------------------------------------------------
    int nlevels = 0;
    std::vector<int> small_list;     // supernodes, grouped by level then size batch
    std::vector<LevelBatch> small_batches;
    std::vector<int> level_ptr;      // nlevels+1 into level_list (all fronts by level)
    std::vector<int> level_list;
    std::vector<int> level_fmax;     // largest front of each level
    std::vector<LargeStep> large_steps;
    // large-front tasks
    std::vector<int> large_asm;      // pairs (front, column)
    // per large_asm task: column base in the factor buffer, (f, j), K-entry
    // range, and its contribution segments (children whose CB has a column
    // mapping to j): CB column offset, relative-index offset, (first row, rows)
    std::vector<int64_t> asm_col, asm_kr, asm_seg_ptr, asm_seg_cb, asm_seg_rel;
    std::vector<int> asm_fj, asm_seg_bc;
    std::vector<int> large_diag;     // pairs (front, k0): diagonal block update, factorization, inverse
    std::vector<int> large_panel;    // triples (front, k0, 32-row block start >= k0 + panel)
    std::vector<int> large_upd;      // quads (front, k0, tile row start, tile col start); the next
                                     // panel's diagonal tile is left to large_diag
    // persistent launches: fronts in topological order (level, then larger
    // first), per large front its column-assembly tasks (first, count) in
    // large_asm / asm_*, fronts per system, largest orders
    std::vector<int> pers_order;
    std::vector<int64_t> pers_asm;   // 2 per supernode (0, 0 for small fronts)
    std::vector<int> sys_nfronts;
    int pers_fmax_large = 0, pers_fmax_small = 0, pers_fmax = 0;
    // solve schedule
    std::vector<SolveStep> solve_steps;
    std::vector<int> solve_pan;      // panels (s, c0, w, slot0, tasks, seg0, nseg)
    std::vector<int> solve_p;        // tasks (panel, r0, r1, index, seg0, nseg); index -1: finish only
    std::vector<int> solve_fin;      // per task: the panel it finishes in the backward sweep
                                     // (c0, w, slot0, tasks), tasks 0 if none
    std::vector<int> solve_seg;      // (child, a0, a1): update-vector entries landing in a task
    // forward sweep: its own steps (j = step index k of the level) and tasks
    // (as solve_p, panel = the step's first panel), with per task (w2,
    // seg0, nseg, 0): the second panel's width (0: one panel) and its pivot
    // rows' contribution segments
    std::vector<SolveStep> fsolve_steps;
    std::vector<int> fsolve_p, fsolve_x;
    std::vector<int> solve_s;        // small fronts (p <= 64, f <= 128) solved by one wave each
    int64_t solve_max_slots = 0;     // tasks in the largest step (partial-sum slots)

    // ---- stats ------------------------------------------------------------
    int64_t nnzL = 0;
    double flops = 0.0, small_flops = 0.0, large_flops = 0.0;   // as executed (padding included)
    int64_t nnzL_exact = 0;          // column counts of the elimination tree (no padding)
    double flops_exact = 0.0;        // sum over columns of c (c + 2), c = below-diagonal count
    std::vector<double> sn_flop_ratio;  // per supernode: exact / executed flops of its pivots
    std::vector<double> sn_nnz_ratio;   // per supernode: exact / stored entries of its L columns
    int max_front = 0;
    int n_large = 0;
    double analyze_seconds = 0.0;
    PlanConfig cfg;
};


}  // namespace ncl
