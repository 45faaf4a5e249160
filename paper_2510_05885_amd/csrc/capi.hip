// capi.hip — C ABI of the KKT factor/solve library (see include/ncl_kkt.h).
//
// Owns the handle: the host plan, every device buffer (allocated once at
// analyze time) and the per-call orchestration of the kernels:
//   factor = assemble K (Sec. 3.3 eq. K1 / Sec. 3.2 eq. K2r) -> norms and
//            static-pivot thresholds -> level-by-level frontal LDL^T ->
//            inertia read-back (Sec. 3.4);
//   solve  = permute -> forward sweep -> D^-1 + backward sweep -> unpermute,
//            then Richardson refinement against the unperturbed K in FP64
//            (Sec. 4.3), with an FP64 refactor when an FP32 factor stalls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/ncl_kkt.h"
#include "analyze.hpp"
#include "kernels.hpp"

using namespace ncl;

namespace {

struct HipError {
    hipError_t e;
};

#define HIPCHK(x)                                  \
    do {                                           \
        hipError_t e_ = (x);                       \
        if (e_ != hipSuccess) throw HipError{e_};  \
    } while (0)

struct Timer {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec { int cls; size_t a, b; double work; int kind; };
    std::vector<Rec> recs;
    ncl_kkt_timing tot{};
};

}  // namespace

// Staging memory of ncl_kkt_backward_noalloc: a file-scope device array, one
// copy per GPU, held until the process ends.  Host code never passes its name
// to a kernel: the device address comes from hipGetSymbolAddress, resolved
// once per device with that device current.
constexpr int64_t kScratchDoubles = int64_t(1) << 21;   // 16 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_on_device(int dev, double** out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

struct ncl_kkt_s {
    Plan P;
    ncl_kkt_options opt{};
    double eps = 0.0;
    int pivot_mode = 0;               // thresholds: 0 global, 1 per block (stabilized), 2 absolute
    // persistent launches (options.persistent)
    bool pers = false;
    int *pers_order = nullptr, *pers_ctr = nullptr, *pers_status = nullptr, *sys_nfronts = nullptr;
    int64_t* pers_asm = nullptr;
    unsigned long long* tstamp = nullptr;
    int pers_grid_f = 0, pers_grid_s = 0, pers_lds_elems = 0, max_lds = 0;
    int64_t pers_ctr_len = 0;
    int* pers_ticket = nullptr;
    unsigned long long pers_timeout = 0;
    double wall_khz = 0.0;
    bool pers_solved = false;
    int nonfinite_bits = 0;           // status word of the last factorization read back
    bool host_only = true;
    int device = 0;
    std::vector<void*> allocs;
    int64_t dev_bytes = 0;
    DevPlan d{};
    int64_t nnzF = 0;
    // schedule arrays (device)
    int *small_list = nullptr, *level_list = nullptr, *large_asm = nullptr, *large_panel = nullptr,
        *large_upd = nullptr, *large_diag = nullptr, *solve_p = nullptr, *solve_seg = nullptr, *solve_s = nullptr,
        *fsolve_p = nullptr;
    int *chunk_row0 = nullptr, *chunk_rows = nullptr, *sys_chunk_ptr = nullptr;
    int nchunks = 0;
    // numeric state
    double *K = nullptr, *partial_norm = nullptr, *norms3 = nullptr, *kmax = nullptr, *kinf = nullptr,
           *thr = nullptr, *rho = nullptr;
    int* nonfinite = nullptr;
    unsigned long long* inertia = nullptr;
    unsigned long long* inertia_part = nullptr;
    double *F64 = nullptr, *D64 = nullptr, *Y64 = nullptr, *U64 = nullptr, *P64 = nullptr, *M64 = nullptr;
    float *F32 = nullptr, *D32 = nullptr, *Y32 = nullptr, *U32 = nullptr, *P32 = nullptr, *M32 = nullptr;
    double *R = nullptr, *DX = nullptr, *Xp = nullptr, *partial_res = nullptr, *res_out = nullptr;
    double *JX = nullptr, *JL = nullptr;
    // slack elimination: J^T in CSC (row, value index per entry), Omega of the
    // last factor_k1s call; `weighted` while the factor is of K1s
    int64_t* Jt_ptr = nullptr;
    int *Jt_row = nullptr, *Jt_k = nullptr;
    double* omega = nullptr;
    bool weighted = false;
    double* sigma_shift = nullptr;   // Sigma + delta of the inertia correction (allocated on first use)
    int *W_row = nullptr, *W_col = nullptr, *Jj = nullptr, *Jrow_sys = nullptr;
    int64_t *Jp = nullptr, *sys_jrow = nullptr;
    double* host_pinned = nullptr;   // read-back staging
    size_t host_pinned_len = 0;
    // host state
    std::vector<double> h_rho, h_kinf;
    std::vector<int64_t> h_inertia;   // 4 per system
    int factored = 0;                 // 1 after a successful factor
    int factor_prec = 0;              // precision of the factor in use (0 FP64, 1 FP32)
    bool inertia_ok = false;
    bool fell_back = false;
    // FP32_IR: smallest max-rho at which an FP32 factor had to be replaced
    double fp32_rho_limit = HUGE_VAL;
    double cur_rho_max = 0.0;
    Timer tm;
    // HIP graphs of the fixed launch sequences (per precision; sweeps per nrhs)
    hipStream_t cap_stream = nullptr;
    // second stream: a level's small fronts run beside its large-front chain
    hipStream_t aux_stream = nullptr;
    std::vector<hipEvent_t> lvl_ev;   // 2 per level: fork, join
    // fourth stream: a level's small-front batches split over two streams
    hipStream_t aux2_stream = nullptr;
    std::vector<hipEvent_t> sb_ev;    // 2 per level: fork, join of the second batch stream
    hipGraphExec_t g_factor[2] = {nullptr, nullptr};
    hipGraphExec_t g_sweep[2][kNrhsMax + 1] = {};
};

namespace {

template <typename T>
T* dalloc(ncl_kkt_s* h, int64_t n) {
    void* p = nullptr;
    if (n <= 0) n = 1;
    HIPCHK(hipMalloc(&p, sizeof(T) * (size_t)n));
    h->allocs.push_back(p);
    h->dev_bytes += (int64_t)(sizeof(T) * (size_t)n);
    return static_cast<T*>(p);
}

template <typename T>
T* upload(ncl_kkt_s* h, const std::vector<T>& v) {
    T* p = dalloc<T>(h, (int64_t)v.size());
    if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return p;
}

// ----- timing helpers ------------------------------------------------------
enum { TM_ASM = 0, TM_SMALL = 1, TM_LASM = 2, TM_PANEL = 3, TM_UPD = 4, TM_SOLVE = 5, TM_RES = 6, TM_DIAG = 7 };

// While a Span is alive (timing enabled), every kernel launched on this
// thread gets its own event pair (the kernel's begin/end timestamps) and
// counts as one launch of class `cls`; the Span's algorithmic work is booked
// once, with its first launch.
struct Span : LaunchTimer {
    ncl_kkt_s* h;
    int cls;
    double work;
    int kind;  // 0 none, 1 update flops, 2 small flops, 3 assembly bytes, 4 solve bytes,
               // 5 panel-solve flops, 6 diagonal-block flops
    LaunchTimer* prev = nullptr;
    bool installed = false;
    Span(ncl_kkt_s* h_, hipStream_t, int c, double w = 0.0, int k = 0) : h(h_), cls(c), work(w), kind(k) {
        if (!h->tm.on) return;
        prev = set_launch_timer(this);
        installed = true;
    }
    ~Span() override {
        if (installed) set_launch_timer(prev);
    }
    bool take(hipEvent_t* e0, hipEvent_t* e1) override {
        if (!h->tm.on) return false;
        if (h->tm.used + 2 > h->tm.pool.size()) { h->tm.on = false; return false; }
        const size_t a = h->tm.used++, b = h->tm.used++;
        *e0 = h->tm.pool[a];
        *e1 = h->tm.pool[b];
        h->tm.recs.push_back({cls, a, b, work, kind});
        work = 0.0;
        return true;
    }
};

void flush_timing(ncl_kkt_s* h) {
    if (h->tm.recs.empty()) { h->tm.used = 0; return; }
    for (auto& r : h->tm.recs) {
        float ms = 0.f;
        HIPCHK(hipEventSynchronize(h->tm.pool[r.b]));
        HIPCHK(hipEventElapsedTime(&ms, h->tm.pool[r.a], h->tm.pool[r.b]));
        h->tm.tot.ms[r.cls] += ms;
        h->tm.tot.launches[r.cls] += 1;
        if (r.kind == 1) h->tm.tot.update_flops += r.work;
        if (r.kind == 2) h->tm.tot.small_flops += r.work;
        if (r.kind == 3) h->tm.tot.assemble_bytes += r.work;
        if (r.kind == 4) h->tm.tot.solve_bytes += r.work;
        if (r.kind == 5) h->tm.tot.panel_flops += r.work;
        if (r.kind == 6) h->tm.tot.diag_flops += r.work;
    }
    h->tm.recs.clear();
    h->tm.used = 0;
}

// ----- device setup ----------------------------------------------------------
void setup_device(ncl_kkt_s* h) {
    Plan& P = h->P;
    HIPCHK(hipGetDevice(&h->device));
    DevPlan& d = h->d;
    d.N = P.N;
    d.n_primal = P.form == NCL_STABILIZED ? P.sys_n[0] : P.N;
    d.S = P.S;
    d.n_fronts = P.nsn;
    d.form = P.form;
    h->nnzF = (int64_t)P.Kj.size();
    std::vector<int> Krow(h->nnzF);
    for (int64_t i = 0; i < P.N; ++i)
        for (int64_t q = P.Kp[i]; q < P.Kp[i + 1]; ++q) Krow[q] = (int)i;
    d.Kp = upload(h, P.Kp);
    d.Kj = upload(h, P.Kj);
    d.Krow = upload(h, Krow);
    d.src_w = upload(h, P.src_w);
    d.src_j = upload(h, P.src_j);
    d.src_flag = upload(h, P.src_flag);
    d.prod_ptr = upload(h, P.prod_ptr);
    d.prod_a = upload(h, P.prod_a);
    d.prod_b = upload(h, P.prod_b);
    d.row_sys = upload(h, P.row_sys);
    d.row_sign = upload(h, P.row_sign);
    d.perm = upload(h, P.perm);
    d.sn_first = upload(h, P.sn_first);
    d.sn_rowptr = upload(h, P.sn_rowptr);
    d.sn_rows = upload(h, P.sn_rows);
    d.child_ptr = upload(h, P.child_ptr);
    d.child_list = upload(h, P.child_list);
    d.sn_sys = upload(h, P.sn_sys);
    d.sn_parent = upload(h, P.sn_parent);
    d.kent_ptr = upload(h, P.kent_ptr);
    d.kent_csr = upload(h, P.kent_csr);
    d.kent_pos = upload(h, P.kent_pos);
    d.kcol_ptr = upload(h, P.kcol_ptr);
    d.kcol_base = upload(h, P.kcol_base);
    d.rel_ptr = upload(h, P.rel_ptr);
    d.rel = upload(h, P.rel);
    d.inv_ptr = upload(h, P.inv_ptr);
    d.inv = upload(h, P.inv);
    d.L_off = upload(h, P.L_off);
    d.CB_off = upload(h, P.CB_off);
    d.CB_ld = upload(h, P.CB_ld);
    std::vector<int64_t> uo(P.U_off);
    for (auto& x : uo) x *= kNrhsMax;
    d.U_off = upload(h, uo);
    d.M_off = upload(h, P.M_off);
    d.asm_col = upload(h, P.asm_col);
    d.asm_fj = upload(h, P.asm_fj);
    d.asm_kr = upload(h, P.asm_kr);
    d.asm_seg_ptr = upload(h, P.asm_seg_ptr);
    d.asm_seg_cb = upload(h, P.asm_seg_cb);
    d.asm_seg_rel = upload(h, P.asm_seg_rel);
    d.asm_seg_bc = upload(h, P.asm_seg_bc);
    h->small_list = upload(h, P.small_list);
    h->level_list = upload(h, P.level_list);
    h->large_asm = upload(h, P.large_asm);
    h->large_diag = upload(h, P.large_diag);
    {
        // every sweep task with its panel's and its front's fields (kTaskRec
        // ints): the backward tasks (with the panel each finishes) and the
        // forward ones (with their second panel)
        auto records = [&](const std::vector<int>& tasks, const std::vector<int>* fin,
                           const std::vector<int>* fx) {
            const size_t nt = tasks.size() / kPTaskInts;
            std::vector<int> rec(std::max<size_t>(nt, 1) * kTaskRec, 0);
            for (size_t t = 0; t < nt; ++t) {
                int* r = rec.data() + t * kTaskRec;
                const int* tk = tasks.data() + t * kPTaskInts;
                const int* pn = P.solve_pan.data() + (size_t)tk[0] * kPanInts;
                const int s = pn[0];
                for (int i = 0; i < kPTaskInts; ++i) r[i] = tk[i];
                for (int i = 0; i < kPanInts; ++i) r[kPTaskInts + i] = pn[i];
                r[13] = P.sn_first[s];
                r[14] = P.sn_first[s + 1] - P.sn_first[s];
                r[15] = (int)(P.sn_rowptr[s + 1] - P.sn_rowptr[s]);
                // U_off as on the device: room for kNrhsMax columns per front
                const int64_t v64[4] = {P.L_off[s], P.U_off[s] * kNrhsMax, P.M_off[s], P.sn_rowptr[s]};
                std::memcpy(r + kTaskRec64, v64, sizeof(v64));
                for (int i = 0; i < 4; ++i) {
                    if (fin) r[kTaskRec64 + 8 + i] = (*fin)[4 * t + i];
                    if (fx) r[kTaskRec64 + 12 + i] = (*fx)[4 * t + i];
                }
            }
            return rec;
        };
        h->solve_p = upload(h, records(P.solve_p, &P.solve_fin, nullptr));
        h->fsolve_p = upload(h, records(P.fsolve_p, nullptr, &P.fsolve_x));
    }
    h->solve_seg = upload(h, P.solve_seg);
    h->solve_s = upload(h, P.solve_s);
    h->large_panel = upload(h, P.large_panel);
    h->large_upd = upload(h, P.large_upd);
    // row chunks (<= 256 rows, never straddling two systems)
    std::vector<int> c0, cn, scp(1, 0);
    for (int s = 0; s < P.S; ++s) {
        for (int64_t r = P.sys_voff[s]; r < P.sys_voff[s + 1]; r += 256) {
            c0.push_back((int)r);
            cn.push_back((int)std::min<int64_t>(256, P.sys_voff[s + 1] - r));
        }
        scp.push_back((int)c0.size());
    }
    h->nchunks = (int)c0.size();
    h->chunk_row0 = upload(h, c0);
    h->chunk_rows = upload(h, cn);
    h->sys_chunk_ptr = upload(h, scp);
    // numeric buffers
    h->K = dalloc<double>(h, h->nnzF);
    h->partial_norm = dalloc<double>(h, 3 * (int64_t)h->nchunks);
    h->norms3 = dalloc<double>(h, 3 * P.S);
    h->kmax = dalloc<double>(h, P.S);
    h->kinf = dalloc<double>(h, P.S);
    h->thr = dalloc<double>(h, 2 * P.S);
    h->rho = dalloc<double>(h, P.S);
    h->nonfinite = dalloc<int>(h, 1);
    h->inertia = dalloc<unsigned long long>(h, 4 * P.S);
    h->inertia_part = dalloc<unsigned long long>(h, 4 * (int64_t)P.S * kInertiaSlots);
    d.sys_thr = h->thr;
    d.inertia = h->inertia;
    d.inertia_part = h->inertia_part;
    d.nonfinite = h->nonfinite;
    h->F64 = dalloc<double>(h, P.factor_elems);
    h->D64 = dalloc<double>(h, P.N);
    h->M64 = dalloc<double>(h, P.M_elems);
    h->Y64 = dalloc<double>(h, 2 * P.N * kNrhsMax);   // right-hand side, then the pivots' y / x
    h->U64 = dalloc<double>(h, P.U_elems * kNrhsMax);
    h->P64 = dalloc<double>(h, 2 * std::max<int64_t>(P.solve_max_slots, 1) * kPanel * kNrhsMax);
    if (h->opt.precision == NCL_FP32_IR) {
        h->F32 = dalloc<float>(h, P.factor_elems);
        h->D32 = dalloc<float>(h, P.N);
        h->M32 = dalloc<float>(h, P.M_elems);
        h->Y32 = dalloc<float>(h, 2 * P.N * kNrhsMax);
        h->U32 = dalloc<float>(h, P.U_elems * kNrhsMax);
        h->P32 = dalloc<float>(h, 2 * std::max<int64_t>(P.solve_max_slots, 1) * kPanel * kNrhsMax);
    }
    h->R = dalloc<double>(h, P.N * kNrhsMax);
    h->DX = dalloc<double>(h, P.N * kNrhsMax);
    h->Xp = dalloc<double>(h, P.N * kNrhsMax);
    h->partial_res = dalloc<double>(h, (int64_t)h->nchunks * kNrhsMax * kResWidth);
    h->res_out = dalloc<double>(h, (int64_t)P.S * kNrhsMax * kResWidth);
    // adjoint structures
    if (P.form == NCL_CONDENSED) {
        h->W_row = upload(h, P.Wrow_of);
        h->W_col = upload(h, P.Wcol_of32);
        h->Jp = upload(h, P.Jp);
        h->Jj = upload(h, P.Jj);
        h->Jrow_sys = upload(h, P.Jrow_sys);
        std::vector<int64_t> sj(P.S + 1, 0);
        for (int64_t r = 0; r < P.nJrows; ++r) sj[P.Jrow_sys[r] + 1]++;
        for (int s = 0; s < P.S; ++s) sj[s + 1] += sj[s];
        h->sys_jrow = upload(h, sj);
        {
            std::vector<int> jrow(P.nnzJ);
            for (int64_t r = 0; r < P.nJrows; ++r)
                for (int64_t k = P.Jp[r]; k < P.Jp[r + 1]; ++k) jrow[k] = (int)r;
            d.jrow_of = upload(h, jrow);
            // J^T: entries of each column in increasing row order
            std::vector<int64_t> tp(P.N + 1, 0);
            for (int64_t k = 0; k < P.nnzJ; ++k) tp[P.Jj[k] + 1]++;
            for (int64_t i = 0; i < P.N; ++i) tp[i + 1] += tp[i];
            std::vector<int> trow(P.nnzJ), tk(P.nnzJ);
            std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
            for (int64_t r = 0; r < P.nJrows; ++r)
                for (int64_t k = P.Jp[r]; k < P.Jp[r + 1]; ++k) {
                    const int64_t q = fill[P.Jj[k]]++;
                    trow[q] = (int)r;
                    tk[q] = (int)k;
                }
            h->Jt_ptr = upload(h, tp);
            h->Jt_row = upload(h, trow);
            h->Jt_k = upload(h, tk);
            h->omega = dalloc<double>(h, std::max<int64_t>(P.nJrows, 1));
        }
        h->JX = dalloc<double>(h, std::max<int64_t>(P.nJrows, 1) * kNrhsMax);
        h->JL = dalloc<double>(h, std::max<int64_t>(P.nJrows, 1) * kNrhsMax);
    }
    if (h->pers) {
        h->pers_order = upload(h, P.pers_order);
        h->pers_asm = upload(h, P.pers_asm);
        h->sys_nfronts = upload(h, P.sys_nfronts);
        // counters, then the ticket 128 bytes past them (a cache line of its own)
        h->pers_ctr_len = ((3 * (int64_t)P.nsn + P.S + 31) / 32) * 32 + 32;
        h->pers_ctr = dalloc<int>(h, h->pers_ctr_len);
        h->pers_ticket = h->pers_ctr + (h->pers_ctr_len - 32);
        h->pers_status = dalloc<int>(h, 1);
        h->tstamp = dalloc<unsigned long long>(h, 1 + 2 * (int64_t)P.S);
        int cus = 0, khz = 0;
        HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
        HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device));
        h->wall_khz = khz;
        h->pers_timeout = (unsigned long long)(2.0 * 1000.0 * khz);   // 2 s of wall_clock64 ticks
        h->pers_grid_f = h->opt.persistent_grid > 0 ? h->opt.persistent_grid : cus;
        h->pers_grid_s = h->opt.persistent_grid > 0 ? h->opt.persistent_grid : 2 * cus;
        h->pers_lds_elems = std::max<int>(P.pers_fmax_small * P.pers_fmax_small, 4 * std::max(P.pers_fmax_large, 1));
    }
    h->host_pinned_len = (size_t)std::max<int64_t>((int64_t)P.S * kNrhsMax * kResWidth + 1, 8 * (int64_t)P.S + 8);
    HIPCHK(hipHostMalloc((void**)&h->host_pinned, sizeof(double) * h->host_pinned_len, hipHostMallocDefault));
    HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&h->aux_stream, hipStreamNonBlocking));
    h->lvl_ev.assign(2 * (size_t)std::max(P.nlevels, 1), nullptr);
    for (auto& e : h->lvl_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPCHK(hipStreamCreateWithFlags(&h->aux2_stream, hipStreamNonBlocking));
    h->sb_ev.assign(2 * (size_t)std::max(P.nlevels, 1), nullptr);
    for (auto& e : h->sb_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    {
        int lds = 0;
        HIPCHK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
        HIPCHK(configure_kernels(lds));
        h->max_lds = lds;
    }
    HIPCHK(hipDeviceSynchronize());
    h->host_only = false;
}

int pick_small_max(int& fmax_out) {
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NCL_ERR_HIP;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return NCL_ERR_HIP;
    int f = (int)std::floor(std::sqrt((double)lds / 8.0));
    fmax_out = std::min(f, 128);
    return NCL_OK;
}

void fill_defaults(ncl_kkt_options* o) {
    o->form = NCL_CONDENSED;
    o->precision = NCL_FP64;
    o->pivot_eps = 0.0;
    o->ir_max_steps = 10;
    o->ir_tol = 1e-12;
    o->ir_stall = 0.5;
    o->ordering = NCL_ORDER_ND;
    o->user_perm = nullptr;
    o->use_graphs = 1;
    o->small_front_max = 0;
    o->relax_big_zeros = -1.0;
    o->fp32_sticky = 1;
    o->pivot_scale = NCL_PIVOT_GLOBAL;
    o->ir_cw_tol = 0.0;
    o->persistent = -1;
    o->persistent_grid = 0;
}

int do_analyze(ncl_kkt_t* out, const ncl_kkt_options* o, const std::vector<SysInput>& sys, bool host_only) {
    if (!out) return NCL_ERR_ARG;
    *out = nullptr;
    ncl_kkt_s* h = new (std::nothrow) ncl_kkt_s();
    if (!h) return NCL_ERR_ALLOC;
    if (o) h->opt = *o; else fill_defaults(&h->opt);
    if (h->opt.form != NCL_CONDENSED && h->opt.form != NCL_STABILIZED) { delete h; return NCL_ERR_ARG; }
    if (h->opt.precision != NCL_FP64 && h->opt.precision != NCL_FP32_IR) { delete h; return NCL_ERR_ARG; }
    if (h->opt.ordering < 0 || h->opt.ordering > 2) { delete h; return NCL_ERR_ARG; }
    if (h->opt.ir_max_steps < 0 || !(h->opt.ir_stall > 0.0)) { delete h; return NCL_ERR_ARG; }
    if (h->opt.pivot_scale < NCL_PIVOT_GLOBAL || h->opt.pivot_scale > NCL_PIVOT_ABSOLUTE) { delete h; return NCL_ERR_ARG; }
    if (!(h->opt.ir_cw_tol >= 0.0)) { delete h; return NCL_ERR_ARG; }
    h->pivot_mode = h->opt.pivot_scale == NCL_PIVOT_ABSOLUTE ? 2
                    : (h->opt.pivot_scale == NCL_PIVOT_BLOCK && h->opt.form == NCL_STABILIZED ? 1 : 0);
    if (sys.size() > 1 && h->opt.form != NCL_CONDENSED) { delete h; return NCL_ERR_ARG; }
    h->eps = h->opt.pivot_eps > 0.0 ? h->opt.pivot_eps : (h->opt.form == NCL_CONDENSED ? 1e-12 : 1e-10);
    // The persistent launches (k_persist_factor / k_persist_solve) are disabled:
    // a batched factor + solve through them once stopped making progress and
    // the cause is not established.  Every handle takes the level-scheduled
    // launches; asking for the persistent ones is an argument error.
    if (h->opt.persistent > 0) { delete h; return NCL_ERR_ARG; }
    h->pers = false;
    PlanConfig cfg;
    if (!host_only) {
        int fm = 90;
        int rc = pick_small_max(fm);
        if (rc) { delete h; return rc; }
        if (h->pers) {
            // the persistent factor keeps a small front in dynamic LDS beside its
            // static LDS (diagonal-block buffers): cap the order so both fit
            int dev = 0, lds = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
                delete h;
                return NCL_ERR_HIP;
            }
            const int st = persist_factor_static_lds(0);
            if (st < 0) { delete h; return NCL_ERR_HIP; }
            fm = std::min(fm, (int)std::floor(std::sqrt((double)(lds - st) / sizeof(double))));
            if (h->opt.small_front_max > fm) { delete h; return NCL_ERR_ARG; }
        }
        cfg.small_front_max = fm;
    }
    if (h->opt.small_front_max > 0) {
        if (h->opt.small_front_max > cfg.small_front_max && !host_only) { delete h; return NCL_ERR_ARG; }
        cfg.small_front_max = std::min(h->opt.small_front_max, kSmallMax);
    }
    if (h->opt.relax_big_zeros >= 0.0) cfg.relax_big_zeros = h->opt.relax_big_zeros;
    std::string err;
    int rc = build_plan(h->P, h->opt.form, sys, h->opt.ordering, h->opt.user_perm, cfg, err);
    if (rc) { delete h; return rc; }
    if (h->pers && !host_only) {
        // a large front's columns (4 per workgroup) must fit the persistent
        // factor's dynamic LDS too; otherwise keep the level-scheduled launches
        int dev = 0, lds = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
            delete h;
            return NCL_ERR_HIP;
        }
        const int64_t need = (int64_t)sizeof(double) * std::max<int64_t>(
            (int64_t)h->P.pers_fmax_small * h->P.pers_fmax_small, 4 * (int64_t)h->P.pers_fmax_large);
        if (need + persist_factor_static_lds(0) > lds) h->pers = false;
    }
    h->h_rho.assign(h->P.S, 1.0);
    h->h_kinf.assign(h->P.S, 0.0);
    h->h_inertia.assign(4 * (size_t)h->P.S, 0);
    if (!host_only) {
        try {
            setup_device(h);
        } catch (const HipError& e) {
            rc = (e.e == hipErrorOutOfMemory) ? NCL_ERR_ALLOC : NCL_ERR_HIP;
        } catch (const std::bad_alloc&) {
            rc = NCL_ERR_ALLOC;
        }
        if (rc) { ncl_kkt_destroy(h); return rc; }
    }
    *out = h;
    return NCL_OK;
}

// ----- numeric factorization -----------------------------------------------
// Algorithmic flops of one step's diagonal-block and panel-solve launches
// (w = panel width): w^3/3 for the LDL^T of each block (its explicit inverse
// is the implementation's extra work and is not counted), plus w_prev * w^2
// for the block's own update after the first panel; rows-below x w^2 for the
// panel solve.  Each front's figures are scaled by its exact / executed flop
// ratio, so amalgamation padding is not counted as work.
double diag_flops(const Plan& P, const LargeStep& ls, size_t k) {
    double fl = 0.0;
    for (int64_t t = ls.diag_first[k]; t < ls.diag_first[k] + ls.diag_count[k]; ++t) {
        const int s = P.large_diag[2 * t], k0 = P.large_diag[2 * t + 1];
        const double w = std::min(kPanel, P.sn_first[s + 1] - P.sn_first[s] - k0);
        fl += (w * w * w / 3.0 + (k0 > 0 ? (double)kPanel * w * w : 0.0)) * P.sn_flop_ratio[s];
    }
    return fl;
}
double panel_flops(const Plan& P, const LargeStep& ls, size_t k) {
    double fl = 0.0;
    for (int64_t t = ls.panel_first[k]; t < ls.panel_first[k] + ls.panel_count[k]; ++t) {
        const int s = P.large_panel[3 * t], k0 = P.large_panel[3 * t + 1], r0 = P.large_panel[3 * t + 2];
        const int f = (int)(P.sn_rowptr[s + 1] - P.sn_rowptr[s]);
        const double w = std::min(kPanel, P.sn_first[s + 1] - P.sn_first[s] - k0);
        fl += (double)std::min(32, f - r0) * w * w * P.sn_flop_ratio[s];
    }
    return fl;
}

template <typename T>
void factor_fronts(ncl_kkt_s* h, T* F, T* D, T* Mb, hipStream_t st) {
    Plan& P = h->P;
    const DevPlan& d = h->d;
    launch_zero_u64(h->inertia_part, 4 * (int64_t)P.S * kInertiaSlots, st);
    if (h->pers) {
        launch_zero_i32(h->pers_ctr, h->pers_ctr_len, st);
        launch_zero_u64(h->tstamp, 1 + (int64_t)P.S, st);
        double fl = 0.0;
        if (h->tm.on) fl = P.flops_exact;
        Span sp(h, st, TM_SMALL, fl, 2);
        launch_persist_factor<T>(d, h->pers_order, P.nsn, h->pers_asm, std::max(P.pers_fmax_large, 1),
                                 h->pers_lds_elems, h->pers_grid_f, h->pers_ctr, h->pers_ticket, h->pers_status,
                                 h->pers_timeout, h->tstamp, h->K, F, D, Mb, st);
        launch_reduce_inertia(d, P.S, st);
        return;
    }
    size_t sb = 0, lb = 0;
    for (int l = 0; l < P.nlevels; ++l) {
        // Fronts of one level are independent: when the level has both kinds,
        // its small fronts go to the second stream (forked after the previous
        // level, joined before the next one).
        const bool has_small = sb < P.small_batches.size() && P.small_batches[sb].level == l;
        const bool has_large = lb < P.large_steps.size() && P.large_steps[lb].level == l;
        const bool fork = has_small && has_large;
        hipStream_t ss = fork ? h->aux_stream : st;
        if (fork) {
            HIPCHK(hipEventRecord(h->lvl_ev[2 * l], st));
            HIPCHK(hipStreamWaitEvent(ss, h->lvl_ev[2 * l], 0));
        }
        // The level's batches (one per front-size class, each a launch) are
        // independent: split them over two streams, each batch to the one
        // with less estimated work (a latency floor plus count x fmax^2).
        size_t nbl = 0;
        while (sb + nbl < P.small_batches.size() && P.small_batches[sb + nbl].level == l) ++nbl;
        const bool split = nbl >= 2;
        if (split) {
            HIPCHK(hipEventRecord(h->sb_ev[2 * l], st));
            HIPCHK(hipStreamWaitEvent(h->aux2_stream, h->sb_ev[2 * l], 0));
        }
        double work[2] = {0.0, 0.0};
        while (sb < P.small_batches.size() && P.small_batches[sb].level == l) {
            const LevelBatch& b = P.small_batches[sb++];
            const int side = split && work[1] < work[0] ? 1 : 0;
            work[side] += 40.0 + (double)b.count * b.fmax * b.fmax / 2e5;
            hipStream_t bs = side ? h->aux2_stream : ss;
            double fl = 0.0;
            if (h->tm.on)
                for (int64_t k = b.first; k < b.first + b.count; ++k) {
                    const int s = P.small_list[k];
                    const double f = (double)(P.sn_rowptr[s + 1] - P.sn_rowptr[s]);
                    const int p = P.sn_first[s + 1] - P.sn_first[s];
                    double ff = 0.0;
                    for (int t = 0; t < p; ++t) { double r = f - t - 1; ff += r + r * (r + 1.0); }
                    fl += ff * P.sn_flop_ratio[s];
                }
            Span sp(h, bs, TM_SMALL, fl, 2);
            launch_small_fronts<T>(d, h->small_list + b.first, (int)b.count, b.fmax, h->K, F, D, bs);
        }
        if (split) HIPCHK(hipEventRecord(h->sb_ev[2 * l + 1], h->aux2_stream));
        if (lb < P.large_steps.size() && P.large_steps[lb].level == l) {
            const LargeStep& ls = P.large_steps[lb++];
            {
                Span sp(h, st, TM_LASM);
                launch_large_asm<T>(d, ls.asm_first, (int)ls.asm_count, ls.asm_fmax, h->K, F, st);
            }
            {
                // Step k: panel TRSM, then one launch with the trailing update
                // and the next panel's diagonal blocks (which update themselves).
                const size_t nsteps = ls.panel_first.size();
                {
                    Span sp(h, st, TM_DIAG, h->tm.on ? diag_flops(P, ls, 0) : 0.0, 6);
                    launch_large_diag<T>(d, h->large_diag + 2 * ls.diag_first[0], (int)ls.diag_count[0], F, D, Mb,
                                         st);
                }
                for (size_t k = 0; k < nsteps; ++k) {
                    {
                        Span sp(h, st, TM_PANEL, h->tm.on ? panel_flops(P, ls, k) : 0.0, 5);
                        launch_large_panel<T>(d, h->large_panel + 3 * ls.panel_first[k], (int)ls.panel_count[k], F, D,
                                              Mb, st);
                    }
                    const int nd = k + 1 < nsteps ? (int)ls.diag_count[k + 1] : 0;
                    const int* dt = nd > 0 ? h->large_diag + 2 * ls.diag_first[k + 1] : nullptr;
                    {
                        Span sp(h, st, TM_UPD, ls.upd_flops[k] + (h->tm.on && nd > 0 ? diag_flops(P, ls, k + 1) : 0.0),
                                1);
                        launch_large_dstep<T>(d, dt, nd, h->large_upd + 4 * ls.upd_first[k], (int)ls.upd_count[k], F,
                                              D, Mb, st);
                    }
                }
            }
        }
        if (fork) {
            HIPCHK(hipEventRecord(h->lvl_ev[2 * l + 1], ss));
            HIPCHK(hipStreamWaitEvent(st, h->lvl_ev[2 * l + 1], 0));
        }
        if (split) HIPCHK(hipStreamWaitEvent(st, h->sb_ev[2 * l + 1], 0));
    }
    launch_reduce_inertia(d, P.S, st);
}

// Runs the frontal factorization; with graphs enabled (and timing off) the
// launch sequence is captured once on a private stream and replayed on the
// caller's stream.  All its pointers are owned by the handle.
template <typename T>
void run_factor(ncl_kkt_s* h, hipStream_t st) {
    const int pr = std::is_same<T, float>::value ? 1 : 0;
    T* F = pr ? (T*)h->F32 : (T*)h->F64;
    T* D = pr ? (T*)h->D32 : (T*)h->D64;
    T* Mb = pr ? (T*)h->M32 : (T*)h->M64;
    if (!h->opt.use_graphs || h->tm.on) {
        factor_fronts<T>(h, F, D, Mb, st);
        return;
    }
    if (!h->g_factor[pr]) {
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
        factor_fronts<T>(h, F, D, Mb, h->cap_stream);
        HIPCHK(hipStreamEndCapture(h->cap_stream, &g));
        hipError_t e = hipGraphInstantiate(&h->g_factor[pr], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(e);
    }
    HIPCHK(hipGraphLaunch(h->g_factor[pr], st));
}

int read_inertia(ncl_kkt_s* h, hipStream_t st) {
    const int S = h->P.S;
    unsigned long long* hp = reinterpret_cast<unsigned long long*>(h->host_pinned);
    HIPCHK(hipMemcpyAsync(hp, h->inertia, sizeof(unsigned long long) * 4 * S, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h->host_pinned + 4 * S, h->nonfinite, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h->host_pinned + 4 * S + 1, h->kinf, sizeof(double) * 1, hipMemcpyDeviceToHost, st));
    if (h->pers)
        HIPCHK(hipMemcpyAsync(h->host_pinned + 4 * S + 2, h->pers_status, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int nonfin = 0, pstat = 0;
    std::memcpy(&nonfin, h->host_pinned + 4 * S, sizeof(int));
    if (h->pers) std::memcpy(&pstat, h->host_pinned + 4 * S + 2, sizeof(int));
    if (pstat & 2) return NCL_ERR_HIP;   // a wait of the persistent launch gave up
    h->nonfinite_bits = nonfin;
    h->inertia_ok = true;
    for (int s = 0; s < S; ++s) {
        for (int k = 0; k < 4; ++k) h->h_inertia[4 * s + k] = (int64_t)hp[4 * s + k];
        const int64_t n = h->P.sys_n[s], m = h->P.sys_m[s];
        const int64_t want_neg = h->P.form == NCL_STABILIZED ? m : 0;
        if (h->h_inertia[4 * s + 0] != n || h->h_inertia[4 * s + 1] != want_neg || h->h_inertia[4 * s + 2] != 0)
            h->inertia_ok = false;
    }
    if (nonfin) return NCL_ERR_NONFINITE;
    return NCL_OK;
}

// Replaces the FP32 factor in use by an FP64 factorization of the same
// assembled K (whose norms and thresholds are already on the device), and
// remembers the rho at which FP32 was insufficient (sticky policy).
int refactor_fp64(ncl_kkt_s* h, hipStream_t st) {
    launch_zero_i32(h->nonfinite, 1, st);
    run_factor<double>(h, st);
    h->factor_prec = 0;
    h->fell_back = true;
    h->fp32_rho_limit = std::min(h->fp32_rho_limit, h->cur_rho_max);
    return read_inertia(h, st);
}

int factor_impl(ncl_kkt_s* h, const double* W, const double* Sigma, const double* J, const double* rho_host,
                hipStream_t st, const double* Sigma_s = nullptr) {
    if (h->host_only) return NCL_ERR_STATE;
    Plan& P = h->P;
    for (int s = 0; s < P.S; ++s)
        if (!(rho_host[s] > 0.0) || !std::isfinite(rho_host[s])) return NCL_ERR_ARG;
    if ((P.nnzW > 0 && !W) || !Sigma || (P.nnzJ > 0 && !J)) return NCL_ERR_ARG;
    h->factored = 0;
    h->fell_back = false;
    try {
        HIPCHK(hipSetDevice(h->device));
        for (int s = 0; s < P.S; ++s) h->host_pinned[s] = rho_host[s];
        HIPCHK(hipMemcpyAsync(h->rho, h->host_pinned, sizeof(double) * P.S, hipMemcpyHostToDevice, st));
        launch_zero_i32(h->nonfinite, 1, st);
        if (h->pers) launch_zero_i32(h->pers_status, 1, st);
        h->pers_solved = false;
        {
            // algorithmic bytes: read W, Sigma, J once, write the lower triangle of K
            const double bytes = 8.0 * ((double)P.nnzW + (double)P.nnzJ + (double)P.N + (double)P.nnz_lower);
            Span sp(h, st, TM_ASM, bytes, 3);
            if (Sigma_s) launch_k1s_omega(P.nJrows, Sigma_s, h->Jrow_sys, h->rho, h->omega, h->nonfinite, st);
            launch_assemble(h->d, h->nnzF, W, Sigma, J, h->rho, Sigma_s ? h->omega : nullptr, h->K, st);
            h->weighted = Sigma_s != nullptr;
            launch_chunk_norms(h->d, h->K, h->chunk_row0, h->chunk_rows, h->nchunks, h->partial_norm, st);
            launch_reduce(h->sys_chunk_ptr, P.S, 3, 3, 0u, h->partial_norm, h->norms3, st);
            launch_thresholds(P.S, h->norms3, h->eps, h->pivot_mode, h->rho, h->kmax, h->kinf, h->thr, h->nonfinite,
                              st);
        }
        HIPCHK(hipGetLastError());
        double rho_max = 0.0;
        for (int s = 0; s < P.S; ++s) rho_max = std::max(rho_max, rho_host[s]);
        h->cur_rho_max = rho_max;
        const bool skip32 = h->opt.fp32_sticky && rho_max >= h->fp32_rho_limit;
        if (h->opt.precision == NCL_FP32_IR && !skip32) {
            run_factor<float>(h, st);
            h->factor_prec = 1;
        } else {
            // FP64, or an FP32 factor failed at a smaller rho of this sequence
            run_factor<double>(h, st);
            h->factor_prec = 0;
            h->fell_back = h->opt.precision == NCL_FP32_IR;
        }
        HIPCHK(hipGetLastError());
        int rc = read_inertia(h, st);
        if (h->factor_prec == 1 && (!h->inertia_ok || rc == NCL_ERR_NONFINITE)) {
            // An FP32 factor with the wrong inertia, or one that met a non-finite
            // pivot (FP32 range) while K itself is finite: refactor in FP64.
            if (rc == NCL_OK || !(h->nonfinite_bits & kNonfiniteInput)) rc = refactor_fp64(h, st);
        }
        if (rc) { flush_timing(h); return rc; }
        // host copy of ||K||_inf per system for the backward error
        HIPCHK(hipMemcpyAsync(h->host_pinned, h->kinf, sizeof(double) * P.S, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int s = 0; s < P.S; ++s) { h->h_kinf[s] = h->host_pinned[s]; h->h_rho[s] = rho_host[s]; }
        flush_timing(h);
    } catch (const HipError& e) {
        return NCL_ERR_HIP;
    }
    h->factored = 1;
    if (!h->inertia_ok) return NCL_WARN_INERTIA;
    return h->fell_back ? NCL_WARN_FELL_BACK_FP64 : NCL_OK;
}

// ----- solve -------------------------------------------------------------------
// LDS of the persistent solve for nrhs columns fits the device limit.
template <typename T>
bool pers_solve_fits(const ncl_kkt_s* h, int nrhs) {
    const size_t need = ((size_t)h->P.pers_fmax * nrhs + 256 * (size_t)nrhs + 64 * 65) * sizeof(T) + 64;
    return h->pers && need <= (size_t)h->max_lds;
}

template <typename T>
void sweeps(ncl_kkt_s* h, int nrhs, const T* F, const T* Z, const T* D, T* Y, T* U, T* partial, hipStream_t st) {
    Plan& P = h->P;
    const DevPlan& d = h->d;
    if (pers_solve_fits<T>(h, nrhs)) {
        launch_zero_i32(h->pers_ctr, h->pers_ctr_len, st);
        Span sp(h, st, TM_SOLVE, 0.0, 0);
        launch_persist_solve<T>(d, h->pers_order, P.nsn, h->sys_nfronts, std::max(P.pers_fmax, 1), h->pers_grid_s,
                                h->pers_ctr, h->pers_ticket, h->pers_status, h->pers_timeout, h->tstamp, F, Z, D, Y,
                                Y + P.N * kNrhsMax, U, nrhs, st);
        return;
    }
    T* Y2 = Y + P.N * kNrhsMax;
    const std::vector<SolveStep>& S = P.solve_steps;
    const std::vector<SolveStep>& FS = P.fsolve_steps;
    // Steps of one level are independent between the one-wave fronts and the
    // panel tasks: when a level has both, the one-wave fronts go to the second
    // stream, forked at the level's first step and joined after its last.
    auto level_end = [&](const std::vector<SolveStep>& V, size_t i) {
        size_t e = i;
        while (e < V.size() && V[e].level == V[i].level) ++e;
        return e;
    };
    auto has_panels = [&](const std::vector<SolveStep>& V, size_t i0, size_t i1) {
        for (size_t i = i0; i < i1; ++i)
            if (V[i].p_count > 0) return true;
        return false;
    };
    for (size_t i0 = 0; i0 < FS.size();) {
        const size_t i1 = level_end(FS, i0);
        const int l = FS[i0].level;
        const bool fork = FS[i0].s_count > 0 && has_panels(FS, i0, i1);
        hipStream_t ss = fork ? h->aux_stream : st;
        if (fork) {
            HIPCHK(hipEventRecord(h->lvl_ev[2 * l], st));
            HIPCHK(hipStreamWaitEvent(ss, h->lvl_ev[2 * l], 0));
        }
        for (size_t i = i0; i < i1; ++i) {
            const SolveStep& ss_ = FS[i];
            if (ss_.s_count > 0) {
                Span sp(h, ss, TM_SOLVE, 0.0, 0);
                launch_fwd_S<T>(d, h->solve_s + ss_.s_first, (int)ss_.s_count, F, Y, Y2, U, nrhs, ss);
            }
            if (ss_.p_count > 0) {
                Span sp(h, st, TM_SOLVE, ss_.fwd_bytes * sizeof(T) / 8.0, 4);
                launch_fwd_P<T>(d, h->fsolve_p + kTaskRec * ss_.p_first, (int)ss_.p_count, h->solve_seg, F, Z, Y,
                                Y2, U, nrhs, st);
            }
        }
        if (fork) {
            HIPCHK(hipEventRecord(h->lvl_ev[2 * l + 1], ss));
            HIPCHK(hipStreamWaitEvent(st, h->lvl_ev[2 * l + 1], 0));
        }
        i0 = i1;
    }
    // backward: levels from the top down, steps of a level in reverse.  The
    // tasks' sums of panel j go to partial half j & 1 and are read by the
    // next launch (panel j - 1, or the level's finish-only records).
    const int64_t half = std::max<int64_t>(P.solve_max_slots, 1) * kPanel * kNrhsMax;
    T* const pbuf[2] = {partial, partial + half};
    std::vector<size_t> starts;
    for (size_t i0 = 0; i0 < S.size(); i0 = level_end(S, i0)) starts.push_back(i0);
    for (auto it = starts.rbegin(); it != starts.rend(); ++it) {
        const size_t i0 = *it, i1 = level_end(S, i0);
        const int l = S[i0].level;
        const bool fork = S[i0].s_count > 0 && has_panels(S, i0, i1);
        hipStream_t ss = fork ? h->aux_stream : st;
        if (fork) {
            HIPCHK(hipEventRecord(h->lvl_ev[2 * l], st));
            HIPCHK(hipStreamWaitEvent(ss, h->lvl_ev[2 * l], 0));
        }
        for (size_t i = i1; i-- > i0;) {
            const SolveStep& ss_ = S[i];
            if (ss_.p_count > 0) {
                Span sp(h, st, TM_SOLVE, ss_.fwd_bytes * sizeof(T) / 8.0, 4);
                launch_bwd_P<T>(d, h->solve_p + kTaskRec * ss_.p_first, (int)ss_.p_count, F, Z, D, Y2,
                                pbuf[ss_.j & 1], pbuf[(ss_.j + 1) & 1], nrhs, st);
            }
            if (ss_.s_count > 0) {
                Span sp(h, ss, TM_SOLVE, 0.0, 0);
                launch_bwd_S<T>(d, h->solve_s + ss_.s_first, (int)ss_.s_count, F, D, Y2, nrhs, ss);
            }
        }
        if (S[i0].f_count > 0) {
            Span sp(h, st, TM_SOLVE, 0.0, 0);
            launch_bwd_P<T>(d, h->solve_p + kTaskRec * S[i0].f_first, (int)S[i0].f_count, F, Z, D, Y2, pbuf[1],
                            pbuf[0], nrhs, st);
        }
        if (fork) {
            HIPCHK(hipEventRecord(h->lvl_ev[2 * l + 1], ss));
            HIPCHK(hipStreamWaitEvent(st, h->lvl_ev[2 * l + 1], 0));
        }
    }
}

template <typename T>
void solve_once(ncl_kkt_s* h, const double* B, int64_t ldb, double* X, int64_t ldx, int nrhs, const T* F,
                const T* Z, const T* D, T* Y, T* U, T* partial, hipStream_t st) {
    const DevPlan& d = h->d;
    launch_permute_in<T>(d, B, ldb, nrhs, Y, st);
    const int pr = std::is_same<T, float>::value ? 1 : 0;
    if (!h->opt.use_graphs || h->tm.on) {
        sweeps<T>(h, nrhs, F, Z, D, Y, U, partial, st);
    } else {
        hipGraphExec_t& ge = h->g_sweep[pr][nrhs];
        if (!ge) {
            hipGraph_t g = nullptr;
            HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
            sweeps<T>(h, nrhs, F, Z, D, Y, U, partial, h->cap_stream);
            HIPCHK(hipStreamEndCapture(h->cap_stream, &g));
            hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIPCHK(e);
        }
        HIPCHK(hipGraphLaunch(ge, st));
    }
    launch_permute_out<T>(d, Y + h->P.N * kNrhsMax, nrhs, X, ldx, st);
}

void solve_with_factor(ncl_kkt_s* h, const double* B, int64_t ldb, double* X, int64_t ldx, int nrhs, hipStream_t st) {
    if (h->factor_prec == 1)
        solve_once<float>(h, B, ldb, X, ldx, nrhs, h->F32, h->M32, h->D32, h->Y32, h->U32, h->P32, st);
    else
        solve_once<double>(h, B, ldb, X, ldx, nrhs, h->F64, h->M64, h->D64, h->Y64, h->U64, h->P64, st);
}

// Backward errors of X against B, each the max over systems and columns.
struct Backward {
    double omega = 0.0;   // normwise
    double cw = 0.0;      // componentwise
    double rel2 = 0.0;    // ||b - Kx||_2 / ||b||_2
};

Backward backward_error(ncl_kkt_s* h, const double* B, int64_t ldb, const double* X, int64_t ldx, int nrhs,
                        hipStream_t st) {
    Plan& P = h->P;
    {
        Span sp(h, st, TM_RES);
        launch_residual(h->d, h->K, B, ldb, X, ldx, h->R, nrhs, h->chunk_row0, h->chunk_rows, h->nchunks,
                        h->partial_res, st);
        launch_reduce(h->sys_chunk_ptr, P.S, kResWidth * nrhs, kResWidth, (1u << 3) | (1u << 4), h->partial_res,
                      h->res_out, st);
    }
    HIPCHK(hipMemcpyAsync(h->host_pinned, h->res_out, sizeof(double) * kResWidth * nrhs * P.S,
                          hipMemcpyDeviceToHost, st));
    int* pstat = reinterpret_cast<int*>(h->host_pinned + (int64_t)kResWidth * nrhs * P.S);
    if (h->pers) HIPCHK(hipMemcpyAsync(pstat, h->pers_status, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h->pers && (*pstat & 2)) throw HipError{hipErrorLaunchTimeOut};   // a wait of the persistent solve gave up
    Backward out;
    auto upd = [](double& m, double w) { m = std::isnan(w) ? INFINITY : std::max(m, w); };
    for (int s = 0; s < P.S; ++s)
        for (int q = 0; q < nrhs; ++q) {
            const double* v = h->host_pinned + ((int64_t)s * nrhs + q) * kResWidth;
            const double den = h->h_kinf[s] * v[1] + v[2];
            upd(out.omega, den > 0.0 ? v[0] / den : (v[0] > 0.0 ? INFINITY : 0.0));
            upd(out.cw, v[5]);
            upd(out.rel2, v[4] > 0.0 ? std::sqrt(v[3] / v[4]) : (v[3] > 0.0 ? INFINITY : 0.0));
        }
    return out;
}

// Distance to the refinement target: <= 1 when converged.
double ir_gap(const ncl_kkt_s* h, const Backward& b) {
    double g = h->opt.ir_tol > 0.0 ? b.omega / h->opt.ir_tol : (b.omega > 0.0 ? INFINITY : 0.0);
    if (h->opt.ir_cw_tol > 0.0) g = std::max(g, b.cw / h->opt.ir_cw_tol);
    return std::isnan(g) ? INFINITY : g;
}
bool converged(const ncl_kkt_s* h, const Backward& b) { return ir_gap(h, b) <= 1.0; }

// One chunk of <= kNrhsMax columns: solve + refinement.  Returns the final
// backward errors; om0 = omega of the unrefined solve.
Backward solve_refine(ncl_kkt_s* h, const double* B, int64_t ldb, double* X, int64_t ldx, int nrhs, hipStream_t st,
                      int& steps, double& om0) {
    const int64_t N = h->P.N;
    solve_with_factor(h, B, ldb, X, ldx, nrhs, st);
    Backward om = backward_error(h, B, ldb, X, ldx, nrhs, st);
    om0 = om.omega;
    steps = 0;
    if (!h->inertia_ok) return om;
    double gap = ir_gap(h, om);
    while (gap > 1.0 && steps < h->opt.ir_max_steps) {
        // correction from the residual left in R by backward_error
        solve_with_factor(h, h->R, N, h->DX, N, nrhs, st);
        launch_copy_cols(h->Xp, N, X, ldx, N, nrhs, st);
        launch_axpy_cols(X, ldx, h->DX, N, nrhs, st);
        const Backward omn = backward_error(h, B, ldb, X, ldx, nrhs, st);
        const double gapn = ir_gap(h, omn);
        ++steps;
        if (!(gapn <= gap)) {          // worse (or NaN): keep the previous iterate
            launch_copy_cols(X, ldx, h->Xp, N, N, nrhs, st);
            // R must match X again for a caller that continues
            backward_error(h, B, ldb, X, ldx, nrhs, st);
            break;
        }
        const bool stalled = gapn > h->opt.ir_stall * gap;
        om = omn;
        gap = gapn;
        if (stalled) break;
    }
    return om;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
namespace {

// Inertia correction: factor with delta = 0, delta_init, delta_init * growth,
// ... until the inertia is the expected one (or delta would pass delta_max).
int factor_regularized(ncl_kkt_s* h, const double* W, const double* Sigma, const double* J, const double* Sigma_s,
                       double rho, double delta_init, double growth, double delta_max, double* delta_out,
                       int32_t* attempts_out, hipStream_t st) {
    const int64_t ns = h->P.form == NCL_CONDENSED ? h->P.N : h->P.sys_n[0];   // length of Sigma
    if (!h->sigma_shift) {
        try {
            h->sigma_shift = dalloc<double>(h, ns);
        } catch (const HipError&) {
            return NCL_ERR_ALLOC;
        }
    }
    double delta = 0.0;
    int attempts = 0, rc = NCL_OK;
    for (;;) {
        const double rh = rho + delta;
        const double* sg = Sigma;
        if (delta > 0.0) {
            try {
                HIPCHK(hipSetDevice(h->device));
                launch_add_scalar(ns, Sigma, delta, h->sigma_shift, st);
                HIPCHK(hipGetLastError());
            } catch (const HipError&) {
                return NCL_ERR_HIP;
            }
            sg = h->sigma_shift;
        }
        rc = factor_impl(h, W, sg, J, &rh, st, Sigma_s);
        ++attempts;
        if (rc < 0) break;
        const double next = delta == 0.0 ? delta_init : delta * growth;
        if (h->inertia_ok || !(next <= delta_max)) break;
        delta = next;
    }
    if (delta_out) *delta_out = delta;
    if (attempts_out) *attempts_out = attempts;
    return rc;
}

// The vector kernels below take rho-hat of each system from the last factor.
int step_ready(ncl_kkt_s* h) {
    if (!h) return NCL_ERR_ARG;
    if (h->host_only || !h->factored) return NCL_ERR_STATE;
    if (h->P.form != NCL_CONDENSED) return NCL_ERR_ARG;
    return NCL_OK;
}

template <typename F>
int run_vec(ncl_kkt_s* h, F&& body) {
    try {
        HIPCHK(hipSetDevice(h->device));
        body();
        HIPCHK(hipGetLastError());
    } catch (const HipError&) {
        return NCL_ERR_HIP;
    }
    return NCL_OK;
}

}  // namespace

extern "C" {

void ncl_kkt_default_options(ncl_kkt_options* o) {
    if (o) fill_defaults(o);
}

int ncl_kkt_analyze(ncl_kkt_t* h, const ncl_kkt_options* o, int32_t n, int32_t m, const int32_t* W_colptr,
                    const int32_t* W_rowidx, const int32_t* J_rowptr, const int32_t* J_colidx) {
    SysInput s{n, m, W_colptr, W_rowidx, J_rowptr, J_colidx};
    return do_analyze(h, o, {s}, false);
}

int ncl_kkt_analyze_host(ncl_kkt_t* h, const ncl_kkt_options* o, int32_t n, int32_t m, const int32_t* W_colptr,
                         const int32_t* W_rowidx, const int32_t* J_rowptr, const int32_t* J_colidx) {
    SysInput s{n, m, W_colptr, W_rowidx, J_rowptr, J_colidx};
    return do_analyze(h, o, {s}, true);
}

int ncl_kkt_analyze_batched(ncl_kkt_t* h, const ncl_kkt_options* o, int32_t count, const int32_t* n,
                            const int32_t* m, const int32_t* const* W_colptr, const int32_t* const* W_rowidx,
                            const int32_t* const* J_rowptr, const int32_t* const* J_colidx) {
    if (!h || count < 1 || !n || !m || !W_colptr || !W_rowidx || !J_rowptr || !J_colidx) return NCL_ERR_ARG;
    std::vector<SysInput> sys(count);
    for (int s = 0; s < count; ++s) sys[s] = SysInput{n[s], m[s], W_colptr[s], W_rowidx[s], J_rowptr[s], J_colidx[s]};
    return do_analyze(h, o, sys, false);
}

int ncl_kkt_factor(ncl_kkt_t h, const double* W_val, const double* Sigma, const double* J_val, double rho,
                   void* stream) {
    if (!h) return NCL_ERR_ARG;
    if (h->P.S != 1) return NCL_ERR_ARG;
    return factor_impl(h, W_val, Sigma, J_val, &rho, (hipStream_t)stream);
}

int ncl_kkt_factor_batched(ncl_kkt_t h, const double* W_val, const double* Sigma, const double* J_val,
                           const double* rho, void* stream) {
    if (!h || !rho) return NCL_ERR_ARG;
    return factor_impl(h, W_val, Sigma, J_val, rho, (hipStream_t)stream);
}

int ncl_kkt_factor_k1s(ncl_kkt_t h, const double* W_val, const double* Sigma_t, const double* J_val,
                       const double* Sigma_s, const double* rho, void* stream) {
    if (!h || !rho || !Sigma_s) return NCL_ERR_ARG;
    if (h->P.form != NCL_CONDENSED) return NCL_ERR_ARG;
    return factor_impl(h, W_val, Sigma_t, J_val, rho, (hipStream_t)stream, Sigma_s);
}

int ncl_kkt_factor_regularized(ncl_kkt_t h, const double* W_val, const double* Sigma, const double* J_val,
                               const double* Sigma_s, double rho, double delta_init, double growth,
                               double delta_max, double* delta_out, int32_t* attempts_out, void* stream) {
    if (!h || h->P.S != 1) return NCL_ERR_ARG;
    if (h->host_only) return NCL_ERR_STATE;
    if (!(delta_init > 0.0) || !(growth > 1.0) || !(delta_max >= 0.0) || !std::isfinite(delta_init)) return NCL_ERR_ARG;
    if (Sigma_s && h->P.form != NCL_CONDENSED) return NCL_ERR_ARG;
    if (!Sigma) return NCL_ERR_ARG;
    return factor_regularized(h, W_val, Sigma, J_val, Sigma_s, rho, delta_init, growth, delta_max, delta_out,
                              attempts_out, (hipStream_t)stream);
}

int ncl_kkt_k1s_rhs(ncl_kkt_t h, const double* J_val, const double* r_t, const double* r_s, const double* Sigma_s,
                    double* b, void* stream) {
    int rc = step_ready(h);
    if (rc) return rc;
    if ((h->P.nnzJ > 0 && !J_val) || !r_t || !r_s || !Sigma_s || !b) return NCL_ERR_ARG;
    return run_vec(h, [&] {
        launch_k1s_rhs(h->P.N, h->Jt_ptr, h->Jt_row, h->Jt_k, J_val, r_t, r_s, Sigma_s, h->Jrow_sys, h->rho,
                       h->d.row_sys, b, (hipStream_t)stream);
    });
}

int ncl_kkt_k1s_recover(ncl_kkt_t h, const double* J_val, const double* dt, const double* r_s,
                        const double* Sigma_s, double* ds, void* stream) {
    int rc = step_ready(h);
    if (rc) return rc;
    if ((h->P.nnzJ > 0 && !J_val) || !dt || !r_s || !Sigma_s || !ds) return NCL_ERR_ARG;
    return run_vec(h, [&] {
        launch_k1s_ds(h->P.nJrows, h->Jp, h->Jj, J_val, dt, r_s, Sigma_s, h->Jrow_sys, h->rho, ds,
                      (hipStream_t)stream);
    });
}

int ncl_kkt_recover_dy(ncl_kkt_t h, const double* J_val, const double* dx, const double* c, const double* y_k,
                       const double* y, double* dy, void* stream) {
    int rc = step_ready(h);
    if (rc) return rc;
    if ((h->P.nnzJ > 0 && !J_val) || !dx || !c || !y_k || !y || !dy) return NCL_ERR_ARG;
    return run_vec(h, [&] {
        launch_recover_dy(h->P.nJrows, h->Jp, h->Jj, J_val, dx, c, y_k, y, h->Jrow_sys, h->rho, dy,
                          (hipStream_t)stream);
    });
}

int ncl_kkt_recover_dr(ncl_kkt_t h, const double* dy, const double* y_k, const double* y, const double* r,
                       double* dr, void* stream) {
    int rc = step_ready(h);
    if (rc) return rc;
    if (!dy || !y_k || !y || !r || !dr) return NCL_ERR_ARG;
    return run_vec(h, [&] {
        launch_recover_dr(h->P.nJrows, dy, y_k, y, r, h->Jrow_sys, h->rho, dr, (hipStream_t)stream);
    });
}

int ncl_kkt_recover_dz(ncl_kkt_t h, const double* x, const double* l, const double* u, const double* z_l,
                       const double* z_u, const double* dx, double mu, double* dz_l, double* dz_u, void* stream) {
    if (!h) return NCL_ERR_ARG;
    if (h->host_only) return NCL_ERR_STATE;
    if (!x || !l || !u || !z_l || !z_u || !dx || !dz_l || !dz_u || !std::isfinite(mu)) return NCL_ERR_ARG;
    return run_vec(h, [&] {
        launch_recover_dz(h->P.N, x, l, u, z_l, z_u, dx, mu, dz_l, dz_u, (hipStream_t)stream);
    });
}

int ncl_kkt_barrier_sigma(ncl_kkt_t h, const double* x, const double* l, const double* u, const double* z_l,
                          const double* z_u, double* sigma, void* stream) {
    if (!h) return NCL_ERR_ARG;
    if (h->host_only) return NCL_ERR_STATE;
    if (!x || !l || !u || !z_l || !z_u || !sigma) return NCL_ERR_ARG;
    return run_vec(h, [&] { launch_barrier_sigma(h->P.N, x, l, u, z_l, z_u, sigma, (hipStream_t)stream); });
}

int ncl_kkt_solve(ncl_kkt_t h, const double* B, int64_t ldb, double* X, int64_t ldx, int32_t nrhs, void* stream,
                  ncl_kkt_solve_info* info) {
    if (!h) return NCL_ERR_ARG;
    if (h->host_only || !h->factored) return NCL_ERR_STATE;
    if (!B || !X || nrhs < 1 || ldb < h->P.N || ldx < h->P.N) return NCL_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    int total_steps = 0;
    Backward om_all;
    double om0_all = 0.0;
    bool fell = h->fell_back;
    try {
        HIPCHK(hipSetDevice(h->device));
        for (int q0 = 0; q0 < nrhs; q0 += kNrhsMax) {
            const int nq = std::min(kNrhsMax, nrhs - q0);
            const double* Bq = B + (int64_t)q0 * ldb;
            double* Xq = X + (int64_t)q0 * ldx;
            int steps = 0;
            double om0 = 0.0;
            Backward om = solve_refine(h, Bq, ldb, Xq, ldx, nq, st, steps, om0);
            if (!converged(h, om) && h->factor_prec == 1 && h->inertia_ok) {
                // FP32 factor not accurate enough: refactor in FP64 from the assembled K
                int rc = refactor_fp64(h, st);
                fell = true;
                if (rc) { flush_timing(h); return rc; }
                int steps2 = 0;
                om = solve_refine(h, Bq, ldb, Xq, ldx, nq, st, steps2, om0);
                steps += steps2;
            }
            total_steps += steps;
            om_all.omega = std::max(om_all.omega, om.omega);
            om_all.cw = std::max(om_all.cw, om.cw);
            om_all.rel2 = std::max(om_all.rel2, om.rel2);
            om0_all = std::max(om0_all, om0);
        }
        flush_timing(h);
        h->pers_solved = h->pers;
    } catch (const HipError&) {
        return NCL_ERR_HIP;
    }
    if (info) {
        info->ir_steps = total_steps;
        info->fell_back_fp64 = fell ? 1 : 0;
        info->backward_error = om_all.omega;
        info->backward_error0 = om0_all;
        info->backward_error_cw = om_all.cw;
        info->resid_rel2 = om_all.rel2;
    }
    if (!h->inertia_ok) return NCL_WARN_INERTIA;
    if (!converged(h, om_all) && h->opt.ir_max_steps > 0) return NCL_WARN_IR_NOT_CONVERGED;
    return fell ? NCL_WARN_FELL_BACK_FP64 : NCL_OK;
}

int ncl_kkt_inertia(ncl_kkt_t h, int64_t* npos, int64_t* nneg, int64_t* nzero, int64_t* nperturbed) {
    if (!h) return NCL_ERR_ARG;
    if (h->host_only || !h->factored) return NCL_ERR_STATE;
    int64_t t[4] = {0, 0, 0, 0};
    for (int s = 0; s < h->P.S; ++s)
        for (int k = 0; k < 4; ++k) t[k] += h->h_inertia[4 * s + k];
    if (npos) *npos = t[0];
    if (nneg) *nneg = t[1];
    if (nzero) *nzero = t[2];
    if (nperturbed) *nperturbed = t[3];
    return NCL_OK;
}

int ncl_kkt_inertia_batched(ncl_kkt_t h, int64_t* out) {
    if (!h || !out) return NCL_ERR_ARG;
    if (h->host_only || !h->factored) return NCL_ERR_STATE;
    std::memcpy(out, h->h_inertia.data(), sizeof(int64_t) * h->h_inertia.size());
    return NCL_OK;
}

int ncl_kkt_backward(ncl_kkt_t h, const double* J_val, const double* X, const double* Lambda, int64_t ld,
                     int32_t nrhs, double* gW, double* gSigma, double* gJ, double* gRho, void* stream) {
    if (!h) return NCL_ERR_ARG;
    if (h->host_only || !h->factored) return NCL_ERR_STATE;
    if (h->P.form != NCL_CONDENSED) return NCL_ERR_ARG;
    if (h->weighted) return NCL_ERR_STATE;   // the adjoint is of K1, not of K1s
    if (!X || !Lambda || nrhs < 1 || nrhs > kNrhsMax || ld < h->P.N) return NCL_ERR_ARG;
    if ((gJ || gRho) && h->P.nnzJ > 0 && !J_val) return NCL_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    try {
        HIPCHK(hipSetDevice(h->device));
        launch_adjoint(h->d, h->P.nnzW, h->W_row, h->W_col, h->P.nJrows, h->Jp, h->Jj, h->Jrow_sys, J_val, h->rho, X,
                       Lambda, ld, nrhs, gW, gSigma, gJ, gRho, h->JX, h->JL, h->sys_jrow, st);
        HIPCHK(hipGetLastError());
    } catch (const HipError&) {
        return NCL_ERR_HIP;
    }
    return NCL_OK;
}

int ncl_kkt_backward_noalloc(ncl_kkt_t h, const double* J_val, const double* X, const double* Lambda, int64_t ld,
                             int32_t nrhs, double* gW, double* gSigma, double* gJ, double* gRho, void* stream) {
    if (!h) return NCL_ERR_ARG;
    if (h->host_only || !h->factored) return NCL_ERR_STATE;
    if (h->P.form != NCL_CONDENSED) return NCL_ERR_ARG;
    if (h->weighted) return NCL_ERR_STATE;   // the adjoint is of K1, not of K1s
    if (!X || !Lambda || nrhs < 1 || nrhs > kNrhsMax || ld < h->P.N) return NCL_ERR_ARG;
    if ((gJ || gRho) && h->P.nnzJ > 0 && !J_val) return NCL_ERR_ARG;
    const int64_t need = 2 * h->P.nJrows * (int64_t)nrhs;   // J X and J Lambda, nJrows x nrhs each
    if (need > kScratchDoubles) return NCL_ERR_SCRATCH;
    hipStream_t st = (hipStream_t)stream;
    try {
        HIPCHK(hipSetDevice(h->device));
        double* ws = nullptr;
        HIPCHK(scratch_on_device(h->device, &ws));
        launch_adjoint(h->d, h->P.nnzW, h->W_row, h->W_col, h->P.nJrows, h->Jp, h->Jj, h->Jrow_sys, J_val, h->rho, X,
                       Lambda, ld, nrhs, gW, gSigma, gJ, gRho, ws, ws + h->P.nJrows * (int64_t)nrhs, h->sys_jrow, st);
        HIPCHK(hipGetLastError());
    } catch (const HipError&) {
        return NCL_ERR_HIP;
    }
    return NCL_OK;
}

int ncl_kkt_get_stats(ncl_kkt_t h, ncl_kkt_stats* st) {
    if (!h || !st) return NCL_ERR_ARG;
    const Plan& P = h->P;
    st->order = P.N;
    st->nnz_K_lower = P.nnz_lower;
    st->nnz_L = P.nnzL;
    st->flops_factor = P.flops;
    st->n_supernodes = P.nsn;
    st->n_levels = P.nlevels;
    st->max_front = P.max_front;
    st->n_large_fronts = P.n_large;
    // host-only handles report the factor buffer they would need in FP64
    st->device_bytes = h->host_only ? P.factor_elems * 8 : h->dev_bytes;
    st->analyze_seconds = P.analyze_seconds;
    st->nnz_L_exact = P.nnzL_exact;
    st->flops_exact = P.flops_exact;
    return NCL_OK;
}

int ncl_kkt_get_perm(ncl_kkt_t h, int32_t* perm) {
    if (!h || !perm) return NCL_ERR_ARG;
    std::memcpy(perm, h->P.perm.data(), sizeof(int32_t) * h->P.perm.size());
    return NCL_OK;
}

int ncl_kkt_get_supernodes(ncl_kkt_t h, int32_t* first, int32_t* parent, int64_t* row_ptr, int32_t* rows) {
    if (!h) return NCL_ERR_ARG;
    const Plan& P = h->P;
    if (first) std::memcpy(first, P.sn_first.data(), sizeof(int32_t) * P.sn_first.size());
    if (parent) std::memcpy(parent, P.sn_parent.data(), sizeof(int32_t) * P.sn_parent.size());
    if (row_ptr) std::memcpy(row_ptr, P.sn_rowptr.data(), sizeof(int64_t) * P.sn_rowptr.size());
    if (rows) std::memcpy(rows, P.sn_rows.data(), sizeof(int32_t) * P.sn_rows.size());
    return NCL_OK;
}

int ncl_kkt_get_system_times(ncl_kkt_t h, double* factor_ms, double* solve_ms) {
    if (!h) return NCL_ERR_ARG;
    if (h->host_only || !h->pers || !h->pers_solved) return NCL_ERR_STATE;
    const int S = h->P.S;
    std::vector<unsigned long long> t(1 + 2 * (size_t)S);
    try {
        HIPCHK(hipSetDevice(h->device));
        HIPCHK(hipMemcpy(t.data(), h->tstamp, sizeof(unsigned long long) * t.size(), hipMemcpyDeviceToHost));
    } catch (const HipError&) {
        return NCL_ERR_HIP;
    }
    const double per_ms = h->wall_khz > 0.0 ? 1.0 / h->wall_khz : 0.0;   // ticks of wall_clock64 -> ms
    for (int s = 0; s < S; ++s) {
        if (factor_ms) factor_ms[s] = (double)(t[1 + s] - t[0]) * per_ms;
        if (solve_ms) solve_ms[s] = (double)(t[1 + S + s] - t[0]) * per_ms;
    }
    return NCL_OK;
}

int ncl_kkt_set_timing(ncl_kkt_t h, int32_t enable) {
    if (!h) return NCL_ERR_ARG;
    if (h->host_only) return NCL_ERR_STATE;
    try {
        if (enable && h->tm.pool.empty()) {
            h->tm.pool.resize(16384);
            for (auto& e : h->tm.pool) HIPCHK(hipEventCreate(&e));
        }
    } catch (const HipError&) {
        return NCL_ERR_HIP;
    }
    h->tm.on = enable != 0;
    h->tm.tot = ncl_kkt_timing{};
    h->tm.recs.clear();
    h->tm.used = 0;
    return NCL_OK;
}

int ncl_kkt_get_timing(ncl_kkt_t h, ncl_kkt_timing* t) {
    if (!h || !t) return NCL_ERR_ARG;
    *t = h->tm.tot;
    return NCL_OK;
}

void ncl_kkt_destroy(ncl_kkt_t h) {
    if (!h) return;
    if (!h->host_only || !h->allocs.empty()) {
        (void)hipSetDevice(h->device);
        (void)hipDeviceSynchronize();
        for (void* p : h->allocs) (void)hipFree(p);
        if (h->host_pinned) (void)hipHostFree(h->host_pinned);
        for (auto& e : h->tm.pool) (void)hipEventDestroy(e);
        for (auto& g : h->g_factor) if (g) (void)hipGraphExecDestroy(g);
        for (auto& row : h->g_sweep)
            for (auto& g : row) if (g) (void)hipGraphExecDestroy(g);
        if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
        if (h->aux_stream) (void)hipStreamDestroy(h->aux_stream);
        if (h->aux2_stream) (void)hipStreamDestroy(h->aux2_stream);
        for (auto& e : h->sb_ev) if (e) (void)hipEventDestroy(e);
        for (auto& e : h->lvl_ev) if (e) (void)hipEventDestroy(e);
    }
    delete h;
}

const char* ncl_kkt_strerror(int code) {
    switch (code) {
        case NCL_OK: return "success";
        case NCL_ERR_ARG: return "invalid argument";
        case NCL_ERR_PATTERN: return "invalid sparsity pattern (unsorted, duplicate, out-of-range or upper entry)";
        case NCL_ERR_ALLOC: return "allocation failed";
        case NCL_ERR_HIP: return "HIP runtime error";
        case NCL_ERR_STATE: return "call out of order (no numeric factorization or host-only handle)";
        case NCL_ERR_NONFINITE: return "NaN or Inf in the assembled matrix or a pivot";
        case NCL_ERR_SCRATCH:
            return "problem too large for the no-allocation entry point's fixed scratch (2 x m x nrhs > 2^21 "
                   "doubles); use the allocating entry point";
        case NCL_WARN_INERTIA: return "warning: inertia differs from the expected (n,0,0) / (n,m,0)";
        case NCL_WARN_IR_NOT_CONVERGED: return "warning: iterative refinement stopped above the tolerance";
        case NCL_WARN_FELL_BACK_FP64: return "warning: FP32 factor replaced by an FP64 refactorization";
        default: return "unknown status";
    }
}

}  // extern "C"
