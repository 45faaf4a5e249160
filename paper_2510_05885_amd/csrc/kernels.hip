// kernels.hip — gfx950 kernels of the KKT hot path.
//
//   assembly   K = W + Sigma + rho J^T J (Sec. 3.3, eq. K1) or the stabilized
//              [[W + Sigma, J^T], [J, -1/rho I]] (Sec. 3.2, eq. K2r) on the
//              fixed pattern, one thread per stored entry, FP64; row and
//              system norms by two-stage deterministic reductions.
//   factor     supernodal multifrontal LDL^T with the static-pivot rule of
//              Sec. 3.1 (|d| < thr -> d = sign * thr, sign of the pivot's
//              block before reordering); fronts processed level by level:
//                * small fronts: one workgroup per front, the whole front in
//                  LDS (assembly, extend-add of the children's contribution
//                  blocks, partial factorization, write-out);
//                * large fronts: the front lives in the factor buffer; one
//                  launch assembles it column by column, then per pivot panel
//                  a one-wave diagonal-block factor, a panel solve, and a
//                  trailing update on MFMA (v_mfma_f64_16x16x4 / f32).
//   solve      level-scheduled multifrontal forward sweep (children's
//              update vectors pulled by the parent: no atomics), D^-1, and
//              backward sweep; right-hand sides chunked through LDS.
//   refinement residual b - K x with per-system max norms.
// All reductions are deterministic; integer atomics only count inertia.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.hpp"

namespace ncl {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ double to_d(double x) { return x; }
__device__ __forceinline__ double to_d(float x) { return (double)x; }

// Static-pivot thresholds of one system (Sec. 3.1): p for pivots of the
// primal block, n for pivots of the dual block (equal unless the thresholds
// are block-scaled), with the reciprocals of the replacement pivots +p, -n.
template <typename T>
struct PivThr {
    double p, n;
    T inv_p, inv_n;
    __device__ PivThr(const DevPlan& d, int sys)
        : p(d.sys_thr[2 * sys]), n(d.sys_thr[2 * sys + 1]), inv_p(T(1) / (T)p), inv_n(-(T(1) / (T)n)) {}
    __device__ __forceinline__ T inv(int sign) const { return sign > 0 ? inv_p : inv_n; }
};

// Static-pivot rule (Sec. 3.1): returns the pivot to use; flags perturbation.
// |d| < t (strict) with t the threshold of the pivot's block is replaced by +t
// for a primal pivot and by -t for a dual one.
template <typename T>
__device__ __forceinline__ T static_pivot(T d, const PivThr<T>& th, int sign, bool& perturbed, bool& bad) {
    const double dd = to_d(d);
    const double t = sign > 0 ? th.p : th.n;
    bad = !isfinite(dd);
    perturbed = fabs(dd) < t;
    if (perturbed) return (T)(sign > 0 ? t : -t);
    return d;
}

// Adds a workgroup's pivot counts to one of the system's partial counters
// (many fronts finish at once; one shared counter would serialize them).
__device__ __forceinline__ void add_inertia(const DevPlan& d, int sys, const unsigned int* cnt, int slot) {
    unsigned long long* in4 = d.inertia_part + 4 * ((int64_t)sys * kInertiaSlots + (slot & (kInertiaSlots - 1)));
    for (int k = 0; k < 4; ++k)
        if (cnt[k]) atomicAdd(&in4[k], (unsigned long long)cnt[k]);
}

__device__ __forceinline__ void count_pivot(unsigned long long* in4, double d, bool pert) {
    if (d > 0.0) atomicAdd(&in4[0], 1ULL);
    else if (d < 0.0) atomicAdd(&in4[1], 1ULL);
    else atomicAdd(&in4[2], 1ULL);
    if (pert) atomicAdd(&in4[3], 1ULL);
}

// 16x16x4 MFMA wrappers.  Operands: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16].  Result item r of lane l is D[row(l / 16, r)][l % 16];
// the row order differs between the f64 and f32 instructions (checked on
// gfx950 with a one-hot probe).
template <typename T> struct Mfma;
//
// run_chained: for an MFMA whose result is read by the very next instruction
// that touches it (the next MFMA of a single-accumulator chain, as SrcC or as
// an operand, or the read-out).  On gfx950 such a dependency needs more
// separation than the compiler inserts: without the 16 wait states below,
// about 3% of the factorizations of a 500k-order system differed from run to
// run, always in one accumulator register pair of one wave, while with them
// every repeat was bitwise identical.  Chains whose consecutive MFMAs write
// different accumulators (the interleaved 64x64 tile update) need only pad()
// before their read-out.
__device__ __forceinline__ void mfma_pad() {
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_nop 15");
    __builtin_amdgcn_sched_barrier(0);
}
template <> struct Mfma<double> {
    typedef f64x4 acc_t;
    static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ acc_t run_chained(double a, double b, acc_t c) {
        acc_t r = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
        mfma_pad();
        return r;
    }
    static __device__ __forceinline__ int row(int lk, int r) { return 4 * r + lk; }
};
template <> struct Mfma<float> {
    typedef f32x4 acc_t;
    static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ acc_t run_chained(float a, float b, acc_t c) {
        acc_t r = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
        mfma_pad();
        return r;
    }
    static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

// 1/d from the hardware reciprocal refined by two Newton steps (within ~1 ulp
// of the rounded quotient); shorter dependent latency than a full division.
__device__ __forceinline__ double fast_rcp(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float fast_rcp(float d) {
    float r = __builtin_amdgcn_rcpf(d);
    const float e = __builtin_fmaf(-d, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}

// Value of `v` held by lane `src` (a compile-time / wave-uniform lane index).
__device__ __forceinline__ double bcast(double v, int src) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float bcast(float v, int src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}

// Compiler-level fence: keeps LDS accesses of one wave in program order.
__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
}

// Partial LDL^T of the leading p columns of an f x f lower-triangular matrix
// held in LDS (column-major, leading dimension lda), with the static-pivot
// rule of Sec. 3.1.  Blocked by 16 columns: wave 0 factors each 16-column
// sub-panel over all rows below it (one row per lane, no workgroup barrier),
// then the four waves apply the rank-16 update to the trailing lower matrix
// on MFMA.  On return A holds L (unit lower, strictly below the diagonal) in
// its first p columns, d_k on the diagonal and in dv[k], and the Schur
// complement in the trailing (f - p) x (f - p) part.  sgn[k] is the block sign
// of pivot k.  Lane 0 of wave 0 accumulates the pivot counts into cnt[4].
// kTwoRows: f may exceed 64 + (sub-panel start), so a lane holds two rows.
// Must be called by all 256 threads; ends with a barrier.
template <typename T, bool kTwoRows>
__device__ void lds_partial_ldlt(T* A, int lda, int f, int p, T* dv, const int8_t* sgn, const PivThr<T>& thr,
                                 unsigned int* cnt, bool& bad_out) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    bool bad_any = false;
    for (int kb = 0; kb < p; kb += 16) {
        const int bw = min(16, p - kb);
        if (wave == 0) {
            // Rows kb + lane and kb + lane + 64 of the sub-panel, in registers.
            // Slots above a row's diagonal are scratch: they take the same
            // unpredicated updates as the rest, are never read for a later
            // pivot, and are not written back.
            const int i0 = kb + lane, i1 = kb + lane + 64;
            T r0[16], r1[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                r0[t] = (t < bw && i0 < f && t <= lane) ? A[i0 + (kb + t) * lda] : T(0);
                r1[t] = (kTwoRows && t < bw && i1 < f) ? A[i1 + (kb + t) * lda] : T(0);
            }
            T mydk = T(0);
            unsigned int np = 0, nn = 0, nz = 0, npt = 0;
            bool anybad = false;
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                if (t >= bw) continue;   // uniform; keeps the loop fully unrolled
                bool pert, bad;
                const T draw = bcast(r0[t], t);
                const T inv0 = fast_rcp(draw);
                const int sg = sgn[kb + t];
                const T dk = static_pivot(draw, thr, sg, pert, bad);
                const T inv = pert ? thr.inv(sg) : inv0;
                T ck[16];
#pragma unroll
                for (int u = t + 1; u < 16; ++u) ck[u] = (u < bw) ? bcast(r0[t], u) : T(0);
                const T l0 = r0[t] * inv;
#pragma unroll
                for (int u = t + 1; u < 16; ++u) r0[u] -= l0 * ck[u];
                r0[t] = (lane == t) ? dk : l0;
                if (kTwoRows) {
                    const T l1 = r1[t] * inv;
#pragma unroll
                    for (int u = t + 1; u < 16; ++u) r1[u] -= l1 * ck[u];
                    r1[t] = l1;
                }
                mydk = (lane == t) ? dk : mydk;
                const double dd = to_d(dk);
                np += dd > 0.0; nn += dd < 0.0; nz += dd == 0.0; npt += pert;
                anybad |= bad;
            }
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                if (t < bw && i0 < f && t <= lane) A[i0 + (kb + t) * lda] = r0[t];
                if (kTwoRows && t < bw && i1 < f) A[i1 + (kb + t) * lda] = r1[t];
            }
            if (lane < bw) dv[kb + lane] = mydk;
            if (lane == 0) {
                cnt[0] += np; cnt[1] += nn; cnt[2] += nz; cnt[3] += npt;
                bad_any |= anybad;
            }
        }
        __syncthreads();
        // trailing update on MFMA: C -= L_panel D L_panel^T for rows/cols >= r0
        const int r0 = kb + bw;
        const int nt = (f - r0 + 15) / 16;
        const int ntiles = nt * (nt + 1) / 2;
        for (int tix = wave; tix < ntiles; tix += 4) {
            int tj = 0, rem = tix;
            while (rem >= nt - tj) { rem -= nt - tj; ++tj; }
            const int ti = tj + rem;
            const int i0 = r0 + 16 * ti, j0 = r0 + 16 * tj;
            T av[4], bv[4];   // operands first: see panel_body
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const int tt = 4 * st + lk;
                const bool tv = tt < bw;
                const int t = kb + tt;
                av[st] = (tv && i0 + lr < f) ? A[(i0 + lr) + t * lda] : T(0);
                bv[st] = (tv && j0 + lr < f) ? A[(j0 + lr) + t * lda] * dv[tv ? t : 0] : T(0);
            }
            typename Mfma<T>::acc_t acc = {0, 0, 0, 0};
#pragma unroll
            for (int st = 0; st < 4; ++st) acc = Mfma<T>::run_chained(av[st], bv[st], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = i0 + Mfma<T>::row(lk, r), gj = j0 + lr;
                if (gi < f && gj < f && gi >= gj) A[gi + gj * lda] -= acc[r];
            }
        }
        __syncthreads();
    }
    bad_out = bad_any;
}

// Value of lane 16 * (lane / 16) + U of each 16-lane row (DPP row_newbcast).
template <int U>
__device__ __forceinline__ double rowbcast(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const long long r = __builtin_amdgcn_update_dpp(b, b, 0x150 + U, 0xf, 0xf, true);
    return __builtin_bit_cast(double, r);
}
template <int U>
__device__ __forceinline__ float rowbcast(float v) {
    const int b = __builtin_bit_cast(int, v);
    const int r = __builtin_amdgcn_update_dpp(b, b, 0x150 + U, 0xf, 0xf, true);
    return __builtin_bit_cast(float, r);
}
template <typename T>
__device__ __forceinline__ T rowbcast_n(T v, int u) {   // u: a compile-time constant after unrolling
    switch (u) {
        case 0: return rowbcast<0>(v);   case 1: return rowbcast<1>(v);   case 2: return rowbcast<2>(v);
        case 3: return rowbcast<3>(v);   case 4: return rowbcast<4>(v);   case 5: return rowbcast<5>(v);
        case 6: return rowbcast<6>(v);   case 7: return rowbcast<7>(v);   case 8: return rowbcast<8>(v);
        case 9: return rowbcast<9>(v);   case 10: return rowbcast<10>(v); case 11: return rowbcast<11>(v);
        case 12: return rowbcast<12>(v); case 13: return rowbcast<13>(v); case 14: return rowbcast<14>(v);
        default: return rowbcast<15>(v);
    }
}

// LDL^T of one kPanel x kPanel diagonal block held in LDS (column-major,
// leading dimension kPanel + 1, lower triangle), with the static-pivot rule of
// Sec. 3.1 for its first w pivots.  The caller pads the block beyond w with
// the identity and zeroes the upper triangle, so every size is a compile-time
// constant: wave 0 factors each 16-column sub-panel in registers (lane = row,
// readlane broadcasts), then the four waves apply its rank-16 update to the
// trailing lower block on MFMA.  Bit c of negmask set = pivot c takes the
// negative sign.  On return: L strictly below the diagonal, d on the diagonal
// and in dv; lane 0 of wave 0 has added the counts of the first w pivots to
// cnt[4].  Called by all 256 threads; ends with a barrier.
template <typename T>
__device__ __forceinline__ void diag_ldlt64(T* B, T* dv, unsigned long long negmask, int w, const PivThr<T>& thr,
                                            unsigned int* cnt, bool& bad_out, int tid) {
    constexpr int LB = kPanel + 1;
    const int wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    bool bad_any = false;
#pragma unroll
    for (int kb = 0; kb < kPanel; kb += 16) {
        if (wave == 0) {
            // Row `lane`, columns kb..kb+15.  Entries above a row's diagonal are
            // scratch: they take the same updates, are never read as a pivot or
            // a multiplier of a lower row, and are not stored.
            T r[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) r[t] = B[lane + (kb + t) * LB];
            T mydk = T(0);
            unsigned int np = 0, nn = 0, nz = 0, npt = 0;
            bool anybad = false;
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int c = kb + t;
                bool pert, bd;
                // The reciprocal starts from the raw pivot; the static-pivot
                // rule (rarely taken) replaces both afterwards, so its test is
                // off the dependent chain.
                const T draw = bcast(r[t], c);
                const T inv0 = fast_rcp(draw);
                const int sg = ((negmask >> c) & 1ULL) ? -1 : 1;
                const T dk = static_pivot(draw, thr, sg, pert, bd);
                const T inv = pert ? thr.inv(sg) : inv0;
                const T l = r[t] * inv;
#pragma unroll
                for (int u = t + 1; u < 16; ++u) r[u] -= l * bcast(r[t], kb + u);
                r[t] = (lane == c) ? dk : l;
                mydk = (lane == c) ? dk : mydk;
                if (c < w) {
                    const double dd = to_d(dk);
                    np += dd > 0.0; nn += dd < 0.0; nz += dd == 0.0; npt += pert;
                    anybad |= bd;
                }
            }
#pragma unroll
            for (int t = 0; t < 16; ++t)
                if (lane >= kb + t) B[lane + (kb + t) * LB] = r[t];
            if (lane >= kb && lane < kb + 16) dv[lane] = mydk;
            if (lane == 0) {
                cnt[0] += np; cnt[1] += nn; cnt[2] += nz; cnt[3] += npt;
                bad_any |= anybad;
            }
        }
        __syncthreads();
        if (kb + 16 < kPanel) {
            // trailing lower block of order kPanel - kb - 16, in 16 x 16 tiles
            const int r0 = kb + 16;
            const int nt = (kPanel - r0) / 16;
            const int ntiles = nt * (nt + 1) / 2;
            for (int tix = wave; tix < ntiles; tix += 4) {
                int tj = 0, rem = tix;
                while (rem >= nt - tj) { rem -= nt - tj; ++tj; }
                const int ti = tj + rem;
                const int i0 = r0 + 16 * ti, j0 = r0 + 16 * tj;
                T av[4], bv[4];   // operands first: see panel_body
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    const int t = kb + 4 * st + lk;
                    av[st] = B[(i0 + lr) + t * LB];
                    bv[st] = B[(j0 + lr) + t * LB] * dv[t];
                }
                typename Mfma<T>::acc_t acc = {0, 0, 0, 0};
#pragma unroll
                for (int st = 0; st < 4; ++st) acc = Mfma<T>::run_chained(av[st], bv[st], acc);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gi = i0 + Mfma<T>::row(lk, r), gj = j0 + lr;
                    if (gi >= gj) B[gi + gj * LB] -= acc[r];
                }
            }
            __syncthreads();
        }
    }
    bad_out = bad_any;
}

// Inverse Z = L^-1 of the unit lower triangle of a factored kPanel x kPanel
// block in LDS (L strictly below the diagonal of B, column-major, leading
// dimension kPanel + 1).  Z is unit lower triangular; its strictly lower part
// is stored transposed in the strictly upper triangle of B (Z[u][t] at
// B[t + u * LB], u > t).  By 16 x 16 blocks: Z_qq = L_qq^-1 by substitution
// (wave q, lane j builds column j), then for distance 1..3 the blocks below,
// Z_iq = -Z_ii (sum_{k=q}^{i-1} L_ik Z_kq), on MFMA.  Called by all 256
// threads; ends with a barrier.
template <typename T>
__device__ __forceinline__ T zget(const T* B, int u, int t) {   // Z[u][t]
    constexpr int LB = kPanel + 1;
    return u > t ? B[t + u * LB] : (u == t ? T(1) : T(0));
}

template <typename T>
__device__ __forceinline__ void tri_inv64(T* B, int tid) {
    constexpr int LB = kPanel + 1;
    const int wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    {
        // wave q: lane (g, j) builds column j of Z_qq (same in each 16-lane
        // row) and holds row j of L_qq; L[i][u] comes from lane i of its row.
        const int o = 16 * wave, j = lr;
        T lrow[16], z[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            lrow[u] = u < j ? B[(o + j) + (o + u) * LB] : T(0);
            z[u] = (u == j) ? T(1) : T(0);
        }
#pragma unroll
        for (int i = 1; i < 16; ++i) {
            // Tie row i's broadcasts to z[i-1]: otherwise all 120 of them are
            // issued up front and held in registers.
#pragma unroll
            for (int u = 0; u < i; ++u) asm volatile("" : "+v"(lrow[u]) : "v"(z[i - 1]));
#pragma unroll
            for (int u = 0; u < i; ++u) z[i] = __builtin_fma(-rowbcast_n(lrow[u], i), z[u], z[i]);
        }
        if (lane < 16) {
#pragma unroll
            for (int i = 1; i < 16; ++i)
                if (i > j) B[(o + j) + (o + i) * LB] = z[i];
        }
    }
    __syncthreads();
    typedef typename Mfma<T>::acc_t acc_t;
#pragma unroll
    for (int dist = 1; dist < 4; ++dist) {
        const int q = wave, i = q + dist;
        if (i < 4) {
            acc_t S = {0, 0, 0, 0};
            for (int k = q; k < i; ++k) {
                T la[4], zb[4];   // operands first: see panel_body
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    const int kk = Mfma<T>::row(lk, st);
                    la[st] = B[(16 * i + lr) + (16 * k + kk) * LB];
                    zb[st] = zget(B, 16 * k + kk, 16 * q + lr);
                }
#pragma unroll
                for (int st = 0; st < 4; ++st) S = Mfma<T>::run_chained(la[st], zb[st], S);
            }
            T zi[4];
#pragma unroll
            for (int st = 0; st < 4; ++st) zi[st] = zget(B, 16 * i + lr, 16 * i + Mfma<T>::row(lk, st));
            acc_t R = {0, 0, 0, 0};
#pragma unroll
            for (int st = 0; st < 4; ++st) R = Mfma<T>::run_chained(zi[st], S[st], R);
#pragma unroll
            for (int r = 0; r < 4; ++r) B[(16 * q + lr) + (16 * i + Mfma<T>::row(lk, r)) * LB] = -R[r];
        }
        __syncthreads();
    }
}

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b runs on XCD
// b mod 8), each XCD with its own L2.  Task index for workgroup b of n such
// that every XCD takes one contiguous range of tasks: neighbouring tiles of a
// front share their panel operands, which then stay in one L2.
__device__ __forceinline__ int xcd_task(int b, int n) {
    const int x = b & 7, q = n >> 3, r = n & 7;
    return x * q + min(x, r) + (b >> 3);
}

inline unsigned int blocks_for(int64_t n, int bs) { return (unsigned int)((n + bs - 1) / bs); }

// ---------------------------------------------------------------------------
// assembly
// ---------------------------------------------------------------------------
__global__ void k_assemble(DevPlan d, int64_t nnzF, const double* __restrict__ W, const double* __restrict__ Sigma,
                           const double* __restrict__ J, const double* __restrict__ sys_rho,
                           const double* __restrict__ omega, double* __restrict__ K) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnzF) return;
    const int row = d.Krow[e];
    const double rho = sys_rho[d.row_sys[row]];
    double v = 0.0;
    const int w = d.src_w[e];
    if (w >= 0) v = W[w];
    const uint8_t fl = d.src_flag[e];
    if (fl & 1) v += Sigma[row];
    const int j = d.src_j[e];
    if (j >= 0) v += J[j];
    const int64_t q0 = d.prod_ptr[e], q1 = d.prod_ptr[e + 1];
    if (q1 > q0) {
        double acc = 0.0;
        // explicit fma in both: with every Omega_rr = 1 the K1s products
        // round exactly like K1's
        if (omega) {
            // K1s: each row r of J weighted by Omega_rr
            for (int64_t q = q0; q < q1; ++q) {
                const int a = d.prod_a[q];
                acc = fma(omega[d.jrow_of[a]] * J[a], J[d.prod_b[q]], acc);
            }
        } else {
            for (int64_t q = q0; q < q1; ++q) acc = fma(J[d.prod_a[q]], J[d.prod_b[q]], acc);
        }
        v += rho * acc;
    }
    if (fl & 2) v += -1.0 / rho;
    K[e] = v;
}

// Block per chunk of rows (one system): max |K_ij|, max row sum of |K|, and
// max |K_ij| over the primal block (i, j < n_primal).  Eight lanes share a row
// (coalesced reads of the row's entries).
__global__ __launch_bounds__(256) void k_chunk_norms(DevPlan d, const double* __restrict__ K,
                                                     const int* __restrict__ chunk_row0,
                                                     const int* __restrict__ chunk_rows, double* partial) {
    const int c = blockIdx.x;
    const int tid = threadIdx.x, sub = tid & 7, grp = tid >> 3;   // 32 row groups of 8 lanes
    double mx = 0.0, rsmax = 0.0, pmx = 0.0;
    bool bad = false;
    for (int r = grp; r < chunk_rows[c]; r += 32) {
        const int row = chunk_row0[c] + r;
        const bool prow = row < d.n_primal;
        double rs = 0.0;
        for (int64_t e = d.Kp[row] + sub; e < d.Kp[row + 1]; e += 8) {
            const double v = K[e];
            bad |= !isfinite(v);
            const double a = fabs(v);
            mx = fmax(mx, a);
            if (prow && d.Kj[e] < d.n_primal) pmx = fmax(pmx, a);
            rs += a;
        }
        for (int o = 4; o > 0; o >>= 1) rs += __shfl_xor(rs, o, 8);
        rsmax = fmax(rsmax, rs);
    }
    if (bad) { mx = INFINITY; rsmax = INFINITY; pmx = INFINITY; }
    __shared__ double sm[3][256];
    sm[0][tid] = mx;
    sm[1][tid] = rsmax;
    sm[2][tid] = pmx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            sm[0][tid] = fmax(sm[0][tid], sm[0][tid + o]);
            sm[1][tid] = fmax(sm[1][tid], sm[1][tid + o]);
            sm[2][tid] = fmax(sm[2][tid], sm[2][tid + o]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        partial[3 * c] = sm[0][0];
        partial[3 * c + 1] = sm[1][0];
        partial[3 * c + 2] = sm[2][0];
    }
}

// Block per (system, column group): reduction over the system's chunks of
// `width` values, in a fixed order (deterministic): a sum for the columns k
// with bit (k mod period) of sum_mask set, a max otherwise.
__global__ __launch_bounds__(256) void k_reduce_partials(const int* __restrict__ sys_chunk_ptr, int width, int period,
                                                         unsigned int sum_mask, const double* __restrict__ partial,
                                                         double* out) {
    const int s = blockIdx.x;
    const int k = blockIdx.y;
    const int tid = threadIdx.x;
    const bool sum = (sum_mask >> (k % period)) & 1u;
    double acc = 0.0;
    for (int c = sys_chunk_ptr[s] + tid; c < sys_chunk_ptr[s + 1]; c += 256) {
        const double v = partial[(int64_t)c * width + k];
        acc = sum ? acc + v : fmax(acc, v);
    }
    __shared__ double sm[256];
    sm[tid] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) sm[tid] = sum ? sm[tid] + sm[tid + o] : fmax(sm[tid], sm[tid + o]);
        __syncthreads();
    }
    if (tid == 0) out[(int64_t)s * width + k] = sm[0];
}

// Per system, from the reduced norms (max |K_ij|, ||K||_inf, max over the
// primal block): kmax, kinf and the two static-pivot thresholds of Sec. 3.1.
// mode 0, global rule: both eps * max |K_ij|.  mode 1, block rule (stabilized
// form): primal pivots eps * max |K_xx|, dual pivots eps / rho, the norm of
// the -1/rho I block of Sec. 3.2, eq. K2r.  mode 2: eps itself for both (the
// pivot epsilon of Sec. 4.3 as an absolute bound).  Non-finite norms set
// kNonfiniteInput.
__global__ void k_thresholds(int S, const double* norms3, double eps, int mode, const double* sys_rho,
                             double* kmax, double* kinf, double* thr, int* nonfinite) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const double a = norms3[3 * s], b = norms3[3 * s + 1], pm = norms3[3 * s + 2];
    kmax[s] = a;
    kinf[s] = b;
    thr[2 * s] = mode == 2 ? eps : (mode == 1 ? pm : a) * eps;
    thr[2 * s + 1] = mode == 2 ? eps : (mode == 1 ? eps / sys_rho[s] : eps * a);
    if (!isfinite(a) || !isfinite(b)) atomicOr(nonfinite, kNonfiniteInput);
}

// ---------------------------------------------------------------------------
// small fronts: one workgroup per front, front in LDS (column-major, ld = f)
// ---------------------------------------------------------------------------
// One front s (f <= kSmallMax) factored by the whole workgroup in LDS (A: f x f
// of T); `slot` spreads the inertia atomics.  Ends with the write-out (no
// trailing barrier).
template <typename T, bool kTwoRows>
__device__ __forceinline__ void small_front_body(const DevPlan& d, int s, int slot, const double* __restrict__ K,
                                                 T* __restrict__ F, T* __restrict__ D, T* A) {
    __shared__ T dv[kSmallMax];
    __shared__ int8_t sgn[kSmallMax];
    const int first = d.sn_first[s];
    const int p = d.sn_first[s + 1] - first;
    const int f = (int)(d.sn_rowptr[s + 1] - d.sn_rowptr[s]);
    const int c = f - p;
    const int tid = threadIdx.x;
    const int ti = tid & 63, tj = tid >> 6;

    // The front's first K entries (position and value, two per thread) are
    // loaded before the LDS zero-fill, so their latency overlaps it.
    const int64_t ke0 = d.kent_ptr[s], ke1 = d.kent_ptr[s + 1];
    int kpos[2];
    T kval[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int64_t e = ke0 + tid + 256 * u;
        if (e < ke1) {
            kpos[u] = d.kent_pos[e];
            kval[u] = (T)K[d.kent_csr[e]];
        }
    }
    for (int t = tid; t < f * f; t += 256) A[t] = T(0);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u)
        if (ke0 + tid + 256 * u < ke1) A[kpos[u]] = kval[u];
    for (int64_t e = ke0 + tid + 512; e < ke1; e += 256) A[d.kent_pos[e]] = (T)K[d.kent_csr[e]];
    __syncthreads();
    // extend-add: pull every child's contribution block, children in order.
    // Entry (a, b) of the child's lower CB is element idx = a + 128 b of a
    // 128-row grid (cc <= f <= 128); 8 loads per thread are issued before
    // their LDS adds.
    static_assert(kSmallMax == 128, "the extend-add grid assumes 128 rows");
    __shared__ int rl[kSmallMax];
    for (int k = d.child_ptr[s]; k < d.child_ptr[s + 1]; ++k) {
        const int ch = d.child_list[k];
        const int fc = (int)(d.sn_rowptr[ch + 1] - d.sn_rowptr[ch]);
        const int cc = fc - (d.sn_first[ch + 1] - d.sn_first[ch]);
        const T* __restrict__ CB = F + d.CB_off[ch];
        const int ld = d.CB_ld[ch];
        const int* __restrict__ r = d.rel + d.rel_ptr[ch];
        const int n2 = kSmallMax * cc;
        // the first batch of the child's entries is loaded before the
        // barrier that publishes its row map, so both round trips overlap
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = tid + 256 * u;
            const int a = min(idx & (kSmallMax - 1), cc - 1), b = min(idx >> 7, cc - 1);
            v[u] = cc > 0 ? CB[a + (int64_t)b * ld] : T(0);
        }
        if (tid < cc) rl[tid] = r[tid];
        __syncthreads();
        for (int base = 0; base < n2; base += 256 * 8) {
            if (base > 0) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int idx = base + tid + 256 * u;
                    const int a = min(idx & (kSmallMax - 1), cc - 1), b = min(idx >> 7, cc - 1);
                    v[u] = CB[a + (int64_t)b * ld];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = base + tid + 256 * u;
                const int a = idx & (kSmallMax - 1), b = idx >> 7;
                if (idx < n2 && a < cc && a >= b) A[rl[a] + rl[b] * f] += v[u];
            }
        }
        __syncthreads();
    }
    // partial LDL^T of the p pivot columns (blocked, MFMA trailing updates)
    const int sys = d.sn_sys[s];
    for (int k = tid; k < p; k += 256) sgn[k] = d.row_sign[d.perm[first + k]];
    __syncthreads();
    unsigned int cnt[4] = {0, 0, 0, 0};
    bool bad = false;
    lds_partial_ldlt<T, kTwoRows>(A, f, f, p, dv, sgn, PivThr<T>(d, sys), cnt, bad);
    if (tid == 0) {
        add_inertia(d, sys, cnt, slot);
        if (bad) atomicOr(d.nonfinite, kNonfiniteFactor);
    }
    for (int k = tid; k < p; k += 256) D[first + k] = dv[k];
    // write L (f x p, ld f) and the contribution block (c x c, ld CB_ld)
    T* __restrict__ L = F + d.L_off[s];
    for (int j = tj; j < p; j += 4)
        for (int i = j + ti; i < f; i += 64) L[i + (int64_t)j * f] = A[i + j * f];
    if (c > 0) {
        T* __restrict__ CB = F + d.CB_off[s];
        const int ld = d.CB_ld[s];
        for (int b = tj; b < c; b += 4)
            for (int a = b + ti; a < c; a += 64) CB[a + (int64_t)b * ld] = A[(p + a) + (p + b) * f];
    }
}

template <typename T, bool kTwoRows>
__global__ __launch_bounds__(256) void k_small_fronts(DevPlan d, const int* __restrict__ list,
                                                      const double* __restrict__ K, T* __restrict__ F,
                                                      T* __restrict__ D) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    small_front_body<T, kTwoRows>(d, list[blockIdx.x], blockIdx.x, K, F, D, reinterpret_cast<T*>(smem_raw));
}

// Fronts of order f <= kTinyMax: one wave per front, four fronts per
// workgroup, no workgroup barrier.  The wave assembles its front in an LDS
// slice (K entries, then the children's contribution blocks one after the
// other), loads row `lane` into registers and eliminates the p pivots right-
// looking with readlane broadcasts (static pivoting of Sec. 3.1), then writes
// L, D and the contribution block like k_small_fronts.
constexpr int kTinyMax = 32;

template <typename T>
__global__ __launch_bounds__(256) void k_tiny_fronts(DevPlan d, const int* __restrict__ list, int count,
                                                     const double* __restrict__ K, T* __restrict__ F,
                                                     T* __restrict__ D) {
    constexpr int LD = kTinyMax;
    __shared__ T Aall[4][kTinyMax * kTinyMax];
    __shared__ int rlall[4][kTinyMax];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = 4 * blockIdx.x + wave;
    if (q >= count) return;
    T* A = Aall[wave];
    int* rl = rlall[wave];
    const int s = list[q];
    const int first = d.sn_first[s];
    const int p = d.sn_first[s + 1] - first;
    const int f = (int)(d.sn_rowptr[s + 1] - d.sn_rowptr[s]);
    const int c = f - p;
    for (int t = lane; t < kTinyMax * kTinyMax; t += 64) A[t] = T(0);
    wave_fence();
    // K entries come with local positions for leading dimension f
    for (int64_t e = d.kent_ptr[s] + lane; e < d.kent_ptr[s + 1]; e += 64) {
        const int pos = d.kent_pos[e];
        A[pos % f + (pos / f) * LD] = (T)K[d.kent_csr[e]];
    }
    wave_fence();
    for (int k = d.child_ptr[s]; k < d.child_ptr[s + 1]; ++k) {
        const int ch = d.child_list[k];
        const int fc = (int)(d.sn_rowptr[ch + 1] - d.sn_rowptr[ch]);
        const int cc = fc - (d.sn_first[ch + 1] - d.sn_first[ch]);
        if (cc <= 0) continue;   // uniform
        const T* __restrict__ CB = F + d.CB_off[ch];
        const int ld = d.CB_ld[ch];
        if (lane < cc) rl[lane] = d.rel[d.rel_ptr[ch] + lane];
        wave_fence();
        T v[kTinyMax * kTinyMax / 64];
#pragma unroll
        for (int u = 0; u < kTinyMax * kTinyMax / 64; ++u) {
            const int idx = lane + 64 * u, a = min(idx % kTinyMax, cc - 1), b = min(idx / kTinyMax, cc - 1);
            v[u] = CB[a + (int64_t)b * ld];
        }
#pragma unroll
        for (int u = 0; u < kTinyMax * kTinyMax / 64; ++u) {
            const int idx = lane + 64 * u, a = idx % kTinyMax, b = idx / kTinyMax;
            if (a < cc && b < cc && a >= b) A[rl[a] + rl[b] * LD] += v[u];
        }
        wave_fence();
    }
    // row `lane` of the front (lanes >= f hold zeros and are never stored)
    T r[kTinyMax];
#pragma unroll
    for (int j = 0; j < kTinyMax; ++j) r[j] = A[(lane & (kTinyMax - 1)) + j * LD];
    const bool neg = lane < p && d.row_sign[d.perm[first + lane]] < 0;
    const unsigned long long negmask = __ballot(neg);
    const int sys = d.sn_sys[s];
    const PivThr<T> thr(d, sys);
    unsigned int np = 0, nn = 0, nz = 0, npt = 0;
    bool anybad = false;
#pragma unroll
    for (int k = 0; k < kTinyMax; ++k) {
        if (k < p) {   // uniform
            bool pert, bd;
            const T draw = bcast(r[k], k);
            const T inv0 = fast_rcp(draw);
            const int sg = ((negmask >> k) & 1ULL) ? -1 : 1;
            const T dk = static_pivot(draw, thr, sg, pert, bd);
            const T inv = pert ? thr.inv(sg) : inv0;
            const T l = r[k] * inv;
#pragma unroll
            for (int j = k + 1; j < kTinyMax; ++j) r[j] -= l * bcast(r[k], j);
            r[k] = (lane == k) ? dk : l;
            const double dd = to_d(dk);
            np += dd > 0.0; nn += dd < 0.0; nz += dd == 0.0; npt += pert;
            anybad |= bd;
        }
    }
    if (lane == 0) {
        const unsigned int cnt[4] = {np, nn, nz, npt};
        add_inertia(d, sys, cnt, q);
        if (anybad) atomicOr(d.nonfinite, kNonfiniteFactor);
    }
    T* __restrict__ L = F + d.L_off[s];
    T* __restrict__ CBo = F + d.CB_off[s];
    const int ldo = d.CB_ld[s];
#pragma unroll
    for (int j = 0; j < kTinyMax; ++j) {
        if (lane < f && lane >= j) {
            if (j < p) L[lane + (int64_t)j * f] = r[j];
            else if (c > 0) CBo[(lane - p) + (int64_t)(j - p) * ldo] = r[j];
        }
    }
    T mine = T(0);
#pragma unroll
    for (int j = 0; j < kTinyMax; ++j) mine = (lane == j) ? r[j] : mine;
    if (lane < p) D[first + lane] = mine;
}

// ---------------------------------------------------------------------------
// large fronts (front stored in the factor buffer, ld = f)
// ---------------------------------------------------------------------------
// Orders one wave's accesses to its column: LDS accesses of a wave execute in
// order; global stores must have completed before other lanes read them back.
template <bool kLds>
__device__ __forceinline__ void asm_fence() {
    if (!kLds) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    wave_fence();
}

// Reads back an element of the column being built.  In global memory (front
// too large for the LDS slice) the read bypasses the CU's L1, which may hold a
// copy of the line from before the wave's own stores.
template <bool kLds, typename T>
__device__ __forceinline__ T col_read(const T* p) {
    if (kLds) return *p;
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One wave per (large front, column j), four columns per workgroup: assemble
// column j (rows >= j) from K and the children's contribution blocks.  The
// task's column base, K-entry range and contribution segments (one per child
// whose CB maps a column onto j) come precomputed, so the wave starts with
// one round of independent loads.  kLds: the column is built in the wave's
// LDS slice (dynamic, 4 x >= f elements) and written once; otherwise in place.
// A wave's LDS accesses execute in order, so no workgroup barrier is needed;
// children are added one after the other (two may map onto the same row).
template <typename T, bool kLds>
__device__ __forceinline__ void asm_column(const DevPlan& d, int64_t t, const double* __restrict__ K,
                                           T* __restrict__ F, T* slice, int lane) {
    const int64_t colbase = d.asm_col[t];
    const int f = d.asm_fj[2 * t], j = d.asm_fj[2 * t + 1];
    const int64_t e0 = d.asm_kr[2 * t], e1 = d.asm_kr[2 * t + 1];
    const int64_t g0 = d.asm_seg_ptr[t], g1 = d.asm_seg_ptr[t + 1];
    T* __restrict__ Acol = F + colbase;                      // Acol[i] = A[i, j]
    T* __restrict__ cv = kLds ? slice : Acol;
    const int64_t jf = (int64_t)j * f;
    for (int i = j + lane; i < f; i += 64) cv[i] = T(0);
    asm_fence<kLds>();
    for (int64_t e = e0 + lane; e < e1; e += 64) cv[d.kent_pos[e] - jf] = (T)K[d.kent_csr[e]];
    asm_fence<kLds>();
    for (int64_t g = g0; g < g1; ++g) {
        const T* __restrict__ CB = F + d.asm_seg_cb[g];
        const int* __restrict__ r = d.rel + d.asm_seg_rel[g];
        const int b = d.asm_seg_bc[2 * g], cc = d.asm_seg_bc[2 * g + 1];
        for (int a0 = b + lane; a0 < cc; a0 += 64 * 4) {
            T v[4];
            int ri[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int a = min(a0 + 64 * u, cc - 1);
                v[u] = CB[a];
                ri[u] = r[a];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (a0 + 64 * u < cc) cv[ri[u]] = col_read<kLds>(cv + ri[u]) + v[u];
        }
        asm_fence<kLds>();
    }
    if (kLds)
        for (int i = j + lane; i < f; i += 64) Acol[i] = cv[i];
}

template <typename T, bool kLds>
__global__ __launch_bounds__(256) void k_large_asm(DevPlan d, int64_t task0, int count, int fcap,
                                                   const double* __restrict__ K, T* __restrict__ F) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t q = 4 * (int64_t)blockIdx.x + wave;
    if (q >= count) return;
    asm_column<T, kLds>(d, task0 + q, K, F, reinterpret_cast<T*>(smem_raw) + (int64_t)wave * fcap, lane);
}

// Writes the factored diagonal block of a panel (in LDS: L strictly below the
// diagonal, Z = L^-1 transposed strictly above it, column-major with leading
// dimension kPanel + 1; dv = pivots) to its consumers: D, the front's L
// (strictly lower part of the block), and Zg = Z (column-major, kPanel x
// kPanel, unit diagonal, identity beyond w) for the panel solves.
template <typename T>
__device__ void publish_diag(T* A, int f, int k0, int w, const T* Bf, const T* dv, T* D, int first, T* Zg, int tid) {
    constexpr int LB = kPanel + 1;
    if (tid < w) D[first + k0 + tid] = dv[tid];
    for (int idx = tid; idx < kPanel * kPanel; idx += 256) {
        const int u = idx & (kPanel - 1), t = idx / kPanel;   // row u, column t
        if (u < w && t < u) A[(k0 + u) + (int64_t)(k0 + t) * f] = Bf[u + t * LB];
        Zg[idx] = zget(Bf, u, t);
    }
}

// Pads the diagonal block beyond its w pivots with the identity and zeroes
// its upper triangle (entries with u < w and t < w on or below the diagonal
// are left to the caller).
template <typename T>
__device__ __forceinline__ void pad_diag(T* Bf, int w, int tid) {
    constexpr int LB = kPanel + 1;
    for (int idx = tid; idx < kPanel * kPanel; idx += 256) {
        const int u = idx & (kPanel - 1), t = idx / kPanel;
        if (u < t) Bf[u + t * LB] = T(0);
        else if (u >= w) Bf[u + t * LB] = (u == t) ? T(1) : T(0);
    }
}

__device__ __forceinline__ unsigned long long neg_mask(const DevPlan& d, int first, int k0, int w, int tid) {
    const int lane = tid & 63;
    const bool neg = lane < w && d.row_sign[d.perm[first + k0 + lane]] < 0;
    return __ballot(neg);
}

// C - L_I D_k L_J^T for the 64x64 tile at rows i0, columns j0 of front A
// (ld f), with panel k = columns [k0, k0 + w): four waves, each a 32x32
// quadrant as 2x2 blocks of 16x16 (v_mfma 16x16x4).  The accumulators start
// from C (prefetched with the operands, clamped addresses) and the B operand
// is negated, so the result is the updated tile.  acc[bi][bj][r] holds entry
// (i0 + wr + 16 bi + row(lk, r), j0 + wc + 16 bj + lr).
template <typename T>
__device__ __forceinline__ void tile_update(const T* __restrict__ A, int f, int k0, int w, int i0, int j0,
                                            const T* __restrict__ Dk, typename Mfma<T>::acc_t (&acc)[2][2], int tid) {
    const int wave = tid >> 6, lane = tid & 63;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            const int gj = min(j0 + wc + 16 * bj + lr, f - 1);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = min(i0 + wr + 16 * bi + Mfma<T>::row(lk, r), f - 1);
                acc[bi][bj][r] = A[gi + (int64_t)gj * f];
            }
        }
    constexpr int KS = kPanel / 4;
    T av[KS][2], bv[KS][2];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int t = 4 * ks + lk;
        const bool tv = t < w;
        const int tc = tv ? t : 0;
        const int64_t cofs = (int64_t)(k0 + tc) * f;
        const T dtr = Dk[tc];
        const T ndt = tv ? -dtr : T(0);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ri = i0 + wr + 16 * h + lr, rj = j0 + wc + 16 * h + lr;
            const T a = A[min(ri, f - 1) + cofs], b = A[min(rj, f - 1) + cofs];
            av[ks][h] = (tv && ri < f) ? a : T(0);
            bv[ks][h] = (rj < f) ? b * ndt : T(0);
        }
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = Mfma<T>::run(av[ks][bi], bv[ks][bj], acc[bi][bj]);
    mfma_pad();   // before the read-out of the last accumulator written
}

// One workgroup per (large front, panel k0): bring the panel's diagonal block
// up to date (for k0 > 0 it applies the previous panel's update to the block
// itself, which the update launch of that panel leaves out, so the two run
// side by side), factor it with the static-pivot rule of Sec. 3.1, count its
// inertia, invert its unit lower triangle and publish L, D and Z = L_kk^-1.
// When the panel is narrower than 64, the block's rows past the last pivot
// belong to the panel rows below it / the contribution block and are written
// back to the front.
template <typename T>
__device__ __forceinline__ void diag_body(const DevPlan& d, int s, int k0, T* F, T* D, T* Zbuf, int tid) {
    const int first = d.sn_first[s];
    const int p = d.sn_first[s + 1] - first;
    const int f = (int)(d.sn_rowptr[s + 1] - d.sn_rowptr[s]);
    const int w = min(kPanel, p - k0);
    T* __restrict__ A = F + d.L_off[s];
    constexpr int LB = kPanel + 1;
    __shared__ T Bf[kPanel * LB];
    __shared__ T dv[kPanel];
    constexpr int kIt = kPanel * kPanel / 256;   // staging: all loads first, then the LDS stores
    if (k0 == 0) {
        T cv[kIt];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int idx = tid + 256 * it, u = idx & (kPanel - 1), t = idx / kPanel;
            cv[it] = A[min(u, w - 1) + (int64_t)min(t, w - 1) * f];
        }
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int idx = tid + 256 * it, u = idx & (kPanel - 1), t = idx / kPanel;
            if (u < w && t <= u) Bf[u + t * LB] = cv[it];
        }
    } else {
        // The block's own update by the previous panel (columns kp = k0 - 64
        // .. k0, all 64 wide), with the operands read from the front as for a
        // trailing-update tile, the result into the block.
        const int kp = k0 - kPanel;
        const int nr = min(kPanel, f - k0);
        typename Mfma<T>::acc_t acc[2][2];
        tile_update<T>(A, f, kp, kPanel, k0, k0, D + first + kp, acc, tid);
        const int wave = tid >> 6, lane = tid & 63;
        const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
        const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int li = wr + bi * 16 + Mfma<T>::row(lk, r), lj = wc + bj * 16 + lr;
                    if (li < lj || li >= nr) continue;
                    const T v = acc[bi][bj][r];
                    if (li < w) Bf[li + lj * LB] = v;
                    else A[(k0 + li) + (int64_t)(k0 + lj) * f] = v;   // rows past the last pivot
                }
        __syncthreads();   // pad_diag below overwrites rows past the last pivot
    }
    pad_diag<T>(Bf, w, tid);
    const unsigned long long negmask = neg_mask(d, first, k0, w, tid);
    __syncthreads();
    const int sys = d.sn_sys[s];
    unsigned int cnt[4] = {0, 0, 0, 0};
    bool bad = false;
    diag_ldlt64<T>(Bf, dv, negmask, w, PivThr<T>(d, sys), cnt, bad, tid);
    tri_inv64<T>(Bf, tid);
    if (tid == 0) {
        add_inertia(d, sys, cnt, s + k0);
        if (bad) atomicOr(d.nonfinite, kNonfiniteFactor);
    }
    publish_diag<T>(A, f, k0, w, Bf, dv, D, first, Zbuf + d.M_off[s] + (int64_t)(k0 / kPanel) * (kPanel * kPanel),
                    tid);
}

// The first panels' diagonal blocks of a level (later ones run in
// k_large_dstep beside the previous panel's trailing update).
template <typename T>
__global__ __launch_bounds__(256) void k_large_diag(DevPlan d, const int* __restrict__ tasks, T* __restrict__ F,
                                                    T* __restrict__ D, T* __restrict__ Zbuf) {
    diag_body<T>(d, tasks[2 * blockIdx.x], tasks[2 * blockIdx.x + 1], F, D, Zbuf, threadIdx.x);
}

// One workgroup per (front, panel, 32-row block) below the panel's diagonal
// block: L[i, k0:k1] = A[i, k0:k1] Z^T D^-1 with Z = L_kk^-1 (published by the
// diagonal-block factorization), on MFMA.  The result is also stored
// transposed in the front's upper triangle (never used by the factorization)
// so that the backward solve reads L^T rows contiguously.  Wave w takes rows r0 + 16 (w & 1)
// and the output column blocks J = w >> 1 and 3 - (w >> 1); Z is lower
// triangular, so block J contracts over k < 16 (J + 1) only.
template <typename T>
__device__ __forceinline__ void panel_body(const DevPlan& d, int s, int k0, int r0, T* F, const T* D,
                                           const T* Zbuf, int tid) {
    const int first = d.sn_first[s];
    const int p = d.sn_first[s + 1] - first;
    const int f = (int)(d.sn_rowptr[s + 1] - d.sn_rowptr[s]);
    const int w = min(kPanel, p - k0);
    T* __restrict__ A = F + d.L_off[s];
    const T* __restrict__ Zt = Zbuf + d.M_off[s] + (int64_t)(k0 / kPanel) * (kPanel * kPanel);
    const int wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int rb = r0 + 16 * (wave & 1);
    const int row = rb + lr;
    const bool rv = row < f;
    T a[4][4];
#pragma unroll
    for (int K = 0; K < 4; ++K)
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int kk = 16 * K + Mfma<T>::row(lk, st);
            a[K][st] = (rv && kk < w) ? A[row + (int64_t)(k0 + kk) * f] : T(0);
        }
    typedef typename Mfma<T>::acc_t acc_t;
    // Z operands of both output blocks (blocks K <= J only: Z is lower
    // triangular), loaded before the padded MFMA chains (the padding's
    // scheduling barriers would otherwise hold each load next to its MFMA and
    // serialize the round trips)
    T zo[2][4][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int J = h ? 3 - (wave >> 1) : (wave >> 1);
#pragma unroll
        for (int K = 0; K < 4; ++K) {
            if (K > J) continue;   // uniform
#pragma unroll
            for (int st = 0; st < 4; ++st) zo[h][K][st] = Zt[(16 * K + Mfma<T>::row(lk, st)) * kPanel + 16 * J + lr];
        }
    }
    // The results overwrite A[rows, panel] in place, and the two waves that
    // share a row block each read all of its panel columns but write only
    // their own output blocks: every wave's loads must have returned before
    // any wave stores.
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int J = h ? 3 - (wave >> 1) : (wave >> 1);
        acc_t acc = {0, 0, 0, 0};
#pragma unroll
        for (int K = 0; K < 4; ++K) {
            if (K > J) continue;   // uniform
#pragma unroll
            for (int st = 0; st < 4; ++st) acc = Mfma<T>::run_chained(a[K][st], zo[h][K][st], acc);
        }
        const int col = 16 * J + lr;
        if (col < w) {
            const T dinv = T(1) / D[first + k0 + col];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = rb + Mfma<T>::row(lk, r);
                if (gi < f) {
                    const T x = acc[r] * dinv;
                    A[gi + (int64_t)(k0 + col) * f] = x;
                    A[(k0 + col) + (int64_t)gi * f] = x;   // L^T in the unused upper triangle
                }
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_large_panel(DevPlan d, const int* __restrict__ tasks, T* __restrict__ F,
                                                     const T* __restrict__ D, const T* __restrict__ Zbuf) {
    panel_body<T>(d, tasks[3 * blockIdx.x], tasks[3 * blockIdx.x + 1], tasks[3 * blockIdx.x + 2], F, D, Zbuf,
                  threadIdx.x);
}

// Trailing update of one 64x64 lower tile: C -= L_I D_k L_J^T on MFMA, with
// the operands read straight from the front (no LDS).  The next panel's
// diagonal tile is not in the task list: its diagonal-block workgroup updates it.
template <typename T>
__device__ __forceinline__ void update_body(const DevPlan& d, int s, int k0, int i0, int j0, T* F, const T* D,
                                            int tid) {
    const int first = d.sn_first[s];
    const int p = d.sn_first[s + 1] - first;
    const int f = (int)(d.sn_rowptr[s + 1] - d.sn_rowptr[s]);
    const int w = min(kPanel, p - k0);
    T* __restrict__ A = F + d.L_off[s];
    typename Mfma<T>::acc_t acc[2][2];
    tile_update<T>(A, f, k0, w, i0, j0, D + first + k0, acc, tid);
    const int wave = tid >> 6, lane = tid & 63;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = i0 + wr + bi * 16 + Mfma<T>::row(lk, r), gj = j0 + wc + bj * 16 + lr;
                if (gi < f && gj < f && gi >= gj) A[gi + (int64_t)gj * f] = acc[bi][bj][r];
            }
}

// Panel k's trailing update and panel k+1's diagonal blocks in one launch
// (they touch disjoint tiles): the first nd workgroups factor the diagonal
// blocks (their own update read from the front, like a tile), workgroups from nd8 = nd rounded up to a
// multiple of 8 take the update tiles with the XCD-contiguous mapping.
template <typename T>
__global__ __launch_bounds__(256) void k_large_dstep(DevPlan d, const int* __restrict__ dtasks, int nd,
                                                     const int* __restrict__ utasks, int nu, T* __restrict__ F,
                                                     T* __restrict__ D, T* __restrict__ Zbuf) {
    const int nd8 = (nd + 7) & ~7;
    const int b = blockIdx.x;
    if (b < nd) {
        diag_body<T>(d, dtasks[2 * b], dtasks[2 * b + 1], F, D, Zbuf, threadIdx.x);
    } else if (b >= nd8) {
        const int* tk = utasks + 4 * xcd_task(b - nd8, nu);
        update_body<T>(d, tk[0], tk[1], tk[2], tk[3], F, D, threadIdx.x);
    }
}

// ---------------------------------------------------------------------------
// solves
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_permute_in(DevPlan d, const double* __restrict__ B, int64_t ldb, int nrhs, T* __restrict__ Y) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d.N) return;
    const int src = d.perm[k];
    for (int q = 0; q < nrhs; ++q) Y[k + q * d.N] = (T)B[src + q * ldb];
}

template <typename T>
__global__ void k_permute_out(DevPlan d, const T* __restrict__ Y, int nrhs, double* __restrict__ X, int64_t ldx) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d.N) return;
    const int dst = d.perm[k];
    for (int q = 0; q < nrhs; ++q) X[dst + q * ldx] = to_d(Y[k + q * d.N]);
}

// ---- sweeps of the fronts outside the one-wave path ----------------------
// One launch per panel step of a level.  Panel = pivot columns [c0, c0 + w),
// w <= kPanel, of front s.  Its triangle is applied through the inverse
// Z = L_kk^-1 that the factorization published (a GEMV, no dependent chain)
// for large fronts, by one-wave substitution otherwise.  The rows below the
// panel are split into tasks, one workgroup each, of solve_task_rows(w) rows:
// the panel's columns are taken 16 at a time, so a narrow panel gives each
// wave more rows instead of leaving waves idle.
//   forward: every task recomputes y = Z b of its panel (b = the pivots' right-
//     hand side, plus the children's update vectors at the first panel),
//     subtracts L[rows, panel] y from its own rows and writes them back; task 0
//     also stores y.  No task reads what another task of the launch writes: the
//     pivots' results go to a second vector Y2 (y after the forward sweep, x
//     after the backward one), the right-hand side stays in Y.
//   backward: every task forms the partial sums L[rows, panel]^T x of its rows
//     (x of rows below the panel is final when it starts).  A one-task panel
//     forms v = y / d - sum and x = Z^T v itself; otherwise the sums are left
//     for the next launch, where the task whose rows begin with the panel's
//     pivots (or a finish-only record) adds them in task order and forms x.
// Panel table (kPanInts ints): s, c0, w, first partial slot, tasks, first and
// count of the pivot rows' contribution segments.  Task (kPTaskInts ints):
// panel, rows [r0, r1) (r0 == r1 = f for a panel with nothing below), index
// within the panel, first and count of its rows' segments.  Segment (3 ints):
// child, entries [a0, a1) of its update vector that land in the rows.
// NR: columns of the right-hand side the kernel is built for (1, or up to
// kNrhsMax).

// acc[q] += sum_{k < n} M[row + (col0 + k) * f] v[k + q * ldv], q < nrhs,
// in chunks of kDotChunk operands loaded before use.
constexpr int kDotChunk = 32;
template <typename T>
__device__ __forceinline__ void row_dot(const T* __restrict__ M, int64_t f, int row, int col0, int n, const T* v,
                                        int ldv, int nrhs, T* acc) {
    for (int kc = 0; kc < n; kc += kDotChunk) {
        T lv[kDotChunk];
#pragma unroll
        for (int k = 0; k < kDotChunk; ++k) lv[k] = (kc + k < n) ? M[row + (int64_t)(col0 + kc + k) * f] : T(0);
        const bool tail = kc + kDotChunk > n;
#pragma unroll
        for (int q = 0; q < kNrhsMax; ++q) {
            if (q >= nrhs) continue;   // uniform
            const T* vq = v + kc + q * ldv;
            T a0 = T(0), a1 = T(0);
            if (!tail) {
#pragma unroll
                for (int k = 0; k < kDotChunk; k += 2) { a0 += lv[k] * vq[k]; a1 += lv[k + 1] * vq[k + 1]; }
            } else {
#pragma unroll
                for (int k = 0; k < kDotChunk; k += 2) {
                    a0 += (kc + k < n) ? lv[k] * vq[k] : T(0);
                    a1 += (kc + k + 1 < n) ? lv[k + 1] * vq[k + 1] : T(0);
                }
            }
            acc[q] += a0 + a1;
        }
    }
}

// Small fronts: the sub-block's unit lower triangle staged in Ld (64 x 65),
// then one wave substitutes (forward: rows; backward: transposed); v has
// leading dimension vld.
template <typename T, bool kBackward>
__device__ __forceinline__ void chain_solve64(const T* __restrict__ L, int f, int c, int ws, T* Ld, T* v, int vld,
                                              int nrhs) {
    const int tid = threadIdx.x, lane = tid & 63;
    {
        T lv[16];   // all loads first, then the LDS stores
#pragma unroll
        for (int it = 0; it < 16; ++it) {
            const int idx = tid + 256 * it, a = idx & 63, b = idx >> 6;
            lv[it] = L[(c + min(a, ws - 1)) + (int64_t)(c + min(b, ws - 1)) * f];
        }
#pragma unroll
        for (int it = 0; it < 16; ++it) {
            const int idx = tid + 256 * it, a = idx & 63, b = idx >> 6;
            if (a < ws && b < a) Ld[a * 65 + b] = lv[it];
        }
    }
    __syncthreads();
    if (tid < 64) {
        // the row (forward) or column (backward) of the triangle is read from
        // LDS at each step: a register copy would set the register budget of
        // every kernel that contains this path
        for (int q = 0; q < nrhs; ++q) {
            T val = lane < ws ? v[lane + q * vld] : T(0);
            if (!kBackward) {
#pragma unroll 8
                for (int k = 0; k < 63; ++k) {
                    const T l = (k < lane && lane < ws) ? Ld[lane * 65 + k] : T(0);
                    val -= l * bcast(val, k);
                }
            } else {
#pragma unroll 8
                for (int k = 63; k > 0; --k) {
                    const T l = (lane < k && k < ws) ? Ld[k * 65 + lane] : T(0);
                    val -= l * bcast(val, k);
                }
            }
            if (lane < ws) v[lane + q * vld] = val;
        }
    }
    __syncthreads();
}

// dst[r - base] += the children's update-vector entries of segments
// [g0, g0 + gn).  The entries of all segments are loaded at once (256 per
// round, one per thread, held in registers), then added segment by segment:
// two children may add to one row, and the order stays the children's.
template <typename T, int NR>
__device__ __forceinline__ void add_segments(const DevPlan& d, const T* __restrict__ U, const int* __restrict__ segs,
                                             int g0, int gn, int base, T* dst, int ld, int nrhs) {
    int total = 0;
    for (int g = g0; g < g0 + gn; ++g) total += segs[3 * g + 2] - segs[3 * g + 1];
    for (int e0 = 0; e0 < total; e0 += 256) {
        const int e = e0 + (int)threadIdx.x;
        int mine = -1, row = 0;
        T val[NR];
        if (e < total) {
            int g = g0, acc = 0;
            for (;; ++g) {
                const int len = segs[3 * g + 2] - segs[3 * g + 1];
                if (e < acc + len) break;
                acc += len;
            }
            const int ch = segs[3 * g], a = segs[3 * g + 1] + (e - acc);
            const int cc = (int)(d.sn_rowptr[ch + 1] - d.sn_rowptr[ch]) - (d.sn_first[ch + 1] - d.sn_first[ch]);
            const T* __restrict__ Uc = U + d.U_off[ch] + a;
            row = d.rel[d.rel_ptr[ch] + a] - base;
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (q < nrhs) val[q] = Uc[(int64_t)q * cc];
            mine = g;
        }
        for (int g = g0; g < g0 + gn; ++g) {
            if (mine == g)
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    if (q < nrhs) dst[row + q * ld] += val[q];
            __syncthreads();
        }
    }
}

// Forward sweep step, one workgroup per task.  With a second panel (w2 > 0,
// large fronts, w = 64) the task owns 64 rows below both panels and forms
// both y itself: y = Z b of the first, the second's b minus L[its pivots,
// first panel] y, y2 = Z2 b2, then its rows -= L[rows, first] y and
// -= L[rows, second] y2.  Every product and sum is the one a step per
// panel would form (the second panel's b as the first panel's task 0
// would update it), in the same order.
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_fwd_P(DevPlan d, const int* __restrict__ tasks,
                                               const int* __restrict__ segs, const T* __restrict__ F,
                                               const T* __restrict__ Zbuf, T* __restrict__ Y, T* __restrict__ Y2,
                                               T* __restrict__ U, int nrhs) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* v = reinterpret_cast<T*>(smem_raw);        // kPanel x nrhs: b of the pivots, then y
    T* rw = v + kPanel * nrhs;                    // kSolveRowsMax x nrhs: the task's rows
    T* part = rw + kSolveRowsMax * nrhs;          // 256 x nrhs
    T* Ld = part + 256 * nrhs;                    // 64 x 65
    T* v2 = Ld + 64 * 65;                         // kPanel x nrhs: the second panel's b, then y
    const int* tk = tasks + kTaskRec * blockIdx.x;
    const int64_t* tk64 = reinterpret_cast<const int64_t*>(tk + kTaskRec64);
    const int c0 = tk[7], w = tk[8];
    const int r0 = tk[1], nr = tk[2] - tk[1], chunk = tk[3];
    const int first = tk[13], p = tk[14], f = tk[15];
    const int w2 = tk[kTaskRec64 + 12];
    const int c02 = c0 + kPanel;
    const int c = f - p;
    const T* __restrict__ L = F + tk64[0];
    T* __restrict__ Us = U + tk64[1];
    const int64_t moff = tk64[2];
    const int tid = threadIdx.x, lane = tid & 63, q4 = tid >> 6;
    const int64_t N = d.N;
    const bool large = moff >= 0;
    const bool pair = w2 > 0;
    // wave q4: row group q4 / nwc (64 rows, lane = row), columns 16 (q4 % nwc) + [0, 16)
    const int nwc = (w + 15) >> 4, ng = 4 / nwc;
    const int rgrp = q4 / nwc, k0 = 16 * (q4 - rgrp * nwc);
    const int myrow = 64 * rgrp + lane;           // row of the task (valid if < nr)
    const int nwc2 = (w2 + 15) >> 4;              // second panel: wave q4 takes its columns 16 q4 + [0, 16)
    // Operands that depend on nothing computed here are loaded first, so
    // their latency overlaps the right-hand side's: Z[lane][16 q4 + j] (large
    // fronts) and this thread's slice of L[rows, panel]; with a second panel
    // also its Z, its slice of L[rows, second panel] and of the block
    // L[second panel's pivots, first panel].
    T z[16], lv[16], z2[16], lv2[16], lb[16];
    if (large) {
        const T* __restrict__ Zb = Zbuf + moff + (int64_t)(c0 / kPanel) * (kPanel * kPanel);
#pragma unroll
        for (int j = 0; j < 16; ++j) z[j] = (lane < w && 16 * q4 + j < w) ? Zb[(16 * q4 + j) * kPanel + lane] : T(0);
    }
    {
        const bool rv = rgrp < ng && myrow < nr;
        const int64_t row = r0 + (rv ? myrow : 0);
#pragma unroll
        for (int j = 0; j < 16; ++j) lv[j] = (rv && k0 + j < w) ? L[row + (int64_t)(c0 + k0 + j) * f] : T(0);
    }
    if (pair) {
        const T* __restrict__ Zb = Zbuf + moff + (int64_t)(c02 / kPanel) * (kPanel * kPanel);
        const bool rv = lane < nr;
        const int64_t row = r0 + (rv ? lane : 0);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int kk = 16 * q4 + j;
            z2[j] = (lane < w2 && kk < w2) ? Zb[kk * kPanel + lane] : T(0);
            lv2[j] = (rv && kk < w2) ? L[row + (int64_t)(c02 + kk) * f] : T(0);
            lb[j] = lane < w2 ? L[(c02 + lane) + (int64_t)(c0 + kk) * f] : T(0);
        }
    }
    for (int q = 0; q < nrhs; ++q) {
        if (tid < kPanel) {
            v[tid + q * kPanel] = tid < w ? Y[first + c0 + tid + q * N] : T(0);
            if (pair) v2[tid + q * kPanel] = tid < w2 ? Y[first + c02 + tid + q * N] : T(0);
        }
        const int gi = r0 + tid;
        T val = T(0);
        if (tid < nr) val = gi < p ? Y[first + gi + q * N] : (c0 == 0 ? T(0) : Us[(gi - p) + (int64_t)q * c]);
        rw[tid + q * kSolveRowsMax] = val;
    }
    __syncthreads();
    if (c0 == 0) {
        add_segments<T, NR>(d, U, segs, tk[11], tk[12], 0, v, kPanel, nrhs);
        if (pair) add_segments<T, NR>(d, U, segs, tk[kTaskRec64 + 13], tk[kTaskRec64 + 14], c02, v2, kPanel, nrhs);
        add_segments<T, NR>(d, U, segs, tk[4], tk[5], r0, rw, kSolveRowsMax, nrhs);
    }
    if (large) {
        // y = Z b: the 4 waves split the contraction, partial sums meet in part
        for (int q = 0; q < nrhs; ++q) {
            const T* vq = v + 16 * q4 + q * kPanel;
            T acc = T(0);
#pragma unroll
            for (int j = 0; j < 16; ++j) acc += z[j] * vq[j];
            part[(q4 * 64 + lane) * nrhs + q] = acc;
        }
        __syncthreads();
        if (tid < w)
            for (int q = 0; q < nrhs; ++q) {
                const T* pp = part + tid * nrhs + q;
                v[tid + q * kPanel] = (pp[0] + pp[64 * nrhs]) + (pp[128 * nrhs] + pp[192 * nrhs]);
            }
        __syncthreads();
    } else {
        chain_solve64<T, false>(L, f, c0, w, Ld, v, kPanel, nrhs);
    }
    if (chunk == 0)
        for (int q = 0; q < nrhs; ++q)
            if (tid < w) Y2[first + c0 + tid + q * N] = v[tid + q * kPanel];
    if (pair) {
        // the second panel's b -= L[its pivots, first panel] y (wave q4: columns
        // 16 q4 + [0, 16), lane = pivot), then y2 = Z2 b
        for (int q = 0; q < nrhs; ++q) {
            const T* vq = v + 16 * q4 + q * kPanel;
            T acc = T(0);
#pragma unroll
            for (int j = 0; j < 16; ++j) acc += lb[j] * vq[j];
            part[(q4 * 64 + lane) * nrhs + q] = acc;
        }
        __syncthreads();
        if (tid < w2)
            for (int q = 0; q < nrhs; ++q) {
                const T* pp = part + tid * nrhs + q;
                T sum = pp[0];
                for (int k = 1; k < 4; ++k) sum += pp[k * 64 * nrhs];
                v2[tid + q * kPanel] -= sum;
            }
        __syncthreads();
        for (int q = 0; q < nrhs; ++q) {
            const T* vq = v2 + 16 * q4 + q * kPanel;
            T acc = T(0);
#pragma unroll
            for (int j = 0; j < 16; ++j) acc += z2[j] * vq[j];
            part[(q4 * 64 + lane) * nrhs + q] = acc;
        }
        __syncthreads();
        if (tid < w2)
            for (int q = 0; q < nrhs; ++q) {
                const T* pp = part + tid * nrhs + q;
                const T y2 = (pp[0] + pp[64 * nrhs]) + (pp[128 * nrhs] + pp[192 * nrhs]);
                v2[tid + q * kPanel] = y2;
                if (chunk == 0) Y2[first + c02 + tid + q * N] = y2;
            }
        __syncthreads();
    }
    if (nr == 0) return;
    // rows: y_i -= L[i, panel] y
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        if (q >= nrhs) continue;
        const T* vq = v + k0 + q * kPanel;
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < 16; ++j) acc += lv[j] * vq[j];
        part[(q4 * 64 + lane) * nrhs + q] = acc;
    }
    __syncthreads();
    if (!pair) {
        if (tid < nr) {
            const int gi = r0 + tid, g = tid >> 6, l = tid & 63;
            for (int q = 0; q < nrhs; ++q) {
                const T* pp = part + ((g * nwc) * 64 + l) * nrhs + q;
                T sum = pp[0];
                for (int k = 1; k < nwc; ++k) sum += pp[k * 64 * nrhs];
                const T val = rw[tid + q * kSolveRowsMax] - sum;
                if (gi < p) Y[first + gi + q * N] = val;
                else Us[(gi - p) + (int64_t)q * c] = val;
            }
        }
        return;
    }
    // two panels: the first panel's update of the rows, then the second's
    if (tid < nr)
        for (int q = 0; q < nrhs; ++q) {
            const T* pp = part + tid * nrhs + q;
            T sum = pp[0];
            for (int k = 1; k < 4; ++k) sum += pp[k * 64 * nrhs];
            rw[tid + q * kSolveRowsMax] -= sum;
        }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        if (q >= nrhs) continue;
        const T* vq = v2 + 16 * q4 + q * kPanel;
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < 16; ++j) acc += lv2[j] * vq[j];
        part[(q4 * 64 + lane) * nrhs + q] = acc;
    }
    __syncthreads();
    if (tid < nr) {
        const int gi = r0 + tid;
        for (int q = 0; q < nrhs; ++q) {
            const T* pp = part + tid * nrhs + q;
            T sum = pp[0];
            for (int k = 1; k < nwc2; ++k) sum += pp[k * 64 * nrhs];
            const T val = rw[tid + q * kSolveRowsMax] - sum;
            if (gi < p) Y[first + gi + q * N] = val;
            else Us[(gi - p) + (int64_t)q * c] = val;
        }
    }
}

// x of a panel's xw pivots from the sums over its rows below (v, kPanel x
// nrhs in LDS): v = y / d - sums, then x = Z^T v with Z = L_kk^-1 (this
// thread's share in zv, staged transposed in Ld; wave q4 takes rows
// 16 q4 .. 16 q4 + 15).  x goes to Y2p (the panel's first pivot) and, when
// xs is given, to the task's rows from xoff.
template <typename T, int NR>
__device__ __forceinline__ void bwd_panel_x(T* v, T* part, T* Ld, const T (&zv)[kPanel * kPanel / 256],
                                            const T (&yv)[NR], T dinv, int xw, int nrhs, T* __restrict__ Y2p,
                                            int64_t N, T* xs, int xoff, int tid) {
    const int lane = tid & 63, q4 = tid >> 6;
    if (tid < kPanel) {
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            if (q >= nrhs) continue;
            v[tid + q * kPanel] = tid < xw ? yv[q] * dinv - v[tid + q * kPanel] : T(0);
        }
    }
#pragma unroll
    for (int it = 0; it < kPanel * kPanel / 256; ++it) {
        const int idx = tid + 256 * it;
        Ld[(idx & 63) + (idx >> 6) * 65] = zv[it];
    }
    __syncthreads();
    for (int q = 0; q < nrhs; ++q) {
        const T* vq = v + 16 * q4 + q * kPanel;
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < 16; ++j) acc += Ld[(16 * q4 + j) + lane * 65] * vq[j];
        part[(q4 * 64 + lane) * nrhs + q] = acc;
    }
    __syncthreads();
    if (tid < xw)
        for (int q = 0; q < nrhs; ++q) {
            const T* pp = part + tid * nrhs + q;
            const T x = (pp[0] + pp[64 * nrhs]) + (pp[128 * nrhs] + pp[192 * nrhs]);
            Y2p[tid + q * N] = x;
            if (xs) xs[xoff + tid + q * kSolveRowsMax] = x;
        }
}

// Backward sweep step, one workgroup per task (rows r0..r1 below a panel):
// the task's sums L[rows, panel]^T x[rows] (a large front keeps L^T in its
// upper triangle).  A panel with one task is finished by it.  A panel with
// several leaves their sums in pw (slots slot0 + index) and is finished in
// the next launch -- ordered on the same stream, so plain loads see the sums
// -- by the first task of the front's previous panel, whose rows start with
// this panel's pivots and which needs their x first, or, for a front's first
// panel, by a finish-only record (index -1) after the level's last step.
// Each panel's sums are added in task order per wave (wave q4: tasks q4,
// q4 + 4, ...), then the four waves' totals.
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_bwd_P(DevPlan d, const int* __restrict__ tasks,
                                               const T* __restrict__ F, const T* __restrict__ Zbuf,
                                               const T* __restrict__ D, T* __restrict__ Y2, T* __restrict__ pw,
                                               const T* __restrict__ pr, int nrhs) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* xs = reinterpret_cast<T*>(smem_raw);       // kSolveRowsMax x nrhs: x of the task's rows
    T* v = xs + kSolveRowsMax * nrhs;             // kPanel x nrhs
    T* part = v + kPanel * nrhs;                  // 256 x nrhs
    T* Ld = part + 256 * nrhs;                    // 64 x 65
    const int* tk = tasks + kTaskRec * blockIdx.x;
    const int64_t* tk64 = reinterpret_cast<const int64_t*>(tk + kTaskRec64);
    const int c0 = tk[7], w = tk[8], slot0 = tk[9], ntask = tk[10];
    const int r0 = tk[1], nr = tk[2] - tk[1], chunk = tk[3];
    const int first = tk[13], p = tk[14], f = tk[15];
    const int fc0 = tk[kTaskRec64 + 8], fw = tk[kTaskRec64 + 9];
    const int fslot0 = tk[kTaskRec64 + 10], fntask = tk[kTaskRec64 + 11];
    const T* __restrict__ L = F + tk64[0];
    const int64_t moff = tk64[2];
    const int* __restrict__ rows = d.sn_rows + tk64[3];
    const bool large = moff >= 0;
    const bool own = chunk >= 0;              // else a finish-only record
    const bool fin = fntask > 0;              // finishes panel fc0 before its own sums
    const bool self = own && ntask == 1;      // finishes its own panel
    const int xc0 = fin ? fc0 : c0;           // the panel it finishes (xw pivots, 0: none)
    const int xw = fin ? fw : (self ? w : 0);
    const int tid = threadIdx.x, lane = tid & 63, q4 = tid >> 6;
    const int64_t N = d.N;
    // thread = (panel column t, row group rg): columns in slots of 16, the
    // row groups take rows rg, rg + nrg, ... (at most 16 per thread)
    const int W16 = 16 * ((w + 15) >> 4), nrg = 256 / W16;
    const int t = tid % W16, rg = tid / W16;
    const bool tact = own && t < w && rg < nrg;
    // Loads that depend on nothing computed here first: this thread's L^T
    // operands, and Z, 1 / d and y of the panel it finishes.
    T lv[16], zv[kPanel * kPanel / 256];
    if (large) {
        const T* __restrict__ lt = L + (c0 + (tact ? t : 0)) + (int64_t)r0 * f;
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int i = rg + nrg * m;
            lv[m] = (tact && i < nr) ? lt[(int64_t)i * f] : T(0);
        }
        const T* __restrict__ Zb = Zbuf + moff + (int64_t)(xc0 / kPanel) * (kPanel * kPanel);
#pragma unroll
        for (int it = 0; it < kPanel * kPanel / 256; ++it) {
            const int idx = tid + 256 * it;
            zv[it] = ((idx & 63) < xw && (idx >> 6) < xw) ? Zb[idx] : T(0);
        }
    }
    const T dinv = tid < xw ? T(1) / D[first + xc0 + tid] : T(0);
    T yv[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) yv[q] = (q < nrhs && tid < xw) ? Y2[first + xc0 + tid + q * N] : T(0);
    if (own)
        for (int q = 0; q < nrhs; ++q) {
            const int gi = r0 + tid;
            xs[tid + q * kSolveRowsMax] = tid >= nr ? T(0) : gi < p ? Y2[first + gi + q * N] : Y2[rows[gi] + q * N];
        }
    if (!large && own && nr > 0) {
        // column-major L only: stage L[rows, panel] as Ld[i + 65 t] (coalesced
        // reads); such fronts have at most 64 rows below a panel (analysis)
        for (int idx = tid; idx < 64 * kPanel; idx += 256) {
            const int i = idx & 63, tt = idx >> 6;
            Ld[i + 65 * tt] = (i < nr && tt < w) ? L[(r0 + i) + (int64_t)(c0 + tt) * f] : T(0);
        }
    }
    if (fin) {
        T acc2[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) acc2[q] = T(0);
        for (int g0 = q4; g0 < fntask; g0 += 32) {
            T pv[8];
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                if (q >= nrhs) continue;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int g = g0 + 4 * u;
                    pv[u] = g < fntask ? pr[((int64_t)(fslot0 + g) * kPanel + lane) * kNrhsMax + q] : T(0);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) acc2[q] += pv[u];
            }
        }
#pragma unroll
        for (int q = 0; q < NR; ++q)
            if (q < nrhs) part[(q4 * 64 + lane) * nrhs + q] = acc2[q];
        __syncthreads();
        if (tid < kPanel)
            for (int q = 0; q < nrhs; ++q) {
                const T* pp = part + tid * nrhs + q;
                v[tid + q * kPanel] = (pp[0] + pp[64 * nrhs]) + (pp[128 * nrhs] + pp[192 * nrhs]);
            }
        __syncthreads();
        bwd_panel_x<T, NR>(v, part, Ld, zv, yv, dinv, fw, nrhs, Y2 + first + fc0, N, own ? xs : nullptr,
                           fc0 - r0, tid);
    }
    if (!own) return;
    __syncthreads();
    // partial sums over the task's rows
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        if (q >= nrhs) continue;
        T a = T(0);
        if (large) {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int i = rg + nrg * m;
                a += lv[m] * xs[min(i, kSolveRowsMax - 1) + q * kSolveRowsMax];
            }
        } else if (tact) {
            for (int m = 0; m < 16; ++m) {
                const int i = rg + nrg * m;
                if (i < 64) a += Ld[i + 65 * t] * xs[i + q * kSolveRowsMax];
            }
        }
        part[tid * nrhs + q] = tact ? a : T(0);
    }
    __syncthreads();
    // this task's sum per panel column
    if (tid < kPanel)
        for (int q = 0; q < nrhs; ++q) {
            T sum = T(0);
            if (tid < w)
                for (int g = 0; g < nrg; ++g) sum += part[(g * W16 + tid) * nrhs + q];
            v[tid + q * kPanel] = sum;
        }
    __syncthreads();
    if (ntask > 1) {
        if (tid < kPanel)
            for (int q = 0; q < nrhs; ++q)
                pw[((int64_t)(slot0 + chunk) * kPanel + tid) * kNrhsMax + q] = v[tid + q * kPanel];
        return;
    }
    if (large) {
        bwd_panel_x<T, NR>(v, part, Ld, zv, yv, dinv, w, nrhs, Y2 + first + c0, N, nullptr, 0, tid);
    } else {
        if (tid < kPanel) {
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                if (q >= nrhs) continue;
                v[tid + q * kPanel] = tid < w ? yv[q] * dinv - v[tid + q * kPanel] : T(0);
            }
        }
        __syncthreads();
        chain_solve64<T, true>(L, f, c0, w, Ld, v, kPanel, nrhs);
        for (int q = 0; q < nrhs; ++q)
            if (tid < w) Y2[first + c0 + tid + q * N] = v[tid + q * kPanel];
    }
}

// Fronts with p <= 64 pivots and f <= kSmallRows rows (L is f x p, ld f).  Each
// wave keeps its front's right-hand-side rows in LDS (ld kSmallRows) and
// synchronizes only with itself; a workgroup carries four fronts.
constexpr int kSmallRows = 128;

// Forward: pull the children's update vectors, substitute the p pivots (lane =
// pivot row, readlane broadcasts), apply them to the rows below, write back.
template <typename T>
__global__ __launch_bounds__(256, 4) void k_fwd_S(DevPlan d, const int* __restrict__ fronts, int count,
                                               const T* __restrict__ F, const T* __restrict__ Y, T* __restrict__ Y2,
                                               T* __restrict__ U, int nrhs) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int task = blockIdx.x * 4 + wv;
    if (task >= count) return;   // whole wave; no workgroup barrier below
    T* ys = reinterpret_cast<T*>(smem_raw) + wv * kSmallRows * nrhs;
    const int s = fronts[task];
    const int first = d.sn_first[s];
    const int p = d.sn_first[s + 1] - first;
    const int f = (int)(d.sn_rowptr[s + 1] - d.sn_rowptr[s]);
    const int c = f - p;
    const T* __restrict__ L = F + d.L_off[s];
    T* __restrict__ Us = U + d.U_off[s];
    const int64_t N = d.N;
    for (int q = 0; q < nrhs; ++q)
        for (int i = lane; i < f; i += 64) ys[i + q * kSmallRows] = i < p ? Y[first + i + q * N] : T(0);
    wave_fence();
    for (int k = d.child_ptr[s]; k < d.child_ptr[s + 1]; ++k) {
        const int ch = d.child_list[k];
        const int cc = (int)(d.sn_rowptr[ch + 1] - d.sn_rowptr[ch]) - (d.sn_first[ch + 1] - d.sn_first[ch]);
        const T* __restrict__ Uc = U + d.U_off[ch];
        const int* __restrict__ r = d.rel + d.rel_ptr[ch];
        for (int q = 0; q < nrhs; ++q)
            for (int a = lane; a < cc; a += 64) ys[r[a] + q * kSmallRows] += Uc[a + (int64_t)q * cc];
        wave_fence();
    }
    // substitution in two 32-column chunks (most small fronts need one)
    const int lr = min(lane, f - 1);
    for (int kc = 0; kc < p; kc += 32) {
        T lrow[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            if (kc + k < p) {
                const T x = L[lr + (int64_t)(kc + k) * f];
                lrow[k] = (kc + k < lane && lane < p) ? x : T(0);
            } else {
                lrow[k] = T(0);
            }
        }
        for (int q = 0; q < nrhs; ++q) {
            T val = lane < p ? ys[lane + q * kSmallRows] : T(0);
#pragma unroll
            for (int k = 0; k < 32; ++k)
                if (kc + k + 1 < p) val -= lrow[k] * bcast(val, kc + k);
            if (lane < p) ys[lane + q * kSmallRows] = val;
        }
        wave_fence();
    }
    for (int i0 = p; i0 < f; i0 += 64) {
        const int i = i0 + lane;
        const int ic = min(i, f - 1);
        T acc[kNrhsMax];
#pragma unroll
        for (int q = 0; q < kNrhsMax; ++q) acc[q] = T(0);
        for (int kc = 0; kc < p; kc += 32) {
            T lv[32];
#pragma unroll
            for (int k = 0; k < 32; ++k) lv[k] = (kc + k < p) ? L[ic + (int64_t)(kc + k) * f] : T(0);
#pragma unroll
            for (int q = 0; q < kNrhsMax; ++q) {
                if (q >= nrhs) continue;
                const T* yq = ys + kc + q * kSmallRows;
                T a = T(0);
#pragma unroll
                for (int k = 0; k < 32; ++k)
                    if (kc + k < p) a += lv[k] * yq[k];
                acc[q] += a;
            }
        }
#pragma unroll
        for (int q = 0; q < kNrhsMax; ++q)
            if (q < nrhs && i < f) ys[i + q * kSmallRows] -= acc[q];
    }
    wave_fence();
    for (int q = 0; q < nrhs; ++q)
        for (int i = lane; i < f; i += 64) {
            const T v = ys[i + q * kSmallRows];
            if (i < p) Y2[first + i + q * N] = v;
            else Us[(i - p) + (int64_t)q * c] = v;
        }
}

// Backward: gather x of the rows below, v_t = y_t / d_t - sum_i L[i][t] x_i
// (lane = pivot column t, its column read contiguously), then the transposed
// substitution from the last pivot up (readlane broadcasts).
template <typename T>
__global__ __launch_bounds__(256, 4) void k_bwd_S(DevPlan d, const int* __restrict__ fronts, int count,
                                               const T* __restrict__ F, const T* __restrict__ D,
                                               T* __restrict__ Y2, int nrhs) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int task = blockIdx.x * 4 + wv;
    if (task >= count) return;   // whole wave; no workgroup barrier below
    T* xs = reinterpret_cast<T*>(smem_raw) + wv * kSmallRows * nrhs;
    const int s = fronts[task];
    const int first = d.sn_first[s];
    const int p = d.sn_first[s + 1] - first;
    const int64_t rb = d.sn_rowptr[s];
    const int f = (int)(d.sn_rowptr[s + 1] - rb);
    const T* __restrict__ L = F + d.L_off[s];
    const int* __restrict__ rows = d.sn_rows + rb;
    const int64_t N = d.N;
    for (int q = 0; q < nrhs; ++q)
        for (int i = lane; i < f; i += 64)
            xs[i + q * kSmallRows] = i < p ? Y2[first + i + q * N] : Y2[rows[i] + q * N];
    wave_fence();
    const int t = lane;
    const bool tv = t < p;
    const T* __restrict__ col = L + (int64_t)min(t, p - 1) * f;
    T acc[kNrhsMax];
#pragma unroll
    for (int q = 0; q < kNrhsMax; ++q) acc[q] = T(0);
    for (int i0 = p; i0 < f; i0 += 32) {
        T lv[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) lv[k] = (i0 + k < f) ? col[i0 + k] : T(0);
#pragma unroll
        for (int q = 0; q < kNrhsMax; ++q) {
            if (q >= nrhs) continue;
            const T* xq = xs + i0 + q * kSmallRows;
            T a = T(0);
#pragma unroll
            for (int k = 0; k < 32; ++k)
                if (i0 + k < f) a += lv[k] * xq[k];
            acc[q] += a;
        }
    }
    // v_t into xs[t], then the transposed substitution in 32-row chunks from
    // the last pivot up (x_k final at lane k when chunk k is reached)
    const T dinv = T(1) / D[first + min(t, p - 1)];
#pragma unroll
    for (int q = 0; q < kNrhsMax; ++q)
        if (q < nrhs && tv) xs[t + q * kSmallRows] = xs[t + q * kSmallRows] * dinv - acc[q];
    wave_fence();
    for (int kc = ((p - 1) / 32) * 32; kc >= 0; kc -= 32) {
        T lcol[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            if (kc + k < p) {
                const T x = col[kc + k];
                lcol[k] = (tv && kc + k > t) ? x : T(0);
            } else {
                lcol[k] = T(0);
            }
        }
        for (int q = 0; q < nrhs; ++q) {
            T val = tv ? xs[t + q * kSmallRows] : T(0);
#pragma unroll
            for (int k = 31; k >= 0; --k)
                if (kc + k < p && kc + k > 0) val -= lcol[k] * bcast(val, kc + k);
            if (tv) xs[t + q * kSmallRows] = val;
        }
        wave_fence();
    }
    for (int q = 0; q < nrhs; ++q)
        if (tv) Y2[first + t + q * N] = xs[t + q * kSmallRows];
}

// ---------------------------------------------------------------------------
// persistent launches: one workgroup per front, fronts from a ticket counter
// ---------------------------------------------------------------------------
// Thread 0 waits until *ctr >= target, then acquires (agent scope: the
// producers ran on other XCDs, whose L2 caches are not coherent with this
// one); the barrier hands the data to the whole workgroup.  Polls back off
// exponentially (up to ~0.9 us apart) and read the shared status word only
// every 64 polls: hundreds of waiting workgroups must not flood one cache
// line.  A wait gives up after `timeout` ticks of wall_clock64 and sets bit 1
// of *status; every later wait then returns within 64 polls, so the grid
// always drains in bounded time.
__device__ __forceinline__ void pers_wait(const int* ctr, int target, int* status, unsigned long long timeout) {
    if (threadIdx.x == 0 && target > 0) {
        const unsigned long long t0 = wall_clock64();
        int backoff = 1;
        for (int n = 1; __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; ++n) {
            if ((n & 63) == 0) {
                if (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2) break;
                if (wall_clock64() - t0 > timeout) {
                    atomicOr(status, 2);
                    break;
                }
            }
            for (int i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(1);
            backoff = min(2 * backoff, 32);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Every wave waits for its stores to reach the L2, then one agent-scope
// release (L2 write-back) publishes them with the counter increment.
__device__ __forceinline__ void pers_signal(int* ctr) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0 && ctr) __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int pers_ticket(int* ctr, int* shared_slot) {
    if (threadIdx.x == 0) *shared_slot = __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int t = *shared_slot;
    __syncthreads();
    return t;
}

// A large front factored by one workgroup: its columns assembled in the
// waves' LDS slices, then the panel steps in order (diagonal block, panel
// solve of every 32-row block, trailing tiles except the next diagonal tile,
// next diagonal block with its own update) -- the steps the level-scheduled
// launches take, one after the other.
template <typename T>
__device__ void large_front_body(const DevPlan& d, int s, int64_t a0, int acnt, int fcap, const double* __restrict__ K,
                                 T* __restrict__ F, T* __restrict__ D, T* __restrict__ Zbuf, T* lds) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int q = wave; q < acnt; q += 4) asm_column<T, true>(d, a0 + q, K, F, lds + (int64_t)wave * fcap, lane);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    const int p = d.sn_first[s + 1] - d.sn_first[s];
    const int f = (int)(d.sn_rowptr[s + 1] - d.sn_rowptr[s]);
    diag_body<T>(d, s, 0, F, D, Zbuf, tid);
    __syncthreads();
    for (int k0 = 0; k0 < p; k0 += kPanel) {
        const int k1 = min(k0 + kPanel, p);
        for (int r0 = k1; r0 < f; r0 += 32) panel_body<T>(d, s, k0, r0, F, D, Zbuf, tid);
        __syncthreads();
        for (int j0 = k1; j0 < f; j0 += kTile)
            for (int i0 = j0; i0 < f; i0 += kTile) {
                if (i0 == k1 && j0 == k1 && k1 < p) continue;
                update_body<T>(d, s, k0, i0, j0, F, D, tid);
            }
        __syncthreads();
        if (k1 < p) {
            diag_body<T>(d, s, k1, F, D, Zbuf, tid);
            __syncthreads();
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_persist_factor(DevPlan d, const int* __restrict__ order, int ntask,
                                                        const int64_t* __restrict__ asm_rng, int fcap, int* ctr,
                                                        int* ticket, int* status, unsigned long long timeout,
                                                        unsigned long long* tstamp,
                                                        const double* __restrict__ K, T* __restrict__ F,
                                                        T* __restrict__ D, T* __restrict__ Zbuf) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    __shared__ int s_t;
    for (;;) {
        const int t = pers_ticket(ticket, &s_t);
        if (t >= ntask) break;
        if (t == 0 && threadIdx.x == 0) tstamp[0] = wall_clock64();
        const int s = order[t];
        pers_wait(ctr + s, d.child_ptr[s + 1] - d.child_ptr[s], status, timeout);
        const int f = (int)(d.sn_rowptr[s + 1] - d.sn_rowptr[s]);
        if (d.M_off[s] < 0) {
            if (f > 64) small_front_body<T, true>(d, s, t, K, F, D, lds);
            else small_front_body<T, false>(d, s, t, K, F, D, lds);
        } else {
            large_front_body<T>(d, s, asm_rng[2 * s], (int)asm_rng[2 * s + 1], fcap, K, F, D, Zbuf, lds);
        }
        const int par = d.sn_parent[s];
        pers_signal(par >= 0 ? ctr + par : nullptr);
        if (par < 0 && threadIdx.x == 0) atomicMax(tstamp + 1 + d.sn_sys[s], (unsigned long long)wall_clock64());
    }
}

// Forward sweep of one front by the workgroup: y (f x nrhs, LDS, ld fcap) =
// its pivots' entries plus the children's update vectors; each 64-column
// block solved (Z = L_kk^-1 for large fronts, substitution by one wave
// otherwise) and applied to the rows below; pivots back to Y, the rest to the
// front's update vector.
template <typename T>
__device__ void front_forward(const DevPlan& d, int s, int fcap, const T* __restrict__ F, const T* __restrict__ Zbuf,
                              const T* __restrict__ Y, T* __restrict__ Y2, T* __restrict__ U, int nrhs, T* ys, T* Ld,
                              T* part) {
    const int tid = threadIdx.x, lane = tid & 63, q4 = tid >> 6;
    const int first = d.sn_first[s];
    const int p = d.sn_first[s + 1] - first;
    const int f = (int)(d.sn_rowptr[s + 1] - d.sn_rowptr[s]);
    const int c = f - p;
    const T* __restrict__ L = F + d.L_off[s];
    T* __restrict__ Us = U + d.U_off[s];
    const int64_t N = d.N;
    for (int q = 0; q < nrhs; ++q)
        for (int i = tid; i < f; i += 256) ys[i + q * fcap] = i < p ? Y[first + i + q * N] : T(0);
    __syncthreads();
    for (int k = d.child_ptr[s]; k < d.child_ptr[s + 1]; ++k) {
        const int ch = d.child_list[k];
        const int cc = (int)(d.sn_rowptr[ch + 1] - d.sn_rowptr[ch]) - (d.sn_first[ch + 1] - d.sn_first[ch]);
        const T* __restrict__ Uc = U + d.U_off[ch];
        const int* __restrict__ r = d.rel + d.rel_ptr[ch];
        for (int q = 0; q < nrhs; ++q)
            for (int a = tid; a < cc; a += 256) ys[r[a] + q * fcap] += Uc[a + (int64_t)q * cc];
        __syncthreads();
    }
    for (int cb = 0; cb < p; cb += kPanel) {
        const int ws = min(kPanel, p - cb);
        if (d.M_off[s] >= 0) {
            // v <- Z v, Z column-major 64 x 64; wave q4 takes columns 16 q4 .. 16 q4 + 15
            const T* __restrict__ Zb = Zbuf + d.M_off[s] + (int64_t)(cb / kPanel) * (kPanel * kPanel);
            T z[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) z[j] = Zb[(16 * q4 + j) * kPanel + lane];
            for (int q = 0; q < nrhs; ++q) {
                T acc = T(0);
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int k = 16 * q4 + j;
                    acc += z[j] * (k < ws ? ys[cb + k + q * fcap] : T(0));
                }
                part[(q4 * 64 + lane) * nrhs + q] = acc;
            }
            __syncthreads();
            if (tid < ws)
                for (int q = 0; q < nrhs; ++q) {
                    const T* pp = part + tid * nrhs + q;
                    ys[cb + tid + q * fcap] = (pp[0] + pp[64 * nrhs]) + (pp[128 * nrhs] + pp[192 * nrhs]);
                }
            __syncthreads();
        } else if (tid < 64) {
            // unit lower substitution on one wave: lane = row of the block
            T lrow[64];
#pragma unroll
            for (int k = 0; k < 64; ++k)
                lrow[k] = (k < lane && lane < ws) ? L[(cb + lane) + (int64_t)(cb + k) * f] : T(0);
            for (int q = 0; q < nrhs; ++q) {
                T val = lane < ws ? ys[cb + lane + q * fcap] : T(0);
#pragma unroll
                for (int k = 0; k < 63; ++k) val -= lrow[k] * bcast(val, k);
                if (lane < ws) ys[cb + lane + q * fcap] = val;
            }
        }
        __syncthreads();
        // rows below the block: y_i -= L[i, cb : cb + ws] y_block
        for (int i = cb + ws + tid; i < f; i += 256) {
            for (int q = 0; q < nrhs; ++q) {
                const T* yb = ys + cb + q * fcap;
                T acc = T(0);
                for (int k = 0; k < ws; ++k) acc += L[i + (int64_t)(cb + k) * f] * yb[k];
                ys[i + q * fcap] -= acc;
            }
        }
        __syncthreads();
    }
    for (int q = 0; q < nrhs; ++q)
        for (int i = tid; i < f; i += 256) {
            const T v = ys[i + q * fcap];
            if (i < p) Y2[first + i + q * N] = v;
            else Us[(i - p) + (int64_t)q * c] = v;
        }
}

// Backward sweep of one front: x of the rows below its pivots (already
// final: they belong to ancestors) gathered from Y, then the pivot blocks from
// the last: v = y / d - L[rows below the block, block]^T x, and the block's
// transposed triangle (Z^T for large fronts, substitution otherwise).
template <typename T>
__device__ void front_backward(const DevPlan& d, int s, int fcap, const T* __restrict__ F,
                               const T* __restrict__ Zbuf, const T* __restrict__ D, T* __restrict__ Y2, int nrhs,
                               T* xs, T* Ld, T* part) {
    const int tid = threadIdx.x, lane = tid & 63, q4 = tid >> 6;
    const int first = d.sn_first[s];
    const int p = d.sn_first[s + 1] - first;
    const int64_t rb = d.sn_rowptr[s];
    const int f = (int)(d.sn_rowptr[s + 1] - rb);
    const T* __restrict__ L = F + d.L_off[s];
    const int* __restrict__ rows = d.sn_rows + rb;
    const int64_t N = d.N;
    for (int q = 0; q < nrhs; ++q)
        for (int i = tid; i < f; i += 256) xs[i + q * fcap] = i < p ? Y2[first + i + q * N] : Y2[rows[i] + q * N];
    __syncthreads();
    for (int cb = ((p - 1) / kPanel) * kPanel; cb >= 0; cb -= kPanel) {
        const int ws = min(kPanel, p - cb);
        const int below = cb + ws;
        // partial dot products: lane = column t of the block, wave q4 takes rows i = below + q4, +4, ...
        for (int q = 0; q < nrhs; ++q) {
            T acc = T(0);
            if (lane < ws)
                for (int i = below + q4; i < f; i += 4) acc += L[i + (int64_t)(cb + lane) * f] * xs[i + q * fcap];
            part[(q4 * 64 + lane) * nrhs + q] = acc;
        }
        __syncthreads();
        if (tid < ws)
            for (int q = 0; q < nrhs; ++q) {
                const T* pp = part + tid * nrhs + q;
                const T sub = (pp[0] + pp[64 * nrhs]) + (pp[128 * nrhs] + pp[192 * nrhs]);
                xs[cb + tid + q * fcap] = xs[cb + tid + q * fcap] / D[first + cb + tid] - sub;
            }
        __syncthreads();
        if (d.M_off[s] >= 0) {
            // v <- Z^T v: wave q4 takes rows 16 q4 .. 16 q4 + 15 of Z, lane = output index
            const T* __restrict__ Zb = Zbuf + d.M_off[s] + (int64_t)(cb / kPanel) * (kPanel * kPanel);
            T z[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) z[j] = Zb[lane * kPanel + 16 * q4 + j];   // Z[16 q4 + j][lane]
            for (int q = 0; q < nrhs; ++q) {
                T acc = T(0);
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int k = 16 * q4 + j;
                    acc += z[j] * (k < ws ? xs[cb + k + q * fcap] : T(0));
                }
                part[(q4 * 64 + lane) * nrhs + q] = acc;
            }
            __syncthreads();
            if (tid < ws)
                for (int q = 0; q < nrhs; ++q) {
                    const T* pp = part + tid * nrhs + q;
                    xs[cb + tid + q * fcap] = (pp[0] + pp[64 * nrhs]) + (pp[128 * nrhs] + pp[192 * nrhs]);
                }
            __syncthreads();
        } else if (tid < 64) {
            // unit upper (L^T) substitution on one wave, from the last row up
            T lcol[64];
#pragma unroll
            for (int k = 0; k < 64; ++k)
                lcol[k] = (lane < k && k < ws) ? L[(cb + k) + (int64_t)(cb + lane) * f] : T(0);
            for (int q = 0; q < nrhs; ++q) {
                T val = lane < ws ? xs[cb + lane + q * fcap] : T(0);
#pragma unroll
                for (int k = 63; k > 0; --k) val -= lcol[k] * bcast(val, k);
                if (lane < ws) xs[cb + lane + q * fcap] = val;
            }
        }
        __syncthreads();
    }
    for (int q = 0; q < nrhs; ++q)
        for (int t = tid; t < p; t += 256) Y2[first + t + q * N] = xs[t + q * fcap];
}

template <typename T>
__global__ __launch_bounds__(256) void k_persist_solve(DevPlan d, const int* __restrict__ order, int nsn,
                                                       const int* __restrict__ sys_nfronts, int fcap, int* ctr,
                                                       int* ticket, int* status, unsigned long long timeout,
                                                       unsigned long long* tstamp,
                                                       const T* __restrict__ F, const T* __restrict__ Zbuf,
                                                       const T* __restrict__ D, const T* __restrict__ Y,
                                                       T* __restrict__ Y2, T* __restrict__ U, int nrhs) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* ys = reinterpret_cast<T*>(smem_raw);                 // fcap x nrhs
    T* part = ys + (int64_t)fcap * nrhs;                    // 256 x nrhs
    T* Ld = part + 256 * nrhs;                              // 64 x 65 (unused scratch)
    __shared__ int s_t;
    int* fwd_kids = ctr;             // children whose forward is done
    int* fwd_done = ctr + nsn;       // forward done (read by the root's backward)
    int* bwd_done = ctr + 2 * nsn;   // backward done (read by the children's backward)
    int* sys_bwd = ctr + 3 * nsn;    // fronts of the system whose backward is done
    for (;;) {
        const int t = pers_ticket(ticket, &s_t);
        if (t >= 2 * nsn) break;
        if (t < nsn) {
            const int s = order[t];
            pers_wait(fwd_kids + s, d.child_ptr[s + 1] - d.child_ptr[s], status, timeout);
            front_forward<T>(d, s, fcap, F, Zbuf, Y, Y2, U, nrhs, ys, Ld, part);
            const int par = d.sn_parent[s];
            pers_signal(par >= 0 ? fwd_kids + par : fwd_done + s);
        } else {
            const int s = order[2 * nsn - 1 - t];
            const int par = d.sn_parent[s];
            pers_wait(par >= 0 ? bwd_done + par : fwd_done + s, 1, status, timeout);
            front_backward<T>(d, s, fcap, F, Zbuf, D, Y2, nrhs, ys, Ld, part);
            pers_signal(bwd_done + s);
            if (threadIdx.x == 0) {
                const int sys = d.sn_sys[s];
                if (atomicAdd(sys_bwd + sys, 1) + 1 == sys_nfronts[sys]) tstamp[1 + d.S + sys] = wall_clock64();
            }
        }
    }
}

// ---------------------------------------------------------------------------
// refinement
// ---------------------------------------------------------------------------
// s = a + b rounded, err = its exact rounding error (a + b = s + err, Knuth's
// two-sum; no reassociation: the build does not allow it).
__device__ __forceinline__ double two_sum(double a, double b, double& err) {
    const double s = a + b;
    const double bb = s - a;
    err = (a - (s - bb)) + (b - bb);
    return s;
}

// Block per chunk of rows (one system); eight lanes share a row.  R = B - K X
// and, per column, the chunk's kResWidth figures: max |r_i|, max |x_i|,
// max |b_i|, sum r_i^2, sum b_i^2, and max_i |r_i| / (|K| |x| + |b|)_i (the
// componentwise backward error; 0/0 counts as 0, r/0 as infinite).  Each row
// sum is compensated (products split with fma, sums with two-sum: the Dot2
// scheme of Ogita, Rump and Oishi, 2005), so r_i is accurate to about one
// rounding of itself rather than of |K||x|_i.

__global__ __launch_bounds__(256) void k_residual(DevPlan d, const double* __restrict__ K,
                                                  const double* __restrict__ B, int64_t ldb,
                                                  const double* __restrict__ X, int64_t ldx, double* __restrict__ R,
                                                  int nrhs, const int* __restrict__ chunk_row0,
                                                  const int* __restrict__ chunk_rows, double* partial) {
    const int c = blockIdx.x;
    const int tid = threadIdx.x, sub = tid & 7, grp = tid >> 3;
    __shared__ double sm[kResWidth][256];
    for (int q = 0; q < nrhs; ++q) {
        const double* __restrict__ x = X + q * ldx;
        double v[kResWidth] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int r = grp; r < chunk_rows[c]; r += 32) {
            const int row = chunk_row0[c] + r;
            // compensated dot product (sum s + c carries about twice the
            // working precision): the residual's own rounding stays near one
            // unit of |b - Kx|, so refinement is not held at the rounding
            // floor of a plain FP64 row sum
            double acc = 0.0, cmp = 0.0, aacc = 0.0;
            for (int64_t e = d.Kp[row] + sub; e < d.Kp[row + 1]; e += 8) {
                const double k = K[e], xv = x[d.Kj[e]];
                const double pr = k * xv;
                const double pe = fma(k, xv, -pr);
                double t;
                acc = two_sum(acc, pr, t);
                cmp += t + pe;
                aacc += fabs(k) * fabs(xv);
            }
            for (int o = 4; o > 0; o >>= 1) {
                double t;
                acc = two_sum(acc, __shfl_xor(acc, o, 8), t);
                cmp += __shfl_xor(cmp, o, 8) + t;
                aacc += __shfl_xor(aacc, o, 8);
            }
            if (sub == 0) {
                const double b = B[row + q * ldb];
                double t;
                const double hi = two_sum(b, -acc, t);
                const double rr = hi + (t - cmp);
                R[row + q * d.N] = rr;
                const bool nan = rr != rr;
                const double den = aacc + fabs(b);
                const double cw = nan ? INFINITY : (den > 0.0 ? fabs(rr) / den : (rr != 0.0 ? INFINITY : 0.0));
                v[0] = nan ? INFINITY : fmax(v[0], fabs(rr));   // NaN residual -> infinite
                v[1] = fmax(v[1], fabs(x[row]));
                v[2] = fmax(v[2], fabs(b));
                v[3] += nan ? INFINITY : rr * rr;
                v[4] += b * b;
                v[5] = fmax(v[5], cw);
            }
        }
#pragma unroll
        for (int k = 0; k < kResWidth; ++k) sm[k][tid] = v[k];
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (tid < o) {
#pragma unroll
                for (int k = 0; k < kResWidth; ++k)
                    sm[k][tid] = (k == 3 || k == 4) ? sm[k][tid] + sm[k][tid + o] : fmax(sm[k][tid], sm[k][tid + o]);
            }
            __syncthreads();
        }
        if (tid < kResWidth) partial[((int64_t)c * nrhs + q) * kResWidth + tid] = sm[tid][0];
        __syncthreads();
    }
}

__global__ void k_axpy_cols(double* X, int64_t ldx, const double* DX, int64_t N, int nrhs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int q = 0; q < nrhs; ++q) X[i + q * ldx] += DX[i + q * N];
}

__global__ void k_copy_cols(double* dst, int64_t ldd, const double* src, int64_t lds, int64_t N, int nrhs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int q = 0; q < nrhs; ++q) dst[i + q * ldd] = src[i + q * lds];
}

__global__ void k_reduce_inertia(DevPlan d, int S) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * S) return;
    const int sys = t >> 2, k = t & 3;
    unsigned long long v = 0;
    for (int q = 0; q < kInertiaSlots; ++q) v += d.inertia_part[4 * ((int64_t)sys * kInertiaSlots + q) + k];
    d.inertia[t] = v;
}

__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ULL;
}
__global__ void k_zero_i32(int* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------
// adjoint (condensed form)
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// slack elimination (K1s) and the recovery of the rest of the Newton step
// ---------------------------------------------------------------------------
// Every row r of J carries Sigma_s[r] >= 0 (its slack's barrier term) or
// +inf (an equality row: Omega = 1, no slack); rho_r = rho-hat of the row's
// system.  Sec. 3.3, Proposition "Condensed KKT system" and its proof.

// Omega_rr = Sigma_s / (rho + Sigma_s); a negative or NaN Sigma_s sets
// kNonfiniteInput.
__global__ void k_k1s_omega(int64_t nrows, const double* __restrict__ Sigma_s, const int* __restrict__ Jrow_sys,
                            const double* __restrict__ sys_rho, double* __restrict__ omega, int* nonfinite) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const double S = Sigma_s[r];
    if (!(S >= 0.0)) {
        atomicOr(nonfinite, kNonfiniteInput);
        omega[r] = 0.0;
        return;
    }
    omega[r] = isinf(S) ? 1.0 : S / (sys_rho[Jrow_sys[r]] + S);
}

// b = r_t + rho J_I^T (Sigma_s + rho I)^-1 r_s: one thread per variable i,
// over the rows of column i of J in increasing order (J^T in CSC: Jt_ptr,
// Jt_row, Jt_k = index of the entry in J's values).
__global__ void k_k1s_rhs(int64_t n, const int64_t* __restrict__ Jt_ptr, const int* __restrict__ Jt_row,
                          const int* __restrict__ Jt_k, const double* __restrict__ J, const double* __restrict__ r_t,
                          const double* __restrict__ r_s, const double* __restrict__ Sigma_s,
                          const int* __restrict__ Jrow_sys, const double* __restrict__ sys_rho,
                          const int* __restrict__ row_sys, double* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int64_t q = Jt_ptr[i]; q < Jt_ptr[i + 1]; ++q) {
        const int r = Jt_row[q];
        const double S = Sigma_s[r];
        if (isinf(S)) continue;
        acc += J[Jt_k[q]] * (r_s[r] / (S + sys_rho[Jrow_sys[r]]));
    }
    b[i] = r_t[i] + sys_rho[row_sys[i]] * acc;
}

// Delta s_r = (rho (J dt)_r + r_s,r) / (Sigma_s,r + rho) on inequality rows, 0
// on equality rows.
__global__ void k_k1s_ds(int64_t nrows, const int64_t* __restrict__ Jp, const int* __restrict__ Jj,
                         const double* __restrict__ J, const double* __restrict__ dt, const double* __restrict__ r_s,
                         const double* __restrict__ Sigma_s, const int* __restrict__ Jrow_sys,
                         const double* __restrict__ sys_rho, double* __restrict__ ds) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const double S = Sigma_s[r];
    if (isinf(S)) {
        ds[r] = 0.0;
        return;
    }
    double a = 0.0;
    for (int64_t k = Jp[r]; k < Jp[r + 1]; ++k) a += J[k] * dt[Jj[k]];
    const double rho = sys_rho[Jrow_sys[r]];
    ds[r] = (rho * a + r_s[r]) / (S + rho);
}

// Delta y = -rho (J dx + c) + y_k - y (Sec. 3.3, eq. K1-elimination).
__global__ void k_recover_dy(int64_t nrows, const int64_t* __restrict__ Jp, const int* __restrict__ Jj,
                             const double* __restrict__ J, const double* __restrict__ dx, const double* __restrict__ c,
                             const double* __restrict__ y_k, const double* __restrict__ y,
                             const int* __restrict__ Jrow_sys, const double* __restrict__ sys_rho,
                             double* __restrict__ dy) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    double a = 0.0;
    for (int64_t k = Jp[r]; k < Jp[r + 1]; ++k) a += J[k] * dx[Jj[k]];
    dy[r] = -sys_rho[Jrow_sys[r]] * (a + c[r]) + y_k[r] - y[r];
}

// Delta r = (Delta y - y_k + y) / rho - r (Sec. 3.2, eq. K2-elimination,
// theta = 1 / rho-hat).
__global__ void k_recover_dr(int64_t nrows, const double* __restrict__ dy, const double* __restrict__ y_k,
                             const double* __restrict__ y, const double* __restrict__ r,
                             const int* __restrict__ Jrow_sys, const double* __restrict__ sys_rho,
                             double* __restrict__ dr) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nrows) return;
    dr[q] = (1.0 / sys_rho[Jrow_sys[q]]) * (dy[q] - y_k[q] + y[q]) - r[q];
}

// Delta z_l = -(Z_l dx - mu) / (x - l) - z_l, Delta z_u = (Z_u dx + mu) / (u - x)
// - z_u (Sec. 3.1, the blocks eliminated from eq. K3); an infinite bound
// makes the quotient 0.
__global__ void k_recover_dz(int64_t n, const double* __restrict__ x, const double* __restrict__ l,
                             const double* __restrict__ u, const double* __restrict__ z_l,
                             const double* __restrict__ z_u, const double* __restrict__ dx, double mu,
                             double* __restrict__ dz_l, double* __restrict__ dz_u) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dz_l[i] = -(z_l[i] * dx[i] - mu) / (x[i] - l[i]) - z_l[i];
    dz_u[i] = (z_u[i] * dx[i] + mu) / (u[i] - x[i]) - z_u[i];
}

// out = in + delta (the primal regularization of eq. K2 applied to Sigma).
__global__ void k_add_scalar(int64_t n, const double* __restrict__ in, double delta, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i] + delta;
}

// Sigma = Z_l / (x - l) + Z_u / (u - x) (Sec. 3.1, below eq. K2unreg).
__global__ void k_barrier_sigma(int64_t n, const double* __restrict__ x, const double* __restrict__ l,
                                const double* __restrict__ u, const double* __restrict__ z_l,
                                const double* __restrict__ z_u, double* __restrict__ sigma) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    sigma[i] = z_l[i] / (x[i] - l[i]) + z_u[i] / (u[i] - x[i]);
}

__global__ void k_jmul(int64_t nrows, const int64_t* __restrict__ Jp, const int* __restrict__ Jj,
                       const double* __restrict__ Jv, const double* __restrict__ X, const double* __restrict__ Lam,
                       int64_t ld, int nrhs, double* JX, double* JL) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    for (int q = 0; q < nrhs; ++q) {
        double a = 0.0, b = 0.0;
        for (int64_t k = Jp[r]; k < Jp[r + 1]; ++k) {
            a += Jv[k] * X[Jj[k] + q * ld];
            b += Jv[k] * Lam[Jj[k] + q * ld];
        }
        JX[r + q * nrows] = a;
        JL[r + q * nrows] = b;
    }
}

__global__ void k_grad_W(int64_t nnzW, const int* __restrict__ Wr, const int* __restrict__ Wc,
                         const double* __restrict__ X, const double* __restrict__ Lam, int64_t ld, int nrhs,
                         double* gW) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnzW) return;
    const int i = Wr[e], j = Wc[e];
    double g = 0.0;
    for (int q = 0; q < nrhs; ++q) {
        g -= Lam[i + q * ld] * X[j + q * ld];
        if (i != j) g -= Lam[j + q * ld] * X[i + q * ld];
    }
    gW[e] = g;
}

__global__ void k_grad_S(int64_t N, const double* __restrict__ X, const double* __restrict__ Lam, int64_t ld,
                         int nrhs, double* gS) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double g = 0.0;
    for (int q = 0; q < nrhs; ++q) g -= Lam[i + q * ld] * X[i + q * ld];
    gS[i] = g;
}

__global__ void k_grad_J(int64_t nrows, const int64_t* __restrict__ Jp, const int* __restrict__ Jj,
                         const int* __restrict__ Jrow_sys, const double* __restrict__ sys_rho,
                         const double* __restrict__ X, const double* __restrict__ Lam, int64_t ld, int nrhs,
                         const double* __restrict__ JX, const double* __restrict__ JL, double* gJ) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const double rho = sys_rho[Jrow_sys[r]];
    for (int64_t k = Jp[r]; k < Jp[r + 1]; ++k) {
        const int i = Jj[k];
        double g = 0.0;
        for (int q = 0; q < nrhs; ++q)
            g += Lam[i + q * ld] * JX[r + q * nrows] + X[i + q * ld] * JL[r + q * nrows];
        gJ[k] = -rho * g;
    }
}

// One block per system: gRho[s] = -sum over the system's J rows and columns of JL * JX.
__global__ __launch_bounds__(256) void k_grad_rho(const int64_t* __restrict__ sys_jrow, int64_t nrows, int nrhs,
                                                  const double* __restrict__ JX, const double* __restrict__ JL,
                                                  double* gRho) {
    const int s = blockIdx.x, tid = threadIdx.x;
    double acc = 0.0;
    for (int q = 0; q < nrhs; ++q)
        for (int64_t r = sys_jrow[s] + tid; r < sys_jrow[s + 1]; r += 256) acc += JL[r + q * nrows] * JX[r + q * nrows];
    __shared__ double sm[256];
    sm[tid] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) sm[tid] += sm[tid + o];
        __syncthreads();
    }
    if (tid == 0) gRho[s] = -sm[0];
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {
thread_local LaunchTimer* tl_timer = nullptr;

template <typename X> struct same_t { using type = X; };

// Every launch goes through here: plain hipLaunchKernelGGL, or the extended
// launch with the installed timer's events.
template <typename... KArgs>
void launch(void (*k)(KArgs...), dim3 grid, dim3 block, uint32_t lds, hipStream_t st,
            typename same_t<KArgs>::type... args) {
    hipEvent_t e0, e1;
    if (tl_timer && tl_timer->take(&e0, &e1))
        hipExtLaunchKernelGGL(k, grid, block, lds, st, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(k, grid, block, lds, st, args...);
}
}  // namespace

LaunchTimer* set_launch_timer(LaunchTimer* t) {
    LaunchTimer* old = tl_timer;
    tl_timer = t;
    return old;
}

void launch_assemble(const DevPlan& d, int64_t nnzF, const double* W, const double* Sigma, const double* J,
                     const double* sys_rho, const double* omega, double* K, hipStream_t st) {
    if (nnzF <= 0) return;
    launch(k_assemble, dim3(blocks_for(nnzF, 256)), dim3(256), 0, st, d, nnzF, W, Sigma, J, sys_rho, omega, K);
}

void launch_k1s_omega(int64_t nrows, const double* Sigma_s, const int* Jrow_sys, const double* sys_rho, double* omega,
                      int* nonfinite, hipStream_t st) {
    if (nrows <= 0) return;
    launch(k_k1s_omega, dim3(blocks_for(nrows, 256)), dim3(256), 0, st, nrows, Sigma_s, Jrow_sys, sys_rho, omega,
           nonfinite);
}

void launch_k1s_rhs(int64_t n, const int64_t* Jt_ptr, const int* Jt_row, const int* Jt_k, const double* J,
                    const double* r_t, const double* r_s, const double* Sigma_s, const int* Jrow_sys,
                    const double* sys_rho, const int* row_sys, double* b, hipStream_t st) {
    if (n <= 0) return;
    launch(k_k1s_rhs, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, Jt_ptr, Jt_row, Jt_k, J, r_t, r_s, Sigma_s,
           Jrow_sys, sys_rho, row_sys, b);
}

void launch_k1s_ds(int64_t nrows, const int64_t* Jp, const int* Jj, const double* J, const double* dt,
                   const double* r_s, const double* Sigma_s, const int* Jrow_sys, const double* sys_rho, double* ds,
                   hipStream_t st) {
    if (nrows <= 0) return;
    launch(k_k1s_ds, dim3(blocks_for(nrows, 256)), dim3(256), 0, st, nrows, Jp, Jj, J, dt, r_s, Sigma_s, Jrow_sys,
           sys_rho, ds);
}

void launch_recover_dy(int64_t nrows, const int64_t* Jp, const int* Jj, const double* J, const double* dx,
                       const double* c, const double* y_k, const double* y, const int* Jrow_sys, const double* sys_rho,
                       double* dy, hipStream_t st) {
    if (nrows <= 0) return;
    launch(k_recover_dy, dim3(blocks_for(nrows, 256)), dim3(256), 0, st, nrows, Jp, Jj, J, dx, c, y_k, y, Jrow_sys,
           sys_rho, dy);
}

void launch_recover_dr(int64_t nrows, const double* dy, const double* y_k, const double* y, const double* r,
                       const int* Jrow_sys, const double* sys_rho, double* dr, hipStream_t st) {
    if (nrows <= 0) return;
    launch(k_recover_dr, dim3(blocks_for(nrows, 256)), dim3(256), 0, st, nrows, dy, y_k, y, r, Jrow_sys, sys_rho, dr);
}

void launch_recover_dz(int64_t n, const double* x, const double* l, const double* u, const double* z_l,
                       const double* z_u, const double* dx, double mu, double* dz_l, double* dz_u, hipStream_t st) {
    if (n <= 0) return;
    launch(k_recover_dz, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, x, l, u, z_l, z_u, dx, mu, dz_l, dz_u);
}

void launch_add_scalar(int64_t n, const double* in, double delta, double* out, hipStream_t st) {
    if (n <= 0) return;
    launch(k_add_scalar, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, in, delta, out);
}

void launch_barrier_sigma(int64_t n, const double* x, const double* l, const double* u, const double* z_l,
                          const double* z_u, double* sigma, hipStream_t st) {
    if (n <= 0) return;
    launch(k_barrier_sigma, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, x, l, u, z_l, z_u, sigma);
}

void launch_chunk_norms(const DevPlan& d, const double* K, const int* chunk_row0, const int* chunk_rows, int nchunks,
                        double* partial, hipStream_t st) {
    launch(k_chunk_norms, dim3(nchunks), dim3(256), 0, st, d, K, chunk_row0, chunk_rows, partial);
}

void launch_reduce(const int* sys_chunk_ptr, int S, int width, int period, unsigned int sum_mask,
                   const double* partial, double* out, hipStream_t st) {
    launch(k_reduce_partials, dim3(S, width), dim3(256), 0, st, sys_chunk_ptr, width, period, sum_mask, partial,
           out);
}

void launch_thresholds(int S, const double* norms3, double eps, int mode, const double* sys_rho, double* kmax,
                       double* kinf, double* thr, int* nonfinite, hipStream_t st) {
    launch(k_thresholds, dim3(blocks_for(S, 64)), dim3(64), 0, st, S, norms3, eps, mode, sys_rho, kmax, kinf, thr,
           nonfinite);
}

template <typename T>
void launch_small_fronts(const DevPlan& d, const int* list, int count, int fmax, const double* K, T* F, T* D,
                         hipStream_t st) {
    if (count <= 0) return;
    if (fmax <= kTinyMax) {
        launch(k_tiny_fronts<T>, dim3((count + 3) / 4), dim3(256), 0, st, d, list, count, K, F, D);
        return;
    }
    const size_t lds = (size_t)fmax * fmax * sizeof(T);
    if (fmax <= 64)
        launch(k_small_fronts<T, false>, dim3(count), dim3(256), lds, st, d, list, K, F, D);
    else
        launch(k_small_fronts<T, true>, dim3(count), dim3(256), lds, st, d, list, K, F, D);
}

template <typename T>
void launch_large_asm(const DevPlan& d, int64_t first, int count, int fmax, const double* K, T* F, hipStream_t st) {
    if (count <= 0) return;
    const size_t lds = 4 * (size_t)fmax * sizeof(T);
    const dim3 grid((count + 3) / 4);
    if (lds <= kAsmLdsMax)
        launch(k_large_asm<T, true>, grid, dim3(256), lds, st, d, first, count, fmax, K, F);
    else
        launch(k_large_asm<T, false>, grid, dim3(256), 0, st, d, first, count, fmax, K, F);
}

template <typename T>
void launch_large_diag(const DevPlan& d, const int* tasks, int count, T* F, T* D, T* M, hipStream_t st) {
    if (count <= 0) return;
    launch(k_large_diag<T>, dim3(count), dim3(256), 0, st, d, tasks, F, D, M);
}

template <typename T>
void launch_large_panel(const DevPlan& d, const int* tasks, int count, T* F, const T* D, const T* M, hipStream_t st) {
    if (count <= 0) return;
    launch(k_large_panel<T>, dim3(count), dim3(256), 0, st, d, tasks, F, D, M);
}

template <typename T>
void launch_large_dstep(const DevPlan& d, const int* dtasks, int nd, const int* utasks, int nu, T* F, T* D, T* M,
                        hipStream_t st) {
    if (nd <= 0 && nu <= 0) return;
    const int nd8 = (nd + 7) & ~7;
    launch(k_large_dstep<T>, dim3(nd8 + nu), dim3(256), 0, st, d, dtasks, nd, utasks, nu, F, D, M);
}


template <typename T>
void launch_persist_factor(const DevPlan& d, const int* order, int ntask, const int64_t* asm_rng, int fcap,
                           int lds_elems, int grid, int* ctr, int* ticket, int* status, unsigned long long timeout,
                           unsigned long long* tstamp, const double* K, T* F, T* D, T* M, hipStream_t st) {
    if (ntask <= 0) return;
    launch(k_persist_factor<T>, dim3(grid < ntask ? grid : ntask), dim3(256), (uint32_t)lds_elems * sizeof(T), st, d,
           order, ntask, asm_rng, fcap, ctr, ticket, status, timeout, tstamp, K, F, D, M);
}

template <typename T>
void launch_persist_solve(const DevPlan& d, const int* order, int nsn, const int* sys_nfronts, int fcap, int grid,
                          int* ctr, int* ticket, int* status, unsigned long long timeout, unsigned long long* tstamp,
                          const T* F, const T* Z, const T* D, const T* Y, T* Y2, T* U, int nrhs, hipStream_t st) {
    if (nsn <= 0) return;
    const size_t lds = ((size_t)fcap * nrhs + 256 * (size_t)nrhs + 64 * 65) * sizeof(T);
    launch(k_persist_solve<T>, dim3(grid < 2 * nsn ? grid : 2 * nsn), dim3(256), (uint32_t)lds, st, d, order, nsn,
           sys_nfronts, fcap, ctr, ticket, status, timeout, tstamp, F, Z, D, Y, Y2, U, nrhs);
}

template <typename T>
void launch_permute_in(const DevPlan& d, const double* B, int64_t ldb, int nrhs, T* Y, hipStream_t st) {
    launch(k_permute_in<T>, dim3(blocks_for(d.N, 256)), dim3(256), 0, st, d, B, ldb, nrhs, Y);
}

template <typename T>
void launch_permute_out(const DevPlan& d, const T* Y, int nrhs, double* X, int64_t ldx, hipStream_t st) {
    launch(k_permute_out<T>, dim3(blocks_for(d.N, 256)), dim3(256), 0, st, d, Y, nrhs, X, ldx);
}

template <typename T>
void launch_fwd_S(const DevPlan& d, const int* fronts, int count, const T* F, const T* Y, T* Y2, T* U, int nrhs,
                  hipStream_t st) {
    if (count <= 0) return;
    const size_t lds = (size_t)4 * kSmallRows * nrhs * sizeof(T);
    launch(k_fwd_S<T>, dim3((count + 3) / 4), dim3(256), lds, st, d, fronts, count, F, Y, Y2, U, nrhs);
}

template <typename T>
void launch_bwd_S(const DevPlan& d, const int* fronts, int count, const T* F, const T* D, T* Y2, int nrhs,
                  hipStream_t st) {
    if (count <= 0) return;
    const size_t lds = (size_t)4 * kSmallRows * nrhs * sizeof(T);
    launch(k_bwd_S<T>, dim3((count + 3) / 4), dim3(256), lds, st, d, fronts, count, F, D, Y2, nrhs);
}

template <typename T>
void launch_fwd_P(const DevPlan& d, const int* tasks, int count, const int* segs, const T* F,
                  const T* Z, T* Y, T* Y2, T* U, int nrhs, hipStream_t st) {
    if (count <= 0) return;
    const size_t lds = (size_t)((2 * kPanel + kSolveRowsMax + 256) * nrhs + 64 * 65) * sizeof(T);
    if (nrhs == 1)
        launch(k_fwd_P<T, 1>, dim3(count), dim3(256), lds, st, d, tasks, segs, F, Z, Y, Y2, U, nrhs);
    else
        launch(k_fwd_P<T, kNrhsMax>, dim3(count), dim3(256), lds, st, d, tasks, segs, F, Z, Y, Y2, U, nrhs);
}

template <typename T>
void launch_bwd_P(const DevPlan& d, const int* tasks, int count, const T* F, const T* Z,
                  const T* D, T* Y2, T* pw, const T* pr, int nrhs, hipStream_t st) {
    if (count <= 0) return;
    const size_t lds = (size_t)((kPanel + kSolveRowsMax + 256) * nrhs + 64 * 65) * sizeof(T);
    if (nrhs == 1)
        launch(k_bwd_P<T, 1>, dim3(count), dim3(256), lds, st, d, tasks, F, Z, D, Y2, pw, pr, nrhs);
    else
        launch(k_bwd_P<T, kNrhsMax>, dim3(count), dim3(256), lds, st, d, tasks, F, Z, D, Y2, pw, pr, nrhs);
}

void launch_residual(const DevPlan& d, const double* K, const double* B, int64_t ldb, const double* X, int64_t ldx,
                     double* R, int nrhs, const int* chunk_row0, const int* chunk_rows, int nchunks, double* partial,
                     hipStream_t st) {
    launch(k_residual, dim3(nchunks), dim3(256), 0, st, d, K, B, ldb, X, ldx, R, nrhs, chunk_row0,
                       chunk_rows, partial);
}

void launch_axpy_cols(double* X, int64_t ldx, const double* DX, int64_t N, int nrhs, hipStream_t st) {
    launch(k_axpy_cols, dim3(blocks_for(N, 256)), dim3(256), 0, st, X, ldx, DX, N, nrhs);
}

void launch_copy_cols(double* dst, int64_t ldd, const double* src, int64_t lds, int64_t N, int nrhs, hipStream_t st) {
    launch(k_copy_cols, dim3(blocks_for(N, 256)), dim3(256), 0, st, dst, ldd, src, lds, N, nrhs);
}

void launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t st) {
    if (n > 0) launch(k_zero_u64, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n);
}

void launch_reduce_inertia(const DevPlan& d, int S, hipStream_t st) {
    launch(k_reduce_inertia, dim3(blocks_for(4 * (int64_t)S, 256)), dim3(256), 0, st, d, S);
}

void launch_zero_i32(int* p, int64_t n, hipStream_t st) {
    if (n > 0) launch(k_zero_i32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n);
}

void launch_adjoint(const DevPlan& d, int64_t nnzW, const int* W_row, const int* W_col, int64_t nJrows,
                    const int64_t* Jp, const int* Jj, const int* Jrow_sys, const double* Jval, const double* sys_rho,
                    const double* X, const double* Lam, int64_t ld, int nrhs, double* gW, double* gSigma,
                    double* gJ, double* gRho, double* JX, double* JL, const int64_t* sys_jrow, hipStream_t st) {
    if (nJrows > 0)
        launch(k_jmul, dim3(blocks_for(nJrows, 256)), dim3(256), 0, st, nJrows, Jp, Jj, Jval, X, Lam, ld,
                           nrhs, JX, JL);
    if (gW && nnzW > 0)
        launch(k_grad_W, dim3(blocks_for(nnzW, 256)), dim3(256), 0, st, nnzW, W_row, W_col, X, Lam, ld,
                           nrhs, gW);
    if (gSigma)
        launch(k_grad_S, dim3(blocks_for(d.N, 256)), dim3(256), 0, st, d.N, X, Lam, ld, nrhs, gSigma);
    if (gJ && nJrows > 0)
        launch(k_grad_J, dim3(blocks_for(nJrows, 256)), dim3(256), 0, st, nJrows, Jp, Jj, Jrow_sys,
                           sys_rho, X, Lam, ld, nrhs, JX, JL, gJ);
    if (gRho)
        launch(k_grad_rho, dim3(d.S), dim3(256), 0, st, sys_jrow, nJrows, nrhs, JX, JL, gRho);
}

int persist_factor_static_lds(int fp32) {
    hipFuncAttributes a{};
    const void* k = fp32 ? (const void*)k_persist_factor<float> : (const void*)k_persist_factor<double>;
    if (hipFuncGetAttributes(&a, k) != hipSuccess) return -1;
    return (int)a.sharedSizeBytes;
}

// Allow the LDS-resident kernels to request more than 64 KiB of dynamic LDS
// (gfx950 has 160 KiB per workgroup).
hipError_t configure_kernels(int max_dynamic_lds) {
    hipError_t e = hipSuccess, r;
    const void* fns[] = {(const void*)k_small_fronts<double, true>, (const void*)k_small_fronts<float, true>,
                         (const void*)k_small_fronts<double, false>, (const void*)k_small_fronts<float, false>,
                         (const void*)k_fwd_P<double, kNrhsMax>, (const void*)k_fwd_P<float, kNrhsMax>,
                         (const void*)k_bwd_P<double, kNrhsMax>, (const void*)k_bwd_P<float, kNrhsMax>,
                         (const void*)k_fwd_S<double>, (const void*)k_fwd_S<float>,
                         (const void*)k_large_asm<double, true>, (const void*)k_large_asm<float, true>,
                         (const void*)k_bwd_S<double>, (const void*)k_bwd_S<float>,
                         (const void*)k_persist_factor<double>, (const void*)k_persist_factor<float>,
                         (const void*)k_persist_solve<double>, (const void*)k_persist_solve<float>};
    for (const void* f : fns) {
        hipFuncAttributes at{};
        r = hipFuncGetAttributes(&at, f);
        if (r != hipSuccess) { e = r; continue; }
        const int dyn = max_dynamic_lds - (int)at.sharedSizeBytes;
        r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
        if (r != hipSuccess) e = r;
    }
    return e;
}

#define NCL_INSTANTIATE(T)                                                                                         \
    template void launch_small_fronts<T>(const DevPlan&, const int*, int, int, const double*, T*, T*, hipStream_t); \
    template void launch_large_asm<T>(const DevPlan&, int64_t, int, int, const double*, T*, hipStream_t);          \
    template void launch_large_diag<T>(const DevPlan&, const int*, int, T*, T*, T*, hipStream_t);                \
    template void launch_large_panel<T>(const DevPlan&, const int*, int, T*, const T*, const T*, hipStream_t);     \
    template void launch_large_dstep<T>(const DevPlan&, const int*, int, const int*, int, T*, T*, T*, hipStream_t); \
    template void launch_persist_factor<T>(const DevPlan&, const int*, int, const int64_t*, int, int, int, int*, int*,  \
                                           int*, unsigned long long, unsigned long long*, const double*, T*, T*, T*,  \
                                           hipStream_t);                                                             \
    template void launch_persist_solve<T>(const DevPlan&, const int*, int, const int*, int, int, int*, int*, int*,      \
                                          unsigned long long, unsigned long long*, const T*, const T*, const T*,       \
                                          const T*, T*, T*, int, hipStream_t);                                      \
    template void launch_permute_in<T>(const DevPlan&, const double*, int64_t, int, T*, hipStream_t);              \
    template void launch_permute_out<T>(const DevPlan&, const T*, int, double*, int64_t, hipStream_t);             \
    template void launch_fwd_S<T>(const DevPlan&, const int*, int, const T*, const T*, T*, T*, int, hipStream_t);  \
    template void launch_bwd_S<T>(const DevPlan&, const int*, int, const T*, const T*, T*, int, hipStream_t);     \
    template void launch_fwd_P<T>(const DevPlan&, const int*, int, const int*, const T*, const T*, T*, T*, T*,    \
                                  int, hipStream_t);                                                               \
    template void launch_bwd_P<T>(const DevPlan&, const int*, int, const T*, const T*, const T*, T*, T*,          \
                                  const T*, int, hipStream_t);

NCL_INSTANTIATE(double)
NCL_INSTANTIATE(float)

}  // namespace ncl
