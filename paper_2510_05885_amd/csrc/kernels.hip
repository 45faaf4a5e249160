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

// Static-pivot rule (Sec. 3.1): returns the pivot to use; flags perturbation.
template <typename T>
__device__ __forceinline__ T static_pivot(T d, double thr, int sign, bool& perturbed, bool& bad) {
    const double dd = to_d(d);
    bad = !isfinite(dd);
    perturbed = fabs(dd) < thr;
    if (perturbed) return (T)(sign > 0 ? thr : -thr);
    return d;
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
template <> struct Mfma<double> {
    typedef f64x4 acc_t;
    static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int r) { return 4 * r + lk; }
};
template <> struct Mfma<float> {
    typedef f32x4 acc_t;
    static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

inline unsigned int blocks_for(int64_t n, int bs) { return (unsigned int)((n + bs - 1) / bs); }

// ---------------------------------------------------------------------------
// assembly
// ---------------------------------------------------------------------------
__global__ void k_assemble(DevPlan d, int64_t nnzF, const double* __restrict__ W, const double* __restrict__ Sigma,
                           const double* __restrict__ J, const double* __restrict__ sys_rho,
                           double* __restrict__ K) {
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
        for (int64_t q = q0; q < q1; ++q) acc += J[d.prod_a[q]] * J[d.prod_b[q]];
        v += rho * acc;
    }
    if (fl & 2) v += -1.0 / rho;
    K[e] = v;
}

// Block per chunk of rows (one system): max |K_ij| and max row sum of |K|.
__global__ __launch_bounds__(256) void k_chunk_norms(DevPlan d, const double* __restrict__ K,
                                                     const int* __restrict__ chunk_row0,
                                                     const int* __restrict__ chunk_rows, double* partial) {
    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    double mx = 0.0, rs = 0.0;
    if (tid < chunk_rows[c]) {
        const int row = chunk_row0[c] + tid;
        bool bad = false;
        for (int64_t e = d.Kp[row]; e < d.Kp[row + 1]; ++e) {
            const double v = K[e];
            bad |= !isfinite(v);
            const double a = fabs(v);
            mx = fmax(mx, a);
            rs += a;
        }
        if (bad) { mx = INFINITY; rs = INFINITY; }
    }
    __shared__ double sm[2][256];
    sm[0][tid] = mx;
    sm[1][tid] = rs;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            sm[0][tid] = fmax(sm[0][tid], sm[0][tid + o]);
            sm[1][tid] = fmax(sm[1][tid], sm[1][tid + o]);
        }
        __syncthreads();
    }
    if (tid == 0) { partial[2 * c] = sm[0][0]; partial[2 * c + 1] = sm[1][0]; }
}

// Block per (system, column group): max over the system's chunks of `width` values.
__global__ __launch_bounds__(256) void k_reduce_partials(const int* __restrict__ sys_chunk_ptr, int width,
                                                         const double* __restrict__ partial, double* out) {
    const int s = blockIdx.x;
    const int k = blockIdx.y;
    const int tid = threadIdx.x;
    double mx = 0.0;
    for (int c = sys_chunk_ptr[s] + tid; c < sys_chunk_ptr[s + 1]; c += 256) mx = fmax(mx, partial[(int64_t)c * width + k]);
    __shared__ double sm[256];
    sm[tid] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) sm[tid] = fmax(sm[tid], sm[tid + o]);
        __syncthreads();
    }
    if (tid == 0) out[(int64_t)s * width + k] = sm[0];
}

__global__ void k_thresholds(int S, const double* norms2, double eps, double* kmax, double* kinf, double* thr,
                             int* nonfinite) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const double a = norms2[2 * s], b = norms2[2 * s + 1];
    kmax[s] = a;
    kinf[s] = b;
    thr[s] = eps * a;
    if (!isfinite(a) || !isfinite(b)) nonfinite[0] = 1;
}

// ---------------------------------------------------------------------------
// small fronts: one workgroup per front, front in LDS (column-major, ld = f)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_small_fronts(DevPlan d, const int* __restrict__ list,
                                                      const double* __restrict__ K, T* __restrict__ F,
                                                      T* __restrict__ D) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* A = reinterpret_cast<T*>(smem_raw);
    const int s = list[blockIdx.x];
    const int first = d.sn_first[s];
    const int p = d.sn_first[s + 1] - first;
    const int f = (int)(d.sn_rowptr[s + 1] - d.sn_rowptr[s]);
    const int c = f - p;
    const int tid = threadIdx.x;
    const int ti = tid & 63, tj = tid >> 6;

    for (int t = tid; t < f * f; t += 256) A[t] = T(0);
    __syncthreads();
    for (int64_t e = d.kent_ptr[s] + tid; e < d.kent_ptr[s + 1]; e += 256) A[d.kent_pos[e]] = (T)K[d.kent_csr[e]];
    __syncthreads();
    // extend-add: pull every child's contribution block, children in order
    for (int k = d.child_ptr[s]; k < d.child_ptr[s + 1]; ++k) {
        const int ch = d.child_list[k];
        const int fc = (int)(d.sn_rowptr[ch + 1] - d.sn_rowptr[ch]);
        const int cc = fc - (d.sn_first[ch + 1] - d.sn_first[ch]);
        const T* __restrict__ CB = F + d.CB_off[ch];
        const int ld = d.CB_ld[ch];
        const int* __restrict__ r = d.rel + d.rel_ptr[ch];
        for (int b = tj; b < cc; b += 4) {
            const int col = r[b] * f;
            for (int a = b + ti; a < cc; a += 64) A[r[a] + col] += CB[a + (int64_t)b * ld];
        }
        __syncthreads();
    }
    // partial LDL^T of the p pivot columns (right-looking, one barrier per pivot)
    const int sys = d.sn_sys[s];
    const double thr = d.sys_thr[sys];
    unsigned long long* in4 = d.inertia + 4 * sys;
    for (int k = 0; k < p; ++k) {
        bool pert, bad;
        const int sign = d.row_sign[d.perm[first + k]];
        const T dk = static_pivot(A[k + k * f], thr, sign, pert, bad);
        const T inv = T(1) / dk;
        for (int i0 = k + 1; i0 < f; i0 += 64) {
            const int i = i0 + ti;
            if (i < f) {
                const T lik = A[i + k * f] * inv;
                for (int j = k + 1 + tj; j <= i; j += 4) A[i + j * f] -= lik * A[j + k * f];
            }
        }
        if (tid == 0) {
            D[first + k] = dk;
            count_pivot(in4, to_d(dk), pert);
            if (bad) d.nonfinite[0] = 1;
        }
        __syncthreads();
        // column k is no longer read by the updates: scale it now
        for (int i = k + 1 + tid; i < f; i += 256) A[i + k * f] *= inv;
        if (tid == 0) A[k + k * f] = dk;
    }
    __syncthreads();
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

// ---------------------------------------------------------------------------
// large fronts (front stored in the factor buffer, ld = f)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_large_asm(DevPlan d, const int* __restrict__ tasks,
                                                   const double* __restrict__ K, T* __restrict__ F) {
    const int s = tasks[2 * blockIdx.x], j = tasks[2 * blockIdx.x + 1];
    const int p = d.sn_first[s + 1] - d.sn_first[s];
    const int f = (int)(d.sn_rowptr[s + 1] - d.sn_rowptr[s]);
    T* __restrict__ A = F + d.L_off[s];
    const int64_t col = (int64_t)j * f;
    const int tid = threadIdx.x;
    for (int i = j + tid; i < f; i += 256) A[i + col] = T(0);
    __syncthreads();
    if (j < p) {
        const int64_t* cp = d.kcol_ptr + d.kcol_base[s];
        for (int64_t e = cp[j] + tid; e < cp[j + 1]; e += 256) A[d.kent_pos[e]] = (T)K[d.kent_csr[e]];
    }
    __syncthreads();
    for (int k = d.child_ptr[s]; k < d.child_ptr[s + 1]; ++k) {
        const int ch = d.child_list[k];
        const int b = d.inv[d.inv_ptr[ch] + j];
        if (b >= 0) {
            const int fc = (int)(d.sn_rowptr[ch + 1] - d.sn_rowptr[ch]);
            const int cc = fc - (d.sn_first[ch + 1] - d.sn_first[ch]);
            const T* __restrict__ CB = F + d.CB_off[ch] + (int64_t)b * d.CB_ld[ch];
            const int* __restrict__ r = d.rel + d.rel_ptr[ch];
            for (int a = b + tid; a < cc; a += 256) A[r[a] + col] += CB[a];
        }
        __syncthreads();
    }
}

// One wave per (front, panel): LDL^T of the diagonal block with the static-pivot rule.
template <typename T>
__global__ __launch_bounds__(64) void k_large_diag(DevPlan d, const int* __restrict__ tasks, T* __restrict__ F,
                                                   T* __restrict__ D) {
    const int s = tasks[2 * blockIdx.x], k0 = tasks[2 * blockIdx.x + 1];
    const int first = d.sn_first[s];
    const int p = d.sn_first[s + 1] - first;
    const int f = (int)(d.sn_rowptr[s + 1] - d.sn_rowptr[s]);
    const int w = min(kPanel, p - k0);
    T* __restrict__ A = F + d.L_off[s];
    __shared__ T B[kPanel][kPanel + 1];
    const int lane = threadIdx.x;
    for (int j = 0; j < w; ++j)
        if (lane >= j && lane < w) B[lane][j] = A[(k0 + lane) + (int64_t)(k0 + j) * f];
    __syncthreads();
    const int sys = d.sn_sys[s];
    const double thr = d.sys_thr[sys];
    unsigned long long* in4 = d.inertia + 4 * sys;
    for (int k = 0; k < w; ++k) {
        bool pert, bad;
        const int sign = d.row_sign[d.perm[first + k0 + k]];
        const T dk = static_pivot(B[k][k], thr, sign, pert, bad);
        const T inv = T(1) / dk;
        if (lane > k && lane < w) {
            const T lik = B[lane][k] * inv;
            for (int j = k + 1; j <= lane; ++j) B[lane][j] -= lik * B[j][k];
        }
        __syncthreads();
        if (lane > k && lane < w) B[lane][k] *= inv;
        if (lane == 0) {
            B[k][k] = dk;
            D[first + k0 + k] = dk;
            count_pivot(in4, to_d(dk), pert);
            if (bad) d.nonfinite[0] = 1;
        }
        __syncthreads();
    }
    for (int j = 0; j < w; ++j)
        if (lane >= j && lane < w) A[(k0 + lane) + (int64_t)(k0 + j) * f] = B[lane][j];
}

// One wave per (front, panel, 64-row block below the diagonal block):
// L[i, k0:k1] = A[i, k0:k1] L_kk^-T D_k^-1, one row per lane.
template <typename T>
__global__ __launch_bounds__(64) void k_large_panel(DevPlan d, const int* __restrict__ tasks, T* __restrict__ F,
                                                    const T* __restrict__ D) {
    const int s = tasks[3 * blockIdx.x], k0 = tasks[3 * blockIdx.x + 1], r0 = tasks[3 * blockIdx.x + 2];
    const int first = d.sn_first[s];
    const int p = d.sn_first[s + 1] - first;
    const int f = (int)(d.sn_rowptr[s + 1] - d.sn_rowptr[s]);
    const int w = min(kPanel, p - k0);
    T* __restrict__ A = F + d.L_off[s];
    __shared__ T M[kPanel][kPanel + 1];   // M[t][u] = L_kk[t][u] * d_u (u < t)
    __shared__ T dinv[kPanel];
    const int lane = threadIdx.x;
    for (int u = 0; u < w; ++u)
        if (lane > u && lane < w) M[lane][u] = A[(k0 + lane) + (int64_t)(k0 + u) * f] * D[first + k0 + u];
    if (lane < w) dinv[lane] = T(1) / D[first + k0 + lane];
    __syncthreads();
    const int row = r0 + lane;
    if (row >= f) return;
    T x[kPanel];
#pragma unroll
    for (int t = 0; t < kPanel; ++t) x[t] = (t < w) ? A[row + (int64_t)(k0 + t) * f] : T(0);
#pragma unroll
    for (int t = 0; t < kPanel; ++t) {
        if (t < w) {
            T v = x[t];
#pragma unroll
            for (int u = 0; u < t; ++u) v -= M[t][u] * x[u];
            x[t] = v * dinv[t];
        }
    }
#pragma unroll
    for (int t = 0; t < kPanel; ++t)
        if (t < w) A[row + (int64_t)(k0 + t) * f] = x[t];
}

// Trailing update of one 64x64 lower tile: C -= L_I D_k L_J^T on MFMA.
// Four waves, each a 32x32 quadrant as 2x2 blocks of 16x16; K-depth = panel.
template <typename T>
__global__ __launch_bounds__(256) void k_large_update(DevPlan d, const int* __restrict__ tasks, T* __restrict__ F,
                                                      const T* __restrict__ D) {
    const int* tk = tasks + 4 * blockIdx.x;
    const int s = tk[0], k0 = tk[1], i0 = tk[2], j0 = tk[3];
    const int first = d.sn_first[s];
    const int p = d.sn_first[s + 1] - first;
    const int f = (int)(d.sn_rowptr[s + 1] - d.sn_rowptr[s]);
    const int w = min(kPanel, p - k0);
    T* __restrict__ A = F + d.L_off[s];
    __shared__ T La[kTile][kPanel + 1];
    __shared__ T Lb[kTile][kPanel + 1];
    const int tid = threadIdx.x;
    for (int idx = tid; idx < kTile * kPanel; idx += 256) {
        const int r = idx & (kTile - 1), t = idx / kTile;
        T a = T(0), b = T(0);
        if (t < w) {
            const int64_t cofs = (int64_t)(k0 + t) * f;
            if (i0 + r < f) a = A[(i0 + r) + cofs];
            if (j0 + r < f) b = A[(j0 + r) + cofs] * D[first + k0 + t];
        }
        La[r][t] = a;
        Lb[r][t] = b;
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
    typedef typename Mfma<T>::acc_t acc_t;
    acc_t acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < kPanel; kk += 4) {
        T a0 = La[wr + lr][kk + lk], a1 = La[wr + 16 + lr][kk + lk];
        T b0 = Lb[wc + lr][kk + lk], b1 = Lb[wc + 16 + lr][kk + lk];
        acc[0][0] = Mfma<T>::run(a0, b0, acc[0][0]);
        acc[0][1] = Mfma<T>::run(a0, b1, acc[0][1]);
        acc[1][0] = Mfma<T>::run(a1, b0, acc[1][0]);
        acc[1][1] = Mfma<T>::run(a1, b1, acc[1][1]);
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = i0 + wr + bi * 16 + Mfma<T>::row(lk, r);
                const int gj = j0 + wc + bj * 16 + lr;
                if (gi < f && gj < f && gi >= gj) A[gi + (int64_t)gj * f] -= acc[bi][bj][r];
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

// Forward sweep of one level: y_p = L11^-1 (b_p + children), u = (children) - L21 y_p.
template <typename T>
__global__ __launch_bounds__(256) void k_forward(DevPlan d, const int* __restrict__ fronts, const T* __restrict__ F,
                                                 T* __restrict__ Y, T* __restrict__ U, int nrhs, int qc) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* v = reinterpret_cast<T*>(smem_raw);
    const int s = fronts[blockIdx.x];
    const int first = d.sn_first[s];
    const int p = d.sn_first[s + 1] - first;
    const int f = (int)(d.sn_rowptr[s + 1] - d.sn_rowptr[s]);
    const int c = f - p;
    const T* __restrict__ L = F + d.L_off[s];
    const int tid = threadIdx.x;
    const int64_t N = d.N;
    for (int q0 = 0; q0 < nrhs; q0 += qc) {
        const int nq = min(qc, nrhs - q0);
        for (int q = 0; q < nq; ++q)
            for (int i = tid; i < f; i += 256) v[i + q * f] = i < p ? Y[first + i + (q0 + q) * N] : T(0);
        __syncthreads();
        for (int k = d.child_ptr[s]; k < d.child_ptr[s + 1]; ++k) {
            const int ch = d.child_list[k];
            const int fc = (int)(d.sn_rowptr[ch + 1] - d.sn_rowptr[ch]);
            const int cc = fc - (d.sn_first[ch + 1] - d.sn_first[ch]);
            const T* __restrict__ Uc = U + d.U_off[ch];
            const int* __restrict__ r = d.rel + d.rel_ptr[ch];
            for (int q = 0; q < nq; ++q)
                for (int a = tid; a < cc; a += 256) v[r[a] + q * f] += Uc[a + (int64_t)(q0 + q) * cc];
            __syncthreads();
        }
        for (int kb = 0; kb < p; kb += 64) {
            const int w = min(64, p - kb);
            if (tid < 64) {
                for (int q = 0; q < nq; ++q) {
                    T val = tid < w ? v[kb + tid + q * f] : T(0);
                    for (int k = 0; k < w; ++k) {
                        const T yk = __shfl(val, k, 64);
                        if (tid > k && tid < w) val -= L[(kb + tid) + (int64_t)(kb + k) * f] * yk;
                    }
                    if (tid < w) v[kb + tid + q * f] = val;
                }
            }
            __syncthreads();
            for (int i = kb + w + tid; i < f; i += 256) {
                for (int q = 0; q < nq; ++q) {
                    T acc = T(0);
                    for (int k = 0; k < w; ++k) acc += L[i + (int64_t)(kb + k) * f] * v[kb + k + q * f];
                    v[i + q * f] -= acc;
                }
            }
            __syncthreads();
        }
        T* __restrict__ Us = U + d.U_off[s];
        for (int q = 0; q < nq; ++q)
            for (int i = tid; i < f; i += 256) {
                if (i < p) Y[first + i + (q0 + q) * N] = v[i + q * f];
                else Us[(i - p) + (int64_t)(q0 + q) * c] = v[i + q * f];
            }
        __syncthreads();
    }
}

// Backward sweep of one level: x_p = L11^-T (D^-1 y_p - L21^T x_c), x_c read from ancestors.
template <typename T>
__global__ __launch_bounds__(256) void k_backward(DevPlan d, const int* __restrict__ fronts, const T* __restrict__ F,
                                                  const T* __restrict__ D, T* __restrict__ Y, int nrhs, int qc) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* Lt = reinterpret_cast<T*>(smem_raw);          // 64 x 65 diagonal block
    T* v = Lt + 64 * 65;
    const int s = fronts[blockIdx.x];
    const int first = d.sn_first[s];
    const int p = d.sn_first[s + 1] - first;
    const int64_t rb = d.sn_rowptr[s];
    const int f = (int)(d.sn_rowptr[s + 1] - rb);
    const T* __restrict__ L = F + d.L_off[s];
    const int* __restrict__ rows = d.sn_rows + rb;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t N = d.N;
    for (int q0 = 0; q0 < nrhs; q0 += qc) {
        const int nq = min(qc, nrhs - q0);
        for (int q = 0; q < nq; ++q)
            for (int i = tid; i < f; i += 256)
                v[i + q * f] = i < p ? Y[first + i + (q0 + q) * N] / D[first + i] : Y[rows[i] + (q0 + q) * N];
        __syncthreads();
        for (int kb = ((p - 1) / 64) * 64; kb >= 0; kb -= 64) {
            const int w = min(64, p - kb);
            const int below = kb + w;
            for (int t = wave; t < w; t += 4) {
                const T* __restrict__ col = L + (int64_t)(kb + t) * f;
                for (int q = 0; q < nq; ++q) {
                    T part = T(0);
                    for (int i = below + lane; i < f; i += 64) part += col[i] * v[i + q * f];
                    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
                    if (lane == 0) v[kb + t + q * f] -= part;
                }
            }
            for (int idx = tid; idx < 64 * w; idx += 256) {
                const int a = idx & 63, b = idx >> 6;
                if (a < w) Lt[a * 65 + b] = L[(kb + a) + (int64_t)(kb + b) * f];
            }
            __syncthreads();
            if (tid < 64) {
                for (int q = 0; q < nq; ++q) {
                    T val = tid < w ? v[kb + tid + q * f] : T(0);
                    for (int k = w - 1; k > 0; --k) {
                        const T xk = __shfl(val, k, 64);
                        if (tid < k) val -= Lt[k * 65 + tid] * xk;
                    }
                    if (tid < w) v[kb + tid + q * f] = val;
                }
            }
            __syncthreads();
        }
        for (int q = 0; q < nq; ++q)
            for (int i = tid; i < p; i += 256) Y[first + i + (q0 + q) * N] = v[i + q * f];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// refinement
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_residual(DevPlan d, const double* __restrict__ K,
                                                  const double* __restrict__ B, int64_t ldb,
                                                  const double* __restrict__ X, int64_t ldx, double* __restrict__ R,
                                                  int nrhs, const int* __restrict__ chunk_row0,
                                                  const int* __restrict__ chunk_rows, double* partial) {
    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    const bool valid = tid < chunk_rows[c];
    const int row = chunk_row0[c] + tid;
    __shared__ double sm[3][256];
    for (int q = 0; q < nrhs; ++q) {
        double r = 0.0, xa = 0.0, ba = 0.0;
        if (valid) {
            const double* __restrict__ x = X + q * ldx;
            double acc = 0.0;
            for (int64_t e = d.Kp[row]; e < d.Kp[row + 1]; ++e) acc += K[e] * x[d.Kj[e]];
            const double b = B[row + q * ldb];
            r = b - acc;
            R[row + q * d.N] = r;
            xa = fabs(x[row]);
            ba = fabs(b);
        }
        sm[0][tid] = fabs(r);
        sm[1][tid] = xa;
        sm[2][tid] = ba;
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
            double* o = partial + ((int64_t)c * nrhs + q) * 3;
            o[0] = sm[0][0]; o[1] = sm[1][0]; o[2] = sm[2][0];
        }
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
void launch_assemble(const DevPlan& d, int64_t nnzF, const double* W, const double* Sigma, const double* J,
                     const double* sys_rho, double* K, hipStream_t st) {
    if (nnzF <= 0) return;
    hipLaunchKernelGGL(k_assemble, dim3(blocks_for(nnzF, 256)), dim3(256), 0, st, d, nnzF, W, Sigma, J, sys_rho, K);
}

void launch_chunk_norms(const DevPlan& d, const double* K, const int* chunk_row0, const int* chunk_rows, int nchunks,
                        double* partial, hipStream_t st) {
    hipLaunchKernelGGL(k_chunk_norms, dim3(nchunks), dim3(256), 0, st, d, K, chunk_row0, chunk_rows, partial);
}

void launch_reduce(const int* sys_chunk_ptr, int S, int width, const double* partial, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(S, width), dim3(256), 0, st, sys_chunk_ptr, width, partial, out);
}

void launch_thresholds(int S, const double* norms2, double eps, double* kmax, double* kinf, double* thr,
                       int* nonfinite, hipStream_t st) {
    hipLaunchKernelGGL(k_thresholds, dim3(blocks_for(S, 64)), dim3(64), 0, st, S, norms2, eps, kmax, kinf, thr,
                       nonfinite);
}

template <typename T>
void launch_small_fronts(const DevPlan& d, const int* list, int count, int fmax, const double* K, T* F, T* D,
                         hipStream_t st) {
    if (count <= 0) return;
    const size_t lds = (size_t)fmax * fmax * sizeof(T);
    hipLaunchKernelGGL(k_small_fronts<T>, dim3(count), dim3(256), lds, st, d, list, K, F, D);
}

template <typename T>
void launch_large_asm(const DevPlan& d, const int* tasks, int count, const double* K, T* F, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_large_asm<T>, dim3(count), dim3(256), 0, st, d, tasks, K, F);
}

template <typename T>
void launch_large_diag(const DevPlan& d, const int* tasks, int count, T* F, T* D, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_large_diag<T>, dim3(count), dim3(64), 0, st, d, tasks, F, D);
}

template <typename T>
void launch_large_panel(const DevPlan& d, const int* tasks, int count, T* F, const T* D, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_large_panel<T>, dim3(count), dim3(64), 0, st, d, tasks, F, D);
}

template <typename T>
void launch_large_update(const DevPlan& d, const int* tasks, int count, T* F, const T* D, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_large_update<T>, dim3(count), dim3(256), 0, st, d, tasks, F, D);
}

template <typename T>
void launch_permute_in(const DevPlan& d, const double* B, int64_t ldb, int nrhs, T* Y, hipStream_t st) {
    hipLaunchKernelGGL(k_permute_in<T>, dim3(blocks_for(d.N, 256)), dim3(256), 0, st, d, B, ldb, nrhs, Y);
}

template <typename T>
void launch_permute_out(const DevPlan& d, const T* Y, int nrhs, double* X, int64_t ldx, hipStream_t st) {
    hipLaunchKernelGGL(k_permute_out<T>, dim3(blocks_for(d.N, 256)), dim3(256), 0, st, d, Y, nrhs, X, ldx);
}

static int solve_chunk(int fmax, int nrhs, size_t elem, size_t budget) {
    int qc = (int)(budget / elem / (size_t)(fmax > 0 ? fmax : 1));
    if (qc > nrhs) qc = nrhs;
    return qc;
}

template <typename T>
void launch_forward(const DevPlan& d, const int* fronts, int count, int fmax, const T* F, T* Y, T* U, int nrhs,
                    hipStream_t st) {
    if (count <= 0) return;
    const int qc = solve_chunk(fmax, nrhs, sizeof(T), 64 * 1024);
    const size_t lds = (size_t)fmax * qc * sizeof(T);
    hipLaunchKernelGGL(k_forward<T>, dim3(count), dim3(256), lds, st, d, fronts, F, Y, U, nrhs, qc);
}

template <typename T>
void launch_backward(const DevPlan& d, const int* fronts, int count, int fmax, const T* F, const T* D, T* Y,
                     int nrhs, hipStream_t st) {
    if (count <= 0) return;
    const size_t diag = 64 * 65 * sizeof(T);
    const int qc = solve_chunk(fmax, nrhs, sizeof(T), 64 * 1024);
    const size_t lds = diag + (size_t)fmax * qc * sizeof(T);
    hipLaunchKernelGGL(k_backward<T>, dim3(count), dim3(256), lds, st, d, fronts, F, D, Y, nrhs, qc);
}

void launch_residual(const DevPlan& d, const double* K, const double* B, int64_t ldb, const double* X, int64_t ldx,
                     double* R, int nrhs, const int* chunk_row0, const int* chunk_rows, int nchunks, double* partial,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_residual, dim3(nchunks), dim3(256), 0, st, d, K, B, ldb, X, ldx, R, nrhs, chunk_row0,
                       chunk_rows, partial);
}

void launch_reduce_partials(const int* sys_chunk_ptr, int S, int width, const double* partial, double* out,
                            hipStream_t st) {
    launch_reduce(sys_chunk_ptr, S, width, partial, out, st);
}

void launch_axpy_cols(double* X, int64_t ldx, const double* DX, int64_t N, int nrhs, hipStream_t st) {
    hipLaunchKernelGGL(k_axpy_cols, dim3(blocks_for(N, 256)), dim3(256), 0, st, X, ldx, DX, N, nrhs);
}

void launch_copy_cols(double* dst, int64_t ldd, const double* src, int64_t lds, int64_t N, int nrhs, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_cols, dim3(blocks_for(N, 256)), dim3(256), 0, st, dst, ldd, src, lds, N, nrhs);
}

void launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_zero_u64, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n);
}

void launch_zero_i32(int* p, int64_t n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_zero_i32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n);
}

void launch_adjoint(const DevPlan& d, int64_t nnzW, const int* W_row, const int* W_col, int64_t nJrows,
                    const int64_t* Jp, const int* Jj, const int* Jrow_sys, const double* Jval, const double* sys_rho,
                    const double* X, const double* Lam, int64_t ld, int nrhs, double* gW, double* gSigma,
                    double* gJ, double* gRho, double* JX, double* JL, const int64_t* sys_jrow, hipStream_t st) {
    if (nJrows > 0)
        hipLaunchKernelGGL(k_jmul, dim3(blocks_for(nJrows, 256)), dim3(256), 0, st, nJrows, Jp, Jj, Jval, X, Lam, ld,
                           nrhs, JX, JL);
    if (gW && nnzW > 0)
        hipLaunchKernelGGL(k_grad_W, dim3(blocks_for(nnzW, 256)), dim3(256), 0, st, nnzW, W_row, W_col, X, Lam, ld,
                           nrhs, gW);
    if (gSigma)
        hipLaunchKernelGGL(k_grad_S, dim3(blocks_for(d.N, 256)), dim3(256), 0, st, d.N, X, Lam, ld, nrhs, gSigma);
    if (gJ && nJrows > 0)
        hipLaunchKernelGGL(k_grad_J, dim3(blocks_for(nJrows, 256)), dim3(256), 0, st, nJrows, Jp, Jj, Jrow_sys,
                           sys_rho, X, Lam, ld, nrhs, JX, JL, gJ);
    if (gRho)
        hipLaunchKernelGGL(k_grad_rho, dim3(d.S), dim3(256), 0, st, sys_jrow, nJrows, nrhs, JX, JL, gRho);
}

// Allow the LDS-resident kernels to request more than 64 KiB of dynamic LDS
// (gfx950 has 160 KiB per workgroup).
hipError_t configure_kernels(int max_dynamic_lds) {
    hipError_t e = hipSuccess, r;
    const void* fns[] = {(const void*)k_small_fronts<double>, (const void*)k_small_fronts<float>,
                         (const void*)k_forward<double>, (const void*)k_forward<float>,
                         (const void*)k_backward<double>, (const void*)k_backward<float>};
    for (const void* f : fns) {
        r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_dynamic_lds);
        if (r != hipSuccess) e = r;
    }
    return e;
}

#define NCL_INSTANTIATE(T)                                                                                         \
    template void launch_small_fronts<T>(const DevPlan&, const int*, int, int, const double*, T*, T*, hipStream_t); \
    template void launch_large_asm<T>(const DevPlan&, const int*, int, const double*, T*, hipStream_t);            \
    template void launch_large_diag<T>(const DevPlan&, const int*, int, T*, T*, hipStream_t);                      \
    template void launch_large_panel<T>(const DevPlan&, const int*, int, T*, const T*, hipStream_t);               \
    template void launch_large_update<T>(const DevPlan&, const int*, int, T*, const T*, hipStream_t);              \
    template void launch_permute_in<T>(const DevPlan&, const double*, int64_t, int, T*, hipStream_t);              \
    template void launch_permute_out<T>(const DevPlan&, const T*, int, double*, int64_t, hipStream_t);             \
    template void launch_forward<T>(const DevPlan&, const int*, int, int, const T*, T*, T*, int, hipStream_t);     \
    template void launch_backward<T>(const DevPlan&, const int*, int, int, const T*, const T*, T*, int, hipStream_t);

NCL_INSTANTIATE(double)
NCL_INSTANTIATE(float)

}  // namespace ncl
