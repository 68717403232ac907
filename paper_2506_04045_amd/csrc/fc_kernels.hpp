// fc_kernels.hpp -- gfx950 (MI355X) kernels of the fuzzy-clustering solver.
//
// Problem (P), section 2: minimise ||S - U U^T||_F^2 over row-stochastic
// U (n x c), i.e. the paper's X = U^T with columns on the unit simplex.
// One accelerated gradient-projection iteration (Alg. 4) is built here from
//   * k_spmm   : Z = S_eff U, the products X s_i of eq. (gradient_column),
//                plus the per-row terms <u_i, (S U)_i> of the loss (Alg. 3)
//   * k_fused  : extrapolation Y = (1+beta) Xbar_c - beta Xbar_p and, by
//                linearity of S, S Y from the stored products; the gradient
//                -4 (S Y - Y G_Y) with Y G_Y on MFMA; the step; the row-wise
//                simplex projection (Alg. 1 semantics, computed by Michelot's
//                finite pivoting); Gram matrices of the new iterate and of
//                the next extrapolated point on MFMA; line-search sums
//   * k_control: one workgroup that turns the reduced sums into the loss,
//                the acceptance test, the inertial update of Alg. 4 and the
//                stop tests, entirely on the device.
//
// Layout: every n x c matrix is stored row-major with a padded width CP (a
// power of two >= max(c, 4)); padded columns hold zeros.  Reductions across
// rows are done per workgroup in double and then combined in a fixed order,
// so results do not depend on scheduling.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "fc_host.hpp"

namespace fc {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T> struct Acc4;
template <> struct Acc4<float> { typedef floatx4 type; };
template <> struct Acc4<double> { typedef doublex4 type; };

// 16x16x4 matrix-core products, D = A B + C, operand layout for lane l:
// A[l % 16][l / 16], B[l / 16][l % 16].  The result registers differ between
// the two types: register q of lane l holds D[4 (l / 16) + q][l % 16] for
// FP32 and D[4 q + l / 16][l % 16] for FP64 (mfma_row gives the row).
__device__ __forceinline__ floatx4 mfma16x16x4(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mfma16x16x4(double a, double b, doublex4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename T> __device__ __forceinline__ int mfma_row(int g, int q) { return 4 * g + q; }
template <> __device__ __forceinline__ int mfma_row<double>(int g, int q) { return 4 * q + g; }

// Component of a row held in slot s by lane group g in the fused kernel.
// The layout is chosen so that the Y G product comes back from the matrix
// cores in the registers that hold y: slot s = 4a + q of lane group g is
// component 16a + mfma_row(g, q).
template <typename T> __device__ __forceinline__ int kslot(int s, int g) {
    return 16 * (s >> 2) + mfma_row<T>(g, s & 3);
}

template <typename T> __device__ __forceinline__ float to_f32(T v) { return (float)v; }
// A stored value in the accumulation type TA (double stays double).
template <typename TA, typename VS> __device__ __forceinline__ TA to_acc(VS v) {
    return (TA)to_f32(v);
}
template <> __device__ __forceinline__ double to_acc<double, double>(double v) { return v; }
template <> __device__ __forceinline__ float to_f32<__half>(__half v) { return __half2float(v); }
template <> __device__ __forceinline__ float to_f32<__hip_bfloat16>(__hip_bfloat16 v) {
    return __bfloat162float(v);
}

__device__ __forceinline__ double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ float shfl_xor_f(float v, int m) { return __shfl_xor(v, m, 64); }

// ---------------------------------------------------------------------------
// Device-resident solver state.  Written by k_control (and by the host only
// between launches); read by every kernel of an iteration.
// ---------------------------------------------------------------------------
enum { ROLE_C = 0, ROLE_P = 1, ROLE_N = 2 };
enum { ERR_NONE = 0, ERR_NONFINITE = 5, ERR_STEP = 6 };
enum { STOP_NONE = 0, STOP_MAXITER = 1, STOP_LOSS = 2, STOP_PGRAD = 3, STOP_ERROR = 4 };

struct DevState {
    int32_t iter;           // accepted iterations
    int32_t target;         // kernels work while iter < target
    int32_t active;         // 1 while iterating
    int32_t stop_reason;
    int32_t trials;         // trials launched and evaluated
    int32_t trial_in_iter;  // trial number within the current iteration (1-based)
    int32_t role[3];        // ring slots of Xbar_c (current), Xbar_p (previous), trial
    int32_t error;
    int32_t max_iter;
    int32_t sched_len;
    int32_t accelerate;
    int32_t backtrack;
    int32_t c;
    int32_t hist_cap;
    double L, tau;          // current trial: tau = 1/L
    double t;               // t_n of Alg. 4 (iteration n = iter + 1)
    double beta;            // Y_n = Xbar_c + beta (Xbar_c - Xbar_p)
    double beta_next;       // weight of the next extrapolation (for G of Y_{n+1})
    double f, f_prev;       // f(Xbar_iter), f(Xbar_{iter-1})
    double r1, r;           // first and latest gradient-mapping norms
    double s2;              // ||S_eff||_F^2
    double mu;              // mean removed from G_Y before the product Y G_Y
    double tol_loss, tol_pgrad, eta;
    double tau0;            // constant step
    double tr_y_last;       // diagnostics of the last trial
    double df_last, rhs_last;
    // deferred loss evaluation (fixed steps): the loss of an accepted iterate
    // is formed during the next trial, from the terms <x_i, (S X)_i> that the
    // fused kernel accumulates while it reads the iterate and its product
    int32_t defer;          // 1: deferred evaluation
    int32_t f_known;        // 1: f holds f(Xbar_iter)
    double gsq_c;           // ||Xbar_iter^T Xbar_iter||_F^2, saved at acceptance
};

// Partial-sum layout of the fused kernel: three CPM x CPM matrices
// (Gram of the trial point, Gram of the next extrapolated point, and the
// line-search cross sum (p + y)^T (p - y)) followed by FUSED_NSCAL scalars.
enum { FS_TRY = 0, FS_LIN = 1, FS_SQ = 2, FS_CORR = 3, FS_BAD = 4, FS_TRC = 5, FUSED_NSCAL = 8 };
template <int CPM> struct FusedLayout {
    static constexpr int MAT = CPM * CPM;
    static constexpr int NE = 3 * MAT + FUSED_NSCAL;
};

// ---------------------------------------------------------------------------
// One problem instance as the kernels see it: the similarity, the heavy-row
// plan of the sparse product, the iterate/product rings, the device state
// and the buffers of partial sums.  The kernels below are written as device
// functions of (instance, block index, block count); thin wrappers run them
// either for one instance (block index = blockIdx) or for a batch, where a
// persistent grid walks a table of (instance, block) pairs.  Each instance's
// blocks do the same work in both cases, so its results do not depend on
// what it is batched with.
// ---------------------------------------------------------------------------
struct Inst {
    const int64_t *row_ptr;
    const int32_t *col;
    const void *val;
    int64_t n;
    int32_t c;
    int32_t diag_unit;
    int64_t light_max, nmed, nchunks, nheavy;
    const int32_t *med_rows;
    const int32_t *chunk_row;
    const int64_t *chunk_beg;
    const int32_t *chunk_len;
    const int32_t *heavy_rows;
    const int32_t *heavy_chunk_ptr;
    void *chunk_sum;
    void *X[3];   // iterate ring (compute type), padded n x CP
    void *Z[3];   // products S X in the same slots
    void *Sh[3];  // bfloat16 shadows of X (mixed precision)
    DevState *st; // NULL: stateless use, ring slot 0
    double *GY64;
    void *GYs;
    double *part_fused;
    double *part_spmm;
    double *red_mats;
    int32_t g_fused, g_spmm, g_comb, g_red;
    int32_t defer;   // 1: products hold S_off X (no unit diagonal, no trace terms)
    int32_t pass_kind; // PASS_*: how the sparse product and controller treat the instance
    int64_t nt_from; // FP32 products gather rows >= nt_from non-temporally (0: none)
    const double *sched;
    double *hist_f, *hist_tau, *hist_r;
    int32_t *hist_trials;
};

// Inst::pass_kind.  PASS_SINGLE: the single-pass iteration (k_single), whose
// controller sees no loss per iteration; PASS_LONG: the copy of a single-pass
// instance that its sparse product pre-pass runs with -- medium and heavy
// rows only, light rows left to k_single.
enum { PASS_DEFAULT = 0, PASS_SINGLE = 1, PASS_LONG = 2 };

// One entry of a batch table: block `blk` of instance `inst`.
struct VBlk {
    int32_t inst;
    int32_t blk;
};

__device__ __forceinline__ int ring_slot(const Inst &I, int role) {
    return I.st ? I.st->role[role] : 0;
}
__device__ __forceinline__ bool inst_active(const Inst &I) { return !I.st || I.st->active; }

// ---------------------------------------------------------------------------
// Deterministic column reduction: out[e] = sum_p in[p * ld + e] for
// e < ne, p < np.  A workgroup owns EB consecutive entries; its 256 threads
// split the p range into 256/EB fixed chunks that are combined in order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void reduce_cols_body(const double *__restrict__ in, int64_t np,
                                                 int64_t ld, int64_t ne, double *__restrict__ out,
                                                 int eb, int64_t blk) {
    // eb entries per workgroup, 256 / eb fixed chunks of the np partial rows;
    // every thread keeps four interleaved sums so its loads overlap.  The
    // order of all additions is fixed, so the result is reproducible.
    __shared__ double sh[256];
    const int tid = threadIdx.x;
    const int el = tid % eb, chunk = tid / eb, nchunk = 256 / eb;
    const int64_t e = blk * eb + el;
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
    if (e < ne) {
        const int64_t per = (np + nchunk - 1) / nchunk;
        const int64_t p0 = chunk * per;
        const int64_t p1 = p0 + per < np ? p0 + per : np;
        int64_t p = p0;
        for (; p + 4 <= p1; p += 4)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                a4[j] += in[(p + j) * ld + e];
        for (int j = 0; p < p1; ++p, ++j)
            a4[j] += in[p * ld + e];
    }
    sh[tid] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
    __syncthreads();
    if (chunk == 0 && e < ne) {
        double s = sh[el];
        for (int k = 1; k < nchunk; ++k)
            s += sh[k * eb + el];
        out[e] = s;
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_reduce_cols(const double *__restrict__ in, int64_t np,
                                                     int64_t ld, int64_t ne,
                                                     double *__restrict__ out, int eb) {
    reduce_cols_body(in, np, ld, ne, out, eb, blockIdx.x);
}

// The fused kernel's partial sums of one instance: entries split in blocks of
// FUSED_RED_EB, each reduced over the instance's g_fused workgroup partials.
constexpr int FUSED_RED_EB = 16;
template <int CPM>
__device__ __forceinline__ void reduce_fused_body(const Inst &I, int64_t blk) {
    constexpr int NE = FusedLayout<CPM>::NE;
    reduce_cols_body(I.part_fused, I.g_fused, NE, NE, I.red_mats, FUSED_RED_EB, blk);
}
template <int CPM> __global__ __launch_bounds__(256) void k_reduce_fused_1(Inst I) {
    if (inst_active(I))
        reduce_fused_body<CPM>(I, blockIdx.x);
}
template <int CPM>
__global__ __launch_bounds__(256) void k_reduce_fused_b(const Inst *__restrict__ insts,
                                                        const VBlk *__restrict__ tab,
                                                        const int32_t *__restrict__ count) {
    for (int64_t vb = blockIdx.x; vb < *count; vb += gridDim.x) {
        __syncthreads();
        const VBlk t = tab[vb];
        const Inst &I = insts[t.inst];
        if (inst_active(I))
            reduce_fused_body<CPM>(I, t.blk);
    }
}

// ---------------------------------------------------------------------------
// Copies between user matrices (rows x c, leading dimension ld, any of
// f64/f32) and the padded internal layout (rows x CP).  A NULL source fills
// the constant 1/c start point.
// ---------------------------------------------------------------------------
template <typename Tin, typename Tout>
__global__ void k_pad_copy(const Tin *__restrict__ src, int64_t ld, Tout *__restrict__ dst,
                           int64_t rows, int c, int cp, const int32_t *__restrict__ rowmap) {
    const int64_t total = rows * cp;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / cp;
        const int k = (int)(idx % cp);
        const int64_t si = rowmap ? (int64_t)rowmap[i] : i;   // internal row i holds user row si
        Tout v = (Tout)0;
        if (k < c)
            v = src ? (Tout)src[si * ld + k] : (Tout)(1.0 / c);
        dst[idx] = v;
    }
}

template <typename Tin, typename Tout>
__global__ void k_unpad_copy(const Tin *__restrict__ src, int cp, Tout *__restrict__ dst,
                             int64_t rows, int c, const int32_t *__restrict__ rowmap) {
    const int64_t total = rows * c;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / c;
        const int k = (int)(idx % c);
        const int64_t si = rowmap ? (int64_t)rowmap[i] : i;   // user row i is internal row si
        dst[idx] = (Tout)src[si * cp + k];
    }
}

template <typename T> __device__ __forceinline__ T from_f32(float v) { return (T)v; }
template <> __device__ __forceinline__ __half from_f32<__half>(float v) { return __float2half_rn(v); }
template <> __device__ __forceinline__ __hip_bfloat16 from_f32<__hip_bfloat16>(float v) {
    return __float2bfloat16(v);
}

// Elementwise conversion (rounding to nearest) between storage types.
template <typename Tin, typename Tout>
__global__ void k_convert(const Tin *__restrict__ src, Tout *__restrict__ dst, int64_t count) {
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < count;
         idx += (int64_t)gridDim.x * blockDim.x)
        dst[idx] = from_f32<Tout>(to_f32(src[idx]));
}

// ---------------------------------------------------------------------------
// Degree relabelling.  The solver may renumber the articles by descending
// number of stored nonzeros (ties by index): internal row i is user row
// perm[i], and user row j is internal row inv[j].  The objective and the
// iteration are equivariant under a simultaneous permutation of S's rows and
// columns and U's rows, so only locality changes: the rows of U that most
// nonzeros gather end up side by side.  Each row keeps the order of its
// nonzeros, so every per-row sum is formed from the same terms in the same
// order as without relabelling.
// ---------------------------------------------------------------------------
__global__ void k_degree_keys(const int64_t *__restrict__ row_ptr, int64_t n,
                              uint32_t *__restrict__ keys, int32_t *__restrict__ ids) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = row_ptr[i + 1] - row_ptr[i];
        keys[i] = ~(uint32_t)d;   // ascending keys = descending degree
        ids[i] = (int32_t)i;
    }
}

__global__ void k_perm_lengths(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ perm,
                               int64_t n, int32_t *__restrict__ inv, int64_t *__restrict__ len) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = perm[i];
        inv[r] = (int32_t)i;
        len[i] = row_ptr[r + 1] - row_ptr[r];
    }
}

// One wave per internal row: copy the user row's nonzeros, renumber their
// columns, convert their values.
template <typename VSin, typename VSout>
__global__ __launch_bounds__(256) void k_permute_csr(const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col,
                                                     const VSin *__restrict__ val,
                                                     const int32_t *__restrict__ perm,
                                                     const int32_t *__restrict__ inv,
                                                     const int64_t *__restrict__ new_row_ptr, int64_t n,
                                                     int32_t *__restrict__ new_col,
                                                     VSout *__restrict__ new_val) {
    const int lane = threadIdx.x & 63;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += (int64_t)gridDim.x * 4) {
        const int64_t src = row_ptr[perm[i]];
        const int64_t dst = new_row_ptr[i], len = new_row_ptr[i + 1] - dst;
        for (int64_t k = lane; k < len; k += 64) {
            new_col[dst + k] = inv[col[src + k]];
            new_val[dst + k] = from_f32<VSout>(to_f32(val[src + k]));
        }
    }
}
template <>
__global__ __launch_bounds__(256) void k_permute_csr<double, double>(
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col, const double *__restrict__ val,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ inv,
    const int64_t *__restrict__ new_row_ptr, int64_t n, int32_t *__restrict__ new_col,
    double *__restrict__ new_val) {
    const int lane = threadIdx.x & 63;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += (int64_t)gridDim.x * 4) {
        const int64_t src = row_ptr[perm[i]];
        const int64_t dst = new_row_ptr[i], len = new_row_ptr[i + 1] - dst;
        for (int64_t k = lane; k < len; k += 64) {
            new_col[dst + k] = inv[col[src + k]];
            new_val[dst + k] = val[src + k];
        }
    }
}

// ---------------------------------------------------------------------------
// Sum of squared stored values (||S||_F^2 without the unit diagonal).
// ---------------------------------------------------------------------------
template <typename VS>
__global__ __launch_bounds__(256) void k_sumsq(const VS *__restrict__ val, int64_t nnz,
                                               double *__restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * 256) {
        const double v = (double)to_f32(val[e]);
        acc += v * v;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = sh[0];
}
template <>
__global__ __launch_bounds__(256) void k_sumsq<double>(const double *__restrict__ val, int64_t nnz,
                                                       double *__restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * 256)
        acc += val[e] * val[e];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = sh[0];
}

// ---------------------------------------------------------------------------
// CSR validation of the stored entries, launched only after the host has
// checked row_ptr (starts at 0, never decreases, ends at nnz), so every row
// range below lies in [0, nnz).  Flags: 2 a column out of range, 4 a stored
// diagonal in unit-diagonal mode, 8 a row not sorted or with a duplicate
// column, 16 an entry (i, j, s) whose mirror (j, i) is missing or holds
// another value (binary search in row j; needs sorted rows).
// ---------------------------------------------------------------------------
template <typename VS>
__global__ void k_check_csr(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                            const VS *__restrict__ val, int64_t n, int64_t nnz, int diag_unit,
                            int check_sym, int32_t *__restrict__ flags) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = row_ptr[i], e = row_ptr[i + 1];
        for (int64_t k = b; k < e; ++k) {
            const int32_t j = col[k];
            if (j < 0 || j >= n) {
                atomicOr(&flags[0], 2);
                break;
            }
            if (diag_unit && j == i)
                atomicOr(&flags[0], 4);
            if (k > b && col[k - 1] >= j)
                atomicOr(&flags[0], 8);  // unsorted or duplicate: symmetry check unavailable
            if (check_sym) {
                // clamped to the stored range as well, so no read leaves it
                int64_t lo = row_ptr[j], hi = row_ptr[j + 1] - 1;
                lo = lo < 0 ? 0 : lo;
                hi = hi > nnz - 1 ? nnz - 1 : hi;
                bool found = false;
                while (lo <= hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    const int32_t cm = col[mid];
                    if (cm == (int32_t)i) {
                        found = to_acc<double>(val[mid]) == to_acc<double>(val[k]);
                        break;
                    }
                    if (cm < (int32_t)i)
                        lo = mid + 1;
                    else
                        hi = mid - 1;
                }
                if (!found)
                    atomicOr(&flags[0], 16);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Sparse product Z = S_eff U (one team of lanes per row).
//
// Each nonzero s_ij gathers the row u_j with GS lanes that each load 16
// bytes, so a team of TEAM lanes works on SLOTS nonzeros of the row at once
// and the slots are summed with cross-lane shuffles.  The epilogue adds u_i
// for the unit diagonal, writes z_i and accumulates <u_i, z_i> in double
// (the per-article products of Alg. 3); workgroups write one partial each.
// Rows are visited in a grid-stride loop over blocks of ROWS_PER_WG rows.
// ---------------------------------------------------------------------------
template <typename T> struct Vec16;
template <> struct Vec16<float> {
    typedef float4 type;
    static constexpr int N = 4;
};
template <> struct Vec16<double> {
    typedef double2 type;
    static constexpr int N = 2;
};
template <> struct Vec16<__hip_bfloat16> {
    typedef uint4 type;  // 8 bf16
    static constexpr int N = 8;
};

// A team of lanes working on one row: GS lanes per nonzero (16 bytes each),
// SLOTS nonzeros side by side.
template <typename TU, int CP, int WANT_SLOTS> struct TeamCfg {
    static constexpr int VEC = Vec16<TU>::N;
    static constexpr int GS = CP / VEC > 0 ? CP / VEC : 1;
    static constexpr int TEAM = GS * WANT_SLOTS > 64 ? 64 : GS * WANT_SLOTS;
    static constexpr int SLOTS = TEAM / GS;
    static constexpr int TEAMS = 256 / TEAM;     // teams per 256-thread workgroup
    static constexpr int LANE_ELEMS = CP / GS;  // elements of the row handled per lane
};
// Short rows (at most SPMM_LIGHT_MAX nonzeros, most rows of a sparse graph)
// get two-slot teams, so a wave works on several rows at once; longer rows
// get whole waves of eight slots.
template <typename TU, int CP> struct SpmmCfg {
    using Light = TeamCfg<TU, CP, 2>;
    using Wide = TeamCfg<TU, CP, 8>;
    static constexpr int ROWS_PER_WG = Light::TEAMS;
};

// Accumulator of LANE_ELEMS values in TA (float or double).
template <typename TA, int NE> struct Frag {
    TA v[NE];
};

template <typename TU, int NE> struct GatherLoad;
template <int NE> struct GatherLoad<float, NE> {
    __device__ __forceinline__ static void load(const float *p, float (&out)[NE]) {
        static_assert(NE % 4 == 0, "float rows load in float4 pieces");
#pragma unroll
        for (int q = 0; q < NE / 4; ++q) {
            const float4 t = reinterpret_cast<const float4 *>(p)[q];
            out[4 * q + 0] = t.x;
            out[4 * q + 1] = t.y;
            out[4 * q + 2] = t.z;
            out[4 * q + 3] = t.w;
        }
    }
};
template <int NE> struct GatherLoad<double, NE> {
    __device__ __forceinline__ static void load(const double *p, double (&out)[NE]) {
        static_assert(NE % 2 == 0, "double rows load in double2 pieces");
#pragma unroll
        for (int q = 0; q < NE / 2; ++q) {
            const double2 t = reinterpret_cast<const double2 *>(p)[q];
            out[2 * q + 0] = t.x;
            out[2 * q + 1] = t.y;
        }
    }
};
template <int NE> struct GatherLoad<__hip_bfloat16, NE> {
    __device__ __forceinline__ static void load(const __hip_bfloat16 *p, float (&out)[NE]) {
        static_assert(NE % 8 == 0, "bf16 rows load in 8-element pieces");
#pragma unroll
        for (int q = 0; q < NE / 8; ++q) {
            const uint4 t = reinterpret_cast<const uint4 *>(p)[q];
            const uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                out[8 * q + 2 * h + 0] = __uint_as_float(w[h] << 16);
                out[8 * q + 2 * h + 1] = __uint_as_float(w[h] & 0xffff0000u);
            }
        }
    }
};

// FP32 rows gathered with the non-temporal hint: rows that are rarely
// gathered again then stay out of the way of the ones that are (the hint
// also keeps them out of the memory-side Infinity Cache).
template <int NE> struct GatherLoadNT {
    __device__ __forceinline__ static void load(const float *p, float (&out)[NE]) {
        static_assert(NE % 4 == 0, "float rows load in float4 pieces");
        typedef float f4v __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int q = 0; q < NE / 4; ++q) {
            const f4v t = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(p) + q);
            out[4 * q + 0] = t.x;
            out[4 * q + 1] = t.y;
            out[4 * q + 2] = t.z;
            out[4 * q + 3] = t.w;
        }
    }
};

template <typename T> struct AccumOf { typedef T type; };
template <> struct AccumOf<__hip_bfloat16> { typedef float type; };

// Sum over the nonzeros e in [beg, end) of a row: a team of SLOTS slots takes
// SLOTS * DEPTH nonzeros per pass, and every slot issues its DEPTH gathers
// (predicated on e < end) before it consumes any of them, so a row shorter
// than one pass costs a single memory round trip.  For FP32 rows the column
// indices and values of the next pass are loaded while the gathers of the
// current one are in flight, which takes one dependent load off every pass
// (measured 28.2 -> 27.4 ms at n = 7e7, c = 32, at seven instead of eight
// waves per SIMD; the bfloat16 product measured slower that way, dropping
// from six waves to five, and it and the FP64 product keep the plain loop).
// Both loops add the same terms in the same order.  FP32 rows at index
// nt_from and beyond (when nt_from > 0) are gathered non-temporally.
template <typename TU, typename VS, int CP, int SLOTS, int DEPTH, typename TA, int NE>
__device__ __forceinline__ void team_row_sum(const int32_t *__restrict__ col,
                                             const VS *__restrict__ val,
                                             const TU *__restrict__ U, int64_t beg, int64_t end,
                                             int slot, int sub, TA (&acc)[NE], int64_t nt_from) {
    if constexpr (std::is_same<TU, float>::value) {
        int32_t jn[DEPTH];   // column of the next pass's nonzero u, -1 past the row's end
        TA sn[DEPTH];
#pragma unroll
        for (int u = 0; u < DEPTH; ++u) {
            const int64_t e = beg + slot + u * SLOTS;
            jn[u] = e < end ? col[e] : -1;
            sn[u] = e < end ? to_acc<TA>(val[e]) : (TA)0;
        }
        for (int64_t e0 = beg + slot; e0 < end; e0 += DEPTH * SLOTS) {
            TA s[DEPTH];
            TA g[DEPTH][NE];
#pragma unroll
            for (int u = 0; u < DEPTH; ++u) {
                s[u] = sn[u];
#pragma unroll
                for (int q = 0; q < NE; ++q)
                    g[u][q] = (TA)0;
                if (jn[u] >= 0) {
                    if (nt_from > 0 && jn[u] >= nt_from)
                        GatherLoadNT<NE>::load(U + (int64_t)jn[u] * CP + sub * NE, g[u]);
                    else
                        GatherLoad<TU, NE>::load(U + (int64_t)jn[u] * CP + sub * NE, g[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < DEPTH; ++u) {
                const int64_t e = e0 + DEPTH * SLOTS + u * SLOTS;
                jn[u] = e < end ? col[e] : -1;
                sn[u] = e < end ? to_acc<TA>(val[e]) : (TA)0;
            }
#pragma unroll
            for (int u = 0; u < DEPTH; ++u)
#pragma unroll
                for (int q = 0; q < NE; ++q)
                    acc[q] += s[u] * g[u][q];
        }
    } else {
        for (int64_t e0 = beg + slot; e0 < end; e0 += DEPTH * SLOTS) {
            TA s[DEPTH];
            TA g[DEPTH][NE];
#pragma unroll
            for (int u = 0; u < DEPTH; ++u) {
                const int64_t e = e0 + u * SLOTS;
                s[u] = (TA)0;
#pragma unroll
                for (int q = 0; q < NE; ++q)
                    g[u][q] = (TA)0;
                if (e < end) {
                    const int64_t j = col[e];
                    s[u] = to_acc<TA>(val[e]);
                    GatherLoad<TU, NE>::load(U + j * CP + sub * NE, g[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < DEPTH; ++u)
#pragma unroll
                for (int q = 0; q < NE; ++q)
                    acc[q] += s[u] * g[u][q];
        }
    }
}

// Add the accumulators of the SLOTS slots of a team (lanes with equal sub).
template <int GS, int TEAM, typename TA, int NE>
__device__ __forceinline__ void team_slot_sum(TA (&acc)[NE]) {
#pragma unroll
    for (int off = GS; off < TEAM; off <<= 1)
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            if constexpr (sizeof(TA) == 8)
                acc[q] += shfl_xor_d(acc[q], off);
            else
                acc[q] += shfl_xor_f(acc[q], off);
        }
}

// Row epilogue of a team whose slots are already summed: slot 0 adds u_i for
// the unit diagonal, writes z_i and returns <u_i, z_i> on its sub-0 lane.
// u_i and z_i are touched once per launch, so they go through the caches as
// non-temporal accesses and leave room for the gathered rows (measured 3 %
// faster at n = 7e7).
template <int GS, typename TA, typename TZ, typename TX, int CP, int NE>
__device__ __forceinline__ double row_epilogue(bool live, int slot, int sub, int64_t row,
                                               const TX *__restrict__ X, TZ *__restrict__ Z,
                                               int diag_unit, int plain, TA (&acc)[NE]) {
    double d = 0.0;
    if (live && slot == 0 && plain) {   // off-diagonal product only
#pragma unroll
        for (int q = 0; q < NE; ++q)
            __builtin_nontemporal_store((TZ)acc[q], &Z[row * CP + sub * NE + q]);
    } else if (live && slot == 0) {
        TA xi[NE];
#pragma unroll
        for (int q = 0; q < NE; ++q)
            xi[q] = (TA)__builtin_nontemporal_load(&X[row * CP + sub * NE + q]);
        if (diag_unit)
#pragma unroll
            for (int q = 0; q < NE; ++q)
                acc[q] += xi[q];
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            __builtin_nontemporal_store((TZ)acc[q], &Z[row * CP + sub * NE + q]);
            d += (double)acc[q] * (double)xi[q];
        }
    }
#pragma unroll
    for (int off = 1; off < GS; off <<= 1)
        d += shfl_xor_d(d, off);
    return (live && slot == 0 && sub == 0) ? d : 0.0;
}

// Z = S_eff U for one instance (S_off U, the stored entries only, with no
// terms <u_i, z_i>, when the loss evaluation is deferred).
//   light rows  (<= SPMM_LIGHT_MAX nonzeros): two-slot teams, in a
//               grid-stride loop over blocks of ROWS_PER_WG rows;
//   medium rows (listed in med_rows): one eight-slot team each;
//   heavy rows  (listed as chunks of their nonzeros): each chunk summed by an
//               eight-slot team into chunk_sum; k_combine adds a row's chunk
//               sums in chunk order.
// TU: type of the gathered rows (f64, f32 or bf16); TZ: output type;
// TX: type of the row u_i used by the epilogue (the master copy);
// VS: type of the stored values.
// DEPTH: gathers each slot keeps in flight.  A slot still adds its nonzeros
// in increasing order whatever DEPTH is, so DEPTH changes speed, never a sum.
template <typename TU, typename TZ, typename TX, typename VS, int CP, int DEPTH = 4>
__device__ __forceinline__ void spmm_body(const Inst &I, int role, int64_t blk, int64_t nblk) {
    using Lc = typename SpmmCfg<TU, CP>::Light;
    using Wc = typename SpmmCfg<TU, CP>::Wide;
    using TA = typename AccumOf<TU>::type;
    constexpr int NE = Lc::LANE_ELEMS;
    static_assert(Lc::GS == Wc::GS, "both team shapes split a row the same way");
    const int slot_role = ring_slot(I, role);
    const TX *__restrict__ X = (const TX *)I.X[slot_role];
    TZ *__restrict__ Z = (TZ *)I.Z[slot_role];
    const TU *__restrict__ U =
        sizeof(TU) == 2 ? (const TU *)I.Sh[slot_role] : (const TU *)I.X[slot_role];
    const int64_t *__restrict__ row_ptr = I.row_ptr;
    const int32_t *__restrict__ col = I.col;
    const VS *__restrict__ val = (const VS *)I.val;
    const int64_t n = I.n, light_max = I.light_max;
    const int diag_unit = I.diag_unit, plain = I.defer;
    const int tid = threadIdx.x;
    double trace_acc = 0.0;

    if (I.pass_kind != PASS_LONG) {   // light rows
        const int team = tid / Lc::TEAM, lt = tid % Lc::TEAM;
        const int slot = lt / Lc::GS, sub = lt % Lc::GS;
        const int64_t nblocks = (n + Lc::TEAMS - 1) / Lc::TEAMS;
        for (int64_t rb = blk; rb < nblocks; rb += nblk) {
            const int64_t row = rb * Lc::TEAMS + team;
            TA acc[NE];
#pragma unroll
            for (int q = 0; q < NE; ++q)
                acc[q] = (TA)0;
            bool live = row < n;
            if (live) {
                const int64_t beg = row_ptr[row], end = row_ptr[row + 1];
                if (end - beg > light_max)
                    live = false;
                else
                    team_row_sum<TU, VS, CP, Lc::SLOTS, DEPTH>(col, val, U, beg, end, slot, sub, acc,
                                                               I.nt_from);
            }
            team_slot_sum<Lc::GS, Lc::TEAM>(acc);
            trace_acc += row_epilogue<Lc::GS, TA, TZ, TX, CP>(live, slot, sub, row, X, Z, diag_unit,
                                                              plain, acc);
        }
    }
    {   // medium rows, then the chunks of heavy rows
        const int team = tid / Wc::TEAM, lt = tid % Wc::TEAM;
        const int slot = lt / Wc::GS, sub = lt % Wc::GS;
        const int32_t *__restrict__ med_rows = I.med_rows;
        for (int64_t m = blk * Wc::TEAMS + team; m < I.nmed; m += nblk * Wc::TEAMS) {
            const int64_t row = med_rows[m];
            TA acc[NE];
#pragma unroll
            for (int q = 0; q < NE; ++q)
                acc[q] = (TA)0;
            team_row_sum<TU, VS, CP, Wc::SLOTS, DEPTH>(col, val, U, row_ptr[row], row_ptr[row + 1],
                                                        slot, sub, acc, I.nt_from);
            team_slot_sum<Wc::GS, Wc::TEAM>(acc);
            trace_acc += row_epilogue<Wc::GS, TA, TZ, TX, CP>(true, slot, sub, row, X, Z, diag_unit,
                                                              plain, acc);
        }
        const int64_t *__restrict__ chunk_beg = I.chunk_beg;
        const int32_t *__restrict__ chunk_len = I.chunk_len;
        TA *__restrict__ chunk_sum = (TA *)I.chunk_sum;
        for (int64_t k = blk * Wc::TEAMS + team; k < I.nchunks; k += nblk * Wc::TEAMS) {
            TA acc[NE];
#pragma unroll
            for (int q = 0; q < NE; ++q)
                acc[q] = (TA)0;
            const int64_t beg = chunk_beg[k];
            team_row_sum<TU, VS, CP, Wc::SLOTS, DEPTH>(col, val, U, beg, beg + chunk_len[k], slot, sub,
                                                        acc, I.nt_from);
            team_slot_sum<Wc::GS, Wc::TEAM>(acc);
            if (slot == 0)
#pragma unroll
                for (int q = 0; q < NE; ++q)
                    chunk_sum[k * CP + sub * NE + q] = acc[q];
        }
    }
    if (plain)   // no loss terms: the products of a deferred instance write no partials
        return;
    __shared__ double sh[256];
    sh[tid] = trace_acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s)
            sh[tid] += sh[tid + s];
        __syncthreads();
    }
    if (tid == 0)
        I.part_spmm[blk] = sh[0];
    __syncthreads();
}

template <typename TU, typename TZ, typename TX, typename VS, int CP>
__global__ __launch_bounds__(256) void k_spmm_1(Inst I, int role) {
    if (inst_active(I))
        spmm_body<TU, TZ, TX, VS, CP>(I, role, blockIdx.x, gridDim.x);
}
template <typename TU, typename TZ, typename TX, typename VS, int CP, int DEPTH = 4>
__global__ __launch_bounds__(256) void k_spmm_b(const Inst *__restrict__ insts,
                                                const VBlk *__restrict__ tab,
                                                const int32_t *__restrict__ count, int role) {
    for (int64_t vb = blockIdx.x; vb < *count; vb += gridDim.x) {
        __syncthreads();
        const VBlk t = tab[vb];
        const Inst &I = insts[t.inst];
        if (inst_active(I))
            spmm_body<TU, TZ, TX, VS, CP, DEPTH>(I, role, t.blk, I.g_spmm);
    }
}

// Heavy rows: z_i = sum of the row's chunk sums in chunk order (+ u_i for the
// unit diagonal), and the terms <u_i, z_i>.  One thread per component of a
// row, 256/CP rows per workgroup step; partials go to trace_part[blockIdx].
template <typename TA, typename TZ, typename TX, int CP>
__device__ __forceinline__ void combine_body(const Inst &I, int role, int64_t blk, int64_t nblk) {
    constexpr int RPB = 256 / CP;
    const int slot_role = ring_slot(I, role);
    const TX *__restrict__ X = (const TX *)I.X[slot_role];
    TZ *__restrict__ Z = (TZ *)I.Z[slot_role];
    const int32_t *__restrict__ heavy_rows = I.heavy_rows;
    const int32_t *__restrict__ heavy_chunk_ptr = I.heavy_chunk_ptr;
    const TA *__restrict__ chunk_sum = (const TA *)I.chunk_sum;
    const int64_t nheavy = I.nheavy;
    const int diag_unit = I.diag_unit;
    const int tid = threadIdx.x, k = tid % CP, rl = tid / CP;
    __shared__ double sh[256];
    double trace_acc = 0.0;
    for (int64_t h0 = blk * RPB; h0 < nheavy; h0 += nblk * RPB) {
        const int64_t h = h0 + rl;
        if (h < nheavy) {
            const int64_t row = heavy_rows[h];
            TA acc = (TA)0;
            for (int32_t q = heavy_chunk_ptr[h]; q < heavy_chunk_ptr[h + 1]; ++q)
                acc += chunk_sum[(int64_t)q * CP + k];
            if (I.defer) {
                Z[row * CP + k] = (TZ)acc;
            } else {
                const TA xi = (TA)X[row * CP + k];
                if (diag_unit)
                    acc += xi;
                Z[row * CP + k] = (TZ)acc;
                trace_acc += (double)acc * (double)xi;
            }
        }
    }
    if (I.defer)
        return;
    sh[tid] = trace_acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s)
            sh[tid] += sh[tid + s];
        __syncthreads();
    }
    if (tid == 0)
        I.part_spmm[I.g_spmm + blk] = sh[0];
    __syncthreads();
}

template <typename TA, typename TZ, typename TX, int CP>
__global__ __launch_bounds__(256) void k_combine_1(Inst I, int role) {
    if (inst_active(I))
        combine_body<TA, TZ, TX, CP>(I, role, blockIdx.x, gridDim.x);
}
template <typename TA, typename TZ, typename TX, int CP>
__global__ __launch_bounds__(256) void k_combine_b(const Inst *__restrict__ insts,
                                                   const VBlk *__restrict__ tab,
                                                   const int32_t *__restrict__ count, int role) {
    for (int64_t vb = blockIdx.x; vb < *count; vb += gridDim.x) {
        __syncthreads();
        const VBlk t = tab[vb];
        const Inst &I = insts[t.inst];
        if (inst_active(I))
            combine_body<TA, TZ, TX, CP>(I, role, t.blk, I.g_comb);
    }
}

// ---------------------------------------------------------------------------
// Gram matrix G = U^T U on the matrix cores (the paper's share = X X^T).
// Each wave walks 16-row tiles; for every output block (a <= b) of 16 x 16
// it issues four 16x16x4 products over the tile's rows, then adds the tile
// result into double accumulators.  Wave partials (CPM x CPM, symmetric) go
// to part[(blockIdx * 4 + wave) * ld].
// ---------------------------------------------------------------------------
template <int M> struct SymBlocks {
    static constexpr int N = M * (M + 1) / 2;
    __device__ __forceinline__ static void ab(int k, int &a, int &b) {
        int r = k;
        a = 0;
        while (r >= M - a) {
            r -= M - a;
            ++a;
        }
        b = a + r;
    }
};

// Rows of X have stride ldx and cx valid components (the rest count as zero).
template <typename T, int CP>
__device__ __forceinline__ void gram_body(const T *__restrict__ X, int64_t ldx, int cx, int64_t n,
                                          double *__restrict__ part, int64_t ld) {
    constexpr int CPM = CP < 16 ? 16 : CP;
    constexpr int M = CPM / 16;
    constexpr int NB = SymBlocks<M>::N;
    using A4 = typename Acc4<T>::type;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    doublex4 acc64[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k)
        acc64[k] = doublex4{0, 0, 0, 0};
    const int64_t ntiles = (n + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
        // operand values: component 16a + r of rows 4t + g of the tile
        T xv[4][M];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t row = tile * 16 + 4 * t + g;
#pragma unroll
            for (int a = 0; a < M; ++a) {
                const int k = 16 * a + r;
                xv[t][a] = (row < n && k < CP && k < cx) ? X[row * ldx + k] : (T)0;
            }
        }
#pragma unroll
        for (int kb = 0; kb < NB; ++kb) {
            int a, b;
            SymBlocks<M>::ab(kb, a, b);
            A4 acc = A4{0, 0, 0, 0};
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc = mfma16x16x4(xv[t][a], xv[t][b], acc);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc64[kb][q] += (double)acc[q];
        }
    }
    double *out = part + ((int64_t)blockIdx.x * 4 + wave) * ld;
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
        int a, b;
        SymBlocks<M>::ab(kb, a, b);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = 16 * a + mfma_row<T>(g, q), j = 16 * b + r;
            out[i * CPM + j] = acc64[kb][q];
            if (a != b)
                out[j * CPM + i] = acc64[kb][q];
        }
    }
}

// Padded rows (stride CP, padding zero): the solver's iterates.
template <typename T, int CP>
__global__ __launch_bounds__(256) void k_gram(const T *__restrict__ X, int64_t n,
                                              double *__restrict__ part, int64_t ld) {
    gram_body<T, CP>(X, CP, CP, n, part, ld);
}

// A caller's matrix read in place: rows of stride ldx with cx components.
template <typename T, int CP>
__global__ __launch_bounds__(256) void k_gram_strided(const T *__restrict__ X, int64_t ldx, int cx,
                                                      int64_t n, double *__restrict__ part,
                                                      int64_t ld) {
    gram_body<T, CP>(X, ldx, cx, n, part, ld);
}

// out[i * c + j] = in[i * ld + j] for i, j < c (the c x c corner of a padded
// matrix, in place of a strided copy).
__global__ void k_corner_copy(const double *__restrict__ in, int ld, int c,
                              double *__restrict__ out) {
    for (int e = threadIdx.x; e < c * c; e += blockDim.x)
        out[e] = in[(e / c) * ld + e % c];
}

// ---------------------------------------------------------------------------
// Row-wise projection onto the unit simplex for rows spread over four lanes
// (lanes r, r+16, r+32, r+48 of a wave hold the components of one row).
// The threshold theta with sum_k max(v_k - theta, 0) = 1 is found by
// Michelot's finite pivoting: theta = (sum of active v - 1) / #active,
// drop every active component with v <= theta, repeat until nothing drops.
// It yields the same threshold as Alg. 1's sort-based search; the sums are
// carried in double.  The loop is wave-uniform and ends after at most
// NC * 4 passes.
// ---------------------------------------------------------------------------
template <typename T, int NC>
__device__ __forceinline__ double simplex_threshold(const T (&v)[NC], const bool (&valid)[NC]) {
    bool act[NC];
#pragma unroll
    for (int s = 0; s < NC; ++s)
        act[s] = valid[s];
    double theta = 0.0;
    for (int pass = 0; pass <= 4 * NC; ++pass) {
        double sum = 0.0;
        int cnt = 0;
#pragma unroll
        for (int s = 0; s < NC; ++s)
            if (act[s]) {
                sum += (double)v[s];
                ++cnt;
            }
        sum += shfl_xor_d(sum, 16);
        sum += shfl_xor_d(sum, 32);
        cnt += __shfl_xor(cnt, 16, 64);
        cnt += __shfl_xor(cnt, 32, 64);
        theta = (sum - 1.0) / (double)(cnt > 0 ? cnt : 1);
        bool changed = false;
#pragma unroll
        for (int s = 0; s < NC; ++s)
            if (act[s] && (double)v[s] <= theta) {
                act[s] = false;
                changed = true;
            }
        if (!__any(changed))
            break;
    }
    return theta;
}

// ---------------------------------------------------------------------------
// Fused iteration kernel.  Rows are processed in 16-row wave tiles, four
// waves (64 rows) per workgroup step, in a grid-stride loop.  Lane l of a
// wave owns row r = l % 16 of the tile and the components
//   k(s) = 16 (s / 4) + 4 (l / 16) + s % 4,   s = 0 .. 4M-1,
// which is exactly the layout in which the 16x16x4 product returns
// (Y G)^T, so Y G needs no data movement: with A = G (rows 16a..) and
// B = Y^T the contraction index is enumerated through the lanes' own slots.
//
// Per row: y = (1+beta) xc - beta xp, sy = (1+beta) zc - beta zp (S Y by
// linearity from the stored products), grad = -4 (sy - y (G_Y - mu 1 1^T)),
// v = y - tau grad, p = P_simplex(v), y' = (1+beta') p - beta' xc.
// The constant mu removed from G_Y changes every gradient row by a
// multiple of the ones vector, which the projection ignores; it is added
// back in the line-search sum.  The workgroup then stages p, y' (and y when
// backtracking) in LDS, writes p from there in contiguous pieces, and each
// wave accumulates some of the 16 x 16 blocks of the Gram matrices of p and
// y' (and of the line-search cross sum (p + y)^T (p - y)) on the matrix
// cores.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t nwt_of(int64_t n) { return (n + 63) / 64; }

// A lane's terms x_k (S_eff x)_k of the loss, from a row of the iterate and of
// its off-diagonal product (padded and missing components are zero): summed
// in the compute type over the lane's components (explicit FMAs, so every
// kernel that calls this forms the same value), then carried in double.
template <typename T, int NC>
__device__ __forceinline__ double trace_terms(const T (&x)[NC], const T (&z)[NC], int diag_unit) {
    T a = (T)0;
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        const T zd = diag_unit ? z[s] + x[s] : z[s];
        a = fma(x[s], zd, a);
    }
    return (double)a;
}

// The fused kernel's scalars of one workgroup: a tree over each wave, then the
// four waves added in order; scalar k goes to out[k], unused slots get zero.
template <int N>
__device__ __forceinline__ void fused_scalars_out(double (&vals)[N], double *__restrict__ out) {
    __shared__ double shs[4][FUSED_NSCAL];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            vals[k] += shfl_xor_d(vals[k], off);
    }
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < N; ++k)
            shs[wave][k] = vals[k];
    __syncthreads();
    if (tid < FUSED_NSCAL) {
        double sum = 0.0;
        if (tid < N)
            sum = ((shs[0][tid] + shs[1][tid]) + shs[2][tid]) + shs[3][tid];
        out[tid] = sum;
    }
    __syncthreads();
}

template <typename T, int CP, bool ACCEL, bool BT, bool SHADOW>
__device__ __forceinline__ void fused_body(const Inst &I, int64_t blk, int64_t nblk) {
    constexpr int CPM = CP < 16 ? 16 : CP;
    constexpr int M = CPM / 16;
    constexpr int NC = 4 * M;
    // LDS row stride: float rows are offset by half the banks between the four
    // row groups an MFMA operand read touches; double rows only need padding
    constexpr int STRIDE = sizeof(T) == 8 ? CPM + 4 : CPM + (CPM == 16 ? 32 : 16);
    // staged tiles: p, the next extrapolated point (ACCEL), y (BT; the
    // line-search operands p + y and p - y are formed from p and y as they
    // are read, which costs a tile of LDS less than staging both)
    constexpr int NMAT = 1 + (ACCEL ? 1 : 0) + (BT ? 1 : 0);
    constexpr int NSYM = SymBlocks<M>::N;
    constexpr int NBLK = NSYM + (ACCEL ? NSYM : 0) + (BT ? M * M : 0);
    constexpr int BPW = (NBLK + 3) / 4;  // Gram blocks per wave
    using A4 = typename Acc4<T>::type;
    using L = FusedLayout<CPM>;

    const DevState *__restrict__ st = I.st;
    T *const *Xring = (T *const *)I.X;
    T *const *Zring = (T *const *)I.Z;
    __hip_bfloat16 *const *shadow_ring = (__hip_bfloat16 *const *)I.Sh;
    const T *__restrict__ GYs = (const T *)I.GYs;
    const int64_t n = I.n;
    const int c = I.c;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    const T *__restrict__ Xc = Xring[st->role[ROLE_C]];
    const T *__restrict__ Xp = Xring[st->role[ROLE_P]];
    T *__restrict__ Xn = Xring[st->role[ROLE_N]];
    const T *__restrict__ Zc = Zring[st->role[ROLE_C]];
    const T *__restrict__ Zp = Zring[st->role[ROLE_P]];
    __hip_bfloat16 *shadow = SHADOW ? shadow_ring[st->role[ROLE_N]] : nullptr;
    const double beta = ACCEL ? st->beta : 0.0;
    const double beta_next = ACCEL ? st->beta_next : 0.0;
    const T tau = (T)st->tau;
    const T b1 = (T)(1.0 + beta), b0 = (T)beta;
    const T bn1 = (T)(1.0 + beta_next), bn0 = (T)beta_next;
    const bool use_prev = ACCEL && beta != 0.0;

    // A operands of Y G: G[16a + r][k(s)] for every block a and slot s.  FP32
    // keeps G_Y in LDS (row stride CPM + 1 spreads the 16 rows a read touches
    // over the banks) and reads the operands next to their use, which keeps
    // the kernel within 128 registers; FP64 holds them in registers.
    constexpr bool G_LDS = sizeof(T) == 4;
    constexpr int GSTR = CPM + 1;
    __shared__ T gsh[G_LDS ? CPM * GSTR : 1];
    T gA[G_LDS ? 1 : M][G_LDS ? 1 : NC];
    if constexpr (G_LDS) {
        for (int e = tid; e < CPM * CPM; e += 256)
            gsh[(e / CPM) * GSTR + e % CPM] = GYs[e];
        __syncthreads();
    } else {
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int s = 0; s < NC; ++s)
                gA[a][s] = GYs[(16 * a + r) * CPM + kslot<T>(s, g)];
    }

    __shared__ __attribute__((aligned(16))) T lds[NMAT][64 * STRIDE];

    double sc_try = 0.0, sc_lin = 0.0, sc_sq = 0.0, sc_corr = 0.0, sc_trc = 0.0;
    int32_t n_bad = 0;   // non-finite step values
    const int defer = I.defer, diag_unit = I.diag_unit;
    doublex4 acc64[BPW];
#pragma unroll
    for (int k = 0; k < BPW; ++k)
        acc64[k] = doublex4{0, 0, 0, 0};

    // The four row streams of one 64-row tile (loading the next tile ahead of
    // the arithmetic was measured slower: the extra registers cost occupancy).
    auto load_tile = [&](int64_t wt, T (&xc)[NC], T (&zc)[NC], T (&xp)[NC], T (&zp)[NC]) {
        const int64_t row = wt * 64 + wave * 16 + r;
        const bool live = wt < nwt_of(n) && row < n;
#pragma unroll
        for (int a = 0; a < M; ++a) {
            const int k0 = 16 * a + 4 * g;
            const bool ok = live && k0 < CP;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                xc[4 * a + q] = (T)0;
                zc[4 * a + q] = (T)0;
                xp[4 * a + q] = (T)0;
                zp[4 * a + q] = (T)0;
            }
            if (ok && sizeof(T) == 4) {   // four consecutive components
                T t4[4];
                GatherLoad<T, 4>::load(Xc + row * CP + k0, t4);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    xc[4 * a + q] = t4[q];
                GatherLoad<T, 4>::load(Zc + row * CP + k0, t4);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    zc[4 * a + q] = t4[q];
                if (use_prev) {
                    GatherLoad<T, 4>::load(Xp + row * CP + k0, t4);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        xp[4 * a + q] = t4[q];
                    GatherLoad<T, 4>::load(Zp + row * CP + k0, t4);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        zp[4 * a + q] = t4[q];
                }
            } else if (live && sizeof(T) == 8) {   // components 16a + 4q + g
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int k = kslot<T>(4 * a + q, g);
                    if (k < CP) {
                        xc[4 * a + q] = Xc[row * CP + k];
                        zc[4 * a + q] = Zc[row * CP + k];
                        if (use_prev) {
                            xp[4 * a + q] = Xp[row * CP + k];
                            zp[4 * a + q] = Zp[row * CP + k];
                        }
                    }
                }
            }
        }
    };
    const int64_t nwt = nwt_of(n);
    for (int64_t wt = blk; wt < nwt; wt += nblk) {
        const int64_t row = wt * 64 + wave * 16 + r;
        const bool live = row < n;
        T xc[NC], xp[NC], zc[NC], zp[NC];
        load_tile(wt, xc, zc, xp, zp);
        if (defer)   // the current iterate's terms <x_i, (S_eff X)_i> for its loss
            sc_trc += trace_terms<T, NC>(xc, zc, diag_unit);
        T y[NC], sy[NC];
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            y[s] = use_prev ? b1 * xc[s] - b0 * xp[s] : xc[s];
            sy[s] = use_prev ? b1 * zc[s] - b0 * zp[s] : zc[s];
        }
        if (defer && diag_unit)   // the stored products lack the unit diagonal
#pragma unroll
            for (int s = 0; s < NC; ++s)
                sy[s] += y[s];
        // Y (G_Y - mu 1 1^T) on the matrix cores, returned in the lane layout of y
        T yg[NC];
#pragma unroll
        for (int a = 0; a < M; ++a) {
            A4 acc = A4{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                T ga;
                if constexpr (G_LDS)
                    ga = gsh[(16 * a + r) * GSTR + kslot<T>(s, g)];
                else
                    ga = gA[a][s];
                acc = mfma16x16x4(ga, y[s], acc);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                yg[4 * a + q] = acc[q];
        }
        T grad[NC], v[NC];
        bool valid[NC];
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const int k = kslot<T>(s, g);
            valid[s] = live && k < c;
            grad[s] = (T)(-4) * (sy[s] - yg[s]);
            v[s] = y[s] - tau * grad[s];
        }
        const double theta = simplex_threshold<T, NC>(v, valid);
        T p[NC];
        double dsum = 0.0, ysum = 0.0;
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const double w = (double)v[s] - theta;
            p[s] = valid[s] && w > 0.0 ? (T)w : (T)0;
            if (valid[s]) {
                const double d = (double)p[s] - (double)y[s];
                sc_sq += d * d;
                if (BT) {
                    sc_try += (double)y[s] * (double)sy[s];
                    sc_lin += (double)grad[s] * d;
                    dsum += d;
                    ysum += (double)y[s];
                }
                if (!(v[s] == v[s]) || v[s] - v[s] != (T)0)
                    n_bad += 1;
            }
        }
        if (BT) {
            dsum += shfl_xor_d(dsum, 16);
            dsum += shfl_xor_d(dsum, 32);
            ysum += shfl_xor_d(ysum, 16);
            ysum += shfl_xor_d(ysum, 32);
            if (g == 0 && live)
                sc_corr += ysum * dsum;
        }
        // stage the tile for the Gram products
        __syncthreads();
        const int lrow = wave * 16 + r;
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const int k = kslot<T>(s, g);
            lds[0][lrow * STRIDE + k] = p[s];
            if constexpr (ACCEL)
                lds[1][lrow * STRIDE + k] = bn1 * p[s] - bn0 * xc[s];
            if constexpr (BT)
                lds[NMAT - 1][lrow * STRIDE + k] = y[s];
        }
        __syncthreads();
        // the new iterate (and its bfloat16 copy for the next sparse product): a
        // wave's 16 rows are contiguous in memory, so they are written from the
        // staged tile in pieces of up to 16 bytes, consecutive lanes on
        // consecutive pieces (a lane's own slots are 4 components of 16 rows)
        {
            constexpr int PER = 16 / (int)sizeof(T);   // components per piece
            constexpr int RP = CP / PER;               // pieces per row
            constexpr int PIECES = 16 * RP;            // pieces of a wave's rows
            using V16 = T __attribute__((ext_vector_type(PER)));
            const int64_t row0 = wt * 64 + wave * 16;
#pragma unroll
            for (int e0 = 0; e0 < PIECES; e0 += 64) {
                const int e = e0 + lane;
                const int lr = e / RP, kc = (e % RP) * PER;
                if ((PIECES % 64 == 0 || e < PIECES) && row0 + lr < n)
                    *reinterpret_cast<V16 *>(Xn + (row0 + lr) * CP + kc) =
                        *reinterpret_cast<const V16 *>(&lds[0][(wave * 16 + lr) * STRIDE + kc]);
            }
            if constexpr (SHADOW) {
                constexpr int SPER = CP < 8 ? CP : 8;      // bfloat16 components per piece
                constexpr int SRP = CP / SPER;
                constexpr int SPIECES = 16 * SRP;
                using W = uint32_t __attribute__((ext_vector_type(SPER / 2)));
#pragma unroll
                for (int e0 = 0; e0 < SPIECES; e0 += 64) {
                    const int e = e0 + lane;
                    const int lr = e / SRP, kc = (e % SRP) * SPER;
                    if ((SPIECES % 64 == 0 || e < SPIECES) && row0 + lr < n) {
                        const T *src = &lds[0][(wave * 16 + lr) * STRIDE + kc];
                        W w;
#pragma unroll
                        for (int h = 0; h < SPER / 2; ++h)
                            w[h] = (uint32_t)__bfloat16_as_ushort(__float2bfloat16((float)src[2 * h])) |
                                   ((uint32_t)__bfloat16_as_ushort(__float2bfloat16((float)src[2 * h + 1])) << 16);
                        *reinterpret_cast<W *>(shadow + (row0 + lr) * CP + kc) = w;
                    }
                }
            }
        }
#pragma unroll
        for (int kk = 0; kk < BPW; ++kk) {
            const int kb = wave + 4 * kk;
            if (kb < NBLK) {
                int m, a, b;
                bool cross = false;   // (p + y)^T (p - y)
                if (kb < NSYM) {
                    m = 0;
                    SymBlocks<M>::ab(kb, a, b);
                } else if (ACCEL && kb < 2 * NSYM) {
                    m = 1;
                    SymBlocks<M>::ab(kb - NSYM, a, b);
                } else {
                    const int q = kb - NSYM - (ACCEL ? NSYM : 0);
                    m = 0;
                    cross = true;
                    a = q / M;
                    b = q % M;
                }
                A4 acc = A4{0, 0, 0, 0};
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const int ia = (4 * t + g) * STRIDE + 16 * a + r, ib = (4 * t + g) * STRIDE + 16 * b + r;
                    T va = lds[m][ia], vb = lds[m][ib];
                    if (BT && cross) {
                        va = va + lds[NMAT - 1][ia];
                        vb = vb - lds[NMAT - 1][ib];
                    }
                    acc = mfma16x16x4(va, vb, acc);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc64[kk][q] += (double)acc[q];
            }
        }
    }

    // write this workgroup's partials
    double *out = I.part_fused + blk * L::NE;
#pragma unroll
    for (int kk = 0; kk < BPW; ++kk) {
        const int kb = wave + 4 * kk;
        if (kb < NBLK) {
            int mat, a, b;
            bool sym = true;
            if (kb < NSYM) {
                mat = 0;
                SymBlocks<M>::ab(kb, a, b);
            } else if (ACCEL && kb < 2 * NSYM) {
                mat = 1;
                SymBlocks<M>::ab(kb - NSYM, a, b);
            } else {
                const int q = kb - NSYM - (ACCEL ? NSYM : 0);
                mat = 2;
                sym = false;
                a = q / M;
                b = q % M;
            }
            double *o = out + mat * L::MAT;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 16 * a + mfma_row<T>(g, q), j = 16 * b + r;
                o[i * CPM + j] = acc64[kk][q];
                if (sym && a != b)
                    o[j * CPM + i] = acc64[kk][q];
            }
        }
    }
    double vals[6] = {sc_try, sc_lin, sc_sq, sc_corr, (double)n_bad, sc_trc};
    fused_scalars_out(vals, out + 3 * L::MAT);
}

// FP32 up to 32 clusters without the line-search sums fits 128 registers:
// ask for four waves per SIMD (measured 6 % faster at c = 32 than the three
// the compiler picks alone); with them it fits 168, three waves (10.6 vs
// 11.1 ms at n = 7e7 against two).  At 64 clusters two waves instead of the
// one the compiler picks alone: 12.5 vs 18.9 ms for the same bytes
// (n = 3.5e7), 11.7 vs 15.6 ms with the line-search sums (a few spilled
// registers).
template <typename T, int CP, bool BT> constexpr int fused_min_waves() {
    return sizeof(T) == 4 ? (CP <= 32 ? (BT ? 3 : 4) : 2) : 1;
}

template <typename T, int CP, bool ACCEL, bool BT, bool SHADOW>
__global__ __launch_bounds__(256, (fused_min_waves<T, CP, BT>())) void k_fused_1(Inst I) {
    if (inst_active(I))
        fused_body<T, CP, ACCEL, BT, SHADOW>(I, blockIdx.x, gridDim.x);
}
// The batched form holds more state per lane; FP32 asks for two waves per
// SIMD (at 64 clusters the compiler alone picks one).
template <typename T, int CP, bool ACCEL, bool BT, bool SHADOW>
__global__ __launch_bounds__(256, (sizeof(T) == 4 ? 2 : 1)) void k_fused_b(const Inst *__restrict__ insts,
                                                 const VBlk *__restrict__ tab,
                                                 const int32_t *__restrict__ count) {
    for (int64_t vb = blockIdx.x; vb < *count; vb += gridDim.x) {
        __syncthreads();
        const VBlk t = tab[vb];
        const Inst &I = insts[t.inst];
        if (inst_active(I))
            fused_body<T, CP, ACCEL, BT, SHADOW>(I, t.blk, I.g_fused);
    }
}

// ---------------------------------------------------------------------------
// Single-pass iteration (constant or scheduled steps): one sweep over the
// rows per iteration that takes the step from the stored extrapolated point
// Y_n instead of re-forming it from two iterates and their products.
//
// A 64-row tile at a time, a workgroup
//   A. sums the tile's rows of S_eff Y_n -- rows of at most light_max stored
//      nonzeros by teams of lanes that gather rows of Y_n (the sparse
//      product's loop), longer rows from the pre-pass, which left their
//      products S_off Y_n in Z -- into LDS;
//   B. with the fused kernel's lane layout reads y_i and xbar_{n-1,i}, adds
//      the unit diagonal, forms grad = -4 (S_eff y - y (G_Y - mu 1 1^T)) (Y G
//      on the matrix cores), v = y - tau grad and its projection p onto the
//      simplex (Xbar_n), and the next extrapolated point
//      y' = (1 + beta') p - beta' xbar_{n-1};
//   C. stages p and y' in LDS, writes p over xbar_{n-1} (each row is read
//      and written by its own tile only) and y' into the other Y buffer, and
//      accumulates the Gram matrix of y' on the matrix cores.
// The partials hold that Gram matrix (the fused layout's second matrix) and
// the scalars ||Y_n - Xbar_n||^2 and the count of non-finite step values.
// S is applied once per iteration, to Y_n, and nothing of size n x c is
// stored besides Xbar and Y; the loss needs S Xbar and is formed only when
// the iterate is read out.
// ---------------------------------------------------------------------------
template <typename T, int CP, bool ACCEL>
__device__ __forceinline__ void single_body(const Inst &I, int64_t blk, int64_t nblk) {
    constexpr int CPM = CP < 16 ? 16 : CP;
    constexpr int M = CPM / 16;
    constexpr int NC = 4 * M;
    constexpr int STRIDE = sizeof(T) == 8 ? CPM + 4 : CPM + (CPM == 16 ? 32 : 16);
    constexpr int NMAT = ACCEL ? 2 : 1;   // staged tiles: p (and the z tile before it), y'
    constexpr int NSYM = SymBlocks<M>::N;
    constexpr int BPW = (NSYM + 3) / 4;
    using A4 = typename Acc4<T>::type;
    using L = FusedLayout<CPM>;
    // light-row teams: where a row takes fewer than four 16-byte lanes the
    // slots of a team sit side by side on one row and each team has one row
    // of the tile; wider rows get one-slot teams that walk RPT consecutive
    // rows, whose row pointers they load together (the tile's gathers wait
    // on fewer dependent loads than with two-slot teams walking more rows)
    constexpr int GS1 = TeamCfg<T, CP, 1>::GS;
    using Lc = TeamCfg<T, CP, (GS1 < 4 ? 4 / GS1 : 1)>;
    constexpr int RPT = Lc::TEAMS >= 64 ? 1 : 64 / Lc::TEAMS;
    constexpr int NE = Lc::LANE_ELEMS;
    constexpr int DEPTH = 4;
    static_assert(64 % Lc::TEAMS == 0 || Lc::TEAMS >= 64, "every wave walks the same rows");

    const DevState *__restrict__ st = I.st;
    T *const *Xring = (T *const *)I.X;
    const T *__restrict__ Y = Xring[st->role[ROLE_P]];     // Y_n: gathered and streamed
    T *__restrict__ Yn = Xring[st->role[ROLE_N]];          // Y_{n+1}
    T *__restrict__ Xb = Xring[st->role[ROLE_C]];          // Xbar_{n-1} -> Xbar_n
    const T *__restrict__ Zl = (const T *)I.Z[st->role[ROLE_P]];   // long rows' S_off Y_n
    const T *__restrict__ GYs = (const T *)I.GYs;
    const int64_t *__restrict__ row_ptr = I.row_ptr;
    const int32_t *__restrict__ col = I.col;
    const T *__restrict__ val = (const T *)I.val;
    const int64_t n = I.n, light_max = I.light_max;
    const int c = I.c, diag_unit = I.diag_unit;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    const double beta_next = ACCEL ? st->beta_next : 0.0;
    const T tau = (T)st->tau;
    const T bn1 = (T)(1.0 + beta_next), bn0 = (T)beta_next;

    constexpr bool G_LDS = sizeof(T) == 4;
    constexpr int GSTR = CPM + 1;
    __shared__ T gsh[G_LDS ? CPM * GSTR : 1];
    T gA[G_LDS ? 1 : M][G_LDS ? 1 : NC];
    if constexpr (G_LDS) {
        for (int e = tid; e < CPM * CPM; e += 256)
            gsh[(e / CPM) * GSTR + e % CPM] = GYs[e];
        __syncthreads();
    } else {
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int s = 0; s < NC; ++s)
                gA[a][s] = GYs[(16 * a + r) * CPM + kslot<T>(s, g)];
    }
    __shared__ __attribute__((aligned(16))) T lds[NMAT][64 * STRIDE];

    double sc_sq = 0.0;
    int32_t n_bad = 0;
    doublex4 acc64[BPW];
#pragma unroll
    for (int k = 0; k < BPW; ++k)
        acc64[k] = doublex4{0, 0, 0, 0};

    // a row of a stream in the lane layout (padded components read as zero)
    auto load_row = [&](const T *__restrict__ src, int64_t row, bool live, T (&out)[NC]) {
#pragma unroll
        for (int a = 0; a < M; ++a) {
            const int k0 = 16 * a + 4 * g;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                out[4 * a + q] = (T)0;
            if constexpr (sizeof(T) == 4) {
                if (live && k0 < CP) {
                    T t4[4];
                    GatherLoad<T, 4>::load(src + row * CP + k0, t4);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        out[4 * a + q] = t4[q];
                }
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int k = kslot<T>(4 * a + q, g);
                    if (live && k < CP)
                        out[4 * a + q] = src[row * CP + k];
                }
            }
        }
    };

    const int64_t nwt = nwt_of(n);
    for (int64_t wt = blk; wt < nwt; wt += nblk) {
        // the lane's own rows of Y_n and Xbar_{n-1} are requested first, so
        // these stream reads are in flight while the gathers below run
        const int64_t row = wt * 64 + wave * 16 + r;
        const bool live = row < n;
        const int lrow = wave * 16 + r;
        T y[NC], xp[NC], z[NC];
        load_row(Y, row, live, y);
        if constexpr (ACCEL)
            load_row(Xb, row, live, xp);
        // A. S_off Y_n for the tile's rows, into lds[0] (row-major, stride STRIDE)
        __syncthreads();   // the previous tile's reads of lds are done
        {
            const int team = tid / Lc::TEAM, lt = tid % Lc::TEAM;
            const int slot = lt / Lc::GS, sub = lt % Lc::GS;
            if (team * RPT < 64) {   // teams past the tile's 64 rows idle
                const int64_t r0 = wt * 64 + team * RPT;
                int64_t rp[RPT + 1];
#pragma unroll
                for (int k = 0; k <= RPT; ++k)
                    rp[k] = row_ptr[r0 + k < n ? r0 + k : n];
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const int rr = team * RPT + k;
                    const int64_t row = r0 + k;
                    T acc[NE];
#pragma unroll
                    for (int q = 0; q < NE; ++q)
                        acc[q] = (T)0;
                    bool longrow = false;
                    if (row < n) {
                        if (rp[k + 1] - rp[k] > light_max)
                            longrow = true;
                        else
                            team_row_sum<T, T, CP, Lc::SLOTS, DEPTH>(col, val, Y, rp[k], rp[k + 1], slot,
                                                                     sub, acc, I.nt_from);
                    }
                    team_slot_sum<Lc::GS, Lc::TEAM>(acc);
                    if (slot == 0) {
                        if (longrow)
#pragma unroll
                            for (int q = 0; q < NE; ++q)
                                acc[q] = Zl[row * CP + sub * NE + q];
#pragma unroll
                        for (int q = 0; q < NE; ++q)
                            lds[0][rr * STRIDE + sub * NE + q] = acc[q];
                    }
                }
            }
        }
        __syncthreads();

        // B. the step, in the fused kernel's lane layout
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const int k = kslot<T>(s, g);
            z[s] = (live && k < CP) ? lds[0][lrow * STRIDE + k] : (T)0;
            if (diag_unit)
                z[s] += y[s];
        }
        T yg[NC];
#pragma unroll
        for (int a = 0; a < M; ++a) {
            A4 acc = A4{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                T ga;
                if constexpr (G_LDS)
                    ga = gsh[(16 * a + r) * GSTR + kslot<T>(s, g)];
                else
                    ga = gA[a][s];
                acc = mfma16x16x4(ga, y[s], acc);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                yg[4 * a + q] = acc[q];
        }
        T v[NC];
        bool valid[NC];
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const int k = kslot<T>(s, g);
            valid[s] = live && k < c;
            const T grad = (T)(-4) * (z[s] - yg[s]);
            v[s] = y[s] - tau * grad;
        }
        const double theta = simplex_threshold<T, NC>(v, valid);
        T p[NC];
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const double w = (double)v[s] - theta;
            p[s] = valid[s] && w > 0.0 ? (T)w : (T)0;
            if (valid[s]) {
                const double d = (double)p[s] - (double)y[s];
                sc_sq += d * d;
                if (!(v[s] == v[s]) || v[s] - v[s] != (T)0)
                    n_bad += 1;
            }
        }

        // C. stage p (over the z tile) and y', write them, Gram of y'
        __syncthreads();
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const int k = kslot<T>(s, g);
            lds[0][lrow * STRIDE + k] = p[s];
            if constexpr (ACCEL)
                lds[1][lrow * STRIDE + k] = bn1 * p[s] - bn0 * xp[s];
        }
        __syncthreads();
        {
            constexpr int PER = 16 / (int)sizeof(T);
            constexpr int RP = CP / PER > 0 ? CP / PER : 1;
            constexpr int PW = CP / PER > 0 ? PER : CP;   // components per piece
            constexpr int PIECES = 16 * RP;
            using V16 = T __attribute__((ext_vector_type(PW)));
            const int64_t row0 = wt * 64 + wave * 16;
#pragma unroll
            for (int e0 = 0; e0 < PIECES; e0 += 64) {
                const int e = e0 + lane;
                const int lr = e / RP, kc = (e % RP) * PW;
                if ((PIECES % 64 == 0 || e < PIECES) && row0 + lr < n) {
                    const int li = (wave * 16 + lr) * STRIDE + kc;
                    *reinterpret_cast<V16 *>(Xb + (row0 + lr) * CP + kc) =
                        *reinterpret_cast<const V16 *>(&lds[0][li]);
                    *reinterpret_cast<V16 *>(Yn + (row0 + lr) * CP + kc) =
                        *reinterpret_cast<const V16 *>(&lds[NMAT - 1][li]);
                }
            }
        }
#pragma unroll
        for (int kk = 0; kk < BPW; ++kk) {
            const int kb = wave + 4 * kk;
            if (kb < NSYM) {
                int a, b;
                SymBlocks<M>::ab(kb, a, b);
                A4 acc = A4{0, 0, 0, 0};
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const T va = lds[NMAT - 1][(4 * t + g) * STRIDE + 16 * a + r];
                    const T vb = lds[NMAT - 1][(4 * t + g) * STRIDE + 16 * b + r];
                    acc = mfma16x16x4(va, vb, acc);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc64[kk][q] += (double)acc[q];
            }
        }
    }

    // partials: the Gram matrix of Y_{n+1} in the second matrix slot
    double *out = I.part_fused + blk * L::NE;
#pragma unroll
    for (int kk = 0; kk < BPW; ++kk) {
        const int kb = wave + 4 * kk;
        if (kb < NSYM) {
            int a, b;
            SymBlocks<M>::ab(kb, a, b);
            double *o = out + L::MAT;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 16 * a + mfma_row<T>(g, q), j = 16 * b + r;
                o[i * CPM + j] = acc64[kk][q];
                if (a != b)
                    o[j * CPM + i] = acc64[kk][q];
            }
        }
    }
    double vals[6] = {0.0, 0.0, sc_sq, 0.0, (double)n_bad, 0.0};
    fused_scalars_out(vals, out + 3 * L::MAT);
}

template <typename T, int CP, bool ACCEL>
__global__ __launch_bounds__(256, (fused_min_waves<T, CP, false>())) void k_single_1(Inst I) {
    if (inst_active(I))
        single_body<T, CP, ACCEL>(I, blockIdx.x, gridDim.x);
}

// Deferred loss of the current iterate: the terms <x_i, (S_eff X)_i> as the
// fused kernel forms them (same tiles, lanes, order and grid), written to
// the same scalar slot of the same partial rows.
template <typename T, int CP>
__global__ __launch_bounds__(256) void k_trace_fused(Inst I) {
    constexpr int CPM = CP < 16 ? 16 : CP;
    constexpr int M = CPM / 16;
    constexpr int NC = 4 * M;
    using L = FusedLayout<CPM>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const T *__restrict__ Xc = (const T *)I.X[I.st->role[ROLE_C]];
    const T *__restrict__ Zc = (const T *)I.Z[I.st->role[ROLE_C]];
    const int64_t n = I.n, nwt = nwt_of(n);
    // a lane's slots of one tile (zero past the end); FP32 slots 4a..4a+3 are
    // four consecutive components, loaded as one 16-byte piece
    auto load = [&](int64_t wt, T (&xc)[NC], T (&zc)[NC]) {
        const int64_t row = wt * 64 + wave * 16 + r;
        const bool live = wt < nwt && row < n;
#pragma unroll
        for (int a = 0; a < M; ++a) {
            if constexpr (sizeof(T) == 4) {
                const int k0 = 16 * a + 4 * g;
                T tx[4] = {0, 0, 0, 0}, tz[4] = {0, 0, 0, 0};
                if (live && k0 < CP) {
                    GatherLoad<T, 4>::load(Xc + row * CP + k0, tx);
                    GatherLoad<T, 4>::load(Zc + row * CP + k0, tz);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    xc[4 * a + q] = tx[q];
                    zc[4 * a + q] = tz[q];
                }
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int k = kslot<T>(4 * a + q, g);
                    const bool ok = live && k < CP;
                    xc[4 * a + q] = ok ? Xc[row * CP + k] : (T)0;
                    zc[4 * a + q] = ok ? Zc[row * CP + k] : (T)0;
                }
            }
        }
    };
    // the next tile's loads are in flight while the current one is summed;
    // the terms are added in tile order, as the fused kernel adds them
    double sc_trc = 0.0;
    T xc[NC], zc[NC], xn[NC], zn[NC];
    load(blockIdx.x, xc, zc);
    for (int64_t wt = blockIdx.x; wt < nwt; wt += gridDim.x) {
        load(wt + gridDim.x, xn, zn);
        sc_trc += trace_terms<T, NC>(xc, zc, I.diag_unit);
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            xc[s] = xn[s];
            zc[s] = zn[s];
        }
    }
    double vals[6] = {0.0, 0.0, 0.0, 0.0, 0.0, sc_trc};
    fused_scalars_out(vals, I.part_fused + (int64_t)blockIdx.x * L::NE + 3 * L::MAT);
}

// One entry of the fused partials reduced exactly as reduce_fused_body does
// (same chunks of partial rows, same order).
template <int CPM> __global__ __launch_bounds__(256) void k_reduce_fused_entry(Inst I, int entry) {
    using L = FusedLayout<CPM>;
    reduce_cols_body(I.part_fused + entry, I.g_fused, L::NE, 1, I.red_mats + entry, FUSED_RED_EB, 0);
}

// ---------------------------------------------------------------------------
// Controller: a single workgroup reads the reduced sums and advances the
// iteration state (Alg. 4: loss, stop test, inertial parameter; backtracking
// acceptance).  mode 0: initialisation after Gram + product of Xbar_0;
// mode 1: after the fused kernel and the product of the trial point.
// ---------------------------------------------------------------------------
// Sum of one double per thread of a 256-thread workgroup in a fixed order:
// a shuffle tree in each wave (lane 0's result), then the four waves in
// order.  Every thread returns the same value.
__device__ __forceinline__ double block_sum_256(double v) {
    __shared__ double wsum[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += shfl_xor_d(v, off);
    if (lane == 0)
        wsum[wave] = v;
    __syncthreads();
    const double r = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
    __syncthreads();   // wsum is reused by the next call
    return r;
}

// The loss terms sum_i <x_i, (S_off X)_i> of a symmetric S, for a read-out:
// from the entries on and below the diagonal only (the one on it at half
// weight; the sum is doubled by the controller), walked as one flat
// sequence of nonzeros rather than row by row (a row-by-row pass over half
// the entries measured nearly as slow as the whole product: its teams wait
// on every row's chain of dependent loads).  Each team of GS lanes (16
// bytes of a row each) takes chunks of LOSS_CHUNK consecutive nonzeros,
// finds the chunk's first row by binary search, and walks the rows it
// touches: the sum z of a row's
// gathered terms, dotted with the row's own x_i when the walk leaves the row
// (a row split between chunks gives each chunk its part of the dot).  The
// next row's end and x_i are loaded ahead.  An entry is gathered in the pass
// that loads it when its column is at most the current row (then it is
// below the diagonal of its own row, which can only be later); the rare
// entry whose row is reached only during the pass is gathered when it is
// added.  Per-lane FP64 dots, summed in a fixed order into part[blockIdx];
// a persistent grid walks the chunks.  At n = 7e7, c = 32 the pass takes
// about 20 ms against 28 ms for the whole product with its epilogue; the
// flat gather probe does the same gathers in 11.5 ms: the walk still waits
// at row boundaries (eight entries per pass instead of four measured the
// same).
constexpr int64_t LOSS_CHUNK = 2048;
template <typename T, int CP, int DEPTH = 4>
__global__ __launch_bounds__(256) void k_loss_lower(const int64_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col,
                                                    const T *__restrict__ val, const T *__restrict__ X,
                                                    int64_t n, int64_t nnz, double *__restrict__ part) {
    using Cfg = TeamCfg<T, CP, 1>;
    constexpr int GS = Cfg::GS, TEAMS = Cfg::TEAMS, NE = Cfg::LANE_ELEMS;
    const int tid = threadIdx.x, team = tid / GS, sub = tid % GS;
    const int64_t nchunks = (nnz + LOSS_CHUNK - 1) / LOSS_CHUNK;
    const int64_t team_id = (int64_t)blockIdx.x * TEAMS + team, nteams = (int64_t)gridDim.x * TEAMS;
    double dot = 0.0;
    auto load_x = [&](int64_t r, T (&x)[NE]) {
#pragma unroll
        for (int q = 0; q < NE; ++q)
            x[q] = (T)0;
        if (r < n)
            GatherLoad<T, NE>::load(X + r * CP + sub * NE, x);
    };
    for (int64_t k = team_id; k < nchunks; k += nteams) {
        const int64_t e0 = k * LOSS_CHUNK, e1 = e0 + LOSS_CHUNK < nnz ? e0 + LOSS_CHUNK : nnz;
        // the last row whose range starts at or before e0
        int64_t lo = 0, hi = n - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (row_ptr[mid] <= e0)
                lo = mid;
            else
                hi = mid - 1;
        }
        int64_t row = lo;
        int64_t rend = row_ptr[row + 1];
        int64_t rend2 = row + 2 <= n ? row_ptr[row + 2] : nnz;
        T xi[NE], xn[NE], z[NE];
        load_x(row, xi);
        load_x(row + 1, xn);
#pragma unroll
        for (int q = 0; q < NE; ++q)
            z[q] = (T)0;
        int32_t jn[DEPTH];
        T sn[DEPTH];
#pragma unroll
        for (int u = 0; u < DEPTH; ++u) {
            const int64_t e = e0 + u;
            jn[u] = e < e1 ? col[e] : -1;
            sn[u] = e < e1 ? val[e] : (T)0;
        }
        for (int64_t eb = e0; eb < e1; eb += DEPTH) {
            int32_t j[DEPTH];
            T s[DEPTH], g[DEPTH][NE];
            bool have[DEPTH];
#pragma unroll
            for (int u = 0; u < DEPTH; ++u) {
                j[u] = jn[u];
                s[u] = sn[u];
                have[u] = j[u] >= 0 && j[u] <= row;
#pragma unroll
                for (int q = 0; q < NE; ++q)
                    g[u][q] = (T)0;
                if (have[u])
                    GatherLoad<T, NE>::load(X + (int64_t)j[u] * CP + sub * NE, g[u]);
            }
#pragma unroll
            for (int u = 0; u < DEPTH; ++u) {
                const int64_t e = eb + DEPTH + u;
                jn[u] = e < e1 ? col[e] : -1;
                sn[u] = e < e1 ? val[e] : (T)0;
            }
#pragma unroll
            for (int u = 0; u < DEPTH; ++u) {
                const int64_t e = eb + u;
                if (e >= e1)
                    break;
                while (e >= rend) {   // the walk leaves the row
#pragma unroll
                    for (int q = 0; q < NE; ++q) {
                        dot += (double)z[q] * (double)xi[q];
                        z[q] = (T)0;
                        xi[q] = xn[q];
                    }
                    ++row;
                    rend = rend2;
                    rend2 = row + 2 <= n ? row_ptr[row + 2] : nnz;
                    load_x(row + 1, xn);
                }
                if (j[u] > row)
                    continue;   // above the diagonal: its mirror entry counts it
                const T w = j[u] == row ? (T)0.5 * s[u] : s[u];
                if (!have[u])
                    GatherLoad<T, NE>::load(X + (int64_t)j[u] * CP + sub * NE, g[u]);
#pragma unroll
                for (int q = 0; q < NE; ++q)
                    z[q] += w * g[u][q];
            }
        }
#pragma unroll
        for (int q = 0; q < NE; ++q)
            dot += (double)z[q] * (double)xi[q];
    }
    const double tot = block_sum_256(dot);
    if (tid == 0)
        part[blockIdx.x] = tot;
}

// K such sums at once, each in exactly the order of block_sum_256 (so each
// result has the same bits), with one pair of barriers for all of them.
template <int K>
__device__ __forceinline__ void block_sums_256(double (&v)[K]) {
    __shared__ double wsum[K][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            v[k] += shfl_xor_d(v[k], off);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k)
            wsum[k][wave] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k)
        v[k] = ((wsum[k][0] + wsum[k][1]) + wsum[k][2]) + wsum[k][3];
    __syncthreads();
}

// The device state as 8-byte words (copies between HBM and LDS).
typedef uint64_t __attribute__((__may_alias__)) state_word;
constexpr int STATE_WORDS = (int)(sizeof(DevState) / sizeof(uint64_t));
static_assert(sizeof(DevState) % sizeof(uint64_t) == 0 && STATE_WORDS <= 256,
              "the state is copied one 8-byte word per thread");

// The controller is one workgroup and latency-bound: its inputs (the state,
// the reduced matrices, the partial sums) are loaded by all threads at
// once, the state is worked on in LDS by one thread and written back by all
// threads, and the four sums are reduced together.  Every value is formed
// exactly as it would be one load after the other.
template <typename T, int CPM>
__device__ __forceinline__ void control_body(const Inst &I, int mode) {
    using L = FusedLayout<CPM>;
    constexpr int PER = (CPM * CPM + 255) / 256;   // matrix entries per thread
    __shared__ int decision;
    __shared__ DevState st_lds;
    DevState *__restrict__ gst = I.st;
    const double *__restrict__ red_mats = I.red_mats;
    double *__restrict__ GY64 = I.GY64;
    T *__restrict__ GYs = (T *)I.GYs;
    const double *__restrict__ sched = I.sched;
    double *__restrict__ hist_f = I.hist_f;
    double *__restrict__ hist_tau = I.hist_tau;
    int32_t *__restrict__ hist_trials = I.hist_trials;
    double *__restrict__ hist_r = I.hist_r;
    const int tid = threadIdx.x;
    // mode 0: initial evaluation; 1: after a trial; 2: deferred evaluation of
    // the current iterate after the trials (nothing else changes); 3: the
    // read-out loss of a single-pass instance (nothing else changes)
    if (mode == 1 && !gst->active)
        return;
    if (tid < STATE_WORDS)
        reinterpret_cast<state_word *>(&st_lds)[tid] = reinterpret_cast<const state_word *>(gst)[tid];
    DevState *__restrict__ st = &st_lds;   // valid after the barrier of the sums below
    const int c = gst->c, accelerate = gst->accelerate, backtrack = gst->backtrack;
    // a single-pass iteration forms no loss terms; its pass leaves the Gram
    // matrix of the next extrapolated point in the second matrix slot
    const bool single = I.pass_kind == PASS_SINGLE;
    const bool single_step = single && mode == 1;
    // the products' terms sum_i <x_i, (S X)_i>: workgroup partials of the
    // sparse product, combined in a fixed order (a deferred instance forms
    // them in the fused pass instead; its products write no partials)
    const bool want_tr = !I.defer && !single_step;
    double sums[4] = {0.0, 0.0, 0.0, 0.0};   // trace terms, ||G_p||^2, <M, G_p + G_Y>, G_next sum
    if (want_tr) {
        const int64_t np = (int64_t)I.g_spmm + I.g_comb;
#pragma unroll 8
        for (int64_t q = tid; q < np; q += 256)   // loads run ahead, adds stay in order
            sums[0] += I.part_spmm[q];
    }
    const double *Gp = red_mats + (single_step ? L::MAT : 0);   // Gram of the new point
    const double *Gnext = single ? Gp : red_mats + (mode == 1 && accelerate ? L::MAT : 0);
    const double *Mx = red_mats + 2 * L::MAT;
    const double *sc = red_mats + 3 * L::MAT;

    // ||G_p||^2, (backtracking) <M, G_p + G_Y>, and the sum over the c x c
    // block of the next extrapolated point's Gram matrix (kept in registers
    // for the copy below), fixed-order tree sums
    const bool want_m = mode == 1 && backtrack;
    double gnext[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = tid + 256 * k;
        gnext[k] = 0.0;
        if (e < CPM * CPM) {
            sums[1] += Gp[e] * Gp[e];
            if (want_m)
                sums[2] += Mx[e] * (Gp[e] + GY64[e]);
            gnext[k] = Gnext[e];
            if (e / CPM < c && e % CPM < c)
                sums[3] += gnext[k];
        }
    }
    block_sums_256(sums);
    const double tr_total = want_tr ? sums[0] : 0.0;
    const double gp_sq = sums[1];
    const double m_dot = want_m ? sums[2] : 0.0;
    const double mu_next = sums[3] / ((double)c * (double)c);

    if (tid == 0) {
        // deferred: the products carry no terms; the fused kernel (or the
        // evaluation pass) summed them for the current iterate
        double tr_p = st->defer ? sc[FS_TRC] : tr_total;
        if (mode == 3) {
            // the read-out's terms come from the entries on and below the
            // diagonal (k_loss_lower): twice them, plus the unit diagonal's
            // sum_i ||x_i||^2, the trace of the read-out's Gram matrix
            double gdiag = 0.0;
            if (I.diag_unit)
                for (int k = 0; k < c; ++k)
                    gdiag += Gp[k * CPM + k];
            tr_p = 2.0 * tr_total + gdiag;
        }
        const double f_p = st->s2 + gp_sq - 2.0 * tr_p;
        int accept = 1;
        if (mode == 0) {
            st->f = f_p;
            st->f_prev = f_p;
            st->iter = 0;
            st->trials = 0;
            st->trial_in_iter = 1;
            st->f_known = 1;
            st->gsq_c = gp_sq;
            if (hist_f)
                hist_f[0] = f_p;
            // the start has no step, trial or gradient mapping: zeros, so
            // that a checkpoint holds no unwritten memory
            if (hist_tau)
                hist_tau[0] = 0.0;
            if (hist_r)
                hist_r[0] = 0.0;
            if (hist_trials)
                hist_trials[0] = 0;
            if (!(f_p == f_p) || f_p - f_p != 0.0) {
                st->error = ERR_NONFINITE;
                st->stop_reason = STOP_ERROR;
                st->active = 0;
                accept = 0;
            }
        } else if (mode == 3) {
            // single pass: the loss of the iterate being read out
            accept = 0;
            st->f_prev = st->f;
            st->f = f_p;
            st->f_known = 1;
            if (st->iter < st->hist_cap && hist_f)
                hist_f[st->iter] = f_p;
            if (!(f_p == f_p) || f_p - f_p != 0.0) {
                st->error = ERR_NONFINITE;
                st->stop_reason = STOP_ERROR;
                st->active = 0;
            }
        } else if (mode == 2 || (st->defer && !st->f_known)) {
            // deferred loss of Xbar_iter: ||G||^2 saved when it was accepted
            accept = mode == 1;
            if (!st->f_known) {
                const double f_c = st->s2 + st->gsq_c - 2.0 * sc[FS_TRC];
                st->f = f_c;
                st->f_known = 1;
                if (st->iter < st->hist_cap && hist_f)
                    hist_f[st->iter] = f_c;
                if (!(f_c == f_c) || f_c - f_c != 0.0) {
                    st->error = ERR_NONFINITE;
                    st->stop_reason = STOP_ERROR;
                    st->active = 0;
                    accept = 0;
                } else if (st->iter >= 1 && st->tol_loss == st->tol_loss &&
                           st->f_prev - f_c <= st->tol_loss) {
                    // the loss test of Alg. 3/4 for Xbar_iter: stop there and
                    // drop the trial computed from it
                    st->stop_reason = STOP_LOSS;
                    st->active = 0;
                    accept = 0;
                }
            }
        }
        if (mode == 1 && accept) {
            const double tr_y = sc[FS_TRY], lin_s = sc[FS_LIN], sq = sc[FS_SQ];
            const double corr = sc[FS_CORR], bad = sc[FS_BAD];
            st->trials += 1;
            // deferred or single pass: f_p is not this trial's loss; check
            // what it provides
            const double f_chk = (st->defer || single) ? gp_sq : f_p;
            const bool finite = (f_chk == f_chk) && (f_chk - f_chk == 0.0) && bad == 0.0;
            if (!finite) {
                st->error = ERR_NONFINITE;
                st->stop_reason = STOP_ERROR;
                st->active = 0;
                accept = 0;
            } else if (st->backtrack) {
                const double lin = lin_s + 4.0 * st->mu * corr;
                const double df = m_dot - 2.0 * (tr_p - tr_y);
                const double rhs = lin + 0.5 * st->L * sq;
                st->tr_y_last = tr_y;
                st->df_last = df;
                st->rhs_last = rhs;
                accept = df <= rhs;
            }
            if (st->active && accept) {
                const int it = st->iter + 1;
                const double rr = sqrt(sq) / st->tau;
                st->iter = it;
                st->f_prev = st->f;
                if (st->defer) {   // f(Xbar_it) follows from the next pass
                    st->f_known = 0;
                    st->gsq_c = gp_sq;
                } else if (single) {   // f(Xbar_it) is formed at the read-out
                    st->f_known = 0;
                } else {
                    st->f = f_p;
                }
                st->r = rr;
                if (it == 1)
                    st->r1 = rr;
                if (it < st->hist_cap) {
                    if (hist_f && !st->defer) hist_f[it] = single ? __longlong_as_double(0x7ff8000000000000ll) : f_p;
                    if (hist_tau) hist_tau[it] = st->tau;
                    if (hist_trials) hist_trials[it] = st->trial_in_iter;
                    if (hist_r) hist_r[it] = rr;
                }
                if (single) {   // Xbar stays in place; Y_{n+1} becomes the current Y
                    const int rp = st->role[ROLE_P];
                    st->role[ROLE_P] = st->role[ROLE_N];
                    st->role[ROLE_N] = rp;
                } else {   // ring: trial -> current, current -> previous, previous -> next trial
                    const int rc = st->role[ROLE_C], rp = st->role[ROLE_P], rn = st->role[ROLE_N];
                    st->role[ROLE_C] = rn;
                    st->role[ROLE_P] = rc;
                    st->role[ROLE_N] = rp;
                }
                // inertial parameter (Alg. 4)
                const double t_next = 0.5 * (1.0 + sqrt(1.0 + 4.0 * st->t * st->t));
                st->beta = st->beta_next;
                st->t = t_next;
                if (st->accelerate) {
                    const double t_after = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t_next * t_next));
                    st->beta_next = (t_next - 1.0) / t_after;
                } else {
                    st->beta_next = 0.0;
                }
                st->trial_in_iter = 1;
                // stop tests (deferred: the loss test runs when f is formed)
                if (!st->defer && st->tol_loss == st->tol_loss && st->f_prev - st->f <= st->tol_loss) {
                    st->stop_reason = STOP_LOSS;
                    st->active = 0;
                } else if (st->tol_pgrad > 0.0 && rr <= st->tol_pgrad * st->r1) {
                    st->stop_reason = STOP_PGRAD;
                    st->active = 0;
                } else if (it >= st->max_iter) {
                    st->stop_reason = STOP_MAXITER;
                    st->active = 0;
                }
                if (it >= st->target)
                    st->active = 0;
                // step of the next iteration
                if (!st->backtrack) {
                    if (sched) {
                        const int k = it < st->sched_len ? it : st->sched_len - 1;
                        st->tau = sched[k];
                    } else {
                        st->tau = st->tau0;
                    }
                    st->L = 1.0 / st->tau;
                }
            } else if (st->active) {
                st->trial_in_iter += 1;
                st->L *= st->eta;
                st->tau = 1.0 / st->L;
                if (!(st->L < 1e300) || st->trial_in_iter > 1000) {
                    st->error = ERR_STEP;
                    st->stop_reason = STOP_ERROR;
                    st->active = 0;
                }
                accept = 0;
            }
        }
        if (accept)
            st->mu = mu_next;
        decision = accept;
    }
    __syncthreads();
    if (tid < STATE_WORDS)
        reinterpret_cast<state_word *>(gst)[tid] = reinterpret_cast<const state_word *>(&st_lds)[tid];
    if (!decision) {
        __syncthreads();   // st_lds is reused by the next call
        return;
    }
    // G of the next extrapolated point: keep it in double and hand the fused
    // kernel a copy with its mean over the c x c block removed.
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = tid + 256 * k;
        if (e < CPM * CPM) {
            const int i = e / CPM, j = e % CPM;
            GY64[e] = gnext[k];
            GYs[e] = (i < c && j < c) ? (T)(gnext[k] - mu_next) : (T)0;
        }
    }
    __syncthreads();
}

template <typename T, int CPM> __global__ __launch_bounds__(256) void k_control_1(Inst I, int mode) {
    control_body<T, CPM>(I, mode);
}
template <typename T, int CPM>
__global__ __launch_bounds__(256) void k_control_b(const Inst *__restrict__ insts,
                                                   const VBlk *__restrict__ tab,
                                                   const int32_t *__restrict__ count) {
    for (int64_t vb = blockIdx.x; vb < *count; vb += gridDim.x) {
        __syncthreads();
        control_body<T, CPM>(insts[tab[vb].inst], 1);
    }
}

// ---------------------------------------------------------------------------
// Power iteration for ||S_eff||_2: w = S_eff v (double), partial sums of
// w_i^2; then v = w / ||w|| once the host-visible estimate is recorded.
// ---------------------------------------------------------------------------
template <typename VS>
__global__ __launch_bounds__(256) void k_spmv_power(const int64_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col,
                                                    const VS *__restrict__ val,
                                                    const double *__restrict__ v,
                                                    double *__restrict__ w, int64_t n, int diag_unit,
                                                    double *__restrict__ part) {
    __shared__ double sh[256];
    const int tid = threadIdx.x, lane8 = tid & 7, row_in = tid >> 3;
    double acc_sq = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * 32; base < n; base += (int64_t)gridDim.x * 32) {
        const int64_t i = base + row_in;
        double acc = 0.0;
        if (i < n) {
            for (int64_t e = row_ptr[i] + lane8; e < row_ptr[i + 1]; e += 8)
                acc += (double)to_f32(val[e]) * v[col[e]];
        }
        for (int off = 1; off < 8; off <<= 1)
            acc += shfl_xor_d(acc, off);
        if (i < n && lane8 == 0) {
            if (diag_unit)
                acc += v[i];
            w[i] = acc;
            acc_sq += acc * acc;
        }
    }
    sh[tid] = acc_sq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s)
            sh[tid] += sh[tid + s];
        __syncthreads();
    }
    if (tid == 0)
        part[blockIdx.x] = sh[0];
}
template <>
__global__ __launch_bounds__(256) void k_spmv_power<double>(const int64_t *__restrict__ row_ptr,
                                                            const int32_t *__restrict__ col,
                                                            const double *__restrict__ val,
                                                            const double *__restrict__ v,
                                                            double *__restrict__ w, int64_t n,
                                                            int diag_unit,
                                                            double *__restrict__ part) {
    __shared__ double sh[256];
    const int tid = threadIdx.x, lane8 = tid & 7, row_in = tid >> 3;
    double acc_sq = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * 32; base < n; base += (int64_t)gridDim.x * 32) {
        const int64_t i = base + row_in;
        double acc = 0.0;
        if (i < n) {
            for (int64_t e = row_ptr[i] + lane8; e < row_ptr[i + 1]; e += 8)
                acc += val[e] * v[col[e]];
        }
        for (int off = 1; off < 8; off <<= 1)
            acc += shfl_xor_d(acc, off);
        if (i < n && lane8 == 0) {
            if (diag_unit)
                acc += v[i];
            w[i] = acc;
            acc_sq += acc * acc;
        }
    }
    sh[tid] = acc_sq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s)
            sh[tid] += sh[tid + s];
        __syncthreads();
    }
    if (tid == 0)
        part[blockIdx.x] = sh[0];
}

// est[it] = ||w||; flag[0] = 1 once |est - prev| <= rtol est.
__global__ void k_power_update(const double *__restrict__ sumsq, double *__restrict__ est, int it,
                               double rtol, int32_t *__restrict__ flag) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double e = sqrt(sumsq[0]);
        est[it] = e;
        if (e == 0.0 || (it > 0 && fabs(e - est[it - 1]) <= rtol * e))
            flag[0] = 1;
    }
}

__global__ void k_power_scale(const double *__restrict__ w, double *__restrict__ v, int64_t n,
                              const double *__restrict__ est, int it,
                              const int32_t *__restrict__ flag) {
    if (flag[0])
        return;
    const double inv = 1.0 / est[it];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v[i] = w[i] * inv;
}

__global__ void k_fill(double *__restrict__ v, int64_t n, double value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v[i] = value;
}

// ---------------------------------------------------------------------------
// Standalone row-wise projection onto the unit simplex (any leading
// dimension), four lanes per row as in the fused kernel.
// ---------------------------------------------------------------------------
template <typename T, int CPM>
__global__ __launch_bounds__(256) void k_project(const T *__restrict__ V, T *__restrict__ out,
                                                 int64_t rows, int c, int64_t ld) {
    constexpr int NC = CPM / 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int64_t ntiles = (rows + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
        const int64_t row = tile * 16 + r;
        T v[NC];
        bool valid[NC];
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const int k = 16 * (s >> 2) + 4 * g + (s & 3);
            valid[s] = row < rows && k < c;
            v[s] = valid[s] ? V[row * ld + k] : (T)0;
        }
        const double theta = simplex_threshold<T, NC>(v, valid);
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const int k = 16 * (s >> 2) + 4 * g + (s & 3);
            if (valid[s]) {
                const double w = (double)v[s] - theta;
                out[row * ld + k] = w > 0.0 ? (T)w : (T)0;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Memory-system probe (a measurement, not a step of the method): gathers, for
// every stored nonzero e in order, the row col[e] of U with the sparse
// product's 16-byte lane loads, and nothing else -- no values, no
// multiplications, no output rows.  A flat, perfectly balanced loop over the
// nonzeros: each team of GS lanes (one 16-byte piece of a row per lane)
// keeps DEPTH gathers in flight and loads the next column indices while they
// are outstanding.  Its time on the product's own column sequence is the
// floor the product's gathers can reach on this memory system.
// ---------------------------------------------------------------------------
template <int GS, int DEPTH>
__global__ __launch_bounds__(256) void k_gather_probe(const int32_t *__restrict__ col, int64_t nnz,
                                                      const uint4 *__restrict__ U, int64_t row_pieces,
                                                      double *__restrict__ checksum) {
    constexpr int TEAMS = 256 / GS;
    const int team = threadIdx.x / GS, sub = threadIdx.x % GS;
    const int64_t nteam = (int64_t)gridDim.x * TEAMS;
    const int64_t t0 = (int64_t)blockIdx.x * TEAMS + team;
    uint32_t acc = 0;
    int32_t jn[DEPTH];
#pragma unroll
    for (int u = 0; u < DEPTH; ++u) {
        const int64_t e = t0 + u * nteam;
        jn[u] = e < nnz ? col[e] : -1;
    }
    for (int64_t e0 = t0; e0 < nnz; e0 += DEPTH * nteam) {
        uint4 g[DEPTH];
#pragma unroll
        for (int u = 0; u < DEPTH; ++u)
            g[u] = jn[u] >= 0 ? U[(int64_t)jn[u] * row_pieces + sub] : uint4{0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < DEPTH; ++u) {
            const int64_t e = e0 + DEPTH * nteam + u * nteam;
            jn[u] = e < nnz ? col[e] : -1;
        }
#pragma unroll
        for (int u = 0; u < DEPTH; ++u)
            acc += g[u].x ^ g[u].y ^ g[u].z ^ g[u].w;
    }
    __shared__ uint32_t sh[256];
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t x = 0;
        for (int k = 0; k < 256; ++k)
            x ^= sh[k];
        atomicAdd(checksum, (double)(x & 0xffff));
    }
}

}  // namespace fc
