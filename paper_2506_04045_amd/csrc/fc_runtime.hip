// fc_runtime.hip -- host runtime and C ABI of the gfx950 fuzzy-clustering
// solver (see include/fc.h for the contract of every entry point).
//
// A solver owns, on one GPU:
//   * a ring of three n x CP iterate buffers (Xbar_c, Xbar_p, trial) and the
//     three matching products S Xbar, so the extrapolated point and S Y are
//     formed inside the fused kernel from stored rows (S is applied once per
//     trial, to the trial point, whose product is reused by the next step);
//   * in mixed precision a half copy of the values of S and a bfloat16
//     shadow of every iterate, which is what the sparse product gathers;
//   * per-workgroup partial sums, their reductions, the device state and the
//     per-iteration history.
// One trial = k_fused -> k_spmm -> two fixed-order reductions -> k_control;
// the host only re-launches that sequence and reads the state back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstddef>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include <hipcub/device/device_radix_sort.hpp>
#include <hipcub/device/device_scan.hpp>
#include <rocprofiler-sdk-roctx/roctx.h>

#include "fc.h"
#include "fc_host.hpp"
#include "fc_kernels.hpp"
#include "fc_second.hpp"

using namespace fc;

namespace {

thread_local std::string g_last_error;

fc_status fail(fc_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

// Named host ranges for timeline tools (rocprofv3 --marker-trace): the
// set-up, each fc_step / fc_solve call, each group of trials between two
// state readbacks, the loss read-out, the stateless calls and the serving
// worker's phases.  Without a tool attached a range costs two calls.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

// Allocation-failure injection (fc_debug_fail_allocations): -1 when off;
// k >= 0 lets k more allocations succeed and fails every later one as out
// of memory.  Every device and pinned allocation of the library goes
// through the three functions below.
std::atomic<int64_t> g_alloc_countdown{-1};

bool injected_alloc_failure() {
    int64_t v = g_alloc_countdown.load(std::memory_order_relaxed);
    while (v >= 0) {
        if (v == 0)
            return true;
        if (g_alloc_countdown.compare_exchange_weak(v, v - 1, std::memory_order_relaxed))
            return false;
    }
    return false;
}

hipError_t lib_malloc(void **p, size_t bytes) {
    return injected_alloc_failure() ? hipErrorOutOfMemory : hipMalloc(p, bytes);
}

hipError_t lib_malloc_async(void **p, size_t bytes, hipStream_t s) {
    return injected_alloc_failure() ? hipErrorOutOfMemory : hipMallocAsync(p, bytes, s);
}

hipError_t lib_host_malloc(void **p, size_t bytes) {
    return injected_alloc_failure() ? hipErrorOutOfMemory : hipHostMalloc(p, bytes, hipHostMallocDefault);
}

#define HIPCHK(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(e_ == hipErrorOutOfMemory ? FC_ERR_OUT_OF_MEMORY : FC_ERR_DEVICE, \
                        std::string(#expr) + ": " + hipGetErrorString(e_));             \
    } while (0)

int cp_of(int c) {
    int cp = 4;
    while (cp < c)
        cp <<= 1;
    return cp;
}
int cpm_of(int cp) { return cp < 16 ? 16 : cp; }

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return cus;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

int grid_1d(int64_t work, int64_t per_block, int64_t cap) {
    int64_t g = cdiv(work, per_block);
    if (g < 1)
        g = 1;
    if (g > cap)
        g = cap;
    return (int)g;
}

size_t dtype_size(fc_dtype d) {
    switch (d) {
    case FC_F64: return 8;
    case FC_F32: return 4;
    case FC_F16: return 2;
    case FC_BF16: return 2;
    }
    return 0;
}

// RAII for temporary device buffers of the stateless entry points.
struct DevBuf {
    void *p = nullptr;
    hipStream_t s = nullptr;
    ~DevBuf() {
        if (p)
            (void)hipFreeAsync(p, s);
    }
};

hipError_t dev_alloc(DevBuf &b, size_t bytes, hipStream_t s) {
    b.s = s;
    return lib_malloc_async(&b.p, bytes > 0 ? bytes : 16, s);
}

// Reduction launch: out[e] = sum over np partial rows of in (row stride ld).
void launch_reduce(const double *in, int64_t np, int64_t ld, int64_t ne, double *out,
                   hipStream_t s) {
    const int eb = ne >= 64 ? 64 : (ne >= 16 ? 16 : 1);
    const int blocks = (int)cdiv(ne, eb);
    hipLaunchKernelGGL(k_reduce_cols, dim3(blocks), dim3(256), 0, s, in, np, ld, ne, out, eb);
}

// Heavy-row plan built on the host from row_ptr.  Device arrays are owned
// by `bufs` (stream-ordered frees).
struct HeavyPlan {
    int64_t nheavy = 0, nchunks = 0, nmed = 0;
    int32_t *med = nullptr;
    int32_t *rows = nullptr, *chunk_ptr = nullptr, *chunk_row = nullptr, *chunk_len = nullptr;
    int64_t *chunk_beg = nullptr;
    void *chunk_sum = nullptr;
    std::vector<void *> bufs;
    hipStream_t s = nullptr;
    ~HeavyPlan() {
        for (void *p : bufs)
            (void)hipFreeAsync(p, s);
    }
    template <typename P> hipError_t alloc(P **p, size_t bytes) {
        void *q = nullptr;
        hipError_t e = lib_malloc_async(&q, bytes > 0 ? bytes : 16, s);
        if (e == hipSuccess) {
            bufs.push_back(q);
            *p = (P *)q;
        }
        return e;
    }
};

fc_status build_heavy_plan(const int64_t *d_row_ptr, int64_t n, size_t acc_bytes, int cp,
                           hipStream_t s, HeavyPlan &plan) {
    plan.s = s;
    std::vector<int64_t> rp(n + 1);
    HIPCHK(hipMemcpyAsync(rp.data(), d_row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    HeavyRows hr = plan_heavy_rows(rp.data(), n);
    const std::vector<int32_t> &rows = hr.rows, &cptr = hr.chunk_ptr, &crow = hr.chunk_row,
                               &clen = hr.chunk_len, &med = hr.med;
    const std::vector<int64_t> &cbeg = hr.chunk_beg;
    plan.nheavy = (int64_t)rows.size();
    plan.nchunks = (int64_t)cbeg.size();
    plan.nmed = (int64_t)med.size();
    if (plan.nmed > 0) {
        HIPCHK(plan.alloc(&plan.med, sizeof(int32_t) * med.size()));
        HIPCHK(hipMemcpyAsync(plan.med, med.data(), sizeof(int32_t) * med.size(), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    if (plan.nheavy == 0)
        return FC_OK;
    HIPCHK(plan.alloc(&plan.rows, sizeof(int32_t) * rows.size()));
    HIPCHK(plan.alloc(&plan.chunk_ptr, sizeof(int32_t) * cptr.size()));
    HIPCHK(plan.alloc(&plan.chunk_row, sizeof(int32_t) * crow.size()));
    HIPCHK(plan.alloc(&plan.chunk_len, sizeof(int32_t) * clen.size()));
    HIPCHK(plan.alloc(&plan.chunk_beg, sizeof(int64_t) * cbeg.size()));
    HIPCHK(plan.alloc(&plan.chunk_sum, acc_bytes * cp * cbeg.size()));
    HIPCHK(hipMemcpyAsync(plan.rows, rows.data(), sizeof(int32_t) * rows.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(plan.chunk_ptr, cptr.data(), sizeof(int32_t) * cptr.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(plan.chunk_row, crow.data(), sizeof(int32_t) * crow.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(plan.chunk_len, clen.data(), sizeof(int32_t) * clen.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(plan.chunk_beg, cbeg.data(), sizeof(int64_t) * cbeg.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return FC_OK;
}

int combine_grid(int64_t nheavy, int rows_per_block) {
    if (nheavy == 0)
        return 0;
    return grid_1d(nheavy, rows_per_block, 1024);
}

// Copy the heavy-row plan into an instance descriptor.
void plan_to_inst(const HeavyPlan &hp, Inst &I) {
    I.light_max = SPMM_LIGHT_MAX;
    I.nmed = hp.nmed;
    I.med_rows = hp.med;
    I.nchunks = hp.nchunks;
    I.nheavy = hp.nheavy;
    I.chunk_row = hp.chunk_row;
    I.chunk_beg = hp.chunk_beg;
    I.chunk_len = hp.chunk_len;
    I.heavy_rows = hp.rows;
    I.heavy_chunk_ptr = hp.chunk_ptr;
    I.chunk_sum = hp.chunk_sum;
    I.g_comb = combine_grid(hp.nheavy, 1);
}

// Sparse product of ring slot `role` of one instance: light rows and chunks,
// then the per-row combination of the chunks (writes g_spmm + g_comb trace
// partials).
template <typename TU, typename TZ, typename TX, typename VS, int CP>
void launch_spmm(const Inst &I, int role, hipStream_t s) {
    using TA = typename AccumOf<TU>::type;
    hipLaunchKernelGGL((k_spmm_1<TU, TZ, TX, VS, CP>), dim3(I.g_spmm), dim3(256), 0, s, I, role);
    if (I.nheavy > 0)
        hipLaunchKernelGGL((k_combine_1<TA, TZ, TX, CP>), dim3(I.g_comb), dim3(256), 0, s, I, role);
}

// Dispatch a functor on the padded width CP in {4, 8, 16, 32, 64}.
template <typename F> fc_status with_cp(int cp, F &&f) {
    switch (cp) {
    case 4: return f(std::integral_constant<int, 4>());
    case 8: return f(std::integral_constant<int, 8>());
    case 16: return f(std::integral_constant<int, 16>());
    case 32: return f(std::integral_constant<int, 32>());
    case 64: return f(std::integral_constant<int, 64>());
    }
    return fail(FC_ERR_UNSUPPORTED, "padded width out of range");
}

fc_status check_csr_args(const fc_csr *S) {
    if (!S)
        return fail(FC_ERR_INVALID_ARG, "S is NULL");
    if (S->n < 1 || S->n > INT32_MAX)
        return fail(FC_ERR_INVALID_ARG, "S->n must be in [1, 2^31 - 1]");
    if (S->nnz < 0)
        return fail(FC_ERR_INVALID_ARG, "S->nnz < 0");
    if (!S->row_ptr || (S->nnz > 0 && (!S->col_idx || !S->values)))
        return fail(FC_ERR_INVALID_ARG, "S arrays are NULL");
    if (S->values_dtype != FC_F64 && S->values_dtype != FC_F32 && S->values_dtype != FC_F16)
        return fail(FC_ERR_INVALID_ARG, "S values must be FC_F64, FC_F32 or FC_F16");
    return FC_OK;
}

// ||S||_F^2 of the stored values, summed on the device in double.
fc_status sum_squares(const fc_csr *S, hipStream_t s, double *out) {
    const int g = grid_1d(S->nnz, 256 * 8, 4096);
    DevBuf part, red;
    HIPCHK(dev_alloc(part, sizeof(double) * g, s));
    HIPCHK(dev_alloc(red, sizeof(double), s));
    switch (S->values_dtype) {
    case FC_F64:
        hipLaunchKernelGGL(k_sumsq<double>, dim3(g), dim3(256), 0, s, (const double *)S->values,
                           S->nnz, (double *)part.p);
        break;
    case FC_F32:
        hipLaunchKernelGGL(k_sumsq<float>, dim3(g), dim3(256), 0, s, (const float *)S->values,
                           S->nnz, (double *)part.p);
        break;
    default:
        hipLaunchKernelGGL(k_sumsq<__half>, dim3(g), dim3(256), 0, s, (const __half *)S->values,
                           S->nnz, (double *)part.p);
        break;
    }
    HIPCHK(hipGetLastError());
    launch_reduce((const double *)part.p, g, 1, 1, (double *)red.p, s);
    HIPCHK(hipMemcpyAsync(out, red.p, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return FC_OK;
}

// Power iteration for ||S_eff||_2 from the normalised ones vector.
fc_status power_norm(const fc_csr *S, int diag_unit, int max_iter, double rtol, hipStream_t s,
                     double *norm_out, int32_t *iters_out) {
    const int64_t n = S->n;
    if (max_iter < 1)
        max_iter = 1;
    const int g = grid_1d(n, 32, 8192);
    DevBuf v, w, part, red, est, flag;
    HIPCHK(dev_alloc(v, sizeof(double) * n, s));
    HIPCHK(dev_alloc(w, sizeof(double) * n, s));
    HIPCHK(dev_alloc(part, sizeof(double) * g, s));
    HIPCHK(dev_alloc(red, sizeof(double), s));
    HIPCHK(dev_alloc(est, sizeof(double) * (max_iter + 1), s));
    HIPCHK(dev_alloc(flag, sizeof(int32_t), s));
    HIPCHK(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(k_fill, dim3(grid_1d(n, 256, 4096)), dim3(256), 0, s, (double *)v.p, n,
                       1.0 / std::sqrt((double)n));
    int it = 0;
    int32_t done = 0;
    for (it = 0; it < max_iter && !done; ++it) {
        switch (S->values_dtype) {
        case FC_F64:
            hipLaunchKernelGGL(k_spmv_power<double>, dim3(g), dim3(256), 0, s, S->row_ptr,
                               S->col_idx, (const double *)S->values, (const double *)v.p,
                               (double *)w.p, n, diag_unit, (double *)part.p);
            break;
        case FC_F32:
            hipLaunchKernelGGL(k_spmv_power<float>, dim3(g), dim3(256), 0, s, S->row_ptr,
                               S->col_idx, (const float *)S->values, (const double *)v.p,
                               (double *)w.p, n, diag_unit, (double *)part.p);
            break;
        default:
            hipLaunchKernelGGL(k_spmv_power<__half>, dim3(g), dim3(256), 0, s, S->row_ptr,
                               S->col_idx, (const __half *)S->values, (const double *)v.p,
                               (double *)w.p, n, diag_unit, (double *)part.p);
            break;
        }
        launch_reduce((const double *)part.p, g, 1, 1, (double *)red.p, s);
        hipLaunchKernelGGL(k_power_update, dim3(1), dim3(64), 0, s, (const double *)red.p,
                           (double *)est.p, it, rtol, (int32_t *)flag.p);
        hipLaunchKernelGGL(k_power_scale, dim3(grid_1d(n, 256, 4096)), dim3(256), 0, s,
                           (const double *)w.p, (double *)v.p, n, (const double *)est.p, it,
                           (const int32_t *)flag.p);
        if ((it + 1) % 16 == 0 || it + 1 == max_iter) {
            HIPCHK(hipMemcpyAsync(&done, flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
    }
    HIPCHK(hipGetLastError());
    // the last recorded estimate is est[k] with k = first converged index or it - 1
    std::vector<double> h(it);
    HIPCHK(hipMemcpyAsync(h.data(), est.p, sizeof(double) * it, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int k = it - 1;
    for (int q = 1; q < it; ++q)
        if (h[q] == 0.0 || std::fabs(h[q] - h[q - 1]) <= rtol * h[q]) {
            k = q;
            break;
        }
    *norm_out = h[k];
    if (iters_out)
        *iters_out = k + 1;
    return FC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// solver object
// ---------------------------------------------------------------------------
struct fc_solver {
    int64_t n = 0, nnz = 0;
    int c = 0, cp = 0, cpm = 0;
    fc_precision prec = FC_PREC_FP32;
    fc_diag diag = FC_DIAG_UNIT;
    int accelerate = 1;
    int backtrack = 0;
    const int64_t *row_ptr = nullptr;
    const int32_t *col = nullptr;
    const void *val = nullptr;  // values used by the kernels (maybe owned)
    fc_dtype vdt = FC_F32;
    void *val_owned = nullptr;
    hipStream_t stream = nullptr;
    void *X[3] = {nullptr, nullptr, nullptr};
    void *Z[3] = {nullptr, nullptr, nullptr};
    void *shadow[3] = {nullptr, nullptr, nullptr};
    DevState *d_state = nullptr;
    DevState h = {};
    double *d_GY64 = nullptr;
    void *d_GYs = nullptr;
    double *d_part_fused = nullptr, *d_part_spmm = nullptr, *d_part_gram = nullptr;
    int g_fused = 1, g_spmm = 1, g_gram = 1, g_comb = 0, g_red = 1;
    HeavyPlan heavy;
    Inst inst = {};
    double *d_red_mats = nullptr;
    double *d_sched = nullptr;
    int sched_len = 0;
    double *d_hist_f = nullptr, *d_hist_tau = nullptr, *d_hist_r = nullptr;
    int32_t *d_hist_trials = nullptr;
    int hist_cap = 65536;
    int check_every = 16;
    int max_iter = 100;
    double spec_norm = 0.0, L_thm = 0.0;
    int reorder = FC_REORDER_NONE;
    int defer = 0;              // deferred loss evaluation (fixed steps)
    int single = 0;             // single-pass iteration (fixed steps)
    Inst inst_long = {};        // its sparse-product pre-pass (rows longer than light_max)
    uint64_t perm_hash = 0;     // FNV-1a of a given order (FC_REORDER_GIVEN), else 0
    int32_t *d_perm = nullptr;  // internal row i is user row d_perm[i]
    int32_t *d_inv = nullptr;   // user row j is internal row d_inv[j]
    std::vector<void *> allocs;
    bool pooled = false;  // stream-ordered allocations (serving instances)
    size_t bytes_held = 0;

    ~fc_solver() {
        for (void *p : allocs) {
            if (pooled)
                (void)hipFreeAsync(p, stream);
            else
                (void)hipFree(p);
        }
    }
    template <typename P> hipError_t alloc(P **p, size_t bytes) {
        void *q = nullptr;
        const size_t b = bytes > 0 ? bytes : 16;
        hipError_t e = pooled ? lib_malloc_async(&q, b, stream) : lib_malloc(&q, b);
        if (e == hipSuccess) {
            allocs.push_back(q);
            bytes_held += b;
            *p = (P *)q;
        }
        return e;
    }
};

namespace {

int fused_ne(int cpm) { return 3 * cpm * cpm + FUSED_NSCAL; }

// Launch one trial: fused step -> sparse product of the trial point ->
// reductions -> controller.
template <typename T, typename TU, typename VS, int CP>
fc_status launch_trial_t(fc_solver *h, hipEvent_t *ev) {
    constexpr int CPM = CP < 16 ? 16 : CP;
    hipStream_t s = h->stream;
    const bool shadow = h->prec == FC_PREC_MIXED;
    const Inst &I = h->inst;
    if (ev)
        HIPCHK(hipEventRecord(ev[0], s));
#define FUSED_LAUNCH(A, B, SH) \
    hipLaunchKernelGGL((k_fused_1<T, CP, A, B, SH>), dim3(h->g_fused), dim3(256), 0, s, I)
    if constexpr (std::is_same<T, float>::value) {
        if (shadow) {
            if (h->accelerate && h->backtrack) FUSED_LAUNCH(true, true, true);
            else if (h->accelerate) FUSED_LAUNCH(true, false, true);
            else if (h->backtrack) FUSED_LAUNCH(false, true, true);
            else FUSED_LAUNCH(false, false, true);
        } else {
            if (h->accelerate && h->backtrack) FUSED_LAUNCH(true, true, false);
            else if (h->accelerate) FUSED_LAUNCH(true, false, false);
            else if (h->backtrack) FUSED_LAUNCH(false, true, false);
            else FUSED_LAUNCH(false, false, false);
        }
    } else {
        if (h->accelerate && h->backtrack) FUSED_LAUNCH(true, true, false);
        else if (h->accelerate) FUSED_LAUNCH(true, false, false);
        else if (h->backtrack) FUSED_LAUNCH(false, true, false);
        else FUSED_LAUNCH(false, false, false);
    }
#undef FUSED_LAUNCH
    if (ev)
        HIPCHK(hipEventRecord(ev[1], s));
    launch_spmm<TU, T, T, VS, CP>(I, (int)ROLE_N, s);
    if (ev)
        HIPCHK(hipEventRecord(ev[2], s));
    hipLaunchKernelGGL((k_reduce_fused_1<CPM>), dim3(h->g_red), dim3(256), 0, s, I);
    if (ev)
        HIPCHK(hipEventRecord(ev[3], s));
    hipLaunchKernelGGL((k_control_1<T, CPM>), dim3(1), dim3(256), 0, s, I, 1);
    if (ev)
        HIPCHK(hipEventRecord(ev[4], s));
    HIPCHK(hipGetLastError());
    return FC_OK;
}

// Deferred loss terms of the current iterate: the fused kernel's sums, formed
// by the evaluation pass and reduced into the same entry.
template <typename T, int CP>
void launch_trace_t(fc_solver *h) {
    constexpr int CPM = CP < 16 ? 16 : CP;
    hipLaunchKernelGGL((k_trace_fused<T, CP>), dim3(h->g_fused), dim3(256), 0, h->stream, h->inst);
    hipLaunchKernelGGL((k_reduce_fused_entry<CPM>), dim3(1), dim3(256), 0, h->stream, h->inst,
                       3 * FusedLayout<CPM>::MAT + (int)FS_TRC);
}

template <typename T, int CP>
fc_status launch_eval_t(fc_solver *h) {
    constexpr int CPM = CP < 16 ? 16 : CP;
    launch_trace_t<T, CP>(h);
    hipLaunchKernelGGL((k_control_1<T, CPM>), dim3(1), dim3(256), 0, h->stream, h->inst, 2);
    HIPCHK(hipGetLastError());
    return FC_OK;
}

// Initial evaluation: Gram and product of Xbar_0, then the controller.
template <typename T, typename TU, typename VS, int CP>
fc_status launch_init_t(fc_solver *h) {
    constexpr int CPM = CP < 16 ? 16 : CP;
    hipStream_t s = h->stream;
    const bool shadow = h->prec == FC_PREC_MIXED;
    const int ld = CPM * CPM;
    hipLaunchKernelGGL((k_gram<T, CP>), dim3(h->g_gram), dim3(256), 0, s, (const T *)h->X[0],
                       h->n, h->d_part_gram, (int64_t)ld);
    if (shadow)
        hipLaunchKernelGGL((k_convert<float, __hip_bfloat16>), dim3(grid_1d(h->n * h->cp, 256, 8192)),
                           dim3(256), 0, s, (const float *)h->X[0], (__hip_bfloat16 *)h->shadow[0],
                           h->n * h->cp);
    launch_reduce(h->d_part_gram, (int64_t)h->g_gram * 4, ld, ld, h->d_red_mats, s);
    launch_spmm<TU, T, T, VS, CP>(h->inst, (int)ROLE_C, s);
    if (h->defer)
        launch_trace_t<T, CP>(h);
    hipLaunchKernelGGL((k_control_1<T, CPM>), dim3(1), dim3(256), 0, s, h->inst, 0);
    HIPCHK(hipGetLastError());
    return FC_OK;
}

// The pre-pass of a single-pass iteration: medium and heavy rows of
// S_off Y_n into Z (light rows are summed inside the single-pass kernel).
template <typename T, int CP>
void launch_single_prepass(fc_solver *h) {
    if (h->heavy.nmed + h->heavy.nheavy > 0)
        launch_spmm<T, T, T, T, CP>(h->inst_long, (int)ROLE_P, h->stream);
}

// One single-pass iteration: the pre-pass, the single-pass kernel, the
// reduction, the controller (events: the pre-pass between ev[0] and ev[1],
// the single-pass kernel between ev[1] and ev[2]).
template <typename T, int CP>
fc_status launch_single_t(fc_solver *h, hipEvent_t *ev) {
    constexpr int CPM = CP < 16 ? 16 : CP;
    hipStream_t s = h->stream;
    const Inst &I = h->inst;
    if (ev)
        HIPCHK(hipEventRecord(ev[0], s));
    launch_single_prepass<T, CP>(h);
    if (ev)
        HIPCHK(hipEventRecord(ev[1], s));
    if (h->accelerate)
        hipLaunchKernelGGL((k_single_1<T, CP, true>), dim3(h->g_fused), dim3(256), 0, s, I);
    else
        hipLaunchKernelGGL((k_single_1<T, CP, false>), dim3(h->g_fused), dim3(256), 0, s, I);
    if (ev)
        HIPCHK(hipEventRecord(ev[2], s));
    hipLaunchKernelGGL((k_reduce_fused_1<CPM>), dim3(h->g_red), dim3(256), 0, s, I);
    if (ev)
        HIPCHK(hipEventRecord(ev[3], s));
    hipLaunchKernelGGL((k_control_1<T, CPM>), dim3(1), dim3(256), 0, s, I, 1);
    if (ev)
        HIPCHK(hipEventRecord(ev[4], s));
    HIPCHK(hipGetLastError());
    return FC_OK;
}

// Loss of the current iterate of a single-pass solver: its Gram matrix and
// S_eff Xbar with the terms <x_i, (S_eff X)_i>, then the controller.
template <typename T, int CP>
fc_status launch_single_eval_t(fc_solver *h) {
    constexpr int CPM = CP < 16 ? 16 : CP;
    hipStream_t s = h->stream;
    const int ld = CPM * CPM;
    const T *Xbar = (const T *)h->X[h->h.role[ROLE_C]];   // the iterate being read out
    hipLaunchKernelGGL((k_gram<T, CP>), dim3(h->g_gram), dim3(256), 0, s, Xbar, h->n, h->d_part_gram,
                       (int64_t)ld);
    launch_reduce(h->d_part_gram, (int64_t)h->g_gram * 4, ld, ld, h->d_red_mats, s);
    // only the loss terms of the read-out iterate are needed: a symmetric S
    // gives them from its entries on and below the diagonal, in one flat pass
    // over the nonzeros (half the gathers; the controller doubles the sum)
    // (a persistent grid of 16 workgroups per CU over chunks of nonzeros; the
    // controller sums that many partials)
    Inst I = h->inst;
    const int64_t chunks = cdiv(h->nnz, LOSS_CHUNK);
    int64_t g_loss = std::min<int64_t>((int64_t)device_cus() * 16, cdiv(chunks, 256 / TeamCfg<T, CP, 1>::GS));
    g_loss = std::max<int64_t>(1, std::min<int64_t>(g_loss, (int64_t)I.g_spmm + I.g_comb));   // partial slots held
    hipLaunchKernelGGL((k_loss_lower<T, CP>), dim3((unsigned)g_loss), dim3(256), 0, s, I.row_ptr, I.col,
                       (const T *)I.val, Xbar, I.n, h->nnz, I.part_spmm);
    I.g_spmm = (int32_t)g_loss;
    I.g_comb = 0;
    hipLaunchKernelGGL((k_control_1<T, CPM>), dim3(1), dim3(256), 0, s, I, 3);
    HIPCHK(hipGetLastError());
    return FC_OK;
}

fc_status launch_trial(fc_solver *h, hipEvent_t *ev = nullptr) {
    return with_cp(h->cp, [&](auto cpc) -> fc_status {
        constexpr int CP = decltype(cpc)::value;
        if (h->single)
            return h->prec == FC_PREC_FP64 ? launch_single_t<double, CP>(h, ev)
                                           : launch_single_t<float, CP>(h, ev);
        if (h->prec == FC_PREC_FP64)
            return launch_trial_t<double, double, double, CP>(h, ev);
        if (h->prec == FC_PREC_FP32)
            return launch_trial_t<float, float, float, CP>(h, ev);
        if constexpr (CP >= 8)
            return launch_trial_t<float, __hip_bfloat16, __half, CP>(h, ev);
        return fail(FC_ERR_UNSUPPORTED, "mixed precision needs c >= 5 (padded width >= 8)");
    });
}

fc_status launch_eval(fc_solver *h) {
    return with_cp(h->cp, [&](auto cpc) -> fc_status {
        constexpr int CP = decltype(cpc)::value;
        if (h->single)
            return h->prec == FC_PREC_FP64 ? launch_single_eval_t<double, CP>(h)
                                           : launch_single_eval_t<float, CP>(h);
        if (h->prec == FC_PREC_FP64)
            return launch_eval_t<double, CP>(h);
        return launch_eval_t<float, CP>(h);
    });
}

fc_status launch_init(fc_solver *h) {
    return with_cp(h->cp, [&](auto cpc) -> fc_status {
        constexpr int CP = decltype(cpc)::value;
        if (h->prec == FC_PREC_FP64)
            return launch_init_t<double, double, double, CP>(h);
        if (h->prec == FC_PREC_FP32)
            return launch_init_t<float, float, float, CP>(h);
        if constexpr (CP >= 8)
            return launch_init_t<float, __hip_bfloat16, __half, CP>(h);
        return fail(FC_ERR_UNSUPPORTED, "mixed precision needs c >= 5 (padded width >= 8)");
    });
}

fc_status read_state(fc_solver *h) {
    HIPCHK(hipMemcpyAsync(&h->h, h->d_state, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return FC_OK;
}

fc_status write_state(fc_solver *h) {
    HIPCHK(hipMemcpyAsync(h->d_state, &h->h, sizeof(DevState), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return FC_OK;
}

void fill_info(const fc_solver *h, fc_info *info) {
    if (!info)
        return;
    info->iter = h->h.iter;
    info->trials = h->h.trials;
    info->stop_reason = h->h.stop_reason;
    info->reserved = 0;
    info->f = h->h.f;
    info->f_prev = h->h.f_prev;
    info->L = h->h.iter > 0 || h->backtrack ? h->h.L : 1.0 / h->h.tau;
    info->t = h->h.t;
    info->beta = h->h.beta;   // the weight that forms Y_{iter+1}
    info->pgrad = h->h.r;
    info->pgrad_rel = h->h.r1 > 0.0 ? h->h.r / h->h.r1 : 0.0;
}

fc_status status_of(const fc_solver *h) {
    if (h->h.error == ERR_NONFINITE)
        return fail(FC_ERR_NONFINITE, "the objective or an iterate became non-finite");
    if (h->h.error == ERR_STEP)
        return fail(FC_ERR_STEP, "backtracking found no acceptable step (L overflow or 1000 trials)");
    return FC_OK;
}

// Events of a profiled run: five per trial, released at the end.
struct EventLog {
    std::vector<hipEvent_t> ev;
    fc_kernel_times *out = nullptr;
    bool single = false;   // slot 0 is the pre-pass (a sparse product), slot 1 the fused pass
    ~EventLog() {
        for (hipEvent_t e : ev)
            (void)hipEventDestroy(e);
    }
    hipError_t add_trial(hipEvent_t **slot) {
        const size_t k = ev.size();
        ev.resize(k + 5, nullptr);
        for (size_t q = k; q < k + 5; ++q) {
            hipError_t e = hipEventCreate(&ev[q]);
            if (e != hipSuccess)
                return e;
        }
        *slot = &ev[k];
        return hipSuccess;
    }
    hipError_t collect() {
        if (!out)
            return hipSuccess;
        std::memset(out, 0, sizeof(*out));
        for (size_t k = 0; k + 5 <= ev.size(); k += 5) {
            float ms[4];
            for (int q = 0; q < 4; ++q) {
                hipError_t e = hipEventElapsedTime(&ms[q], ev[k + q], ev[k + q + 1]);
                if (e != hipSuccess)
                    return e;
            }
            out->fused_ms += single ? ms[1] : ms[0];
            out->spmm_ms += single ? ms[0] : ms[1];
            out->reduce_ms += ms[2];
            out->control_ms += ms[3];
            out->launches += 1;
        }
        return hipSuccess;
    }
};

// Run until `target` accepted iterations (or a stop) with the given budget.
fc_status run_until(fc_solver *h, int32_t target, int32_t max_iter, EventLog *log = nullptr) {
    if (h->h.error != ERR_NONE)
        return status_of(h);
    h->h.target = target;
    h->h.max_iter = max_iter;
    h->h.active = h->h.iter < target && h->h.iter < max_iter ? 1 : 0;
    if (h->h.active)
        h->h.stop_reason = STOP_NONE;
    fc_status st = write_state(h);
    if (st != FC_OK)
        return st;
    while (h->h.active) {
        TraceRange trace_range("trials and state readback");
        int launches = h->backtrack ? h->check_every : (target - h->h.iter);
        if (launches < 1)
            launches = 1;
        for (int k = 0; k < launches; ++k) {
            hipEvent_t *ev = nullptr;
            if (log)
                HIPCHK(log->add_trial(&ev));
            st = launch_trial(h, ev);
            if (st != FC_OK)
                return st;
        }
        st = read_state(h);
        if (st != FC_OK)
            return st;
    }
    if (log)
        HIPCHK(log->collect());
    if ((h->defer || h->single) && !h->h.f_known && h->h.error == ERR_NONE) {
        // the loss of the last accepted iterate
        TraceRange trace_range("loss read-out");
        st = launch_eval(h);
        if (st == FC_OK)
            st = read_state(h);
        if (st != FC_OK)
            return st;
    }
    return status_of(h);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void fc_options_default(fc_options *opt) {
    if (!opt)
        return;
    std::memset(opt, 0, sizeof(*opt));
    opt->struct_size = sizeof(fc_options);
    opt->c = 0;
    opt->precision = FC_PREC_FP32;
    opt->diag = FC_DIAG_UNIT;
    opt->accelerate = 1;
    opt->step_rule = FC_STEP_FIXED;
    opt->step = 0.0;
    opt->L0 = 0.0;
    opt->eta = 2.0;
    opt->max_iter = 100;
    opt->check_every = 16;
    opt->tol_loss = std::nan("");
    opt->tol_pgrad = 0.0;
    opt->validate = 0;
    opt->step_schedule = nullptr;
    opt->step_schedule_len = 0;
}

const char *fc_last_error(void) { return g_last_error.c_str(); }

void fc_debug_fail_allocations(int64_t after) { g_alloc_countdown.store(after < 0 ? -1 : after); }

}  // extern "C"

namespace {

// Set-up shared by fc_create and the serving engine: `hist_cap` iterations
// of history, allocations from the stream-ordered pool when `pooled`.
// Renumber the articles: by descending degree (FC_REORDER_DEGREE), where a
// stable radix sort of the complemented row lengths gives perm, or in the
// caller's order `given` (FC_REORDER_GIVEN, a host array already checked to be
// a permutation); then the permuted CSR is written into library-owned arrays
// with values of type vdt_out.
fc_status build_order(fc_solver *h, const fc_csr *S, fc_dtype vdt_out, const int32_t *given,
                      hipStream_t s) {
    const int64_t n = S->n, nnz = S->nnz;
    if (n > (int64_t)INT32_MAX)
        return fail(FC_ERR_UNSUPPORTED, "relabelling needs n < 2^31");
    int64_t *rp_new = nullptr;
    int32_t *col_new = nullptr;
    void *val_new = nullptr;
    const size_t vbytes = vdt_out == FC_F64 ? 8 : (vdt_out == FC_F32 ? 4 : 2);
    if (h->alloc(&h->d_perm, sizeof(int32_t) * n) != hipSuccess ||
        h->alloc(&h->d_inv, sizeof(int32_t) * n) != hipSuccess ||
        h->alloc(&rp_new, sizeof(int64_t) * (n + 1)) != hipSuccess ||
        h->alloc(&col_new, sizeof(int32_t) * nnz) != hipSuccess ||
        h->alloc(&val_new, vbytes * nnz) != hipSuccess)
        return fail(FC_ERR_OUT_OF_MEMORY, "relabelled copy of S");
    DevBuf keys, keys_out, ids, len, tmp;
    if (dev_alloc(len, sizeof(int64_t) * n, s) != hipSuccess)
        return fail(FC_ERR_OUT_OF_MEMORY, "relabelling scratch");
    const int g = grid_1d(n, 256, 16384);
    size_t sort_bytes = 0, scan_bytes = 0;
    if (!given) {
        if (dev_alloc(keys, sizeof(uint32_t) * n, s) != hipSuccess ||
            dev_alloc(keys_out, sizeof(uint32_t) * n, s) != hipSuccess ||
            dev_alloc(ids, sizeof(int32_t) * n, s) != hipSuccess)
            return fail(FC_ERR_OUT_OF_MEMORY, "relabelling scratch");
        hipLaunchKernelGGL(k_degree_keys, dim3(g), dim3(256), 0, s, S->row_ptr, n, (uint32_t *)keys.p,
                           (int32_t *)ids.p);
        HIPCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (const uint32_t *)keys.p,
                                                  (uint32_t *)keys_out.p, (const int32_t *)ids.p,
                                                  h->d_perm, (int)n, 0, 32, s));
    }
    HIPCHK(hipcub::DeviceScan::InclusiveSum(nullptr, scan_bytes, (const int64_t *)len.p, rp_new + 1,
                                            (int)n, s));
    if (dev_alloc(tmp, std::max(sort_bytes, scan_bytes), s) != hipSuccess)
        return fail(FC_ERR_OUT_OF_MEMORY, "relabelling scratch");
    if (given) {   // the caller's array is read before fc_create goes on
        HIPCHK(hipMemcpyAsync(h->d_perm, given, sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    } else {
        HIPCHK(hipcub::DeviceRadixSort::SortPairs(tmp.p, sort_bytes, (const uint32_t *)keys.p,
                                                  (uint32_t *)keys_out.p, (const int32_t *)ids.p,
                                                  h->d_perm, (int)n, 0, 32, s));
    }
    hipLaunchKernelGGL(k_perm_lengths, dim3(g), dim3(256), 0, s, S->row_ptr, h->d_perm, n, h->d_inv,
                       (int64_t *)len.p);
    HIPCHK(hipMemsetAsync(rp_new, 0, sizeof(int64_t), s));
    HIPCHK(hipcub::DeviceScan::InclusiveSum(tmp.p, scan_bytes, (const int64_t *)len.p, rp_new + 1,
                                            (int)n, s));
    const int gw = grid_1d(n, 4, 65536);
    const bool to_half = vdt_out == FC_F16;
    if (S->values_dtype == FC_F64)
        hipLaunchKernelGGL((k_permute_csr<double, double>), dim3(gw), dim3(256), 0, s, S->row_ptr,
                           S->col_idx, (const double *)S->values, h->d_perm, h->d_inv, rp_new, n, col_new,
                           (double *)val_new);
    else if (S->values_dtype == FC_F32 && !to_half)
        hipLaunchKernelGGL((k_permute_csr<float, float>), dim3(gw), dim3(256), 0, s, S->row_ptr,
                           S->col_idx, (const float *)S->values, h->d_perm, h->d_inv, rp_new, n, col_new,
                           (float *)val_new);
    else if (S->values_dtype == FC_F32)
        hipLaunchKernelGGL((k_permute_csr<float, __half>), dim3(gw), dim3(256), 0, s, S->row_ptr,
                           S->col_idx, (const float *)S->values, h->d_perm, h->d_inv, rp_new, n, col_new,
                           (__half *)val_new);
    else
        hipLaunchKernelGGL((k_permute_csr<__half, __half>), dim3(gw), dim3(256), 0, s, S->row_ptr,
                           S->col_idx, (const __half *)S->values, h->d_perm, h->d_inv, rp_new, n, col_new,
                           (__half *)val_new);
    HIPCHK(hipGetLastError());
    h->row_ptr = rp_new;
    h->col = col_new;
    h->val = val_new;
    h->vdt = vdt_out;
    h->reorder = given ? FC_REORDER_GIVEN : FC_REORDER_DEGREE;
    return FC_OK;
}

fc_status create_impl(const fc_csr *S, const fc_options *opt, const void *U0, fc_dtype u0_dtype,
                      hipStream_t stream, int hist_cap, bool pooled, fc_solver **out) {
    if (!out)
        return fail(FC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    fc_status st = check_csr_args(S);
    if (st != FC_OK)
        return st;
    if (!opt || opt->struct_size != sizeof(fc_options))
        return fail(FC_ERR_INVALID_ARG, "options missing or struct_size mismatch (call fc_options_default)");
    if (opt->c < 1 || opt->c > 64)
        return fail(FC_ERR_INVALID_ARG, "c must be in [1, 64]");
    if (opt->precision != FC_PREC_FP64 && opt->precision != FC_PREC_FP32 &&
        opt->precision != FC_PREC_MIXED)
        return fail(FC_ERR_INVALID_ARG, "unknown precision");
    if (opt->diag != FC_DIAG_STORED && opt->diag != FC_DIAG_UNIT)
        return fail(FC_ERR_INVALID_ARG, "unknown diagonal mode");
    if (opt->step_rule != FC_STEP_FIXED && opt->step_rule != FC_STEP_BACKTRACK)
        return fail(FC_ERR_INVALID_ARG, "unknown step rule");
    if (opt->step_rule == FC_STEP_BACKTRACK && !(opt->eta > 1.0))
        return fail(FC_ERR_INVALID_ARG, "eta must be > 1");
    if (opt->max_iter < 0)
        return fail(FC_ERR_INVALID_ARG, "max_iter < 0");
    if (opt->step_schedule && opt->step_schedule_len < 1)
        return fail(FC_ERR_INVALID_ARG, "step_schedule_len must be >= 1");
    if (opt->norm_estimate != 0 && opt->norm_estimate != 1)
        return fail(FC_ERR_INVALID_ARG, "norm_estimate must be 0 or 1");
    if (opt->reorder != FC_REORDER_NONE && opt->reorder != FC_REORDER_DEGREE &&
        opt->reorder != FC_REORDER_GIVEN)
        return fail(FC_ERR_INVALID_ARG, "unknown reorder mode");
    uint64_t perm_hash = 0;
    if (opt->reorder == FC_REORDER_GIVEN) {   // checked before any device work reads it
        if (!opt->perm)
            return fail(FC_ERR_INVALID_ARG, "FC_REORDER_GIVEN needs options.perm");
        if (S->n > (int64_t)INT32_MAX)
            return fail(FC_ERR_UNSUPPORTED, "relabelling needs n < 2^31");
        int64_t bad = 0;
        const int pc = check_permutation(opt->perm, S->n, &bad);
        if (pc != PERM_OK)
            return fail(FC_ERR_INVALID_ARG,
                        "perm is not a permutation of the rows: entry " + std::to_string(bad) +
                            (pc == PERM_RANGE ? " is outside 0..n-1" : " repeats an earlier entry"));
        perm_hash = order_fingerprint(opt->perm, S->n);
    }
    if (opt->defer_loss != 0 && opt->defer_loss != 1)
        return fail(FC_ERR_INVALID_ARG, "defer_loss must be 0 or 1");
    if (opt->defer_loss && opt->step_rule != FC_STEP_FIXED)
        return fail(FC_ERR_INVALID_ARG, "defer_loss needs FC_STEP_FIXED (backtracking tests each trial's loss)");
    if (U0 && u0_dtype != FC_F64 && u0_dtype != FC_F32)
        return fail(FC_ERR_INVALID_ARG, "U0 must be FC_F64 or FC_F32");
    if (opt->precision == FC_PREC_FP64 && S->values_dtype != FC_F64)
        return fail(FC_ERR_INVALID_ARG, "FP64 precision needs FC_F64 values");
    if (opt->precision == FC_PREC_FP32 && S->values_dtype != FC_F32)
        return fail(FC_ERR_INVALID_ARG, "FP32 precision needs FC_F32 values");
    if (opt->precision == FC_PREC_MIXED && S->values_dtype == FC_F64)
        return fail(FC_ERR_INVALID_ARG, "mixed precision needs FC_F32 or FC_F16 values");
    if (opt->precision == FC_PREC_MIXED && cp_of(opt->c) < 8)
        return fail(FC_ERR_UNSUPPORTED, "mixed precision needs c >= 5");

    fc_solver *h = new (std::nothrow) fc_solver();
    if (!h)
        return fail(FC_ERR_OUT_OF_MEMORY, "host allocation failed");
    auto cleanup = [&](fc_status s) {
        delete h;
        return s;
    };
    h->n = S->n;
    h->nnz = S->nnz;
    h->c = opt->c;
    h->cp = cp_of(opt->c);
    h->cpm = cpm_of(h->cp);
    h->prec = opt->precision;
    h->diag = opt->diag;
    h->accelerate = opt->accelerate ? 1 : 0;
    h->backtrack = opt->step_rule == FC_STEP_BACKTRACK ? 1 : 0;
    h->row_ptr = S->row_ptr;
    h->col = S->col_idx;
    h->val = S->values;
    h->vdt = S->values_dtype;
    h->stream = stream;
    h->pooled = pooled;
    h->hist_cap = hist_cap;
    h->check_every = opt->check_every > 0 ? opt->check_every : 16;
    h->defer = opt->defer_loss ? 1 : 0;
    h->single = opt->single_pass ? 1 : 0;
    h->max_iter = opt->max_iter;
    if (h->single) {
        if (h->backtrack)
            return cleanup(fail(FC_ERR_UNSUPPORTED, "the single-pass iteration takes constant or scheduled steps"));
        if (h->prec == FC_PREC_MIXED)
            return cleanup(fail(FC_ERR_UNSUPPORTED, "the single-pass iteration runs in FP64 or FP32"));
        if (opt->tol_loss == opt->tol_loss)
            return cleanup(fail(FC_ERR_UNSUPPORTED, "the single-pass iteration has no per-iteration loss (tol_loss must be NaN)"));
        h->defer = 0;
    }
    hipStream_t s = h->stream;

    if (opt->validate) {
        // row_ptr on the host first: the entry checks below index rows by it
        std::vector<int64_t> rp(S->n + 1);
        if (hipMemcpyAsync(rp.data(), S->row_ptr, sizeof(int64_t) * (S->n + 1), hipMemcpyDeviceToHost,
                           s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return cleanup(fail(FC_ERR_DEVICE, "validation: row_ptr readback"));
        int64_t bad = 0;
        const int rpc = check_row_ptr(rp.data(), S->n, S->nnz, &bad);
        if (rpc != RP_OK)
            return cleanup(fail(FC_ERR_NOT_SYMMETRIC,
                                std::string("CSR structure invalid: row_ptr ") +
                                    (rpc == RP_FIRST ? "does not start at 0"
                                     : rpc == RP_DECREASING ? "decreases after row " + std::to_string(bad)
                                                            : "does not end at nnz")));
        int32_t *flags = nullptr;
        if (h->alloc(&flags, sizeof(int32_t)) != hipSuccess)
            return cleanup(fail(FC_ERR_OUT_OF_MEMORY, "validation buffer"));
        if (hipMemsetAsync(flags, 0, sizeof(int32_t), s) != hipSuccess)
            return cleanup(fail(FC_ERR_DEVICE, "memset"));
        const int g = grid_1d(S->n, 256, 8192);
        if (S->values_dtype == FC_F64)
            hipLaunchKernelGGL(k_check_csr<double>, dim3(g), dim3(256), 0, s, S->row_ptr, S->col_idx,
                               (const double *)S->values, S->n, S->nnz, (int)(opt->diag == FC_DIAG_UNIT),
                               1, flags);
        else if (S->values_dtype == FC_F32)
            hipLaunchKernelGGL(k_check_csr<float>, dim3(g), dim3(256), 0, s, S->row_ptr, S->col_idx,
                               (const float *)S->values, S->n, S->nnz, (int)(opt->diag == FC_DIAG_UNIT),
                               1, flags);
        else
            hipLaunchKernelGGL(k_check_csr<__half>, dim3(g), dim3(256), 0, s, S->row_ptr, S->col_idx,
                               (const __half *)S->values, S->n, S->nnz, (int)(opt->diag == FC_DIAG_UNIT),
                               1, flags);
        int32_t hf = 0;
        if (hipMemcpyAsync(&hf, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return cleanup(fail(FC_ERR_DEVICE, "validation readback"));
        if (hf & 2)
            return cleanup(fail(FC_ERR_NOT_SYMMETRIC, "CSR structure invalid: col_idx out of range"));
        if (hf & 4)
            return cleanup(fail(FC_ERR_INVALID_ARG, "FC_DIAG_UNIT requires no stored diagonal entries"));
        if (hf & 8)
            return cleanup(fail(FC_ERR_NOT_SYMMETRIC, "validation needs sorted, duplicate-free rows"));
        if (hf & 16)
            return cleanup(fail(FC_ERR_NOT_SYMMETRIC, "S is not symmetric"));
    }

    const size_t esz = h->prec == FC_PREC_FP64 ? 8 : 4;
    const size_t mat_bytes = (size_t)h->n * h->cp * esz;
    for (int k = 0; k < 3; ++k) {
        // the single-pass iteration keeps one product buffer: the long rows
        // of S Y_n within an iteration, S Xbar at a read-out
        if (h->single && k > 0) {
            if (h->alloc(&h->X[k], mat_bytes) != hipSuccess)
                return cleanup(fail(FC_ERR_OUT_OF_MEMORY, "iterate buffers"));
            h->Z[k] = h->Z[0];
            continue;
        }
        if (h->alloc(&h->X[k], mat_bytes) != hipSuccess || h->alloc(&h->Z[k], mat_bytes) != hipSuccess)
            return cleanup(fail(FC_ERR_OUT_OF_MEMORY, "iterate buffers"));
        if (h->prec == FC_PREC_MIXED &&
            h->alloc(&h->shadow[k], (size_t)h->n * h->cp * 2) != hipSuccess)
            return cleanup(fail(FC_ERR_OUT_OF_MEMORY, "bfloat16 shadow buffers"));
    }
    // the ring slots the set-up does not write start as zeros (a checkpoint
    // taken before they are first written then holds no unwritten memory)
    for (int k = 1; k < 3; ++k) {
        if (hipMemsetAsync(h->X[k], 0, mat_bytes, s) != hipSuccess ||
            (h->Z[k] != h->Z[0] && hipMemsetAsync(h->Z[k], 0, mat_bytes, s) != hipSuccess) ||
            (h->shadow[k] && hipMemsetAsync(h->shadow[k], 0, (size_t)h->n * h->cp * 2, s) != hipSuccess))
            return cleanup(fail(FC_ERR_DEVICE, "clearing the iterate buffers"));
    }
    if (opt->reorder == FC_REORDER_DEGREE || opt->reorder == FC_REORDER_GIVEN) {
        const fc_dtype vout = h->prec == FC_PREC_MIXED ? FC_F16 : S->values_dtype;
        st = build_order(h, S, vout, opt->reorder == FC_REORDER_GIVEN ? opt->perm : nullptr, s);
        if (st != FC_OK)
            return cleanup(st);
        h->perm_hash = perm_hash;
    } else if (h->prec == FC_PREC_MIXED && S->values_dtype == FC_F32) {
        if (h->alloc(&h->val_owned, (size_t)S->nnz * 2) != hipSuccess)
            return cleanup(fail(FC_ERR_OUT_OF_MEMORY, "half copy of S"));
        hipLaunchKernelGGL((k_convert<float, __half>), dim3(grid_1d(S->nnz, 256, 8192)), dim3(256), 0, s,
                           (const float *)S->values, (__half *)h->val_owned, S->nnz);
        h->val = h->val_owned;
        h->vdt = FC_F16;
    }
    if (h->alloc(&h->d_state, sizeof(DevState)) != hipSuccess ||
        h->alloc(&h->d_GY64, sizeof(double) * h->cpm * h->cpm) != hipSuccess ||
        h->alloc(&h->d_GYs, esz * h->cpm * h->cpm) != hipSuccess)
        return cleanup(fail(FC_ERR_OUT_OF_MEMORY, "solver state"));

    // launch geometry: persistent grids sized to the device (the fused
    // kernel's count by the rule served instances share)
    const int cus = device_cus();
    h->g_fused = (int)fused_grid(h->n, cus);
    h->g_gram = grid_1d(cdiv(h->n, 16), 4, (int64_t)cus * 2);
    {
        int rows_per_wg = 1;
        with_cp(h->cp, [&](auto cpc) -> fc_status {
            constexpr int CP = decltype(cpc)::value;
            if (h->prec == FC_PREC_FP64)
                rows_per_wg = SpmmCfg<double, CP>::ROWS_PER_WG;
            else if (h->prec == FC_PREC_FP32)
                rows_per_wg = SpmmCfg<float, CP>::ROWS_PER_WG;
            else
                rows_per_wg = SpmmCfg<__hip_bfloat16, CP>::ROWS_PER_WG;
            return FC_OK;
        });
        // persistent workgroups per CU (measured 28.3 vs 29.0 ms at n = 7e7,
        // c = 32, with 1024 instead of 64 per CU; the controller sums the
        // workgroups' loss partials, when there are any, in about 0.1 ms)
        h->g_spmm = grid_1d(h->n, rows_per_wg, (int64_t)cus * 1024);
    }
    st = build_heavy_plan(h->row_ptr, S->n, h->prec == FC_PREC_FP64 ? 8 : 4, h->cp, s, h->heavy);
    if (st != FC_OK)
        return cleanup(st);
    h->g_comb = combine_grid(h->heavy.nheavy, 256 / h->cp);
    h->g_red = (int)cdiv(fused_ne(h->cpm), FUSED_RED_EB);
    const int ne = fused_ne(h->cpm);
    if (h->alloc(&h->d_part_fused, sizeof(double) * (size_t)h->g_fused * ne) != hipSuccess ||
        h->alloc(&h->d_part_spmm, sizeof(double) * (size_t)(h->g_spmm + h->g_comb)) != hipSuccess ||
        h->alloc(&h->d_part_gram, sizeof(double) * (size_t)h->g_gram * 4 * h->cpm * h->cpm) != hipSuccess ||
        h->alloc(&h->d_red_mats, sizeof(double) * ne) != hipSuccess ||
        h->alloc(&h->d_hist_f, sizeof(double) * h->hist_cap) != hipSuccess ||
        h->alloc(&h->d_hist_tau, sizeof(double) * h->hist_cap) != hipSuccess ||
        h->alloc(&h->d_hist_r, sizeof(double) * h->hist_cap) != hipSuccess ||
        h->alloc(&h->d_hist_trials, sizeof(int32_t) * h->hist_cap) != hipSuccess)
        return cleanup(fail(FC_ERR_OUT_OF_MEMORY, "partial-sum buffers"));
    {
        Inst &I = h->inst;
        I.row_ptr = h->row_ptr;
        I.col = h->col;
        I.val = h->val;
        I.n = h->n;
        I.c = h->c;
        I.diag_unit = h->diag == FC_DIAG_UNIT ? 1 : 0;
        plan_to_inst(h->heavy, I);
        for (int k = 0; k < 3; ++k) {
            I.X[k] = h->X[k];
            I.Z[k] = h->Z[k];
            I.Sh[k] = h->shadow[k];
        }
        I.st = h->d_state;
        I.GY64 = h->d_GY64;
        I.GYs = h->d_GYs;
        I.part_fused = h->d_part_fused;
        I.part_spmm = h->d_part_spmm;
        I.red_mats = h->d_red_mats;
        I.g_fused = h->g_fused;
        I.g_spmm = h->g_spmm;
        I.g_comb = h->g_comb;
        I.g_red = h->g_red;
        I.hist_f = h->d_hist_f;
        I.hist_tau = h->d_hist_tau;
        I.hist_r = h->d_hist_r;
        I.hist_trials = h->d_hist_trials;
        I.sched = nullptr;
        I.defer = h->defer;
        I.pass_kind = h->single ? PASS_SINGLE : PASS_DEFAULT;
        // relabelled FP32 instances whose rows fill whole 128-byte lines: the
        // rows past the first 256 MB of X (the size of MI355X's Infinity
        // Cache; the most-gathered rows come first) are gathered
        // non-temporally, which keeps the cache for the hot rows (27.3 ->
        // 26.7 ms at n = 7e7, c = 32; 1, 4 and 8 times the size: 26.8, 26.9,
        // 27.2 ms).  Rows that share a line (64-byte bfloat16 rows) measured
        // slower with the hint.
        const int64_t cache_rows = (int64_t)(256ll << 20) / ((int64_t)h->cp * 4);
        I.nt_from = h->reorder == FC_REORDER_DEGREE && h->prec == FC_PREC_FP32 && h->cp >= 32 &&
                            cache_rows < h->n
                        ? cache_rows
                        : 0;
    }
    if (h->single) {   // the pre-pass: stored products of the long rows only
        h->inst_long = h->inst;
        h->inst_long.defer = 1;
        h->inst_long.pass_kind = PASS_LONG;
    }
    if (hipMemsetAsync(h->d_red_mats, 0, sizeof(double) * ne, s) != hipSuccess ||
        hipMemsetAsync(h->d_hist_trials, 0, sizeof(int32_t) * h->hist_cap, s) != hipSuccess)
        return cleanup(fail(FC_ERR_DEVICE, "memset"));
    if (opt->step_schedule) {
        h->sched_len = opt->step_schedule_len;
        if (h->alloc(&h->d_sched, sizeof(double) * h->sched_len) != hipSuccess)
            return cleanup(fail(FC_ERR_OUT_OF_MEMORY, "step schedule"));
        if (hipMemcpyAsync(h->d_sched, opt->step_schedule, sizeof(double) * h->sched_len,
                           hipMemcpyHostToDevice, s) != hipSuccess)
            return cleanup(fail(FC_ERR_DEVICE, "step schedule copy"));
        for (int k = 0; k < h->sched_len; ++k)
            if (!(opt->step_schedule[k] > 0.0))
                return cleanup(fail(FC_ERR_INVALID_ARG, "step schedule entries must be > 0"));
        h->inst.sched = h->d_sched;
        h->inst_long.sched = h->d_sched;
    }

    // Xbar_0 (the other two ring slots start as copies of it)
    for (int k = 0; k < 3; ++k) {
        const int g = grid_1d((int64_t)h->n * h->cp, 256, 8192);
        if (h->prec == FC_PREC_FP64) {
            if (!U0 || u0_dtype == FC_F64)
                hipLaunchKernelGGL((k_pad_copy<double, double>), dim3(g), dim3(256), 0, s,
                                   (const double *)U0, (int64_t)h->c, (double *)h->X[k], h->n, h->c, h->cp,
                                   (const int32_t *)h->d_perm);
            else
                hipLaunchKernelGGL((k_pad_copy<float, double>), dim3(g), dim3(256), 0, s,
                                   (const float *)U0, (int64_t)h->c, (double *)h->X[k], h->n, h->c, h->cp,
                                   (const int32_t *)h->d_perm);
        } else {
            if (!U0 || u0_dtype == FC_F32)
                hipLaunchKernelGGL((k_pad_copy<float, float>), dim3(g), dim3(256), 0, s,
                                   (const float *)U0, (int64_t)h->c, (float *)h->X[k], h->n, h->c, h->cp,
                                   (const int32_t *)h->d_perm);
            else
                hipLaunchKernelGGL((k_pad_copy<double, float>), dim3(g), dim3(256), 0, s,
                                   (const double *)U0, (int64_t)h->c, (float *)h->X[k], h->n, h->c, h->cp,
                                   (const int32_t *)h->d_perm);
        }
        if (hipMemsetAsync(h->Z[k], 0, mat_bytes, s) != hipSuccess)
            return cleanup(fail(FC_ERR_DEVICE, "memset"));
    }
    if (hipGetLastError() != hipSuccess)
        return cleanup(fail(FC_ERR_DEVICE, "start-point copy launch"));

    // ||S_eff||_F^2 and the step bound of Theorem 3.1
    double s2 = 0.0;
    fc_csr Sv = *S;
    Sv.row_ptr = h->row_ptr;
    Sv.col_idx = h->col;
    Sv.values = h->val;
    Sv.values_dtype = h->vdt;
    st = sum_squares(&Sv, s, &s2);
    if (st != FC_OK)
        return cleanup(st);
    if (h->diag == FC_DIAG_UNIT)
        s2 += (double)h->n;
    const bool need_L = (!h->backtrack && !(opt->step > 0.0) && !opt->step_schedule) ||
                        (h->backtrack && !(opt->L0 > 0.0));
    if (need_L) {
        if (opt->norm_estimate == 1) {
            h->spec_norm = std::sqrt(s2);   // ||S_eff||_F >= ||S_eff||_2
        } else {
            int32_t its = 0;
            st = power_norm(&Sv, (int)(h->diag == FC_DIAG_UNIT), 1000, 1e-12, s, &h->spec_norm, &its);
            if (st != FC_OK)
                return cleanup(st);
        }
        h->L_thm = 4.0 * h->spec_norm + 12.0 * (double)h->n;
    }

    DevState &d = h->h;
    std::memset(&d, 0, sizeof(d));
    d.role[ROLE_C] = 0;
    d.role[ROLE_P] = 1;
    d.role[ROLE_N] = 2;
    d.active = 1;
    d.target = 0;
    d.max_iter = INT_MAX;
    d.accelerate = h->accelerate;
    d.backtrack = h->backtrack;
    d.defer = h->defer;
    d.f_known = 1;
    d.c = h->c;
    d.hist_cap = h->hist_cap;
    d.sched_len = h->sched_len;
    d.t = 1.0;
    d.beta = 0.0;
    d.beta_next = 0.0;
    d.s2 = s2;
    d.tol_loss = opt->tol_loss;
    d.tol_pgrad = opt->tol_pgrad;
    d.eta = opt->eta > 1.0 ? opt->eta : 2.0;
    if (h->backtrack) {
        d.L = opt->L0 > 0.0 ? opt->L0 : h->L_thm / 100.0;
        d.tau = 1.0 / d.L;
    } else {
        d.tau0 = opt->step_schedule ? opt->step_schedule[0] : (opt->step > 0.0 ? opt->step : 1.0 / h->L_thm);
        d.tau = d.tau0;
        d.L = 1.0 / d.tau;
    }
    st = write_state(h);
    if (st != FC_OK)
        return cleanup(st);
    st = launch_init(h);
    if (st != FC_OK)
        return cleanup(st);
    st = read_state(h);
    if (st != FC_OK)
        return cleanup(st);
    if (h->h.error != ERR_NONE)
        return cleanup(status_of(h));
    *out = h;
    return FC_OK;
}

}  // namespace

extern "C" {

fc_status fc_create(const fc_csr *S, const fc_options *opt, const void *U0, fc_dtype u0_dtype,
                    void *stream, fc_solver **out) {
    g_last_error.clear();
    TraceRange trace_range("fc_create");
    return create_impl(S, opt, U0, u0_dtype, (hipStream_t)stream, 65536, false, out);
}

fc_status fc_step(fc_solver *h, int32_t iters, fc_info *info) {
    g_last_error.clear();
    TraceRange trace_range("fc_step");
    if (!h)
        return fail(FC_ERR_INVALID_ARG, "solver is NULL");
    if (iters < 0)
        return fail(FC_ERR_INVALID_ARG, "iters < 0");
    fc_status st = FC_OK;
    if (iters > 0) {
        const int64_t target = (int64_t)h->h.iter + iters;
        st = run_until(h, (int32_t)(target > INT_MAX ? INT_MAX : target), INT_MAX);
    }
    fill_info(h, info);
    return st;
}

fc_status fc_step_profiled(fc_solver *h, int32_t iters, fc_info *info, fc_kernel_times *times) {
    g_last_error.clear();
    TraceRange trace_range("fc_step_profiled");
    if (!h || !times)
        return fail(FC_ERR_INVALID_ARG, "solver or times is NULL");
    if (iters < 0)
        return fail(FC_ERR_INVALID_ARG, "iters < 0");
    std::memset(times, 0, sizeof(*times));
    fc_status st = FC_OK;
    if (iters > 0) {
        EventLog log;
        log.out = times;
        log.single = h->single != 0;
        const int64_t target = (int64_t)h->h.iter + iters;
        st = run_until(h, (int32_t)(target > INT_MAX ? INT_MAX : target), INT_MAX, &log);
    }
    fill_info(h, info);
    return st;
}

fc_status fc_solve(fc_solver *h, fc_info *info) {
    g_last_error.clear();
    TraceRange trace_range("fc_solve");
    if (!h)
        return fail(FC_ERR_INVALID_ARG, "solver is NULL");
    fc_status st = FC_OK;
    if (h->h.iter < h->max_iter &&
        !(h->h.stop_reason == STOP_LOSS || h->h.stop_reason == STOP_PGRAD))
        st = run_until(h, h->max_iter, h->max_iter);
    else if (h->h.iter >= h->max_iter && h->h.stop_reason == STOP_NONE)
        h->h.stop_reason = STOP_MAXITER;
    fill_info(h, info);
    return st;
}

fc_status fc_get_u(const fc_solver *h, void *U_out, fc_dtype dtype) {
    g_last_error.clear();
    if (!h || !U_out)
        return fail(FC_ERR_INVALID_ARG, "NULL argument");
    if (dtype != FC_F64 && dtype != FC_F32)
        return fail(FC_ERR_INVALID_ARG, "U_out must be FC_F64 or FC_F32");
    const void *src = h->X[h->h.role[ROLE_C]];
    const int g = grid_1d(h->n * h->c, 256, 8192);
    hipStream_t s = h->stream;
    if (h->prec == FC_PREC_FP64) {
        if (dtype == FC_F64)
            hipLaunchKernelGGL((k_unpad_copy<double, double>), dim3(g), dim3(256), 0, s,
                               (const double *)src, h->cp, (double *)U_out, h->n, h->c, (const int32_t *)h->d_inv);
        else
            hipLaunchKernelGGL((k_unpad_copy<double, float>), dim3(g), dim3(256), 0, s,
                               (const double *)src, h->cp, (float *)U_out, h->n, h->c, (const int32_t *)h->d_inv);
    } else {
        if (dtype == FC_F64)
            hipLaunchKernelGGL((k_unpad_copy<float, double>), dim3(g), dim3(256), 0, s,
                               (const float *)src, h->cp, (double *)U_out, h->n, h->c, (const int32_t *)h->d_inv);
        else
            hipLaunchKernelGGL((k_unpad_copy<float, float>), dim3(g), dim3(256), 0, s,
                               (const float *)src, h->cp, (float *)U_out, h->n, h->c, (const int32_t *)h->d_inv);
    }
    HIPCHK(hipGetLastError());
    return FC_OK;
}

fc_status fc_get_history(const fc_solver *h, int32_t cap, double *f_log, double *step_log,
                         int32_t *trials_log, double *r_log, int32_t *count) {
    g_last_error.clear();
    if (!h || cap < 0)
        return fail(FC_ERR_INVALID_ARG, "bad argument");
    int32_t k = h->h.iter + 1;
    if (k > h->hist_cap)
        k = h->hist_cap;
    if (k > cap)
        k = cap;
    hipStream_t s = h->stream;
    if (f_log && k > 0)
        HIPCHK(hipMemcpyAsync(f_log, h->d_hist_f, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    if (step_log && k > 0)
        HIPCHK(hipMemcpyAsync(step_log, h->d_hist_tau, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    if (trials_log && k > 0)
        HIPCHK(hipMemcpyAsync(trials_log, h->d_hist_trials, sizeof(int32_t) * k, hipMemcpyDeviceToHost, s));
    if (r_log && k > 0)
        HIPCHK(hipMemcpyAsync(r_log, h->d_hist_r, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (step_log && k > 0)
        step_log[0] = 0.0;
    if (r_log && k > 0)
        r_log[0] = 0.0;
    if (trials_log && k > 0)
        trials_log[0] = 0;
    if (count)
        *count = k;
    return FC_OK;
}

}  // extern "C"

namespace {

// Checkpoint layout: header, then Xbar_c, Xbar_p, S Xbar_c, S Xbar_p
// (n x CP each, padded layout), G_Y in double and in the compute type, and
// the history of the first iter + 1 iterations.  Restoring all of these makes
// a resumed run bitwise equal to an uninterrupted one.
struct CkptHeader {
    uint64_t magic;
    uint32_t version;
    uint32_t header_bytes;
    int64_t n;
    int32_t c, cp, prec, accelerate, backtrack, diag;
    int32_t hist_len, reorder;
    int32_t defer, reserved;   // reserved: the single-pass flag
    uint64_t perm_hash;        // fingerprint of a given order (FC_REORDER_GIVEN), else 0
    DevState st;
};
constexpr uint64_t CKPT_MAGIC = 0x3130545043434646ull;  // "FFCCPT01"

size_t ckpt_bytes(const fc_solver *h, int32_t hist_len) {
    const size_t esz = h->prec == FC_PREC_FP64 ? 8 : 4;
    const size_t mat = (size_t)h->n * h->cp * esz;
    const size_t g = (size_t)h->cpm * h->cpm;
    return sizeof(CkptHeader) + 4 * mat + g * 8 + g * esz +
           (size_t)hist_len * (3 * sizeof(double) + sizeof(int32_t));
}

}  // namespace

extern "C" {

fc_status fc_get_state(const fc_solver *h, void *buf, size_t *bytes) {
    g_last_error.clear();
    if (!h || !bytes)
        return fail(FC_ERR_INVALID_ARG, "solver or bytes is NULL");
    int32_t hist_len = h->h.iter + 1 < h->hist_cap ? h->h.iter + 1 : h->hist_cap;
    const size_t need = ckpt_bytes(h, hist_len);
    if (!buf) {
        *bytes = need;
        return FC_OK;
    }
    if (*bytes < need)
        return fail(FC_ERR_INVALID_ARG, "checkpoint buffer too small");
    *bytes = need;
    hipStream_t s = h->stream;
    CkptHeader hd = {};
    hd.magic = CKPT_MAGIC;
    hd.version = 3;
    hd.header_bytes = sizeof(CkptHeader);
    hd.n = h->n;
    hd.c = h->c;
    hd.cp = h->cp;
    hd.prec = (int32_t)h->prec;
    hd.accelerate = h->accelerate;
    hd.backtrack = h->backtrack;
    hd.diag = (int32_t)h->diag;
    hd.reorder = h->reorder;
    hd.defer = h->defer;
    hd.reserved = h->single;
    hd.perm_hash = h->perm_hash;
    hd.hist_len = hist_len;
    hd.st = h->h;
    char *p = (char *)buf;
    std::memcpy(p, &hd, sizeof(hd));
    p += sizeof(hd);
    const size_t esz = h->prec == FC_PREC_FP64 ? 8 : 4;
    const size_t mat = (size_t)h->n * h->cp * esz;
    const void *src[4] = {h->X[h->h.role[ROLE_C]], h->X[h->h.role[ROLE_P]], h->Z[h->h.role[ROLE_C]],
                          h->Z[h->h.role[ROLE_P]]};
    for (int k = 0; k < 4; ++k, p += mat)
        HIPCHK(hipMemcpyAsync(p, src[k], mat, hipMemcpyDeviceToHost, s));
    const size_t g = (size_t)h->cpm * h->cpm;
    HIPCHK(hipMemcpyAsync(p, h->d_GY64, g * 8, hipMemcpyDeviceToHost, s));
    p += g * 8;
    HIPCHK(hipMemcpyAsync(p, h->d_GYs, g * esz, hipMemcpyDeviceToHost, s));
    p += g * esz;
    HIPCHK(hipMemcpyAsync(p, h->d_hist_f, sizeof(double) * hist_len, hipMemcpyDeviceToHost, s));
    p += sizeof(double) * hist_len;
    HIPCHK(hipMemcpyAsync(p, h->d_hist_tau, sizeof(double) * hist_len, hipMemcpyDeviceToHost, s));
    p += sizeof(double) * hist_len;
    HIPCHK(hipMemcpyAsync(p, h->d_hist_r, sizeof(double) * hist_len, hipMemcpyDeviceToHost, s));
    p += sizeof(double) * hist_len;
    HIPCHK(hipMemcpyAsync(p, h->d_hist_trials, sizeof(int32_t) * hist_len, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return FC_OK;
}

fc_status fc_set_state(fc_solver *h, const void *buf, size_t bytes) {
    g_last_error.clear();
    if (!h || !buf)
        return fail(FC_ERR_INVALID_ARG, "solver or buffer is NULL");
    if (bytes < sizeof(CkptHeader))
        return fail(FC_ERR_INVALID_ARG, "checkpoint buffer too small");
    CkptHeader hd;
    std::memcpy(&hd, buf, sizeof(hd));
    if (hd.magic != CKPT_MAGIC || hd.version != 3 || hd.header_bytes != sizeof(CkptHeader))
        return fail(FC_ERR_INVALID_ARG, "not a checkpoint of this library version");
    if (hd.n != h->n || hd.c != h->c || hd.cp != h->cp || hd.prec != (int32_t)h->prec ||
        hd.accelerate != h->accelerate || hd.backtrack != h->backtrack || hd.diag != (int32_t)h->diag ||
        hd.reorder != h->reorder || hd.defer != h->defer || hd.reserved != h->single)
        return fail(FC_ERR_INVALID_ARG, "checkpoint was taken from a solver with other n, c or options");
    if (hd.perm_hash != h->perm_hash)
        return fail(FC_ERR_INVALID_ARG, "checkpoint was taken under another given article order");
    if (hd.hist_len < 1 || hd.hist_len > h->hist_cap || bytes < ckpt_bytes(h, hd.hist_len))
        return fail(FC_ERR_INVALID_ARG, "checkpoint buffer truncated");
    hipStream_t s = h->stream;
    const char *p = (const char *)buf + sizeof(CkptHeader);
    const size_t esz = h->prec == FC_PREC_FP64 ? 8 : 4;
    const size_t mat = (size_t)h->n * h->cp * esz;
    void *dst[4] = {h->X[0], h->X[1], h->Z[0], h->Z[1]};
    for (int k = 0; k < 4; ++k, p += mat)
        HIPCHK(hipMemcpyAsync(dst[k], p, mat, hipMemcpyHostToDevice, s));
    const size_t g = (size_t)h->cpm * h->cpm;
    HIPCHK(hipMemcpyAsync(h->d_GY64, p, g * 8, hipMemcpyHostToDevice, s));
    p += g * 8;
    HIPCHK(hipMemcpyAsync(h->d_GYs, p, g * esz, hipMemcpyHostToDevice, s));
    p += g * esz;
    const int32_t hl = hd.hist_len;
    HIPCHK(hipMemcpyAsync(h->d_hist_f, p, sizeof(double) * hl, hipMemcpyHostToDevice, s));
    p += sizeof(double) * hl;
    HIPCHK(hipMemcpyAsync(h->d_hist_tau, p, sizeof(double) * hl, hipMemcpyHostToDevice, s));
    p += sizeof(double) * hl;
    HIPCHK(hipMemcpyAsync(h->d_hist_r, p, sizeof(double) * hl, hipMemcpyHostToDevice, s));
    p += sizeof(double) * hl;
    HIPCHK(hipMemcpyAsync(h->d_hist_trials, p, sizeof(int32_t) * hl, hipMemcpyHostToDevice, s));
    if (h->prec == FC_PREC_MIXED)
        for (int k = 0; k < 2; ++k)
            hipLaunchKernelGGL((k_convert<float, __hip_bfloat16>), dim3(grid_1d(h->n * h->cp, 256, 8192)),
                               dim3(256), 0, s, (const float *)h->X[k], (__hip_bfloat16 *)h->shadow[k],
                               h->n * h->cp);
    HIPCHK(hipGetLastError());
    DevState st = hd.st;
    st.role[ROLE_C] = 0;
    st.role[ROLE_P] = 1;
    st.role[ROLE_N] = 2;
    st.hist_cap = h->hist_cap;
    h->h = st;
    return write_state(h);
}

void fc_destroy(fc_solver *h) {
    if (!h)
        return;
    if (h->stream)
        (void)hipStreamSynchronize(h->stream);
    else
        (void)hipDeviceSynchronize();
    delete h;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// stateless entry points
// ---------------------------------------------------------------------------
namespace {

template <typename T, typename VS, int CP>
fc_status spmm_and_gram_t(const fc_csr *S, fc_diag diag, const T *Upad, T *Zpad, bool want_gram,
                          hipStream_t s, double *trace_out, double *G_out) {
    constexpr int CPM = CP < 16 ? 16 : CP;
    using Cfg = SpmmCfg<T, CP>;
    const int64_t n = S->n;
    const int cus = device_cus();
    HeavyPlan hp;
    fc_status st = build_heavy_plan(S->row_ptr, n, sizeof(T), CP, s, hp);
    if (st != FC_OK)
        return st;
    Inst I = {};
    I.row_ptr = S->row_ptr;
    I.col = S->col_idx;
    I.val = S->values;
    I.n = n;
    I.c = CP;
    I.diag_unit = diag == FC_DIAG_UNIT ? 1 : 0;
    plan_to_inst(hp, I);
    I.g_spmm = grid_1d(n, Cfg::ROWS_PER_WG, (int64_t)cus * 64);
    I.g_comb = combine_grid(hp.nheavy, 256 / CP);
    I.X[0] = (void *)Upad;
    I.Z[0] = Zpad;
    DevBuf part, red;
    HIPCHK(dev_alloc(part, sizeof(double) * (I.g_spmm + I.g_comb), s));
    HIPCHK(dev_alloc(red, sizeof(double) * (1 + CPM * CPM), s));
    I.part_spmm = (double *)part.p;
    launch_spmm<T, T, T, VS, CP>(I, 0, s);
    launch_reduce((const double *)part.p, I.g_spmm + I.g_comb, 1, 1, (double *)red.p, s);
    DevBuf gpart;
    if (want_gram) {
        const int g_gram = grid_1d(cdiv(n, 16), 4, (int64_t)cus * 2);
        HIPCHK(dev_alloc(gpart, sizeof(double) * (size_t)g_gram * 4 * CPM * CPM, s));
        hipLaunchKernelGGL((k_gram<T, CP>), dim3(g_gram), dim3(256), 0, s, Upad, n,
                           (double *)gpart.p, (int64_t)(CPM * CPM));
        launch_reduce((const double *)gpart.p, (int64_t)g_gram * 4, CPM * CPM, CPM * CPM,
                      (double *)red.p + 1, s);
    }
    HIPCHK(hipGetLastError());
    std::vector<double> hbuf(1 + CPM * CPM);
    HIPCHK(hipMemcpyAsync(hbuf.data(), red.p, sizeof(double) * (want_gram ? 1 + CPM * CPM : 1),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (trace_out)
        *trace_out = hbuf[0];
    if (G_out && want_gram)
        std::memcpy(G_out, hbuf.data() + 1, sizeof(double) * CPM * CPM);
    return FC_OK;
}

// Copy a user matrix (n x c, ld = c) into a padded device buffer of type T.
template <typename T>
fc_status pad_user(const void *U, fc_dtype dt, int64_t n, int c, int cp, T *dst, hipStream_t s) {
    const int g = grid_1d(n * cp, 256, 8192);
    if (dt == FC_F64)
        hipLaunchKernelGGL((k_pad_copy<double, T>), dim3(g), dim3(256), 0, s, (const double *)U,
                           (int64_t)c, dst, n, c, cp, (const int32_t *)nullptr);
    else
        hipLaunchKernelGGL((k_pad_copy<float, T>), dim3(g), dim3(256), 0, s, (const float *)U,
                           (int64_t)c, dst, n, c, cp, (const int32_t *)nullptr);
    HIPCHK(hipGetLastError());
    return FC_OK;
}

}  // namespace

extern "C" {

fc_status fc_spmm(const fc_csr *S, fc_diag diag, const void *U, void *Z, fc_dtype dtype, int32_t c,
                  void *stream) {
    g_last_error.clear();
    TraceRange trace_range("fc_spmm");
    fc_status st = check_csr_args(S);
    if (st != FC_OK)
        return st;
    if (!U || !Z)
        return fail(FC_ERR_INVALID_ARG, "U or Z is NULL");
    if (c < 1 || c > 64)
        return fail(FC_ERR_INVALID_ARG, "c must be in [1, 64]");
    if (dtype != FC_F64 && dtype != FC_F32)
        return fail(FC_ERR_INVALID_ARG, "dtype must be FC_F64 or FC_F32");
    if ((dtype == FC_F64) != (S->values_dtype == FC_F64))
        return fail(FC_ERR_INVALID_ARG, "S values and U must both be FC_F64, or FC_F32/FC_F16 with FC_F32 U");
    hipStream_t s = (hipStream_t)stream;
    const int cp = cp_of(c);
    const size_t esz = dtype == FC_F64 ? 8 : 4;
    DevBuf up, zp;
    HIPCHK(dev_alloc(up, esz * S->n * cp, s));
    HIPCHK(dev_alloc(zp, esz * S->n * cp, s));
    return with_cp(cp, [&](auto cpc) -> fc_status {
        constexpr int CP = decltype(cpc)::value;
        fc_status r;
        const int g = grid_1d(S->n * c, 256, 8192);
        if (dtype == FC_F64) {
            r = pad_user<double>(U, dtype, S->n, c, CP, (double *)up.p, s);
            if (r != FC_OK)
                return r;
            r = spmm_and_gram_t<double, double, CP>(S, diag, (const double *)up.p, (double *)zp.p,
                                                    false, s, nullptr, nullptr);
            if (r != FC_OK)
                return r;
            hipLaunchKernelGGL((k_unpad_copy<double, double>), dim3(g), dim3(256), 0, s,
                               (const double *)zp.p, CP, (double *)Z, S->n, c,
                               (const int32_t *)nullptr);
        } else {
            r = pad_user<float>(U, dtype, S->n, c, CP, (float *)up.p, s);
            if (r != FC_OK)
                return r;
            if (S->values_dtype == FC_F16)
                r = spmm_and_gram_t<float, __half, CP>(S, diag, (const float *)up.p, (float *)zp.p,
                                                       false, s, nullptr, nullptr);
            else
                r = spmm_and_gram_t<float, float, CP>(S, diag, (const float *)up.p, (float *)zp.p,
                                                      false, s, nullptr, nullptr);
            if (r != FC_OK)
                return r;
            hipLaunchKernelGGL((k_unpad_copy<float, float>), dim3(g), dim3(256), 0, s,
                               (const float *)zp.p, CP, (float *)Z, S->n, c,
                               (const int32_t *)nullptr);
        }
        HIPCHK(hipGetLastError());
        return FC_OK;
    });
}

fc_status fc_objective(const fc_csr *S, fc_diag diag, const void *U, fc_dtype u_dtype, int32_t c,
                       void *stream, double *f_out) {
    g_last_error.clear();
    TraceRange trace_range("fc_objective");
    fc_status st = check_csr_args(S);
    if (st != FC_OK)
        return st;
    if (!U || !f_out)
        return fail(FC_ERR_INVALID_ARG, "U or f_out is NULL");
    if (c < 1 || c > 64)
        return fail(FC_ERR_INVALID_ARG, "c must be in [1, 64]");
    if (u_dtype != FC_F64 && u_dtype != FC_F32)
        return fail(FC_ERR_INVALID_ARG, "u_dtype must be FC_F64 or FC_F32");
    if ((u_dtype == FC_F64) != (S->values_dtype == FC_F64))
        return fail(FC_ERR_INVALID_ARG, "S values and U must both be FC_F64, or FC_F32/FC_F16 with FC_F32 U");
    hipStream_t s = (hipStream_t)stream;
    const int cp = cp_of(c);
    const int cpm = cpm_of(cp);
    double s2 = 0.0;
    st = sum_squares(S, s, &s2);
    if (st != FC_OK)
        return st;
    if (diag == FC_DIAG_UNIT)
        s2 += (double)S->n;
    const size_t esz = u_dtype == FC_F64 ? 8 : 4;
    DevBuf up, zp;
    HIPCHK(dev_alloc(up, esz * S->n * cp, s));
    HIPCHK(dev_alloc(zp, esz * S->n * cp, s));
    std::vector<double> G(cpm * cpm);
    double tr = 0.0;
    st = with_cp(cp, [&](auto cpc) -> fc_status {
        constexpr int CP = decltype(cpc)::value;
        fc_status r;
        if (u_dtype == FC_F64) {
            r = pad_user<double>(U, u_dtype, S->n, c, CP, (double *)up.p, s);
            if (r != FC_OK)
                return r;
            return spmm_and_gram_t<double, double, CP>(S, diag, (const double *)up.p, (double *)zp.p,
                                                       true, s, &tr, G.data());
        }
        r = pad_user<float>(U, u_dtype, S->n, c, CP, (float *)up.p, s);
        if (r != FC_OK)
            return r;
        if (S->values_dtype == FC_F16)
            return spmm_and_gram_t<float, __half, CP>(S, diag, (const float *)up.p, (float *)zp.p, true,
                                                      s, &tr, G.data());
        return spmm_and_gram_t<float, float, CP>(S, diag, (const float *)up.p, (float *)zp.p, true, s,
                                                 &tr, G.data());
    });
    if (st != FC_OK)
        return st;
    double gsq = 0.0;
    for (double g : G)
        gsq += g * g;
    *f_out = s2 + gsq - 2.0 * tr;
    return FC_OK;
}

fc_status fc_gram(const void *U, fc_dtype dtype, int64_t n, int32_t c, void *stream, double *G_out) {
    g_last_error.clear();
    TraceRange trace_range("fc_gram");
    if (!U || !G_out)
        return fail(FC_ERR_INVALID_ARG, "U or G_out is NULL");
    if (n < 1 || c < 1 || c > 64)
        return fail(FC_ERR_INVALID_ARG, "need n >= 1 and c in [1, 64]");
    if (dtype != FC_F64 && dtype != FC_F32)
        return fail(FC_ERR_INVALID_ARG, "dtype must be FC_F64 or FC_F32");
    hipStream_t s = (hipStream_t)stream;
    const int cp = cp_of(c);
    const int cpm = cpm_of(cp);
    const size_t esz = dtype == FC_F64 ? 8 : 4;
    DevBuf up, gpart, red;
    HIPCHK(dev_alloc(up, esz * n * cp, s));
    const int cus = device_cus();
    const int g_gram = grid_1d(cdiv(n, 16), 4, (int64_t)cus * 2);
    HIPCHK(dev_alloc(gpart, sizeof(double) * (size_t)g_gram * 4 * cpm * cpm, s));
    HIPCHK(dev_alloc(red, sizeof(double) * cpm * cpm, s));
    fc_status st = with_cp(cp, [&](auto cpc) -> fc_status {
        constexpr int CP = decltype(cpc)::value;
        fc_status r;
        if (dtype == FC_F64) {
            r = pad_user<double>(U, dtype, n, c, CP, (double *)up.p, s);
            if (r != FC_OK)
                return r;
            hipLaunchKernelGGL((k_gram<double, CP>), dim3(g_gram), dim3(256), 0, s,
                               (const double *)up.p, n, (double *)gpart.p, (int64_t)(cpm * cpm));
        } else {
            r = pad_user<float>(U, dtype, n, c, CP, (float *)up.p, s);
            if (r != FC_OK)
                return r;
            hipLaunchKernelGGL((k_gram<float, CP>), dim3(g_gram), dim3(256), 0, s,
                               (const float *)up.p, n, (double *)gpart.p, (int64_t)(cpm * cpm));
        }
        HIPCHK(hipGetLastError());
        return FC_OK;
    });
    if (st != FC_OK)
        return st;
    launch_reduce((const double *)gpart.p, (int64_t)g_gram * 4, cpm * cpm, cpm * cpm, (double *)red.p, s);
    std::vector<double> G(cpm * cpm);
    HIPCHK(hipMemcpyAsync(G.data(), red.p, sizeof(double) * cpm * cpm, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int i = 0; i < c; ++i)
        for (int j = 0; j < c; ++j)
            G_out[i * c + j] = G[i * cpm + j];
    return FC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free Gram matrix.  Its partial sums live in one static device
// array per GPU; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (the array's own name is a host
// stand-in there).  Calls on one GPU share the array, so calls that overlap
// on the same GPU race.
// ---------------------------------------------------------------------------
namespace {

constexpr int NOALLOC_MAX_WG = 256;                    // workgroups of the Gram pass
constexpr int64_t NOALLOC_PARTS = 4 * NOALLOC_MAX_WG;  // one partial per wave
constexpr int64_t NOALLOC_MAT = 64 * 64;               // largest padded c x c block
constexpr int64_t NOALLOC_WORDS = NOALLOC_PARTS * NOALLOC_MAT + NOALLOC_MAT;
static_assert(NOALLOC_WORDS * 8 == FC_GRAM_NOALLOC_SCRATCH_BYTES,
              "fc.h states the scratch size");

static __device__ __align__(256) double scratch[NOALLOC_WORDS];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};

// The array's device address on the current device, looked up once per device.
fc_status scratch_on_current_device(double **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES)
        return fail(FC_ERR_UNSUPPORTED, "device index beyond the library's table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p)
            return fail(FC_ERR_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return FC_OK;
}

}  // namespace

extern "C" {

fc_status fc_gram_noalloc(const void *U, fc_dtype dtype, int64_t n, int32_t c, int64_t ld,
                          void *stream, double *G_out) {
    g_last_error.clear();
    if (!U || !G_out)
        return fail(FC_ERR_INVALID_ARG, "U or G_out is NULL");
    if (n < 1 || c < 1 || c > 64 || ld < c)
        return fail(FC_ERR_INVALID_ARG, "need n >= 1, c in [1, 64] and ld >= c");
    if (dtype != FC_F64 && dtype != FC_F32)
        return fail(FC_ERR_INVALID_ARG, "dtype must be FC_F64 or FC_F32");
    const int cp = cp_of(c);
    const int cpm = cpm_of(cp);
    const int64_t mat = (int64_t)cpm * cpm;
    const int cus = device_cus();
    // the grid of fc_gram, capped so that the partials fit the scratch array
    const int g = grid_1d(cdiv(n, 16), 4, std::min<int64_t>((int64_t)cus * 2, NOALLOC_MAX_WG));
    if ((int64_t)g * 4 * mat + mat > NOALLOC_WORDS)
        return fail(FC_ERR_INVALID_ARG, "partial sums exceed the scratch array");
    double *base = nullptr;
    fc_status st = scratch_on_current_device(&base);
    if (st != FC_OK)
        return st;
    double *part = base, *red = base + NOALLOC_PARTS * NOALLOC_MAT;
    hipStream_t s = (hipStream_t)stream;
    st = with_cp(cp, [&](auto cpc) -> fc_status {
        constexpr int CP = decltype(cpc)::value;
        if (dtype == FC_F64)
            hipLaunchKernelGGL((k_gram_strided<double, CP>), dim3(g), dim3(256), 0, s,
                               (const double *)U, ld, c, n, part, mat);
        else
            hipLaunchKernelGGL((k_gram_strided<float, CP>), dim3(g), dim3(256), 0, s,
                               (const float *)U, ld, c, n, part, mat);
        HIPCHK(hipGetLastError());
        return FC_OK;
    });
    if (st != FC_OK)
        return st;
    // every wave writes its whole partial block, so nothing needs clearing
    launch_reduce(part, (int64_t)g * 4, mat, mat, red, s);
    hipLaunchKernelGGL(k_corner_copy, dim3(1), dim3(256), 0, s, (const double *)red, cpm, c, G_out);
    HIPCHK(hipGetLastError());
    return FC_OK;
}

fc_status fc_project(const void *V, void *out, fc_dtype dtype, int64_t rows, int32_t c, int64_t ld,
                     void *stream) {
    g_last_error.clear();
    if (rows < 0 || c < 1 || c > 64 || ld < c)
        return fail(FC_ERR_INVALID_ARG, "need rows >= 0, c in [1, 64], ld >= c");
    if (dtype != FC_F64 && dtype != FC_F32)
        return fail(FC_ERR_INVALID_ARG, "dtype must be FC_F64 or FC_F32");
    if (rows == 0)
        return FC_OK;
    if (!V || !out)
        return fail(FC_ERR_INVALID_ARG, "V or out is NULL");
    hipStream_t s = (hipStream_t)stream;
    const int cpm = cpm_of(cp_of(c));
    const int cus = device_cus();
    const int g = grid_1d(cdiv(rows, 16), 4, (int64_t)cus * 8);
#define PROJ(T, CPMV)                                                                             \
    hipLaunchKernelGGL((k_project<T, CPMV>), dim3(g), dim3(256), 0, s, (const T *)V, (T *)out, rows, \
                       c, ld)
    if (dtype == FC_F64) {
        if (cpm == 16) PROJ(double, 16);
        else if (cpm == 32) PROJ(double, 32);
        else PROJ(double, 64);
    } else {
        if (cpm == 16) PROJ(float, 16);
        else if (cpm == 32) PROJ(float, 32);
        else PROJ(float, 64);
    }
#undef PROJ
    HIPCHK(hipGetLastError());
    return FC_OK;
}

fc_status fc_gather_probe(const int32_t *col_idx, int64_t nnz, const void *U, int64_t rows,
                          int32_t row_bytes, int32_t wg_per_cu, int32_t reps, void *stream,
                          double *ms_out) {
    g_last_error.clear();
    if (!col_idx || !U || !ms_out || nnz < 1 || rows < 1 || reps < 1)
        return fail(FC_ERR_INVALID_ARG, "need col_idx, U, ms_out, nnz >= 1, rows >= 1, reps >= 1");
    if (row_bytes != 32 && row_bytes != 64 && row_bytes != 128 && row_bytes != 256)
        return fail(FC_ERR_INVALID_ARG, "row_bytes must be 32, 64, 128 or 256");
    if (wg_per_cu < 1 || wg_per_cu > 64)
        return fail(FC_ERR_INVALID_ARG, "wg_per_cu must be in [1, 64]");
    hipStream_t s = (hipStream_t)stream;
    const int64_t pieces = row_bytes / 16;
    const int teams = 256 / (int)pieces;
    const int g = grid_1d(cdiv(nnz, teams), 1, (int64_t)device_cus() * wg_per_cu);
    DevBuf sum;
    HIPCHK(dev_alloc(sum, sizeof(double), s));
    HIPCHK(hipMemsetAsync(sum.p, 0, sizeof(double), s));
    auto launch = [&]() {
        const uint4 *u = (const uint4 *)U;
        double *cs = (double *)sum.p;
        switch (pieces) {
        case 2: hipLaunchKernelGGL((k_gather_probe<2, 4>), dim3(g), dim3(256), 0, s, col_idx, nnz, u, pieces, cs); break;
        case 4: hipLaunchKernelGGL((k_gather_probe<4, 4>), dim3(g), dim3(256), 0, s, col_idx, nnz, u, pieces, cs); break;
        case 8: hipLaunchKernelGGL((k_gather_probe<8, 4>), dim3(g), dim3(256), 0, s, col_idx, nnz, u, pieces, cs); break;
        default: hipLaunchKernelGGL((k_gather_probe<16, 4>), dim3(g), dim3(256), 0, s, col_idx, nnz, u, pieces, cs); break;
        }
    };
    launch();   // warm-up
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r)
        launch();
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(e);
    HIPCHK(hipGetLastError());
    *ms_out = (double)ms / reps;
    return FC_OK;
}

fc_status fc_spectral_norm(const fc_csr *S, fc_diag diag, int32_t max_iter, double rtol, void *stream,
                           double *norm_out, int32_t *iters_out) {
    g_last_error.clear();
    fc_status st = check_csr_args(S);
    if (st != FC_OK)
        return st;
    if (!norm_out)
        return fail(FC_ERR_INVALID_ARG, "norm_out is NULL");
    return power_norm(S, (int)(diag == FC_DIAG_UNIT), max_iter, rtol, (hipStream_t)stream, norm_out,
                      iters_out);
}

}  // extern "C"

#include "fc_server.inc"
#include "fc_second.inc"
