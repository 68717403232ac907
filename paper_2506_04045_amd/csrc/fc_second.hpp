// Second-order check of Theorem 4.1: the Hessian of f applied to a
// direction, eq. (hessian), and the pieces of a Lanczos search for negative
// curvature over the face of Omega at an iterate (directions whose rows sum
// to zero and that keep every zero component at zero).
//
// In the row layout (u_i = x_i, v_i the rows of the direction) the Hessian
// applied to V is, row by row,
//   h_i = -4 (S_eff V)_i + 4 v_i G + 4 u_i (C + C^T),   G = U^T U, C = U^T V,
// the transpose of -4 V (S - X^T X) + 4 X (V^T X + X^T V).  The product S_eff V
// is the solver's sparse product; G and C come from the matrix cores.
#pragma once

#include "fc_kernels.hpp"

namespace fc {

// C = U^T V (CPM x CPM, every block) over 16-row tiles: lane (r, g) holds
// component 16a + r of rows 4t + g, as in k_gram.  Wave partials go to
// part[(blockIdx * 4 + wave) * ld].
template <typename T, int CP>
__global__ __launch_bounds__(256) void k_cross_gram(const T *__restrict__ U, const T *__restrict__ V,
                                                    int64_t n, double *__restrict__ part, int64_t ld) {
    constexpr int CPM = CP < 16 ? 16 : CP;
    constexpr int M = CPM / 16;
    using A4 = typename Acc4<T>::type;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    doublex4 acc64[M][M];
#pragma unroll
    for (int a = 0; a < M; ++a)
#pragma unroll
        for (int b = 0; b < M; ++b)
            acc64[a][b] = doublex4{0, 0, 0, 0};
    const int64_t ntiles = (n + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
        T uv[4][M], vv[4][M];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t row = tile * 16 + 4 * t + g;
#pragma unroll
            for (int a = 0; a < M; ++a) {
                const int k = 16 * a + r;
                const bool ok = row < n && k < CP;
                uv[t][a] = ok ? U[row * CP + k] : (T)0;
                vv[t][a] = ok ? V[row * CP + k] : (T)0;
            }
        }
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int b = 0; b < M; ++b) {
                A4 acc = A4{0, 0, 0, 0};
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc = mfma16x16x4(uv[t][a], vv[t][b], acc);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc64[a][b][q] += (double)acc[q];
            }
    }
    double *out = part + ((int64_t)blockIdx.x * 4 + wave) * ld;
#pragma unroll
    for (int a = 0; a < M; ++a)
#pragma unroll
        for (int b = 0; b < M; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                out[(16 * a + mfma_row<T>(g, q)) * CPM + 16 * b + r] = acc64[a][b][q];
}

// h_ik = -4 z_ik + 4 sum_l v_il G_lk + 4 sum_l u_il (C_lk + C_kl) for k < c, in
// double; padded components are written as zero.  G and C are CPM x CPM.
template <typename T, int CP>
__global__ __launch_bounds__(256) void k_hvp_rows(const T *__restrict__ U, const T *__restrict__ V,
                                                  const T *__restrict__ Z, const double *__restrict__ G,
                                                  const double *__restrict__ C, int64_t n, int c,
                                                  T *__restrict__ HV) {
    constexpr int CPM = CP < 16 ? 16 : CP;
    __shared__ double gs[CP * CP], ms[CP * CP];
    for (int e = threadIdx.x; e < CP * CP; e += blockDim.x) {
        const int k = e / CP, l = e % CP;
        gs[e] = G[k * CPM + l];
        ms[e] = C[k * CPM + l] + C[l * CPM + k];
    }
    __syncthreads();
    const int64_t total = n * CP;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / CP;
        const int k = (int)(idx % CP);
        double h = 0.0;
        if (k < c) {
            double a = 0.0, b = 0.0;
            for (int l = 0; l < c; ++l) {
                a += (double)V[i * CP + l] * gs[l * CP + k];
                b += (double)U[i * CP + l] * ms[l * CP + k];
            }
            h = -4.0 * (double)Z[idx] + 4.0 * a + 4.0 * b;
        }
        HV[idx] = (T)h;
    }
}

// Orthogonal projection onto the face directions at U: per row, components
// k >= c or with u_ik <= zero_tol are zeroed, the others lose their mean.
template <typename T, int CP>
__global__ void k_face_project(const T *__restrict__ U, double zero_tol, int c, int64_t n,
                               T *__restrict__ W) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double sum = 0.0;
        int cnt = 0;
        for (int k = 0; k < c; ++k)
            if ((double)U[i * CP + k] > zero_tol) {
                sum += (double)W[i * CP + k];
                ++cnt;
            }
        const double mean = cnt > 0 ? sum / cnt : 0.0;
        for (int k = 0; k < CP; ++k) {
            const bool act = k < c && (double)U[i * CP + k] > zero_tol;
            W[i * CP + k] = act ? (T)((double)W[i * CP + k] - mean) : (T)0;
        }
    }
}

// part[j * gridDim.x + blockIdx.x] = sum over this block's stretch of
// w[e] q_j[e], for the vector j = blockIdx.y of the stack Q (stride len).
template <typename T>
__global__ __launch_bounds__(256) void k_multidot(const T *__restrict__ W, const T *__restrict__ Q,
                                                  int64_t len, double *__restrict__ part) {
    __shared__ double sh[256];
    const T *__restrict__ q = Q + (int64_t)blockIdx.y * len;
    double a = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < len; e += (int64_t)gridDim.x * 256)
        a += (double)W[e] * (double)q[e];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = sh[0];
}

// out[e] = scale * (base[e] - sum_{j < m} coef[j] q_j[e]) in double; base may
// be NULL (zero) and out may alias base.
template <typename T>
__global__ void k_combine_vectors(const T *base, const T *__restrict__ Q, const double *__restrict__ coef,
                                  int m, int64_t len, double scale, T *out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
         e += (int64_t)gridDim.x * blockDim.x) {
        double a = base ? (double)base[e] : 0.0;
        for (int j = 0; j < m; ++j)
            a -= coef[j] * (double)Q[(int64_t)j * len + e];
        out[e] = (T)(scale * a);
    }
}

}  // namespace fc
