/* Runs every entry point of the C oracle (oracle/fcref.c) on small random
 * instances, built by the CPU tests with the address and undefined-behaviour
 * sanitizers.  Beyond running clean it checks a few facts that fix the
 * results: projected rows lie on the simplex, the structured loss equals the
 * double-sum definition, and the solver's logs are filled as documented.
 * Exit status 0 when everything holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t accelerate, max_iter, backtrack, reserved;
    double step, L0, eta, tol_loss, tol_pgrad;
    const double *step_schedule;
} fcref_opts;

double fcref_norm_s_sq(int64_t n, const int64_t *row_ptr, const double *val, int diag_unit);
void fcref_x_s(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *val,
               int diag_unit, int C, const double *X, double *XS);
void fcref_share(int64_t n, int C, const double *X, double *share);
void fcref_x_s_rows(int64_t m, const int64_t *rows, const int64_t *sub_row_ptr,
                    const int32_t *sub_col_idx, const double *sub_val, int diag_unit, int C,
                    const double *X, double *XS);
void fcref_project_simplex(int C, const double *x, double *y);
void fcref_project_columns(int64_t n, int C, const double *V, double *out);
double fcref_loss(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *val,
                  int diag_unit, int C, const double *X);
void fcref_gradient(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *val,
                    int diag_unit, int C, const double *X, double *grad);
void fcref_hvp(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *val,
               int diag_unit, int C, const double *X, const double *V, double *HV);
double fcref_spectral_norm(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                           const double *val, int diag_unit, int max_iter, double rtol, int *iters);
int fcref_solve(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *val,
                int diag_unit, int C, const double *X0, const fcref_opts *opt, double *X_out,
                double *f_log, double *tau_log, int32_t *trials_log, double *r_log,
                int32_t *stop_reason);

static int failures = 0;
#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);   \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

static uint64_t state = 88172645463325252ull;
static double urand(void) {   /* xorshift64, uniform in [0, 1) */
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

int main(void) {
    enum { N = 40, C = 5 };
    /* dense symmetric S with zero diagonal, then CSR */
    static double A[N][N];
    for (int i = 0; i < N; ++i)
        for (int j = i + 1; j < N; ++j)
            if (urand() < 0.2)
                A[i][j] = A[j][i] = urand();
    int64_t row_ptr[N + 1];
    int32_t col[N * N];
    double val[N * N];
    int64_t nnz = 0;
    row_ptr[0] = 0;
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j < N; ++j)
            if (A[i][j] != 0.0) {
                col[nnz] = j;
                val[nnz] = A[i][j];
                ++nnz;
            }
        row_ptr[i + 1] = nnz;
    }
    double X[N * C], Y[N * C], XS[N * C], G[C * C], grad[N * C], HV[N * C];
    for (int i = 0; i < N; ++i) {
        double s = 0.0;
        for (int k = 0; k < C; ++k)
            s += (X[i * C + k] = urand() + 1e-3);
        for (int k = 0; k < C; ++k)
            X[i * C + k] /= s;
    }
    /* projection: rows land on the simplex, wide and one-wide rows too */
    for (int t = 0; t < 200; ++t) {
        double v[64], y[64];
        const int c = 1 + t % 64;
        for (int k = 0; k < c; ++k)
            v[k] = (urand() - 0.5) * (t % 3 == 0 ? 1e6 : 3.0);
        fcref_project_simplex(c, v, y);
        double s = 0.0;
        for (int k = 0; k < c; ++k) {
            CHECK(y[k] >= 0.0);
            s += y[k];
        }
        CHECK(fabs(s - 1.0) <= 1e-9);
    }
    for (int i = 0; i < N * C; ++i)
        Y[i] = X[i] + 0.3 * (urand() - 0.5);
    fcref_project_columns(N, C, Y, Y);
    /* structured loss against the double sum, both diagonal modes */
    for (int unit = 0; unit < 2; ++unit) {
        double def = 0.0;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                double d = 0.0;
                for (int k = 0; k < C; ++k)
                    d += X[i * C + k] * X[j * C + k];
                const double s = A[i][j] + (unit && i == j ? 1.0 : 0.0);
                def += (s - d) * (s - d);
            }
        const double f = fcref_loss(N, row_ptr, col, val, unit, C, X);
        CHECK(fabs(f - def) <= 1e-11 * def);
    }
    CHECK(fcref_norm_s_sq(N, row_ptr, val, 1) > (double)N);
    fcref_x_s(N, row_ptr, col, val, 1, C, X, XS);
    fcref_share(N, C, X, G);
    fcref_gradient(N, row_ptr, col, val, 1, C, X, grad);
    fcref_hvp(N, row_ptr, col, val, 1, C, X, Y, HV);
    {
        int64_t rows[3] = {0, 7, N - 1};
        int64_t sub_rp[4] = {0};
        int32_t sub_col[3 * N];
        double sub_val[3 * N], sub_xs[3 * C];
        for (int r = 0; r < 3; ++r) {
            const int64_t i = rows[r], len = row_ptr[i + 1] - row_ptr[i];
            memcpy(sub_col + sub_rp[r], col + row_ptr[i], sizeof(int32_t) * len);
            memcpy(sub_val + sub_rp[r], val + row_ptr[i], sizeof(double) * len);
            sub_rp[r + 1] = sub_rp[r] + len;
        }
        fcref_x_s_rows(3, rows, sub_rp, sub_col, sub_val, 1, C, X, sub_xs);
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < C; ++k)
                CHECK(fabs(sub_xs[r * C + k] - XS[rows[r] * C + k]) <= 1e-14);
    }
    int its = 0;
    const double spec = fcref_spectral_norm(N, row_ptr, col, val, 1, 1000, 1e-12, &its);
    CHECK(spec > 1.0 && its >= 1);
    /* solver: GPA, FISTA, backtracking, a schedule and the stop rules */
    const int K = 12;
    double f_log[K + 1], tau_log[K + 1], r_log[K + 1], Xout[N * C], sched[K];
    int32_t trials[K + 1], reason = -1;
    for (int k = 0; k < K; ++k)
        sched[k] = 1e-3 * (1 + k % 3);
    for (int mode = 0; mode < 5; ++mode) {
        fcref_opts o;
        memset(&o, 0, sizeof(o));
        o.accelerate = mode != 0;
        o.max_iter = K;
        o.backtrack = mode == 2;
        o.step = 1.0 / (4.0 * spec + 12.0 * N);
        o.L0 = 1.0;
        o.eta = 2.0;
        o.tol_loss = mode == 4 ? 0.0 : NAN;
        o.tol_pgrad = mode == 3 ? 0.5 : 0.0;
        o.step_schedule = mode == 1 ? sched : NULL;
        const int done = fcref_solve(N, row_ptr, col, val, 1, C, X, &o, Xout, f_log, tau_log, trials,
                                     r_log, &reason);
        CHECK(done >= 1 && done <= K);
        for (int i = 0; i < N; ++i) {
            double s = 0.0;
            for (int k = 0; k < C; ++k)
                s += Xout[i * C + k];
            CHECK(fabs(s - 1.0) <= 1e-12);
        }
        for (int it = 1; it <= done; ++it)
            CHECK(isfinite(f_log[it]) && tau_log[it] > 0.0 && trials[it] >= 1 && r_log[it] >= 0.0);
    }
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle: all checks passed\n");
    return 0;
}
