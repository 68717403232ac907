/*
 * fcref.c -- FP64 CPU oracle for similarity-based fuzzy clustering by
 * (accelerated) gradient projection.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * HIP path is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the library never does.  It
 * shares no code, header or table with the HIP path.
 *
 * Problem (P), section 2: minimise f(X) = sum_i sum_j (s_ij - x_i . x_j)^2
 * = ||S - X^T X||_F^2 over X in Omega, the product of N unit simplices
 * (one per column x_i of the C x N membership matrix X).
 *
 * Memory layout: X is C x N with column x_i (the memberships of article i)
 * stored contiguously, i.e. X[i*C + k] = x_{k i}.  S is sparse, symmetric and
 * given in CSR form; because S is symmetric its column s_i equals its row i,
 * so the products X s_i of section 3 are read row by row from the CSR arrays.
 *
 * Diagonal convention: with diag_unit = 1 the similarity used is S + I (the
 * paper builds S from the adjacency matrix plus ones on the diagonal, Example
 * 4.1 and the hyperparameter paragraph of section 5) and the CSR arrays must
 * hold no diagonal entry; with diag_unit = 0 the CSR arrays are S itself.
 *
 * Arithmetic is IEEE double throughout.  Reductions that combine values from
 * different columns run in a fixed order (sequentially in column order, or in
 * fixed blocks of consecutive columns added in block order), so every result
 * is the same for any number of OpenMP threads.
 */
#define _POSIX_C_SOURCE 199309L
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of OpenMP threads the parallel loops below use (1 without OpenMP). */
int fcref_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ||S||_F^2 of the similarity in use: the sum of squared stored values, plus
 * N ones from the implicit unit diagonal when diag_unit = 1.  This is the
 * constant first term of the structured loss (section 3, "Loss Update"). */
double fcref_norm_s_sq(int64_t n, const int64_t *row_ptr, const double *val,
                       int diag_unit)
{
    double acc = 0.0;
    for (int64_t e = 0; e < row_ptr[n]; ++e)
        acc += val[e] * val[e];
    if (diag_unit)
        acc += (double)n;
    return acc;
}

/* The N products X s_i of eq. (gradient_column), one C-vector per article:
 * (X s_i)_k = sum_j x_{kj} s_{ji}.  Output XS has the layout of X. */
void fcref_x_s(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
               const double *val, int diag_unit, int C, const double *X,
               double *XS)
{
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double *out = XS + i * C;
        for (int k = 0; k < C; ++k)
            out[k] = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const double s = val[e];
            const double *xj = X + (int64_t)col_idx[e] * C;
            for (int k = 0; k < C; ++k)
                out[k] += s * xj[k];
        }
        if (diag_unit) {
            const double *xi = X + i * C;
            for (int k = 0; k < C; ++k)
                out[k] += xi[k];
        }
    }
}

/* share = X X^T, the C x C matrix shared by all column updates (Alg. 2):
 * the sum of the outer products x_i x_i^T over the columns.  The columns are
 * taken in blocks of SHARE_BLOCK consecutive indices; each block is summed in
 * column order and the block sums are added in block order, so the result is
 * the same for any number of threads. */
#define SHARE_BLOCK 65536
void fcref_share(int64_t n, int C, const double *X, double *share)
{
    const int64_t nb = (n + SHARE_BLOCK - 1) / SHARE_BLOCK;
    const size_t cc = (size_t)C * (size_t)C;
    memset(share, 0, sizeof(double) * cc);
    if (nb == 0)
        return;
    double *part = (double *)calloc((size_t)nb * cc, sizeof(double));
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < nb; ++b) {
        double *pb = part + (size_t)b * cc;
        const int64_t end = (b + 1) * SHARE_BLOCK < n ? (b + 1) * SHARE_BLOCK : n;
        for (int64_t i = b * SHARE_BLOCK; i < end; ++i) {
            const double *xi = X + i * C;
            for (int k = 0; k < C; ++k)
                for (int l = 0; l < C; ++l)
                    pb[k * C + l] += xi[k] * xi[l];
        }
    }
    for (int64_t b = 0; b < nb; ++b)
        for (size_t q = 0; q < cc; ++q)
            share[q] += part[(size_t)b * cc + q];
    free(part);
}

/* The products X s_i of eq. (gradient_column) for a list of m articles only:
 * rows[r] is the article, and sub_row_ptr / sub_col_idx / sub_val hold that
 * article's row of S (its column, S being symmetric) as entries
 * sub_row_ptr[r] .. sub_row_ptr[r+1]-1 of the two arrays.  X is the full
 * C x N membership matrix.  Output XS is m x C. */
void fcref_x_s_rows(int64_t m, const int64_t *rows, const int64_t *sub_row_ptr,
                    const int32_t *sub_col_idx, const double *sub_val, int diag_unit,
                    int C, const double *X, double *XS)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < m; ++r) {
        double *out = XS + r * C;
        for (int k = 0; k < C; ++k)
            out[k] = 0.0;
        for (int64_t e = sub_row_ptr[r]; e < sub_row_ptr[r + 1]; ++e) {
            const double s = sub_val[e];
            const double *xj = X + (int64_t)sub_col_idx[e] * C;
            for (int k = 0; k < C; ++k)
                out[k] += s * xj[k];
        }
        if (diag_unit) {
            const double *xi = X + rows[r] * C;
            for (int k = 0; k < C; ++k)
                out[k] += xi[k];
        }
    }
}

/* Euclidean projection of one C-vector onto the unit simplex (the projection
 * problem of section 2), written from its optimality conditions rather than
 * from the sorting procedure of Alg. 1.  The minimiser is y_k = max(x_k - theta, 0)
 * for the one theta at which h(theta) = sum_k max(x_k - theta, 0) equals 1.
 * h is continuous and non-increasing, h(max_k x_k - 1) >= 1 (the largest term
 * alone is 1) and h(max_k x_k) = 0, so theta lies in that bracket and bisection
 * narrows it until the two ends are adjacent doubles (or 200 halvings).  The
 * bracket then fixes the support A = {k : x_k > lo}, and theta is formed from
 * the support alone as (sum_{k in A} x_k - 1) / |A|, the condition h = 1
 * restricted to A.  A component that lies inside the final bracket changes
 * that value by no more than the bracket's width, so including it is harmless.
 * x and y may alias. */
static double simplex_excess(int C, const double *x, double theta)
{
    double h = 0.0;
    for (int k = 0; k < C; ++k)
        if (x[k] > theta)
            h += x[k] - theta;
    return h - 1.0;
}

void fcref_project_simplex(int C, const double *x, double *y)
{
    double top = x[0];
    for (int k = 1; k < C; ++k)
        if (x[k] > top)
            top = x[k];
    double lo = top - 1.0, hi = top;  /* h(lo) >= 0 > h(hi) */
    for (int pass = 0; pass < 200; ++pass) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi))
            break;
        if (simplex_excess(C, x, mid) >= 0.0)
            lo = mid;
        else
            hi = mid;
    }
    double sum = 0.0;
    int count = 0;
    for (int k = 0; k < C; ++k)
        if (x[k] > lo) {
            sum += x[k];
            ++count;
        }
    const double theta = (sum - 1.0) / (double)count;
    for (int k = 0; k < C; ++k) {
        const double v = x[k] - theta;
        y[k] = v > 0.0 ? v : 0.0;
    }
}

/* P_Omega applied column by column (section 2, "Projection onto Omega"). */
void fcref_project_columns(int64_t n, int C, const double *V, double *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        fcref_project_simplex(C, V + i * C, out + i * C);
}

/* Structured loss of Alg. 3: f(X) = ||S||_F^2 + ||share||_F^2 - 2 merge with
 * merge = sum_i prod_i and prod_i = <X s_i, x_i>.  Given share and the
 * products X s_i already computed, no N x N matrix is formed. */
static double loss_from_parts(int64_t n, int C, double s_sq, const double *share,
                              const double *X, const double *XS, double *prod)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double p = 0.0;
        for (int k = 0; k < C; ++k)
            p += XS[i * C + k] * X[i * C + k];
        prod[i] = p;
    }
    double merge = 0.0;
    for (int64_t i = 0; i < n; ++i)
        merge += prod[i];
    double share_sq = 0.0;
    for (int k = 0; k < C * C; ++k)
        share_sq += share[k] * share[k];
    return s_sq + share_sq - 2.0 * merge;
}

double fcref_loss(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                  const double *val, int diag_unit, int C, const double *X)
{
    double *XS = (double *)malloc(sizeof(double) * (size_t)n * C);
    double *prod = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *share = (double *)malloc(sizeof(double) * (size_t)C * C);
    fcref_x_s(n, row_ptr, col_idx, val, diag_unit, C, X, XS);
    fcref_share(n, C, X, share);
    const double s_sq = fcref_norm_s_sq(n, row_ptr, val, diag_unit);
    const double f = loss_from_parts(n, C, s_sq, share, X, XS, prod);
    free(XS);
    free(prod);
    free(share);
    return f;
}

/* Column i of the gradient, eq. (gradient_column): -4 (X s_i - share x_i). */
static void gradient_from_parts(int64_t n, int C, const double *share,
                                const double *X, const double *XS, double *grad)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double *xi = X + i * C;
        for (int k = 0; k < C; ++k) {
            double sx = 0.0;
            for (int l = 0; l < C; ++l)
                sx += share[k * C + l] * xi[l];
            grad[i * C + k] = -4.0 * (XS[i * C + k] - sx);
        }
    }
}

void fcref_gradient(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                    const double *val, int diag_unit, int C, const double *X,
                    double *grad)
{
    double *XS = (double *)malloc(sizeof(double) * (size_t)n * C);
    double *share = (double *)malloc(sizeof(double) * (size_t)C * C);
    fcref_x_s(n, row_ptr, col_idx, val, diag_unit, C, X, XS);
    fcref_share(n, C, X, share);
    gradient_from_parts(n, C, share, X, XS, grad);
    free(XS);
    free(share);
}

/* The Hessian of f at X applied to a direction V, eq. (hessian) of
 * Theorem 4.1: -4 V (S - X^T X) + 4 X (V^T X + X^T V).  Column i of it is
 *   -4 (V s_i - sum_j v_j (x_j . x_i)) + 4 sum_j x_j ((v_j . x_i) + (x_j . v_i)),
 * which with share = X X^T and cross = X V^T (both C x C) is
 *   -4 V s_i + 4 (cross^T + cross) x_i + 4 share v_i
 * (the term V X^T x_i = cross^T x_i).  X, V and the result HV share the
 * layout of X. */
void fcref_hvp(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
               const double *val, int diag_unit, int C, const double *X,
               const double *V, double *HV)
{
    double *VS = (double *)malloc(sizeof(double) * (size_t)n * C);
    double *share = (double *)malloc(sizeof(double) * (size_t)C * C);
    double *cross = (double *)calloc((size_t)C * C, sizeof(double));
    fcref_x_s(n, row_ptr, col_idx, val, diag_unit, C, V, VS);
    fcref_share(n, C, X, share);
    for (int64_t j = 0; j < n; ++j) {          /* cross = sum_j x_j v_j^T */
        const double *xj = X + j * C, *vj = V + j * C;
        for (int k = 0; k < C; ++k)
            for (int l = 0; l < C; ++l)
                cross[k * C + l] += xj[k] * vj[l];
    }
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double *xi = X + i * C, *vi = V + i * C;
        for (int k = 0; k < C; ++k) {
            double a = 0.0, b = 0.0;
            for (int l = 0; l < C; ++l) {
                a += (cross[l * C + k] + cross[k * C + l]) * xi[l];
                b += share[k * C + l] * vi[l];
            }
            HV[i * C + k] = -4.0 * VS[i * C + k] + 4.0 * a + 4.0 * b;
        }
    }
    free(VS);
    free(share);
    free(cross);
}

/* Spectral norm ||S||_2 of the (symmetric, nonnegative) similarity in use, by
 * power iteration from the normalised all-ones vector: v <- S v / ||S v||,
 * estimate ||S v||.  Stops when the estimate changes by less than rtol
 * relatively, or after max_iter products.  Theorem 3.1 needs ||S||_2 for its
 * step-size bound 1/(4 ||S||_2 + 12 N). */
double fcref_spectral_norm(int64_t n, const int64_t *row_ptr,
                           const int32_t *col_idx, const double *val,
                           int diag_unit, int max_iter, double rtol, int *iters)
{
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        v[i] = 1.0 / sqrt((double)n);
    double est = 0.0;
    int it = 0;
    for (it = 1; it <= max_iter; ++it) {
        fcref_x_s(n, row_ptr, col_idx, val, diag_unit, 1, v, w);
        double nrm = 0.0;
        for (int64_t i = 0; i < n; ++i)
            nrm += w[i] * w[i];
        nrm = sqrt(nrm);
        const double prev = est;
        est = nrm;
        if (nrm == 0.0)
            break;
        for (int64_t i = 0; i < n; ++i)
            v[i] = w[i] / nrm;
        if (it > 1 && fabs(est - prev) <= rtol * est)
            break;
    }
    if (iters)
        *iters = it > max_iter ? max_iter : it;
    free(v);
    free(w);
    return est;
}

/* Options of fcref_solve. */
typedef struct {
    int32_t accelerate;   /* 1: parallel FISTA (Alg. 4); 0: parallel GPA (Alg. 2/3) */
    int32_t max_iter;     /* number of projected-gradient steps n = 1..max_iter */
    int32_t backtrack;    /* 0: constant step; 1: backtracking on L (Beck and Teboulle) */
    int32_t reserved;
    double step;          /* constant step size tau (backtrack = 0, no schedule) */
    double L0;            /* backtracking: initial L */
    double eta;           /* backtracking: growth factor of L on a rejected trial */
    double tol_loss;      /* loss-decrease stop of Alg. 3/4; NaN disables it */
    double tol_pgrad;     /* stop when r_n <= tol_pgrad * r_1; <= 0 disables it */
    const double *step_schedule; /* if non-NULL: tau_n for n = 1..max_iter */
} fcref_opts;

/* Stop reasons written to *stop_reason. */
enum { FCREF_STOP_MAXITER = 0, FCREF_STOP_LOSS = 1, FCREF_STOP_PGRAD = 2,
       FCREF_STOP_STEP = 3 };

/* The solver of Alg. 4 (accelerate = 1) and of Alg. 2/3 (accelerate = 0, no
 * inertial term, so every step starts from the previous output).
 *
 * State: the latest output Xbar, the output before it, the point Y at which
 * the next gradient is taken, and the scalar t of the inertial sequence.  All
 * three points start at X0, t starts at 1, and the loss of X0 is recorded.
 * Each iteration n takes a projected gradient step from Y_n: the gradient is
 * formed column by column from share = Y_n Y_n^T and the products Y_n s_i
 * (eq. gradient_column), every column of Y_n - tau_n grad is projected onto
 * the simplex, and the result becomes Xbar_n, whose loss is formed from its
 * own share and products (the structured loss of Alg. 3).  The run ends after
 * max_iter iterations, or earlier when the loss fell by no more than tol_loss
 * (read as a decrease test; Xbar_n is the output).  Otherwise t is advanced by
 * t <- (1 + sqrt(1 + 4 t^2)) / 2 and Y_{n+1} moves from Xbar_n along
 * Xbar_n - Xbar_{n-1} by the weight (t_old - 1) / t_new (zero for GPA).
 *
 * Step size: a constant tau, a given schedule tau_n, or backtracking on
 * L = 1/tau: starting from L_{n-1}, accept the trial p = P(Y - grad/L) when
 * f(p) <= f(Y) + <grad, p - Y> + (L/2) ||p - Y||^2, else multiply L by eta.
 * The paper cites this rule for FISTA but runs constant steps only.
 *
 * Gradient-mapping measure: r_n = ||Y_n - Xbar_n||_F / tau_n, the norm of the
 * projected-gradient step taken at iteration n; the relative stop compares it
 * with r_1.
 *
 * Logs (each may be NULL): f_log[0..it], tau_log[1..it], trials_log[1..it],
 * r_log[1..it].  Returns the number of completed iterations; X_out receives
 * the output Xbar of the last completed iteration.
 *
 * Parity unpinned (inertial trajectory): the paper prints no value of an
 * accelerated run, so the inertial sequence is checked only through what
 * fixes it otherwise -- with the inertial term dropped it is the GPA of
 * Example 4.1 and Theorem 3.1 (pinned); a planted exact factorisation is a
 * fixed point; the first two steps coincide with GPA (beta_1 = 0) and the
 * third differs; and an independent dense re-implementation agrees.  The
 * backtracking rule is not in the paper either: it is checked by its
 * acceptance test and the minimality of the accepted L.
 */
int fcref_solve_timed(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                      const double *val, int diag_unit, int C, const double *X0,
                      const fcref_opts *opt, double *X_out, double *f_log,
                      double *tau_log, int32_t *trials_log, double *r_log,
                      int32_t *stop_reason, double *seconds_log);

int fcref_solve(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                const double *val, int diag_unit, int C, const double *X0,
                const fcref_opts *opt, double *X_out, double *f_log,
                double *tau_log, int32_t *trials_log, double *r_log,
                int32_t *stop_reason)
{
    return fcref_solve_timed(n, row_ptr, col_idx, val, diag_unit, C, X0, opt, X_out, f_log,
                             tau_log, trials_log, r_log, stop_reason, NULL);
}

static double wall_seconds(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* fcref_solve, also recording the wall time of every iteration in
 * seconds_log[1..it] (may be NULL); the arithmetic is the same. */
int fcref_solve_timed(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                      const double *val, int diag_unit, int C, const double *X0,
                      const fcref_opts *opt, double *X_out, double *f_log,
                      double *tau_log, int32_t *trials_log, double *r_log,
                      int32_t *stop_reason, double *seconds_log)
{
    const size_t nc = (size_t)n * (size_t)C;
    double *Xbar = (double *)malloc(sizeof(double) * nc);      /* Xbar_n     */
    double *Xprev = (double *)malloc(sizeof(double) * nc);     /* Xbar_{n-1} */
    double *Y = (double *)malloc(sizeof(double) * nc);         /* Y_n        */
    double *YS = (double *)malloc(sizeof(double) * nc);        /* Y_n s_i    */
    double *grad = (double *)malloc(sizeof(double) * nc);
    double *V = (double *)malloc(sizeof(double) * nc);
    double *P = (double *)malloc(sizeof(double) * nc);         /* trial      */
    double *PS = (double *)malloc(sizeof(double) * nc);
    double *prod = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *share = (double *)malloc(sizeof(double) * (size_t)C * C);
    double *share_p = (double *)malloc(sizeof(double) * (size_t)C * C);

    const double s_sq = fcref_norm_s_sq(n, row_ptr, val, diag_unit);

    memcpy(Xbar, X0, sizeof(double) * nc);
    memcpy(Xprev, X0, sizeof(double) * nc);
    memcpy(Y, X0, sizeof(double) * nc);
    fcref_x_s(n, row_ptr, col_idx, val, diag_unit, C, X0, PS);
    fcref_share(n, C, X0, share_p);
    double loss_prev = loss_from_parts(n, C, s_sq, share_p, X0, PS, prod);
    if (f_log)
        f_log[0] = loss_prev;
    memcpy(X_out, X0, sizeof(double) * nc);

    double t = 1.0, L = opt->backtrack ? opt->L0 : 0.0, r1 = 0.0;
    int completed = 0, failed = 0;
    int32_t reason = FCREF_STOP_MAXITER;
    for (int it = 1; it <= opt->max_iter; ++it) {
        const double t_start = wall_seconds();
        /* projected gradient step at Y_n */
        fcref_x_s(n, row_ptr, col_idx, val, diag_unit, C, Y, YS);
        fcref_share(n, C, Y, share);
        gradient_from_parts(n, C, share, Y, YS, grad);

        double tau;
        int trials = 1;
        double loss_p;
        if (!opt->backtrack) {
            tau = opt->step_schedule ? opt->step_schedule[it - 1] : opt->step;
            #pragma omp parallel for schedule(static)
            for (int64_t e = 0; e < (int64_t)nc; ++e)
                V[e] = Y[e] - tau * grad[e];
            fcref_project_columns(n, C, V, P);
            fcref_x_s(n, row_ptr, col_idx, val, diag_unit, C, P, PS);
            fcref_share(n, C, P, share_p);
            loss_p = loss_from_parts(n, C, s_sq, share_p, P, PS, prod);
        } else {
            const double loss_y = loss_from_parts(n, C, s_sq, share, Y, YS, prod);
            for (;;) {
                tau = 1.0 / L;
                #pragma omp parallel for schedule(static)
                for (int64_t e = 0; e < (int64_t)nc; ++e)
                    V[e] = Y[e] - tau * grad[e];
                fcref_project_columns(n, C, V, P);
                fcref_x_s(n, row_ptr, col_idx, val, diag_unit, C, P, PS);
                fcref_share(n, C, P, share_p);
                loss_p = loss_from_parts(n, C, s_sq, share_p, P, PS, prod);
                double lin = 0.0, sq = 0.0;
                for (size_t e = 0; e < nc; ++e) {
                    const double d = P[e] - Y[e];
                    lin += grad[e] * d;
                    sq += d * d;
                }
                if (loss_p <= loss_y + lin + 0.5 * L * sq)
                    break;
                if (!isfinite(L) || trials >= 1000) {
                    reason = FCREF_STOP_STEP;
                    failed = 1;
                    break;
                }
                L *= opt->eta;
                ++trials;
            }
            if (failed)
                break;
        }

        /* Xbar_n := trial; keep Xbar_{n-1} for the inertial term */
        double *tmp = Xprev;
        Xprev = Xbar;
        Xbar = P;
        P = tmp;
        completed = it;

        double r2 = 0.0;
        for (size_t e = 0; e < nc; ++e) {
            const double d = Y[e] - Xbar[e];
            r2 += d * d;
        }
        const double r = sqrt(r2) / tau;
        if (it == 1)
            r1 = r;
        if (f_log)
            f_log[it] = loss_p;
        if (tau_log)
            tau_log[it] = tau;
        if (trials_log)
            trials_log[it] = trials;
        if (r_log)
            r_log[it] = r;
        memcpy(X_out, Xbar, sizeof(double) * nc);

        if (!isnan(opt->tol_loss) && loss_prev - loss_p <= opt->tol_loss) {
            reason = FCREF_STOP_LOSS;
            break;
        }
        if (opt->tol_pgrad > 0.0 && r <= opt->tol_pgrad * r1) {
            reason = FCREF_STOP_PGRAD;
            break;
        }
        loss_prev = loss_p;

        /* inertial parameter and accelerated term */
        const double t_next = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
        const double beta = opt->accelerate ? (t - 1.0) / t_next : 0.0;
        #pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < (int64_t)nc; ++e)
            Y[e] = Xbar[e] + beta * (Xbar[e] - Xprev[e]);
        t = t_next;
        if (seconds_log)
            seconds_log[it] = wall_seconds() - t_start;
    }

    if (stop_reason)
        *stop_reason = reason;
    free(Xbar);
    free(Xprev);
    free(Y);
    free(YS);
    free(grad);
    free(V);
    free(P);
    free(PS);
    free(prod);
    free(share);
    free(share_p);
    return completed;
}
