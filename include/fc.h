/*
 * fc.h -- C ABI of the MI355X (gfx950) solver for similarity-based fuzzy
 * clustering by accelerated gradient projection.
 *
 * Problem (P), section 2: given a sparse symmetric similarity S (N x N) and a
 * number of clusters C, minimise f(X) = ||S - X^T X||_F^2 over membership
 * matrices X whose N columns lie on the unit simplex of R^C.  This library
 * stores X^T: U is an n x c row-major matrix whose row i is the column x_i of
 * the paper (n = N, c = C), so every row of U is non-negative and sums to 1.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named "device" must be HIP device memory (hipMalloc'd, or a
 *   torch CUDA tensor's data_ptr()).  Pointers named "host" are host memory.
 * - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *   All device work is enqueued on that stream.  Calls that return scalars
 *   (fc_step, fc_solve, fc_objective, fc_gram, fc_spectral_norm, fc_create,
 *   fc_curvature) and fc_hessian_vector synchronise that stream before
 *   returning; fc_project, fc_spmm and fc_get_u only enqueue work.
 * - S is borrowed: the caller keeps its arrays alive and unmodified until
 *   fc_destroy of every solver built on it.  U0 is copied at fc_create.
 *   Output buffers are caller-allocated.
 * - Every call returns an fc_status; no C++ exception crosses this ABI.
 *   On an error the thread-local message of fc_last_error() says what failed.
 *   A solver handle stays valid after FC_ERR_NONFINITE or FC_ERR_STEP and
 *   keeps the last accepted iterate.
 * - One handle must not be used by two threads at once; distinct handles
 *   are independent.
 * - Arithmetic: FC_PREC_FP64 computes in double; FC_PREC_FP32 stores U, the
 *   products S U and S values in float and accumulates in float, with every
 *   reduction across rows (Gram matrices, the trace term, the line-search
 *   quantities, the simplex threshold sums) carried in double;
 *   FC_PREC_MIXED additionally stores S values as half and keeps a bfloat16
 *   copy of U for the sparse product.
 */
#ifndef FC_H
#define FC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FC_OK = 0,
    FC_ERR_INVALID_ARG = 1,   /* a pointer, size or option is out of range */
    FC_ERR_UNSUPPORTED = 2,   /* a valid request this build does not implement */
    FC_ERR_OUT_OF_MEMORY = 3, /* a device allocation failed */
    FC_ERR_DEVICE = 4,        /* a HIP runtime call failed */
    FC_ERR_NONFINITE = 5,     /* the objective or an iterate became NaN/Inf */
    FC_ERR_STEP = 6,          /* backtracking could not find an acceptable L */
    FC_ERR_NOT_SYMMETRIC = 7, /* validation found S != S^T or a bad CSR */
    FC_ERR_CANCELLED = 8      /* a served request stopped by fc_server_cancel */
} fc_status;

typedef enum { FC_F64 = 0, FC_F32 = 1, FC_F16 = 2, FC_BF16 = 3 } fc_dtype;
typedef enum { FC_PREC_FP64 = 0, FC_PREC_FP32 = 1, FC_PREC_MIXED = 2 } fc_precision;

/* Diagonal of the similarity.  The objective sums over all pairs (i, j)
 * including i = j (problem (P)).  FC_DIAG_STORED uses the CSR arrays as S.
 * FC_DIAG_UNIT uses S + I: the paper builds S as the adjacency matrix plus
 * ones on the diagonal (Example 4.1; hyperparameters of section 5), and in
 * this mode the CSR arrays must not store diagonal entries. */
typedef enum { FC_DIAG_STORED = 0, FC_DIAG_UNIT = 1 } fc_diag;

/* Step rule.  FC_STEP_FIXED: a constant step size tau (Alg. 2-4), or the
 * per-iteration schedule of fc_options.step_schedule.  FC_STEP_BACKTRACK:
 * L = 1/tau grows by eta until the sufficient-decrease test
 * f(p) <= f(Y) + <grad f(Y), p - Y> + (L/2) ||p - Y||^2 holds (the FISTA
 * backtracking rule of Beck and Teboulle, which the paper cites for FISTA). */
typedef enum { FC_STEP_FIXED = 0, FC_STEP_BACKTRACK = 1 } fc_step_rule;

typedef enum {
    FC_STOP_NONE = 0,     /* still running / stopped by the iteration budget */
    FC_STOP_MAXITER = 1,  /* fc_options.max_iter accepted iterations done */
    FC_STOP_LOSS = 2,     /* loss decrease <= tol_loss (Alg. 3 and Alg. 4) */
    FC_STOP_PGRAD = 3,    /* gradient-mapping norm <= tol_pgrad * first one */
    FC_STOP_ERROR = 4     /* FC_ERR_NONFINITE or FC_ERR_STEP */
} fc_stop_reason;

/* Symmetric sparse similarity in CSR form (device arrays).  row_ptr has
 * n + 1 int64 entries with row_ptr[0] = 0 and row_ptr[n] = nnz; col_idx has
 * nnz int32 column indices in [0, n); values has nnz entries of
 * values_dtype (FC_F64, FC_F32 or FC_F16).  Column order within a row is
 * free.  S must equal S^T: the gradient formula of eq. (gradient_matrix)
 * holds only for symmetric S. */
typedef struct {
    int64_t n;
    int64_t nnz;
    const int64_t *row_ptr;
    const int32_t *col_idx;
    const void *values;
    fc_dtype values_dtype;
} fc_csr;

typedef struct {
    uint32_t struct_size;      /* sizeof(fc_options), set by fc_options_default */
    int32_t c;                 /* number of clusters C, 1 <= c <= 64 */
    fc_precision precision;
    fc_diag diag;
    int32_t accelerate;        /* 1: parallel FISTA (Alg. 4); 0: parallel GPA (Alg. 2/3) */
    fc_step_rule step_rule;
    double step;               /* FC_STEP_FIXED: tau; <= 0 means tau = 1/L_thm with
                                  L_thm = 4 ||S||_2 + 12 n (Theorem 3.1), ||S||_2 by
                                  power iteration on the device */
    double L0;                 /* FC_STEP_BACKTRACK: initial L; <= 0 means L_thm / 100 */
    double eta;                /* FC_STEP_BACKTRACK: growth factor of L (> 1; default 2) */
    int32_t max_iter;          /* accepted-iteration budget of fc_solve */
    int32_t check_every;       /* fc_solve/fc_step read the device state back every
                                  check_every launched trials (default 16) */
    double tol_loss;           /* stop when f(Xbar_{n-1}) - f(Xbar_n) <= tol_loss
                                  (Alg. 3/4); NaN disables (default) */
    double tol_pgrad;          /* stop when r_n <= tol_pgrad * r_1, with
                                  r_n = ||Y_n - Xbar_n||_F / tau_n; 0 disables */
    int32_t validate;          /* 1: check CSR structure and symmetry at fc_create */
    int32_t norm_estimate;     /* ||S||_2 in L_thm: 0 = power iteration (default);
                                  1 = the Frobenius norm ||S||_F, an upper bound, as the
                                  paper's experiments do (section 5, hyperparameters) */
    const double *step_schedule; /* host: tau_n for n = 1..step_schedule_len, copied at
                                    fc_create; used by FC_STEP_FIXED when non-NULL */
    int32_t step_schedule_len;
    int32_t reorder;           /* fc_reorder: FC_REORDER_NONE (default),
                                  FC_REORDER_DEGREE or FC_REORDER_GIVEN, see below */
    int32_t defer_loss;        /* 1: deferred loss evaluation, see below (default 0) */
    int32_t single_pass;       /* 1: single-pass iteration, see below (default 0) */
    const int32_t *perm;       /* host, n entries, FC_REORDER_GIVEN only: internal row
                                  i is the caller's row perm[i]; read during
                                  fc_create only (default NULL) */
} fc_options;

/* Internal numbering of the articles.  FC_REORDER_DEGREE renumbers them by
 * descending number of stored nonzeros (ties by index) inside fc_create: the
 * library keeps a permuted copy of S (row_ptr, col_idx and values: 12 bytes
 * per nonzero in FP32, plus 8 bytes per row) and permutes U0 on the way in
 * and the iterate on the way out (fc_get_u), so callers see their own order.
 * Problem (P) is invariant under renumbering the articles, and every row of
 * the sparse product sums the same terms in the same order; only the order of
 * the cross-article reductions (share, the loss terms) changes, so results
 * agree with FC_REORDER_NONE to rounding.  On power-law graphs it places the
 * rows that most nonzeros gather next to each other, which raises cache reuse
 * in the sparse product.  FC_REORDER_GIVEN takes the caller's order instead
 * (options.perm, a host array), for orders built outside the library, such as
 * a breadth-first (Cuthill-McKee) or community order.  fc_create checks on the
 * host that perm holds every row of 0..n-1 exactly once, before any device
 * work reads it, and fails with FC_ERR_INVALID_ARG otherwise.  It then keeps
 * the same permuted copy of S as for FC_REORDER_DEGREE, with the same results
 * up to rounding.  Given the descending-degree order itself, results equal
 * FC_REORDER_DEGREE bit for bit.  Relabelling needs n < 2^31.  Checkpoints
 * record the mode, and for FC_REORDER_GIVEN a 64-bit fingerprint (FNV-1a) of
 * perm.  fc_set_state rejects a state taken under another numbering.  The
 * serving engine checks perm in fc_server_submit and keeps its own copy, so
 * the caller's array may be released when submit returns. */
typedef enum { FC_REORDER_NONE = 0, FC_REORDER_DEGREE = 1, FC_REORDER_GIVEN = 2 } fc_reorder;

/* Deferred loss evaluation (defer_loss = 1, constant or scheduled steps only:
 * backtracking needs each trial's loss at once and rejects it).  The
 * structured loss of Alg. 3 needs sum_i <x_i, (S X)_i> for every accepted
 * iterate.  By default the sparse product forms these terms as it writes
 * S Xbar_n, which makes it read Xbar_n's own rows once more.  With
 * defer_loss = 1 the product stores only the off-diagonal part S_off Xbar_n
 * and the next fused pass, which reads Xbar_n and that product anyway, adds
 * the unit diagonal back (S_eff Y = S_off Y + Y) and forms the terms; the
 * loss of the last iterate of an fc_step or fc_solve call is formed by one
 * extra pass over Xbar and its product before the call returns.  Every
 * loss is still computed and logged; the loss stop test runs when the loss
 * is known, so a stop at iteration k discards the trial computed from
 * Xbar_k and returns Xbar_k with the same iteration count, loss and stop
 * reason as the default mode.  Iterates agree with the default mode to
 * rounding.  Checkpoints record the mode; the serving engine does not
 * accept it (FC_ERR_UNSUPPORTED). */

/* Single-pass iteration (single_pass = 1; constant or scheduled steps,
 * FC_PREC_FP64 or FC_PREC_FP32, tol_loss NaN).  Each iteration sweeps the
 * rows once: it applies S to the stored extrapolated point Y_n (eq.
 * gradient_column), takes the projected step (Alg. 2 step, Alg. 1) and forms
 * the next extrapolated point Y_{n+1} of Alg. 4 in the same pass, so S is
 * applied once per iteration and only Xbar and the two Y buffers are kept
 * (the default mode stores S Xbar and re-forms Y from two iterates).  The
 * structured loss of Alg. 3 needs S Xbar_n, which this mode never forms
 * inside the iteration: it is evaluated once at the end of every fc_step /
 * fc_solve call, by one pass over the stored entries on and below the
 * diagonal (the cross term sum_i <xbar_i, (S Xbar)_i> is twice that half's
 * sum, diagonal once, which holds because S = S^T), so info.f is the loss of the
 * returned iterate and info.f_prev that of the previous read-out, and the
 * history holds losses only at read-outs (NaN elsewhere).  The gradient-
 * mapping stop is available, the loss stop is not (FC_ERR_UNSUPPORTED).
 * Iterates agree with the default mode to rounding.  Xbar is updated in
 * place, so after FC_ERR_NONFINITE the handle holds the failed iterate.
 * Checkpoints record the mode; the serving engine does not accept it. */

/* Per-solver progress, returned by fc_step and fc_solve. */
typedef struct {
    int32_t iter;          /* accepted iterations so far */
    int32_t trials;        /* step-size trials so far (= iter for fixed steps) */
    int32_t stop_reason;   /* fc_stop_reason */
    int32_t reserved;
    double f;              /* f(Xbar_iter), structured objective, double */
    double f_prev;         /* f(Xbar_{iter-1}) */
    double L;              /* 1 / tau of the last accepted step */
    double t;              /* inertial parameter t_{iter+1} of Alg. 4 */
    double beta;           /* (t_iter - 1) / t_{iter+1}, weight of the next extrapolation */
    double pgrad;          /* r_iter */
    double pgrad_rel;      /* r_iter / r_1 */
} fc_info;

typedef struct fc_solver fc_solver;

/* Fill *opt with defaults: c = 0 (must be set), FP32, unit diagonal,
 * FISTA, fixed step with tau from Theorem 3.1, eta = 2, max_iter = 100,
 * check_every = 16, tol_loss = NaN, tol_pgrad = 0, no validation. */
void fc_options_default(fc_options *opt);

/* Set up a solve of problem (P) (Alg. 4, initialisation): copies U0
 * (device, n x c row-major of u0_dtype; NULL = the constant 1/c start) to
 * Xbar_0, computes ||S||_F^2 and, if needed, ||S||_2 by power iteration,
 * and evaluates f(Xbar_0).  Allocates all device work buffers (six n x c
 * iterate/product buffers, S copies for mixed precision, partial sums).
 * Errors: FC_ERR_INVALID_ARG (NULL pointers, n < 1, c outside [1, 64],
 * dtype/precision mismatch), FC_ERR_NOT_SYMMETRIC (validate = 1),
 * FC_ERR_OUT_OF_MEMORY, FC_ERR_DEVICE.  *out is NULL on error. */
fc_status fc_create(const fc_csr *S, const fc_options *opt, const void *U0,
                    fc_dtype u0_dtype, void *stream, fc_solver **out);

/* Device time per kernel of the launches made by fc_step_profiled. */
typedef struct {
    double fused_ms;    /* extrapolation, gradient, step, projection and Grams (single-
                           pass mode: the single-pass kernel, light rows' products included) */
    double spmm_ms;     /* sparse product S Xbar of the trial point (single-pass mode: its
                           pre-pass over the rows longer than 64 stored nonzeros) */
    double reduce_ms;   /* the fixed-order reductions of the partial sums */
    double control_ms;  /* the one-workgroup controller */
    int32_t launches;   /* trials launched (one launch of each kernel per trial) */
    int32_t reserved;
} fc_kernel_times;

/* Run exactly `iters` more accepted iterations of Alg. 4 (Alg. 2/3 when
 * accelerate = 0) unless a stop rule fires first.  One iteration: the
 * extrapolated point Y_n, the gradient -4 (S Y_n - Y_n Y_n^T Y_n) of
 * eq. (gradient_column), the step and the row-wise simplex projection
 * (Alg. 1), and the structured loss of Alg. 3 at the new iterate.  Fills
 * *info (may be NULL).  Returns FC_ERR_NONFINITE or FC_ERR_STEP when the
 * iteration failed; the handle then holds the last good iterate. */
fc_status fc_step(fc_solver *h, int32_t iters, fc_info *info);

/* fc_step with HIP events recorded on the solver's stream between the
 * kernels of every trial; *times receives the summed device time per kernel
 * (for measurement: the events add a few microseconds per trial). */
fc_status fc_step_profiled(fc_solver *h, int32_t iters, fc_info *info,
                           fc_kernel_times *times);

/* Iterate until a stop rule fires or max_iter accepted iterations are
 * done (counted from fc_create).  Same errors as fc_step. */
fc_status fc_solve(fc_solver *h, fc_info *info);

/* Copy the current iterate Xbar (n x c, row-major, dense) to U_out (device)
 * as FC_F64 or FC_F32.  Enqueued on the solver's stream. */
fc_status fc_get_u(const fc_solver *h, void *U_out, fc_dtype dtype);

/* Per-iteration history (host outputs, each may be NULL): f_log[0..k] the
 * loss of Xbar_0..Xbar_k, step_log[1..k] the accepted tau_n,
 * trials_log[1..k] the trials per iteration, r_log[1..k] the gradient-
 * mapping norms.  `cap` is the capacity of each array in entries; *count
 * receives k + 1.  The solver keeps the history of its first 65,536
 * iterations. */
fc_status fc_get_history(const fc_solver *h, int32_t cap, double *f_log,
                         double *step_log, int32_t *trials_log, double *r_log,
                         int32_t *count);

/* Checkpoint: serialise the solver state (Xbar_n, Xbar_{n-1}, their
 * products S Xbar, the Gram matrix of the next extrapolated point, t, L, f,
 * the iteration counters and the history) into host memory `buf` of
 * *bytes bytes.  With buf = NULL, *bytes receives the size needed; a
 * smaller buffer is FC_ERR_INVALID_ARG.  fc_set_state restores a state taken
 * from a solver built on the same S with the same n, c and options
 * (FC_ERR_INVALID_ARG otherwise); iterating after a restore gives the same
 * results, bit for bit, as iterating without the interruption.
 * Both synchronise the solver's stream. */
fc_status fc_get_state(const fc_solver *h, void *buf, size_t *bytes);
fc_status fc_set_state(fc_solver *h, const void *buf, size_t bytes);

void fc_destroy(fc_solver *h);

/* Structured objective of Alg. 3 for a given U (device, n x c row-major of
 * u_dtype = FC_F64 or FC_F32): f = ||S||_F^2 + ||U^T U||_F^2
 * - 2 sum_i <u_i, (S U)_i>, computed in the precision of u_dtype with the
 * sums across rows in double.  *f_out is a host double. */
fc_status fc_objective(const fc_csr *S, fc_diag diag, const void *U,
                       fc_dtype u_dtype, int32_t c, void *stream, double *f_out);

/* Row-wise Euclidean projection onto the unit simplex (Alg. 1 applied to
 * every row; section 2, "Projection onto Omega"): out_i = P(V_i).  V and out
 * are device arrays of `rows` rows with leading dimension ld >= c (in
 * elements) of dtype FC_F64 or FC_F32; in-place (out == V) is allowed.
 * The threshold sums are carried in double.  Asynchronous. */
fc_status fc_project(const void *V, void *out, fc_dtype dtype, int64_t rows,
                     int32_t c, int64_t ld, void *stream);

/* Kernel-level entry points (the steps of one iteration, for testing and
 * profiling).  fc_spmm: Z = S_eff U for U, Z device n x c row-major of
 * dtype (FC_F64/FC_F32; S values must be of the same type, or FC_F16 with
 * FC_F32 U), i.e. row i of Z is the product X s_i of eq. (gradient_column);
 * asynchronous.  fc_gram: G = U^T U (the paper's share = X X^T, Alg. 2)
 * into a host double c x c array.  fc_spectral_norm: ||S_eff||_2 by power
 * iteration from the normalised ones vector (relative change < rtol or
 * max_iter products), for the step bound of Theorem 3.1. */
fc_status fc_spmm(const fc_csr *S, fc_diag diag, const void *U, void *Z,
                  fc_dtype dtype, int32_t c, void *stream);
fc_status fc_gram(const void *U, fc_dtype dtype, int64_t n, int32_t c,
                  void *stream, double *G_out);
fc_status fc_spectral_norm(const fc_csr *S, fc_diag diag, int32_t max_iter,
                           double rtol, void *stream, double *norm_out,
                           int32_t *iters_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the Gram
 * matrix of fc_gram, G = U^T U, with no allocation of any kind.
 *   U      device, n x c, row i at U + i * ld (ld >= c elements), FC_F64 or
 *          FC_F32; read in place (no padded copy).
 *   G_out  device, c x c doubles, row-major; written on `stream`.
 * The call is asynchronous (it only enqueues kernels on `stream` and never
 * synchronises).  Its partial sums live in a library-owned static device
 * array of FC_GRAM_NOALLOC_SCRATCH_BYTES bytes (about 32 MiB) on each GPU the
 * library runs on, held until the process ends: at most 1,024 wave partials
 * of a 64 x 64 block plus the reduced block, which bounds the workgroups of
 * the pass (every n and every c <= 64 fits).  Every call on one GPU shares
 * that GPU's array, so calls that overlap on the same GPU (two streams, two
 * threads) race: serialise them, e.g. on one stream.  Each call overwrites
 * all the scratch it reads, so no clearing is needed between calls.  The
 * result equals fc_gram's to rounding (the per-tile sums are the same; the
 * cross-tile order may differ for large n).  Errors: FC_ERR_INVALID_ARG
 * (NULL pointers, n < 1, c outside [1, 64], ld < c, dtype), FC_ERR_DEVICE. */
#define FC_GRAM_NOALLOC_SCRATCH_BYTES 33587200
fc_status fc_gram_noalloc(const void *U, fc_dtype dtype, int64_t n, int32_t c, int64_t ld,
                          void *stream, double *G_out);

/* Measurement of the memory system on the sparse product's access pattern
 * (not a step of the method; used to state the product's practical ceiling).
 * For every e in [0, nnz), in order, gathers row col_idx[e] of U (device,
 * `rows` rows of row_bytes = 32, 64, 128 or 256 bytes each, e.g. 32 FP32 or
 * 64 bfloat16 clusters per row, 16-byte aligned) with the product's 16-byte
 * lane loads and folds the bits into a checksum; no values, products or
 * output rows.  Every col_idx[e] must lie in [0, rows) (not checked on the
 * device).  A persistent grid of wg_per_cu (1..64) workgroups per compute
 * unit; one untimed launch, then `reps` timed launches on `stream`;
 * *ms_out (host) receives the mean device time per launch.  Synchronises
 * the stream.  Errors: FC_ERR_INVALID_ARG, FC_ERR_DEVICE. */
fc_status fc_gather_probe(const int32_t *col_idx, int64_t nnz, const void *U, int64_t rows,
                          int32_t row_bytes, int32_t wg_per_cu, int32_t reps, void *stream,
                          double *ms_out);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char *fc_last_error(void);

/* Test hook for the error paths (callers: tests of out-of-memory handling).
 * after >= 0: the next `after` device or pinned-host allocations the library
 * makes (any thread: solvers, stateless calls, the serving worker) succeed
 * and every later one fails as if the GPU were out of memory, until the hook
 * is called again; after < 0 turns it off (the default).  The failing call
 * returns FC_ERR_OUT_OF_MEMORY (a served request gets it as its status) and
 * frees what it had allocated.  Process-wide; not for production use. */
void fc_debug_fail_allocations(int64_t after);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of many solves of problem (P) on one GPU.
 *
 * fc_server_submit queues a solve (any n and c <= 64; FP32; FISTA with a
 * fixed step or backtracking; stop rules as in fc_options).  A worker thread
 * admits queued requests in arrival order while the device memory held by
 * admitted requests stays within hbm_budget and fewer than max_active are
 * running; it sets each one up on its own stream, then advances all running
 * requests together, one trial per tick, with batched kernels grouped by
 * padded c and step rule.  A newly admitted request runs its first trials
 * on its own at once, beside the batch in flight, and joins the batched
 * kernels at the next state poll.  A request gets exactly the arithmetic of
 * fc_create + fc_solve with the same options, so its result does not depend
 * on what it is batched with or when it joins.  Finished requests wait in the server (holding their
 * memory) until fc_server_release.
 * ------------------------------------------------------------------------ */
typedef struct fc_server fc_server;

typedef struct {
    uint32_t struct_size;   /* sizeof(fc_server_opts), set by fc_server_opts_default */
    int32_t max_active;     /* requests iterating at once (default 64) */
    double hbm_budget;      /* bytes of device memory admitted requests may hold
                               (default 32 GiB); a request larger than the whole
                               budget finishes with FC_ERR_OUT_OF_MEMORY */
    int32_t ticks_per_poll; /* trials launched between reads of the request states
                               (default 16) */
    int32_t use_graph;      /* 1: replay each tick from a captured hipGraph on the
                               server's stream; 0 (default): direct launches, one
                               stream per group of requests */
    /* Launch table of the batched kernels, indexed by padded width (0..4 for
       4, 8, 16, 32, 64 columns): persistent workgroups per compute unit that
       walk the (instance, block) tables of the fused kernel (grid_fused) and
       of the sparse product (grid_spmm); 0 = built-in (2 and 8), otherwise
       1..64.  Every table entry does the same work whichever workgroup takes
       it, so these choices change the speed and never a result;
       fc_server_tune measures them. */
    int32_t grid_fused[5];
    int32_t grid_spmm[5];
    /* Solo lane: while at most solo_max requests are active (0..8; default
       4, the hardware queues the GPU gives one process), a newly admitted
       request runs unbatched on a stream of its own, in chunks of
       ticks_per_poll trials, as fc_solve runs it; the worker checks its
       chunks by events instead of a poll of every stream.  0 batches every
       request. */
    int32_t solo_max;
    /* Tile shape of the batched sparse product per padded width: gathers
       each lane slot keeps in flight (2, 4 or 8; 0 = built-in 4).  Every
       slot adds its nonzeros in the same order whatever this is, so it
       changes the speed, never a result; fc_server_tune measures it. */
    int32_t spmm_depth[5];
    int32_t reserved;
} fc_server_opts;

typedef struct {
    uint64_t req_id;
    int32_t status;         /* fc_status of the solve */
    int32_t iter;           /* accepted iterations */
    int32_t trials;
    int32_t stop_reason;    /* fc_stop_reason */
    double f;               /* final loss */
    /* seconds on fc_server_clock(): submission; set-up finished (admitted);
       result seen by the worker's state poll; set-up started (the request
       left the queue); first trial launched */
    double t_submit, t_admit, t_finish, t_setup, t_start;
} fc_result;

void fc_server_opts_default(fc_server_opts *opts);
double fc_server_clock(void);

/* Start a server on the device current in the calling thread; `stream`
 * (hipStream_t on that device, NULL = a new stream) carries the batch tables,
 * the state polls and, with use_graph, the captured ticks; without use_graph
 * each group of requests (padded c, step rule) ticks on a stream of its own
 * so that the groups' kernels overlap.  Errors: FC_ERR_INVALID_ARG,
 * FC_ERR_DEVICE. */
fc_status fc_server_create(const fc_server_opts *opts, void *stream, fc_server **out);

/* Queue one solve.  S (device CSR, FC_F32 values) and U0 (device n x c,
 * FC_F32 or FC_F64, NULL = 1/c) are borrowed until the request's result has
 * been released.  opt must ask for FC_PREC_FP32 and accelerate = 1 and no
 * step schedule (FC_ERR_UNSUPPORTED otherwise).  req_id must be unique among
 * requests not yet released.  Does not block. */
fc_status fc_server_submit(fc_server *sv, const fc_csr *S, const fc_options *opt,
                           const void *U0, fc_dtype u0_dtype, uint64_t req_id);

/* Up to `max` results of finished requests not reported before, waiting up
 * to timeout_us microseconds for at least one; *n_out receives the count. */
fc_status fc_server_poll(fc_server *sv, fc_result *out, int32_t max, int32_t timeout_us,
                         int32_t *n_out);

/* Copy a finished request's memberships (n x c) to U_out (device); blocks
 * until the copy is done.  fc_server_release frees the request's memory. */
fc_status fc_server_get_u(fc_server *sv, uint64_t req_id, void *U_out, fc_dtype dtype);
fc_status fc_server_release(fc_server *sv, uint64_t req_id);

/* Stop a request that is queued or running.  Asynchronous: the worker
 * removes it at its next state poll and reports it through fc_server_poll
 * with status FC_ERR_CANCELLED; a request that had started keeps its last
 * accepted iterate (fc_server_get_u) and its iteration count and loss, one
 * still queued has none.  A request that has already finished is left as it
 * is (FC_OK).  Errors: FC_ERR_INVALID_ARG for an id that is neither queued,
 * running nor finished and unreleased. */
fc_status fc_server_cancel(fc_server *sv, uint64_t req_id);

/* Queue lengths and the device memory held by admitted requests. */
fc_status fc_server_stats(fc_server *sv, int32_t *n_pending, int32_t *n_active,
                          int64_t *n_done, double *bytes_in_use);

/* Stop the worker and free everything, including unreleased results. */
void fc_server_destroy(fc_server *sv);

/* Autotuner of the serving schedule.  Solves the n_req sample requests
 * (S[i], opt[i], U0[i]; U0 may be NULL, or hold NULL entries, for the 1/c
 * start; the same rules as fc_server_submit) through servers created from
 * *base with candidate schedules and keeps the fastest, by coordinate
 * search: first graph replay (off, on) x ticks_per_poll (4, 8, 16, 32) on
 * all requests, then for each padded width present in the sample
 * grid_fused (1, 2, 4), grid_spmm (4, 8, 16, 32) and the sparse product's
 * tile shape spmm_depth (2, 4, 8) on that width's requests alone.  A candidate's time runs from the first submission to the
 * last result (set-up included), all requests submitted at once.  Every run
 * must return, for every request, the same status, iteration and trial
 * counts and bitwise the same final loss as the first run; otherwise
 * FC_ERR_DEVICE.  On FC_OK *best holds *base with the chosen schedule,
 * *solves_per_s the rate of a final run of all requests with it, and
 * *n_runs (may be NULL) the number of server runs made.  Blocks until done;
 * every request's memory is released before it returns.  Errors: those of
 * the fc_server_* calls, FC_ERR_INVALID_ARG for n_req < 1 or missing
 * arrays. */
fc_status fc_server_tune(const fc_server_opts *base, int32_t n_req, const fc_csr *S,
                         const fc_options *opt, const void *const *U0, fc_dtype u0_dtype,
                         void *stream, fc_server_opts *best, double *solves_per_s,
                         int32_t *n_runs);

/* ------------------------------------------------------------------------
 * Second-order check (section 4, Theorem 4.1)
 * ---------------------------------------------------------------------- */

/* HV = Hess f(U) V, eq. (hessian) of Theorem 4.1 in the row layout:
 *   row i of HV = -4 (S_eff V)_i + 4 v_i (U^T U) + 4 u_i (U^T V + V^T U).
 * S as for fc_create (values FC_F64 with dtype FC_F64, or FC_F32 with
 * FC_F32); U, V, HV: device, n x c row-major of dtype (HV must not alias U
 * or V).  The sparse product and the c x c products U^T U, U^T V run on the
 * GPU (matrix cores for the latter); the row combination is in double.
 * Synchronises the stream before returning.  Errors: FC_ERR_INVALID_ARG. */
fc_status fc_hessian_vector(const fc_csr *S, fc_diag diag, const void *U, const void *V, void *HV,
                            fc_dtype dtype, int32_t c, void *stream);

/* Smallest curvature of f at U over the face directions
 *   K(U) = { V : every row of V sums to 0, v_ik = 0 where u_ik <= zero_tol },
 * the tangent directions of Omega at U (the cone in the proof of Theorem 4.1)
 * that keep each zero component at zero; at a critical point they satisfy
 * <grad f(U), V> = 0, so Theorem 4.1 requires <Hess f(U) V, V> >= 0 on K(U)
 * for a local minimiser.  Lanczos on the Hessian restricted to K(U), started
 * from the projection of V0 (device, n x c, caller-chosen, e.g. random),
 * with full reorthogonalisation (two Gram-Schmidt passes per step) for
 * `krylov` steps (1..512) or until an invariant subspace is reached; the
 * Ritz pair with the smallest value of the small tridiagonal matrix (cyclic
 * Jacobi) gives *lambda_min and, if V_out (device, n x c) is non-NULL, the
 * unit-norm Ritz direction.  *lambda_min < 0 certifies that U is not a local
 * minimiser (V_out is a direction of negative curvature); a value >= 0 is
 * evidence, not proof, of the converse.  *steps (may be NULL) receives the
 * number of Lanczos steps.  The Krylov basis takes (krylov + 1) n c' words
 * (c' = padded c): FC_ERR_OUT_OF_MEMORY when it would not fit.  dtype and S
 * as for fc_hessian_vector.  Synchronises the stream. */
fc_status fc_curvature(const fc_csr *S, fc_diag diag, const void *U, const void *V0, fc_dtype dtype,
                       int32_t c, int32_t krylov, double zero_tol, double *lambda_min, void *V_out,
                       int32_t *steps, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FC_H */
