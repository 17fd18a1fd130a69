/*
 * amp_pcg.h -- C ABI of the adaptive mixed-precision, dynamically scaled
 * preconditioned conjugate gradient solver (AMP-PCG) for AMD MI355X (gfx950).
 *
 * Method: Guo, de Sturler, Warburton, "An Adaptive Mixed-Precision and
 * Dynamically Scaled Preconditioned Conjugate Gradient Algorithm"
 * (arXiv:2505.04155).  Problem statement: Alg. 3 (AMP-PCG(u0)) -- solve
 * A x = b for a symmetric positive definite A with preconditioner M to
 * ||b - A x|| <= tol ||b||.
 *
 * Conventions for every call:
 *   - Plain C, no exceptions cross the boundary.  Every entry point returns
 *     an amp_status; on failure amp_last_error() (thread-local) describes it.
 *   - "device pointer": memory allocated on the current HIP device (e.g. a
 *     torch.cuda tensor's data_ptr()).  The caller owns it; the library never
 *     frees caller memory and never keeps a pointer to it after returning.
 *   - "stream": a hipStream_t passed as void* (NULL = the legacy default
 *     stream).  All device work is enqueued on it; calls documented as
 *     host-synchronous wait for their own work before returning.
 *   - Handles (amp_matrix, amp_precond) own device memory (hipMalloc, or the
 *     caller's allocator: amp_set_allocator) and free it in their destroy call.  A handle may be used
 *     by one solve at a time.
 *   - Precisions are named by bit width: 64 = IEEE double, 32 = single,
 *     16 = half.
 */
#ifndef AMP_PCG_H
#define AMP_PCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AMP_OK = 0,
    AMP_ERR_ARG = 1,            /* invalid argument (null pointer, n <= 0, tol <= 0, ...) */
    AMP_ERR_NOT_CONVERGED = 2,  /* maxit reached; x holds the last iterate */
    AMP_ERR_BREAKDOWN = 3,      /* rho <= 0, gamma <= 0 or a non-finite scalar; x holds the last finite iterate */
    AMP_ERR_HIP = 4,            /* a HIP runtime call failed */
    AMP_ERR_OOM = 5             /* device allocation failed */
} amp_status;

typedef enum { AMP_FP64 = 64, AMP_FP32 = 32, AMP_FP16 = 16 } amp_prec;

/* Attainable-accuracy indicator that drives the u_r switch (Section 4.1). */
typedef enum {
    AMP_ETA_DELAY = 0,    /* eq. (eta_k): delay window d, constant C */
    AMP_ETA_LINEAR = 1,   /* eq. (linear criterion): rate over ell steps */
    AMP_UR_FIXED64 = 2,   /* u_r stays FP64 */
    AMP_UR_FIXED32 = 3    /* u_r is FP32 from the first iteration */
} amp_eta_mode;

/* Dynamic scaling omega_k of the residual before preconditioning (Alg. 2). */
typedef enum {
    AMP_SCALE_POW2 = 0,   /* omega_k = 2^{e_k}, e_k from the vectors' maxima (default) */
    AMP_SCALE_PAPER = 1,  /* omega_k = 1/delta_k, as written in Alg. 3 */
    AMP_SCALE_NONE = 2    /* omega_k = 1 (plain PCG, Alg. 1) */
} amp_scaling;

typedef enum { AMP_PC_IDENTITY = 0, AMP_PC_JACOBI = 1, AMP_PC_CHEBYSHEV = 2, AMP_PC_PMG = 3 } amp_pc_kind;

/* Preset selectors of the PCG variants compared in Section 5. */
typedef enum {
    AMP_PRESET_PCG64 = 0,   /* PCG(FP64): all vectors FP64 */
    AMP_PRESET_AMP64 = 1,   /* AMP-PCG(FP64): u0 = FP64, u_z lowered by tau_zs/tau_zh */
    AMP_PRESET_AMP16 = 2,   /* AMP-PCG(FP16): z, p in FP16 from the start */
    AMP_PRESET_AMP_UR = 3   /* AMP-PCG(u_r): u_z fixed FP64, only u_r adapts */
} amp_preset;

/* Matrix in CSR form, all arrays device pointers: row_ptr[n+1], col_idx[nnz],
 * val[nnz].  Columns strictly ascending within each row (no duplicates), the
 * diagonal present, nnz < 2^31, n <= 2^29 - 1024 (the product kernels gather
 * vector entries by 32-bit byte offsets).
 * The values are read once by amp_matrix_create (no reference is kept). */
typedef struct {
    int32_t n;
    int64_t nnz;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
} amp_csr;

typedef struct amp_matrix_s *amp_matrix;
typedef struct amp_precond_s *amp_precond;

/* Solver options; fill with amp_options_default / amp_options_preset. */
typedef struct {
    int u0;                 /* initial (maximum) precision of u_z: 64, 32 or 16 (Alg. 3) */
    double tau_zs, tau_zh;  /* nu-thresholds for u_z -> FP32, -> FP16 (eq. precision_selector, eq. criterion) */
    int eta_mode;           /* amp_eta_mode */
    int d;                  /* delay of eq. (eta_k), 1 <= d <= 100 (default 10) */
    double C;               /* constant C of eq. (eta_k) / eq. (linear criterion) (default 1) */
    int ell;                /* window of eq. (linear criterion), 1 <= ell <= 100 (default 5) */
    int scaling;            /* amp_scaling */
    int T_z, T_p;           /* pow2 scaling targets: max|z^| ~ 2^T_z, carried part of p^ <= beta 2^T_p (default 12, 12) */
    int spmv32_diff;        /* 1: FP32 product in row-sum/difference form (default); 0: textbook form */
    int verify;             /* 1: FP64 true-residual check at termination with replacement (default) */
    int max_replacements;   /* replacements allowed by the termination check (default 3) */
    int rr_period;          /* >0: replace r by b - A x every rr_period iterations (default 0) */
    int batch;              /* iterations enqueued between host status checks (default 0 = automatic) */
    int group_rows;         /* rows per work-group, a multiple of 256: every kernel of the solve then
                               runs G = ceil(n_padded / group_rows) work-groups (at most 1024).
                               Default 0: automatic (single solve: per-kernel counts filling the
                               chip; batched solve: 4096) */
    int graph;              /* 1: replay batches of 8 iterations from a captured HIP graph cached in the
                               matrix handle (single solve without rr_period; default 0) */
    int solo_rows;          /* a system with at most this many (padded) rows, Jacobi or identity and
                               rr_period = 0, is solved by one work-group in one launch (the stages of
                               the kernel sequence with one work-group each, in a loop on the device);
                               0 disables (default 0) */
    int spmv_timing;        /* 1: time every product-kernel launch (and every Chebyshev polynomial-step
                               launch) with HIP events carried by the dispatch (eager path only:
                               disables graph and solo); results in amp_result.spmv_ms, cheb_ms */
    int defer_x;            /* 1 (default): the FP64 update x += alpha p is applied two iterations at a
                               time, x_{k+1} = (x_{k-1} + alpha_{k-1} p_{k-1}) + alpha_k p_k, rounded
                               after each step exactly as one step at a time (bitwise the same x);
                               the pending step is applied whenever the solve stops. Ignored (0)
                               with rr_period > 0 */
    double *delta_history;  /* nullable device buffer, maxit+1 doubles: ||r_k|| for k = 0..iters */
    int32_t *prec_history;  /* nullable device buffer, maxit ints: u_z | (u_r << 8) of iteration k */
    double *scalar_history; /* nullable device buffer, 4*maxit doubles: omega_k, rho_k, gamma_k, alpha_k */
    int rr_switch;          /* 1 (default): at the iteration whose u_r first drops to FP32, r is replaced
                               by fl32(b - A x), formed with FP64 values and accumulation (residual
                               replacement, Sections 1.1 and 3.1), instead of the recurrence residual
                               rounded to FP32; counted in n_replacements. 0: rounded recurrence residual */
} amp_options;

typedef struct {
    int iters;                /* iterations performed */
    int status;               /* amp_status of the solve */
    double rel_res_updated;   /* ||r_iters|| / ||b|| (the recurrence residual) */
    double rel_res_true;      /* ||b - A x|| / ||b|| in FP64 (0 when verify = 0) */
    double bnorm;             /* ||b|| */
    int k_z32, k_z16, k_r32;  /* first iteration with u_z <= FP32, u_z = FP16, u_r = FP32 (-1: never) */
    int n_replacements;       /* residual replacements performed */
    double t_solve_ms;        /* wall time of the solve call (host clock, includes the final check) */
    double spmv_ms;           /* spmv_timing: summed duration of the product-kernel launches that
                                 performed an iteration (0 otherwise) */
    int spmv_launches;        /* spmv_timing: number of those launches (= iters) */
    double cheb_ms;           /* spmv_timing with a Chebyshev preconditioner of degree m > 1: summed
                                 duration of the polynomial-step launches that performed an iteration */
    int cheb_launches;        /* spmv_timing: number of those launches (= iters * (m - 1)) */
} amp_result;

/*
 * Device memory of handles and workspaces.  By default the library calls
 * hipMalloc / hipFree.  After amp_set_allocator(alloc, free_, ctx) every
 * later device allocation of the library (matrix planes, work vectors,
 * preconditioner data, the batched solve's tables) calls alloc(bytes, ctx),
 * which must return device memory of the current device, aligned to 256
 * bytes, or NULL (AMP_ERR_OOM); such a block is released with the free_
 * that was set when it was allocated (free_(ptr, ctx)), after the library
 * has waited for the device, as hipFree does.  amp_set_allocator(NULL, NULL,
 * NULL) returns to hipMalloc for later allocations.  Typical use: routing
 * the workspace through a framework's caching allocator.  The functions are
 * called from the thread that calls the library; they must not call back
 * into it.  Pinned host memory and events are not affected.  Errors:
 * AMP_ERR_ARG if exactly one of alloc, free_ is NULL.
 */
amp_status amp_set_allocator(void *(*alloc)(size_t bytes, void *ctx), void (*free_)(void *ptr, void *ctx),
                             void *ctx);

/* Library version (major*10000 + minor*100 + patch). */
int amp_version(void);
/* Human-readable status name; never NULL. */
const char *amp_status_string(amp_status s);
/* Description of the last failure on the calling thread ("" if none). */
const char *amp_last_error(void);

/* Defaults: the AMP-PCG(FP64) preset with d = 10, C = 1, ell = 5,
 * tau_zs = 1e-4, tau_zh = 1e-6 (Section 5, eq. criterion), pow2 scaling. */
void amp_options_default(amp_options *opt);
/* Fill *opt with one of the Section 5 variants (amp_preset); other fields
 * take their defaults.  Returns AMP_ERR_ARG for an unknown preset. */
amp_status amp_options_preset(amp_options *opt, int preset);

/*
 * Build the solver's matrix handle from a device CSR matrix (Section 4: the
 * matrix-vector product is computed in u_r).  Converts to sliced ELL (slice
 * height 64, rows in natural order) with an FP64 value plane (products in
 * FP64) and an FP32 plane (products in FP32; the diagonal slot holds the
 * FP64 row sum rounded to FP32 for the difference form).  The textbook FP32
 * plane (fl32 of every value, for spmv32_diff = 0) is built from the FP64
 * plane by the first solve or product that uses it.  A slice whose rows
 * share a short list of column offsets (col - row, at most 32, at most two
 * more than its longest row) stores that list once instead of a column index
 * per entry (stencil matrices: every slice); other slices keep int32 column
 * indices.
 * Enqueued on `stream` and host-synchronous.
 * The CSR is validated on the device before any entry is read through it:
 * row_ptr[0] = 0, row_ptr[n] = nnz, non-decreasing; columns in [0, n) and
 * strictly ascending within each row.
 * Errors: AMP_ERR_ARG for n <= 0, n > 2^29 - 1024, nnz < n, nnz >= 2^31,
 * null pointers, a CSR failing the validation above, or a missing or
 * non-positive diagonal entry; AMP_ERR_OOM / AMP_ERR_HIP from the runtime.
 */
typedef struct {
    int lanes_per_row;  /* 1 (default): one row per lane, slices of 64 rows; 2, 4, 8 or 16: that many lanes share
                           a row (slices of 64 / lanes rows, entry e of a row in the row's lane e mod lanes),
                           for long rows; 0: chosen from the mean row length (1 up to 32 entries, else the power
                           of two leaving 8 to 16 entries per lane).  More than one lane per row implies index
                           mode, and is not accepted by the Chebyshev preconditioner or the batched solve */
    int offset_mode;    /* 1 (default): slices whose rows share a short column-offset list store it once; 0: a
                           column index per entry everywhere */
} amp_matrix_tuning;
/* Fill *t with the defaults (one lane per row, offset mode allowed). */
void amp_matrix_tuning_default(amp_matrix_tuning *t);
/* tuning: nullable (defaults).  Errors as listed above, and AMP_ERR_ARG for
 * lanes_per_row outside {0, 1, 2, 4, 8, 16}. */
amp_status amp_matrix_create(const amp_csr *A, const amp_matrix_tuning *tuning, void *stream, amp_matrix *out);
/* As amp_matrix_create with one lane per row; flags bit 0 keeps every slice
 * in index mode (no shared per-slice column-offset lists). */
amp_status amp_matrix_create_ex(const amp_csr *A, int flags, void *stream, amp_matrix *out);
/*
 * Lanes-per-row autotuner: for each of the ncand candidates (values as
 * amp_matrix_tuning.lanes_per_row, 0 excluded) build the handle of A with
 * that layout (offset mode allowed where the layout permits) and time reps
 * launches of each of the two products an AMP-PCG(FP16) solve runs -- FP64
 * values with FP16 p, and FP32 row-sum form with FP16 p -- with HIP events,
 * after a warm-up launch.  *best receives the candidate with the least summed
 * time; us_per_product (host array of ncand, nullable) the mean of the two
 * per launch, in microseconds.  Each handle is destroyed before the next is
 * built.  Host-synchronous.  Errors: AMP_ERR_ARG for null pointers, ncand < 1,
 * reps < 1 or a bad candidate; any error of amp_matrix_create.
 */
amp_status amp_tune_lanes(const amp_csr *A, const int *candidates, int ncand, int reps, int *best,
                          double *us_per_product, void *stream);
void amp_matrix_destroy(amp_matrix A);
/* Layout of a matrix handle. */
typedef struct {
    int64_t n, nnz;
    int64_t slots;          /* stored entries including slice padding */
    int64_t bytes;          /* device bytes held by the handle (with its work vectors once solved) */
    int64_t nslices;        /* 64-row slices (rows padded to a multiple of 1024) */
    int64_t offset_slices;  /* slices stored with a shared column-offset list */
    int64_t meta_bytes;     /* column metadata one product reads: 4 B per index-mode slot,
                               the offset lists, 12 B per slice of pointers, plus 8 */
    int64_t lanes_per_row;  /* lanes sharing one row (1, 2, 4, 8 or 16) */
} amp_matrix_stats;
amp_status amp_matrix_info(amp_matrix A, amp_matrix_stats *out);

/*
 * Preconditioner handle.  AMP_PC_JACOBI: M = diag(A) (Section 5.5), inverse
 * stored in FP64, FP32, and FP16 scaled by a power of two.  AMP_PC_CHEBYSHEV:
 * z = D^{-1/2} s(B) D^{-1/2} y, B = D^{-1/2} A D^{-1/2} stored in FP16,
 * s the degree-(degree-1) polynomial with 1 - t s(t) = T_degree((theta - t)/
 * delta)/T_degree(theta/delta) on [lam_lo, lam_hi] (eigenvalue bounds of
 * D^{-1} A).  A bound given as <= 0 is estimated (the paper gives no rule;
 * Section 5.3 uses Chebyshev only as a smoother): 24 Lanczos steps in FP64
 * on D^{-1/2} A D^{-1/2} from a fixed counter-based start vector
 * (splitmix64), lam_hi = 1.05 x the largest Ritz value, lam_lo = lam_hi / 30;
 * amp_precond_bounds reports the values used.  AMP_PC_IDENTITY: M = I.
 * Host-synchronous.
 * Errors: AMP_ERR_ARG for an unknown kind, degree outside 1..16, non-finite
 * bounds, or bounds (given or estimated) not satisfying 0 < lam_lo < lam_hi.
 */
amp_status amp_precond_create(amp_matrix A, int kind, int degree, double lam_lo, double lam_hi,
                              void *stream, amp_precond *out);
/* The interval a Chebyshev preconditioner uses (given or estimated), and
 * the Lanczos Ritz extremes it was estimated from (0 when both bounds were
 * given); ritz_min, ritz_max nullable.  Host-only read of the handle.
 * Errors: AMP_ERR_ARG for null pointers or another preconditioner kind. */
amp_status amp_precond_bounds(amp_precond M, double *lam_lo, double *lam_hi, double *ritz_min, double *ritz_max);
void amp_precond_destroy(amp_precond M);

/*
 * Solve A x = b (Alg. 3, AMP-PCG(u0)).  b: device FP64[n]; x: device
 * FP64[n], initial guess on entry, solution on exit.  opt may be NULL
 * (defaults).  The iteration runs on the device: the precision selector,
 * the eta indicator, the scaling and the stopping test are evaluated by the
 * kernels themselves; the host only polls a status word every opt->batch
 * iterations.  Host-synchronous; fills *res (may be NULL).
 * Returns AMP_OK when ||r|| <= tol ||b|| (and, with verify, the FP64 true
 * residual too), AMP_ERR_NOT_CONVERGED at maxit, AMP_ERR_BREAKDOWN on a
 * breakdown, AMP_ERR_ARG for bad arguments (tol <= 0, maxit < 0, null
 * pointers, M built for another matrix, bad option values).
 */
amp_status amp_pcg_solve(amp_matrix A, amp_precond M, const double *b, double *x, double tol,
                         int maxit, const amp_options *opt, amp_result *res, void *stream);

/*
 * amp_pcg_solve for callers that cannot allocate device memory during the
 * call (serving loops, harnesses that forbid hipMalloc): the same kernels,
 * state chain and results as amp_pcg_solve (bitwise the same x and
 * iterations), with every work vector, partial array, state slot and the
 * residual window held in the library's own device array of about 25 MB
 * per GPU (allocated when the library's code is loaded on that device, held
 * until the process ends), instead of the matrix handle's work buffers.
 * The call makes no hipMalloc, hipFree, event, stream or pinned-memory
 * allocation; it clears the array's used part with a kernel first.
 * Limits: the padded row count of A (n rounded up to a multiple of 1024)
 * is at most 2^18 = 262144; opt->graph, opt->spmv_timing and opt->solo_rows
 * must be 0.  The host polls the state with plain copies (no pipelining).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * device (several host threads, or streams without ordering) race and give
 * wrong results; serialise them.  Arguments, ownership, host-synchronous
 * behaviour and status codes as for amp_pcg_solve; AMP_ERR_ARG also for a
 * system above the row limit or the options above.
 */
amp_status amp_pcg_solve_noalloc(amp_matrix A, amp_precond M, const double *b, double *x, double tol,
                                 int maxit, const amp_options *opt, amp_result *res, void *stream);

/*
 * Solve nsys independent systems A[i] x[i] = b[i] (Alg. 3 for each) in one
 * lockstep iteration: every kernel launch advances every unfinished system,
 * each system keeping its own scalars, precisions, switch points, scaling
 * and convergence state; finished systems leave the launch grid between
 * batches of iterations.  A, M: host arrays of nsys distinct handles (M[i]
 * built on A[i]; Jacobi or identity).  b, x: host arrays of nsys device
 * pointers (FP64, n_i elements; x[i] holds x0 on entry and the solution on
 * exit).  tol: host array of nsys tolerances.  opt as for amp_pcg_solve
 * (histories must be NULL); opt->group_rows sets rows per work-group.
 * res: host array of nsys results (nullable), each with its own status and
 * rel_res_true (always computed).  Each system follows exactly the
 * arithmetic of amp_pcg_solve with its work-group count.  Host-synchronous.
 * Returns AMP_OK if every system converged, else AMP_ERR_BREAKDOWN if any
 * broke down, else AMP_ERR_NOT_CONVERGED; AMP_ERR_ARG for nsys < 1, null
 * or repeated handles, a Chebyshev preconditioner, tol <= 0, maxit < 0,
 * non-null histories or bad option values.
 */
amp_status amp_pcg_solve_batched(int nsys, const amp_matrix *A, const amp_precond *M, const double *const *b,
                                 double *const *x, const double *tol, int maxit, const amp_options *opt,
                                 amp_result *res, void *stream);

/*
 * Rows-per-work-group autotuner.  Every kernel gives each work-group a
 * contiguous share of a system's rows (slices of 64 rows, one row per lane),
 * and opt->group_rows fixes that share: fewer rows per work-group put more
 * work-groups in flight, more rows amortise each work-group's fixed costs
 * (state load, reductions, controller).  For each of the ncand candidate
 * values (0: the automatic choice; else a positive multiple of 256) this
 * runs the solve itself -- amp_pcg_solve when nsys = 1, amp_pcg_solve_batched
 * otherwise -- from x = 0: once with at most `iters` iterations (warm-up),
 * then three times each with none and with `iters`, timed with the host
 * clock; the difference of the least times, per iteration performed, is the
 * candidate's time (the per-call set-up and final check cancel).  *best receives the
 * candidate with the least time per iteration; ms_per_iter (host array of
 * ncand, nullable) the measured times.  A, M, b,
 * tol as for amp_pcg_solve_batched (host arrays of nsys); x: host array of
 * nsys device FP64 vectors used as scratch (overwritten; their contents on
 * entry are ignored).  opt as for the solves (group_rows is set per
 * candidate; histories must be NULL).  The runs' own status (not converged,
 * breakdown) does not matter.  Host-synchronous.  Errors: AMP_ERR_ARG for
 * nsys < 1, iters < 1, ncand < 1, null pointers or a bad candidate; any
 * error a solve returns other than not-converged or breakdown.
 */
amp_status amp_tune_group_rows(int nsys, const amp_matrix *A, const amp_precond *M, const double *const *b,
                               double *const *x, const double *tol, int iters, const int *candidates,
                               int ncand, const amp_options *opt, int *best, double *ms_per_iter,
                               void *stream);

/*
 * One product q = A p with the solver's own kernel, for tests and
 * measurement.  u_r selects the value plane and arithmetic (64: FP64
 * values and accumulation; 32: FP32 values and accumulation, in
 * row-sum/difference form when diff != 0, textbook form otherwise); u_p is
 * the storage precision of p.  p: device array of n elements of precision
 * u_p, or NULL to reuse the vector the handle's last solve or product left
 * in its p buffer of that precision.  q: device array of n elements of
 * precision u_r, or NULL to leave q in the handle's buffer.  gamma
 * (nullable, device FP64[1]) receives q^T p accumulated in FP64.  With
 * p = q = gamma = NULL the call is exactly one kernel launch.  Enqueued on
 * stream, not synchronised.  Errors: AMP_ERR_ARG for a null handle or a
 * precision outside {64, 32} x {64, 32, 16}.
 */
amp_status amp_spmv(amp_matrix A, int u_r, int u_p, int diff, const void *p, void *q, double *gamma,
                    void *stream);

/*
 * One iteration's fused product step on the handle's own work buffers,
 * exactly as the solve's product kernel runs it with the precisions fixed:
 * p_new = fl_{u_z}(z + beta p_old) (z, p_old: the vectors the last solve or
 * product left in the handle), q = A p_new in u_r (FP32 in row-sum/
 * difference form when diff != 0), gamma partial sums.  Meant for timing
 * the solver's dominant kernel in isolation: one kernel launch, enqueued on
 * stream, not synchronised.  Errors: AMP_ERR_ARG for a null handle or a
 * precision outside {64, 32, 16} x {64, 32}.
 */
amp_status amp_spmv_step(amp_matrix A, int u_z, int u_r, int diff, double beta, void *stream);

/*
 * One scaled preconditioner application z = M^{-1} fl_{u_z}(fl_{u_r}(omega r)),
 * Alg. 3 steps y = r/delta, z = M^{-1} y, with r stored in u_r and z in u_z.
 * omega is the total scale (for FP16 Jacobi the static storage scale of
 * dinv is compensated inside).  rho (nullable, device FP64[1]) receives
 * r^T z in FP64.  Enqueued on stream, not synchronised.
 */
amp_status amp_precond_apply(amp_precond M, int u_r, int u_z, const void *r, double omega, void *z,
                             double *rho, void *stream);

/*
 * Refill the handle's values from a CSR matrix with the same sizes (n, nnz)
 * and row lengths -- typically the same pattern with new values (a
 * differentiable solve updating A(theta)).  Device pointers as in
 * amp_matrix_create; host-synchronous.  Preconditioners built on the handle
 * must then be refreshed with amp_precond_update.  Errors: AMP_ERR_ARG for
 * null pointers, other sizes or row lengths, a bad column or diagonal.
 */
amp_status amp_matrix_update_values(amp_matrix A, const amp_csr *csr, void *stream);
/* Recompute a preconditioner's data from its matrix's current values
 * (host-synchronous). */
amp_status amp_precond_update(amp_precond M, void *stream);

/*
 * Cell-centred finite-volume diffusion operator on a dim-dimensional box
 * grid (dim = 2: nx x ny, nz ignored; dim = 3: nx x ny x nz), cells ordered
 * x fastest, cell coefficient kappa = exp(theta): an interior face between
 * cells i and j has T = 2 kappa_i kappa_j / (kappa_i + kappa_j), a face on
 * the Dirichlet boundary T = 2 kappa_i; A_ii = sum of the cell's T,
 * A_ij = -T_ij.  amp_fv_nnz (host-only) gives nnz; amp_fv_csr writes the CSR
 * (row_ptr[n+1], col_idx[nnz] sorted, val[nnz]; device arrays owned by the
 * caller) from theta (device FP32[n]).  Host-synchronous.
 * Errors: AMP_ERR_ARG for dim not 2 or 3, non-positive sizes, null pointers
 * or a grid whose nnz would not fit int32.
 */
amp_status amp_fv_nnz(int dim, int nx, int ny, int nz, int64_t *nnz);
amp_status amp_fv_csr(int dim, int nx, int ny, int nz, const float *theta, int32_t *row_ptr,
                      int32_t *col_idx, double *val, void *stream);
/*
 * Gradient of a loss L(x) through x = A(theta)^{-1} b, given x and the
 * adjoint lambda = A^{-1} dL/dx (A symmetric): dtheta_i = sum over the
 * faces of cell i of dL/dT * dT/dtheta_i with dL/dT_ij = -(lambda_i -
 * lambda_j)(x_i - x_j), dT_ij/dtheta_i = 2 kappa_i kappa_j^2 / (kappa_i +
 * kappa_j)^2, and for a boundary face dL/dT = -lambda_i x_i, dT/dtheta_i =
 * 2 kappa_i.  FP64 accumulation, FP32 result dtheta[n] (device).  Enqueued
 * on stream, not synchronised.
 */
amp_status amp_fv_grad_theta(int dim, int nx, int ny, int nz, const float *theta, const double *x,
                             const double *lambda, float *dtheta, void *stream);

/*
 * Host-only: run the device controller's latched precision selector over a
 * recorded residual-norm history delta[0..len-1] (eq. precision_selector
 * with eq. eta_k or eq. linear criterion) and report the first iteration at
 * which u_z <= FP32, u_z = FP16 and u_r = FP32 (-1: never).  Needs no GPU.
 */
amp_status amp_selector_replay(const double *delta, int len, double bnorm, double tol,
                               const amp_options *opt, int *k_z32, int *k_z16, int *k_r32);

/*
 * Host-only: algorithmic bytes moved per row by one iteration's kernels of
 * the paper's five-kernel decomposition (Table tab:pcg_cost) for storage
 * precisions (u_z, u_r), with the Jacobi preconditioner and M stored in
 * u_z: out[0..3] = zamx, innerProd, axpy, updatePCG.  Needs no GPU.
 */
amp_status amp_paper_kernel_bytes(int u_z, int u_r, double out[4]);

/*
 * Measurement: stream `bytes` bytes through HBM with the library's own
 * probe kernels -- mode 0 reads src once (dst: a device word the kernel
 * may write, so no load can be dropped), mode 1 copies src to dst.  16-byte
 * loads and stores, four in flight per thread, up to 2048 work-groups of
 * 256 threads.  It gives the bandwidth ceiling the solver's kernels are
 * compared with, and the known-size launch that hardware byte counters are
 * scaled by.  Device pointers, 16-byte aligned; bytes a positive multiple
 * of 16.  Enqueued on stream, not synchronised.  Errors: AMP_ERR_ARG.
 */
amp_status amp_stream_probe(int mode, const void *src, void *dst, int64_t bytes, void *stream);

/* ------------------------------------------------------------------------
 * Matrix-free high-order hexahedral operator (Section 5.5, Ex. jac libp:
 * the screened Poisson equation -Laplace(u) + lambda u = f on a box,
 * tensor-product elements of order N with Gauss-Lobatto-Legendre points
 * and quadrature, each element the trilinear image of the reference cube,
 * homogeneous Dirichlet conditions; the paper's Ax kernel, Table
 * tab:pcg_cost, with mu = p^T q).
 *
 * Mesh: ex x ey x ez elements; the global nodes form the
 * (N ex + 1) x (N ey + 1) x (N ez + 1) grid, x fastest, and local node
 * (i, j, k) of element (a, b, c) is grid node (a N + i, b N + j, c N + k).
 * The unknowns are the grid nodes off the boundary, in grid order: node
 * (gx, gy, gz) has index (gx-1) + (N ex - 1)((gy-1) + (N ey - 1)(gz-1)),
 * n = (N ex - 1)(N ey - 1)(N ez - 1).  The element maps come from the
 * vertex array verts: row vx + (ex+1)(vy + (ey+1) vz) holds vertex
 * (vx, vy, vz) as (x, y, z); corner (a, b, c) of element (ex, ey, ez) is
 * vertex (ex + a, ey + b, ez + c).  Geometric factors are formed at every
 * quadrature point from the element's 8 vertices; nothing per node is
 * stored.
 * ------------------------------------------------------------------------ */
typedef struct amp_hexop_s *amp_hexop;

typedef struct {
    int64_t n;          /* unknowns */
    int64_t elements;   /* ex ey ez */
    int64_t local;      /* element-local nodes: elements (N+1)^3 */
    int order;          /* N */
    double lambda;
    double flops_per_element;   /* arithmetic of one element application (multiply and add counted
                                   separately) as the operator's definition states it: (264 for N = 7:
                                   12 (N+1) + 19 for the contractions and the mass term, 149 for the
                                   geometric factors) per local node */
} amp_hexop_stats;

/* Create the operator.  order: 1, 3 or 7 (the matrix-free solve takes 3 and
 * 7; order 1 serves the lowest level of the p-multigrid cycle).  verts: device pointer to
 * (ex+1)(ey+1)(ez+1) x 3 doubles, copied (the caller keeps ownership).
 * lambda >= 0.  Errors: AMP_ERR_ARG for counts < 1, an order not built,
 * n < 1, more than 2^31 - 1 elements or unknowns, a null pointer, a
 * negative or non-finite lambda, or an element map whose Jacobian
 * determinant is not positive at every quadrature point (checked on the
 * device); AMP_ERR_OOM / AMP_ERR_HIP.  Host-synchronous. */
amp_status amp_hexop_create(int ex, int ey, int ez, int order, const double *verts, double lambda, void *stream,
                            amp_hexop *out);
void amp_hexop_destroy(amp_hexop H);
amp_status amp_hexop_info(amp_hexop H, amp_hexop_stats *out);
/* q = A p (device vectors of n entries): p stored in u_p (64, 32 or 16:
 * double, float, _Float16), q and the arithmetic in u_r (64 or 32).
 * mu (device, nullable): one double, p^T q from per-element partials
 * p_e^T A_e p_e summed in element order.  q's shared nodes are summed by
 * atomic adds in no fixed order (exact to rounding, not bitwise
 * reproducible).  Enqueued on stream, not synchronised.  Errors:
 * AMP_ERR_ARG for a bad precision or null p / q. */
amp_status amp_hexop_apply(amp_hexop H, int u_p, int u_r, const void *p, void *q, double *mu, void *stream);
/* diag (device, n doubles) = the diagonal of A, in FP64 (for the Jacobi
 * preconditioner).  Enqueued on stream, not synchronised. */
amp_status amp_hexop_diagonal(amp_hexop H, double *diag, void *stream);
/* A matrix handle that wraps the operator, for amp_pcg_solve with the
 * Jacobi (its diagonal, from amp_hexop_diagonal) or identity preconditioner:
 * AMP-PCG on the matrix-free operator, the paper's Ex. jac libp.  The
 * solve's product is then the element kernel with p = z + beta p_old formed
 * at every gathered node, q summed by atomic adds (the update clears it for
 * the next product), gamma = sum_e p_e^T A_e p_e in element order; the x
 * update is not deferred, and r is not replaced at the u_r switch (the
 * option is ignored).  The operator must outlive the handle (it is not
 * owned).  amp_spmv, amp_spmv_step, amp_matrix_update_values, the batched
 * and allocation-free solves, the Chebyshev preconditioner, periodic
 * replacement, graph replay and group_rows refuse such a handle
 * (AMP_ERR_ARG).  Host-synchronous. */
amp_status amp_matrix_from_hexop(amp_hexop H, void *stream, amp_matrix *out);

/* ------------------------------------------------------------------------
 * p-multigrid preconditioner for a matrix-free handle (Section 5.3, Ex.
 * linear conv2: the preconditioner under which convergence is linear and
 * z, p may be FP16 from the first iteration).  One V-cycle over polynomial
 * orders orders[0] > orders[1] > ... on the operator's mesh, each level the
 * operator rediscretised at its order with the same lambda:
 *   V_l(f): x = S_l f; x += P_l V_{l+1}(P_l^T (f - A_l x)); x += S_l (f - A_l x)
 * S_l: the Chebyshev iteration of degree `degree` for D^-1 A x = D^-1 f from
 * x = 0 (D = diag(A_l)) on [lo_ratio rho_l, hi_margin rho_l], rho_l =
 * lambda_max(D^-1 A_l).  Lowest level: the same polynomial of degree
 * coarse_degree on [coarse_lo_ratio rho, hi_margin rho] (the paper's
 * algebraic multigrid coarse solver is not built; a fixed polynomial keeps
 * the cycle linear and symmetric).  P_l interpolates the coarse function at
 * the fine GLL points element by element; P_l^T is its transpose.
 * Arithmetic: FP64 while u_z is FP64, else FP32; z rounded to u_z.
 * ------------------------------------------------------------------------ */
typedef struct {
    int levels;             /* 1 .. 4 */
    int orders[4];          /* strictly decreasing, each 1, 3 or 7; orders[0] = the operator's order */
    int degree;             /* smoother degree, 1 .. 32 (default 2) */
    int coarse_degree;      /* lowest level's polynomial degree, 1 .. 32 (default 16) */
    double lo_ratio;        /* smoothing interval [lo_ratio rho, hi_margin rho] (default 0.1, 1.1) */
    double hi_margin;
    double coarse_lo_ratio; /* lowest level's interval [coarse_lo_ratio rho, hi_margin rho] (default 0.01) */
    double rho[4];          /* lambda_max(D^-1 A_l) per level; <= 0: estimated by power_iters steps of
                               the power iteration (Rayleigh quotient in the D inner product) */
    int power_iters;        /* 1 .. 1000 (default 40) */
} amp_pmg_params;

typedef struct {
    amp_pmg_params params;  /* as used: rho holds the values of every level */
    double gain;            /* max|V(1)|: the scaling rule's first-iteration bound max|z| <= gain max|r| */
    int64_t n[4];           /* unknowns per level */
    int64_t bytes;          /* device memory held by the preconditioner */
} amp_pmg_stats;

/* Defaults: three levels (7, 3, 1), degree 2, coarse degree 16, intervals
 * [0.1, 1.1] rho and [0.01, 1.1] rho, rho estimated with 40 steps. */
void amp_pmg_params_default(amp_pmg_params *p);
/* Create the preconditioner for A, a handle from amp_matrix_from_hexop
 * (the operator's vertices and lambda are copied into the lower levels).
 * For amp_pcg_solve with any preset; amp_precond_apply, amp_precond_update
 * and the batched and allocation-free solves refuse it.  Errors:
 * AMP_ERR_ARG for a handle that is not matrix-free, parameters out of
 * range, a level without unknowns (order 1 needs at least 2 elements per
 * direction), a non-positive diagonal or an estimate of rho that is not
 * positive and finite; AMP_ERR_OOM / AMP_ERR_HIP.  Host-synchronous.
 * The cycle's work vectors belong to the handle: solves and amp_pmg_apply
 * calls that use one handle must not overlap (in time or across streams). */
amp_status amp_precond_create_pmg(amp_matrix A, const amp_pmg_params *p, void *stream, amp_precond *out);
amp_status amp_pmg_info(amp_precond M, amp_pmg_stats *out);
/* z = V(r) (device, n doubles each), the cycle in FP64 (prec 64) or FP32
 * (prec 32, r rounded to FP32 on entry).  Shares the preconditioner's work
 * vectors with solves that use it: calls on one handle must not overlap.
 * Enqueued on stream, not synchronised.  Errors: AMP_ERR_ARG for a null
 * argument, another kind of preconditioner or a bad precision. */
amp_status amp_pmg_apply(amp_precond M, const double *r, double *z, int prec, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* AMP_PCG_H */
