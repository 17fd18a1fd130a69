/*
 * FP64 CPU oracle for the preconditioned conjugate gradient method.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source
 * with the GPU solver.
 *
 * What it computes (all in IEEE double precision, plain CSR):
 *   oracle_pcg          -- Alg. 1 (PCG) of Section 3.3, step by step:
 *                          r0 = b - A x0, beta_{-1} = 0; for k = 0, 1, ...:
 *                          z = M^{-1} r, rho = r^T z, beta = rho/rho_prev (k>0),
 *                          p = z + beta p, q = A p, gamma = q^T p,
 *                          alpha = rho/gamma, x += alpha p, r -= alpha q,
 *                          stop when ||r|| <= tol ||b||.
 *                          A pre-loop test returns 0 iterations when
 *                          ||r0|| <= tol ||b|| (Alg. 1 would otherwise
 *                          divide 0 by 0 when r0 = 0).
 *   M (preconditioner)  -- identity, Jacobi M = diag(A) (Section 5.5), or a
 *                          Chebyshev polynomial: z = D^{-1/2} s(B) D^{-1/2} r
 *                          with B = D^{-1/2} A D^{-1/2}, where s has degree
 *                          m-1 and 1 - t s(t) = T_m((theta - t)/delta) /
 *                          T_m(theta/delta) on [lam_lo, lam_hi]; evaluated by
 *                          the classical three-term Chebyshev iteration for
 *                          B w = v from w = 0 (m-1 products with B).
 *   oracle_spmv         -- y = A x.
 *   oracle_precond      -- z = M^{-1} r alone.
 *
 * Reductions are summed in fixed chunks of ORACLE_CHUNK entries whose
 * partial sums are added in index order, so results do not depend on the
 * OpenMP thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_CHUNK 8192

enum { PC_IDENTITY = 0, PC_JACOBI = 1, PC_CHEBYSHEV = 2 };
enum { ST_CONVERGED = 0, ST_ARG = 1, ST_MAXIT = 2, ST_BREAKDOWN = 3 };

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

void oracle_spmv(int n, const int32_t *rp, const int32_t *ci, const double *val,
                 const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t j = rp[i]; j < rp[i + 1]; ++j) s += val[j] * x[ci[j]];
        y[i] = s;
    }
}

static double dot(int n, const double *a, const double *b) {
    int nchunk = (n + ORACLE_CHUNK - 1) / ORACLE_CHUNK;
    double *part = (double *)malloc(sizeof(double) * (size_t)(nchunk > 0 ? nchunk : 1));
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nchunk; ++c) {
        int lo = c * ORACLE_CHUNK, hi = lo + ORACLE_CHUNK < n ? lo + ORACLE_CHUNK : n;
        double s = 0.0;
        for (int i = lo; i < hi; ++i) s += a[i] * b[i];
        part[c] = s;
    }
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[c];
    free(part);
    return s;
}

static void diagonal(int n, const int32_t *rp, const int32_t *ci, const double *val, double *d) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        d[i] = 0.0;
        for (int32_t j = rp[i]; j < rp[i + 1]; ++j)
            if (ci[j] == i) d[i] = val[j];
    }
}

typedef struct {
    int kind, degree;
    double lam_lo, lam_hi;
    const double *diag; /* diag(A) */
    double *isq;        /* D^{-1/2} (Chebyshev) */
    double *v, *w, *res, *dir, *tmp, *tmp2; /* Chebyshev work vectors */
} precond_t;

/* B u = D^{-1/2} A D^{-1/2} u */
static void apply_B(int n, const int32_t *rp, const int32_t *ci, const double *val,
                    const precond_t *P, const double *u, double *out) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) P->tmp2[i] = P->isq[i] * u[i];
    oracle_spmv(n, rp, ci, val, P->tmp2, out);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) out[i] *= P->isq[i];
}

static void apply_M(int n, const int32_t *rp, const int32_t *ci, const double *val,
                    const precond_t *P, const double *r, double *z) {
    if (P->kind == PC_IDENTITY) {
        memcpy(z, r, sizeof(double) * (size_t)n);
        return;
    }
    if (P->kind == PC_JACOBI) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) z[i] = r[i] / P->diag[i];
        return;
    }
    /* Chebyshev iteration on B w = v, v = D^{-1/2} r, w0 = 0. */
    const double theta = 0.5 * (P->lam_hi + P->lam_lo);
    const double delta = 0.5 * (P->lam_hi - P->lam_lo);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        P->v[i] = P->isq[i] * r[i];
        P->res[i] = P->v[i];           /* residual of w0 = 0 */
        P->dir[i] = P->v[i] / theta;   /* first correction */
        P->w[i] = 0.0;
    }
    for (int k = 0; k < P->degree; ++k) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) P->w[i] += P->dir[i];
        if (k == P->degree - 1) break;
        apply_B(n, rp, ci, val, P, P->dir, P->tmp);
        const double rho_next = 1.0 / (2.0 * sigma - rho);
        const double c1 = rho_next * rho, c2 = 2.0 * rho_next / delta;
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            P->res[i] -= P->tmp[i];
            P->dir[i] = c1 * P->dir[i] + c2 * P->res[i];
        }
        rho = rho_next;
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) z[i] = P->isq[i] * P->w[i];
}

static int precond_init(precond_t *P, int n, const int32_t *rp, const int32_t *ci,
                        const double *val, int kind, int degree, double lo, double hi,
                        double *diag_buf) {
    memset(P, 0, sizeof(*P));
    P->kind = kind;
    P->degree = degree;
    P->lam_lo = lo;
    P->lam_hi = hi;
    diagonal(n, rp, ci, val, diag_buf);
    P->diag = diag_buf;
    if (kind == PC_JACOBI || kind == PC_CHEBYSHEV)
        for (int i = 0; i < n; ++i)
            if (!(diag_buf[i] > 0.0)) return ST_ARG;
    if (kind == PC_CHEBYSHEV) {
        if (degree < 1 || !(hi > lo) || !(lo > 0.0)) return ST_ARG;
        size_t bytes = sizeof(double) * (size_t)n;
        P->isq = (double *)malloc(bytes);
        P->v = (double *)malloc(bytes);
        P->w = (double *)malloc(bytes);
        P->res = (double *)malloc(bytes);
        P->dir = (double *)malloc(bytes);
        P->tmp = (double *)malloc(bytes);
        P->tmp2 = (double *)malloc(bytes);
        for (int i = 0; i < n; ++i) P->isq[i] = 1.0 / sqrt(diag_buf[i]);
    } else if (kind != PC_IDENTITY && kind != PC_JACOBI) {
        return ST_ARG;
    }
    return ST_CONVERGED;
}

static void precond_free(precond_t *P) {
    free(P->isq); free(P->v); free(P->w); free(P->res); free(P->dir); free(P->tmp); free(P->tmp2);
}

int oracle_precond(int n, const int32_t *rp, const int32_t *ci, const double *val, int kind,
                   int degree, double lam_lo, double lam_hi, const double *r, double *z) {
    double *diag = (double *)malloc(sizeof(double) * (size_t)n);
    precond_t P;
    int st = precond_init(&P, n, rp, ci, val, kind, degree, lam_lo, lam_hi, diag);
    if (st == ST_CONVERGED) apply_M(n, rp, ci, val, &P, r, z);
    precond_free(&P);
    free(diag);
    return st;
}

/*
 * out[0] = iterations, out[1] = status, out[2] = ||r_k||/||b|| (updated),
 * out[3] = ||b - A x||/||b|| (true), out[4] = ||b||.
 * delta_hist[k] = ||r_k|| for k = 0..iters; alpha_hist[k], beta_hist[k]
 * (beta_hist[k] = beta_{k-1}, 0 for k = 0) for k = 0..iters-1.  Any history
 * pointer may be NULL; non-NULL ones must hold maxit+1 entries.
 * max_iters_timed > 0 stops after that many iterations (a bounded sample).
 */
int oracle_pcg(int n, const int32_t *rp, const int32_t *ci, const double *val,
               const double *b, double *x, double tol, int maxit, int pc_kind,
               int cheb_degree, double lam_lo, double lam_hi, double *delta_hist,
               double *alpha_hist, double *beta_hist, double *out) {
    for (int i = 0; i < 5; ++i) out[i] = 0.0;
    if (n <= 0 || !(tol > 0.0) || maxit < 0) { out[1] = ST_ARG; return ST_ARG; }
    size_t bytes = sizeof(double) * (size_t)n;
    double *r = (double *)malloc(bytes), *z = (double *)malloc(bytes);
    double *p = (double *)malloc(bytes), *q = (double *)malloc(bytes);
    double *diag = (double *)malloc(bytes);
    precond_t P;
    int status = precond_init(&P, n, rp, ci, val, pc_kind, cheb_degree, lam_lo, lam_hi, diag);
    int iters = 0;
    double bnorm = sqrt(dot(n, b, b)), delta = 0.0;
    if (status != ST_CONVERGED) goto done;

    oracle_spmv(n, rp, ci, val, x, q);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) { r[i] = b[i] - q[i]; p[i] = 0.0; }
    delta = sqrt(dot(n, r, r));
    if (delta_hist) delta_hist[0] = delta;
    if (delta <= tol * bnorm) { status = ST_CONVERGED; goto done; }

    status = ST_MAXIT;
    double rho_prev = 0.0;
    for (int k = 0; k < maxit; ++k) {
        apply_M(n, rp, ci, val, &P, r, z);
        double rho = dot(n, r, z);
        double beta = (k > 0) ? rho / rho_prev : 0.0;
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        oracle_spmv(n, rp, ci, val, p, q);
        double gamma = dot(n, q, p);
        double alpha = rho / gamma;
        if (beta_hist) beta_hist[k] = beta;
        if (alpha_hist) alpha_hist[k] = alpha;
        if (!(rho > 0.0) || !(gamma > 0.0) || !isfinite(alpha)) { status = ST_BREAKDOWN; break; }
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        delta = sqrt(dot(n, r, r));
        iters = k + 1;
        if (delta_hist) delta_hist[k + 1] = delta;
        rho_prev = rho;
        if (delta <= tol * bnorm) { status = ST_CONVERGED; break; }
    }

done:
    out[0] = iters;
    out[1] = status;
    out[4] = bnorm;
    if (status != ST_ARG && bnorm > 0.0) {
        out[2] = delta / bnorm;
        oracle_spmv(n, rp, ci, val, x, q);
        double s = 0.0;
        for (int i = 0; i < n; ++i) { double t = b[i] - q[i]; s += t * t; }
        out[3] = sqrt(s) / bnorm;
    }
    precond_free(&P);
    free(r); free(z); free(p); free(q); free(diag);
    return status;
}
