/*
 * Plain FP64 CPU oracle for the deflated, block-Jacobi-preconditioned conjugate
 * gradient method (A-DEF2) of Agathos, Dodwell, Chatzi and Bordas.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline leg
 * do.  It shares no source with the GPU library.
 *
 * What it computes, in the paper's order and notation (W is called Z here):
 *   - block-Jacobi preconditioner M = blockdiag(K_BB) over a partition of the
 *     unknowns into contiguous blocks (Sec. 3.4, eqs. block_jacobi and
 *     block_jacobi_enr); M^{-1} r is applied by a dense Cholesky solve per block;
 *   - coarse matrix E = Z^T K Z (Sec. 3.2, definition of Q), formed as Z^T (K Z)
 *     and symmetrised as (E + E^T)/2, factorised by dense Cholesky;
 *   - the A-DEF2 initial solution (Algorithm 2: two coarse solves),
 *   - the A-DEF2 preconditioner (Algorithm 3: y = M^{-1} r, two coarse solves
 *     with right-hand sides Z^T K y and Z^T r, z = y + Z(lambda - mu)), with an
 *     explicit product K y,
 *   - preconditioned CG (Algorithm 1, Fletcher-Reeves beta), stopped when
 *     ||r_i||_2 <= tol ||f||_2 for the recursively updated residual (Sec. 4:
 *     relative tolerance 1e-8), tested after each residual update and once on r_0.
 *
 * Readings where the paper is silent: the iteration count is the number of K p
 * products; a breakdown is p^T K p <= 0 or a non-finite alpha or r^T z; f = 0
 * gives u = 0 after 0 iterations.
 *
 * Parallelism: row loops of sparse products and independent block solves use
 * OpenMP; every sum is taken sequentially in index order, so results do not depend
 * on the thread count.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#else
static int omp_get_num_threads(void) { return 1; }
#endif

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_EINVAL (-1)
#define OR_EBLOCK_NOT_SPD (-3)
#define OR_ECOARSE_NOT_SPD (-4)
#define OR_EBREAKDOWN (-5)
#define OR_ENONFINITE (-7)

typedef struct {
    int64_t n;
    int32_t k;
    int64_t *kp; int32_t *kc; double *kv;    /* K, CSR n x n */
    int64_t *zp; int32_t *zc; double *zv;    /* Z, CSR n x k */
    int32_t nblocks; int32_t *bp;            /* block partition, nblocks+1 */
    int64_t *lb_off;                         /* offset of each block's factor in lb */
    double *lb;                              /* dense lower Cholesky factors of K_BB */
    double *le;                              /* dense lower Cholesky factor of E (k x k) */
    double *ework;                           /* E itself (k x k), kept for inspection */
} oracle_t;

/* ---------------------------------------------------------------- basic ops */

/* y = K x (CSR). */
static void spmv(const oracle_t *o, const double *x, double *y) {
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < o->n; i++) {
        double s = 0.0;
        for (int64_t e = o->kp[i]; e < o->kp[i + 1]; e++) s += o->kv[e] * x[o->kc[e]];
        y[i] = s;
    }
}

/* b = Z^T x (k-vector), accumulated row by row in index order. */
static void zt_times(const oracle_t *o, const double *x, double *b) {
    for (int32_t j = 0; j < o->k; j++) b[j] = 0.0;
    for (int64_t i = 0; i < o->n; i++)
        for (int64_t e = o->zp[i]; e < o->zp[i + 1]; e++) b[o->zc[e]] += o->zv[e] * x[i];
}

/* y = x + Z c. */
static void x_plus_z_times(const oracle_t *o, const double *x, const double *c, double *y) {
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < o->n; i++) {
        double s = 0.0;
        for (int64_t e = o->zp[i]; e < o->zp[i + 1]; e++) s += o->zv[e] * c[o->zc[e]];
        y[i] = x[i] + s;
    }
}

static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

/* In-place dense Cholesky A = L L^T of an m x m row-major matrix (lower triangle
 * read, L written to the lower triangle, upper triangle zeroed).  Returns 0, or
 * -1 when a pivot is not finite or not above m * DBL_EPSILON times the matrix's
 * own diagonal entry (A not SPD to working precision). */
static int cholesky(double *A, int64_t m) {
    for (int64_t j = 0; j < m; j++) {
        double d = A[j * m + j];
        double floor_ = (double)m * DBL_EPSILON * fabs(d);
        for (int64_t p = 0; p < j; p++) d -= A[j * m + p] * A[j * m + p];
        if (!(d > floor_) || !isfinite(d)) return -1;
        double ljj = sqrt(d);
        A[j * m + j] = ljj;
        int64_t i;
#pragma omp parallel for schedule(static) if (m - j > 256)
        for (i = j + 1; i < m; i++) {
            double s = A[i * m + j];
            for (int64_t p = 0; p < j; p++) s -= A[i * m + p] * A[j * m + p];
            A[i * m + j] = s / ljj;
        }
    }
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = i + 1; j < m; j++) A[i * m + j] = 0.0;
    return 0;
}

/* Solve L L^T x = b in place (x holds b on entry). */
static void chol_solve(const double *L, int64_t m, double *x) {
    for (int64_t i = 0; i < m; i++) {
        double s = x[i];
        for (int64_t p = 0; p < i; p++) s -= L[i * m + p] * x[p];
        x[i] = s / L[i * m + i];
    }
    for (int64_t i = m - 1; i >= 0; i--) {
        double s = x[i];
        for (int64_t p = i + 1; p < m; p++) s -= L[p * m + i] * x[p];
        x[i] = s / L[i * m + i];
    }
}

/* y = M^{-1} r: one dense Cholesky solve per diagonal block K_BB (eq. block_jacobi). */
static void bj_apply(const oracle_t *o, const double *r, double *y) {
    int32_t b;
#pragma omp parallel for schedule(static)
    for (b = 0; b < o->nblocks; b++) {
        int64_t s = o->bp[b], m = o->bp[b + 1] - o->bp[b];
        for (int64_t i = 0; i < m; i++) y[s + i] = r[s + i];
        chol_solve(o->lb + o->lb_off[b], m, y + s);
    }
}

/* x = E^{-1} b by the Cholesky factor of E. */
static void coarse_solve(const oracle_t *o, const double *b, double *x) {
    memcpy(x, b, sizeof(double) * (size_t)o->k);
    chol_solve(o->le, o->k, x);
}

/* ---------------------------------------------------------------- setup */

static void *xdup(const void *p, size_t bytes) {
    void *q = malloc(bytes ? bytes : 1);
    if (q && bytes) memcpy(q, p, bytes);
    return q;
}

void oracle_destroy(oracle_t *o) {
    if (!o) return;
    free(o->kp); free(o->kc); free(o->kv);
    free(o->zp); free(o->zc); free(o->zv);
    free(o->bp); free(o->lb_off); free(o->lb); free(o->le); free(o->ework);
    free(o);
}

/* Copies K, Z and the block partition; factorises every K_BB and E = Z^T K Z.
 * Returns OR_OK, OR_EINVAL, OR_EBLOCK_NOT_SPD (bad = block) or
 * OR_ECOARSE_NOT_SPD (Z not of full column rank). */
int oracle_setup(oracle_t **out, int64_t n,
                 const int64_t *kp, const int32_t *kc, const double *kv,
                 int32_t k, const int64_t *zp, const int32_t *zc, const double *zv,
                 int32_t nblocks, const int32_t *bp, int64_t *bad) {
    *out = NULL;
    *bad = -1;
    if (n <= 0 || k < 0 || nblocks <= 0 || bp[0] != 0 || bp[nblocks] != n) return OR_EINVAL;
    oracle_t *o = (oracle_t *)calloc(1, sizeof(oracle_t));
    o->n = n; o->k = k; o->nblocks = nblocks;
    o->kp = xdup(kp, sizeof(int64_t) * (size_t)(n + 1));
    o->kc = xdup(kc, sizeof(int32_t) * (size_t)kp[n]);
    o->kv = xdup(kv, sizeof(double) * (size_t)kp[n]);
    o->zp = xdup(zp, sizeof(int64_t) * (size_t)(n + 1));
    o->zc = xdup(zc, sizeof(int32_t) * (size_t)zp[n]);
    o->zv = xdup(zv, sizeof(double) * (size_t)zp[n]);
    o->bp = xdup(bp, sizeof(int32_t) * (size_t)(nblocks + 1));

    /* block-Jacobi: extract each K_BB densely and factorise it */
    o->lb_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nblocks + 1));
    o->lb_off[0] = 0;
    for (int32_t b = 0; b < nblocks; b++) {
        int64_t m = bp[b + 1] - bp[b];
        if (m <= 0) { oracle_destroy(o); return OR_EINVAL; }
        o->lb_off[b + 1] = o->lb_off[b] + m * m;
    }
    o->lb = (double *)calloc((size_t)o->lb_off[nblocks], sizeof(double));
    int failed = -1;
    int32_t b;
#pragma omp parallel for schedule(dynamic, 64)
    for (b = 0; b < nblocks; b++) {
        int64_t s = bp[b], m = bp[b + 1] - bp[b];
        double *A = o->lb + o->lb_off[b];
        for (int64_t i = 0; i < m; i++)
            for (int64_t e = kp[s + i]; e < kp[s + i + 1]; e++) {
                int64_t c = kc[e];
                if (c >= s && c < s + m) A[i * m + (c - s)] = kv[e];
            }
        if (cholesky(A, m) != 0) {
#pragma omp critical
            { if (failed < 0 || b < failed) failed = b; }
        }
    }
    if (failed >= 0) { *bad = failed; oracle_destroy(o); return OR_EBLOCK_NOT_SPD; }

    /* coarse matrix E = Z^T (K Z): K Z row by row, then E += Z[r,:]^T (KZ)[r,:] */
    if (k > 0) {
        double *E = (double *)calloc((size_t)k * (size_t)k, sizeof(double));
        double *acc = (double *)calloc((size_t)k, sizeof(double));
        int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
        char *mark = (char *)calloc((size_t)k, 1);
        for (int64_t r = 0; r < n; r++) {
            int32_t nt = 0;
            for (int64_t e = kp[r]; e < kp[r + 1]; e++) {
                int64_t c = kc[e];
                for (int64_t f = zp[c]; f < zp[c + 1]; f++) {
                    int32_t j = zc[f];
                    if (!mark[j]) { mark[j] = 1; touched[nt++] = j; }
                    acc[j] += kv[e] * zv[f];
                }
            }
            for (int64_t f = zp[r]; f < zp[r + 1]; f++) {
                double zri = zv[f];
                double *Erow = E + (int64_t)zc[f] * k;
                for (int32_t t = 0; t < nt; t++) Erow[touched[t]] += zri * acc[touched[t]];
            }
            for (int32_t t = 0; t < nt; t++) { acc[touched[t]] = 0.0; mark[touched[t]] = 0; }
        }
        free(touched);
        free(mark);
        free(acc);
        for (int32_t i = 0; i < k; i++)
            for (int32_t j = i + 1; j < k; j++) {
                double s = 0.5 * (E[(int64_t)i * k + j] + E[(int64_t)j * k + i]);
                E[(int64_t)i * k + j] = s;
                E[(int64_t)j * k + i] = s;
            }
        o->ework = E;
        o->le = (double *)xdup(E, sizeof(double) * (size_t)k * (size_t)k);
        if (cholesky(o->le, k) != 0) { oracle_destroy(o); return OR_ECOARSE_NOT_SPD; }
    }
    *out = o;
    return OR_OK;
}

/* ---------------------------------------------------------------- algorithms */

/* Algorithm 2: u0 = u_{-1} + Z(mu - lambda) with E lambda = Z^T K u_{-1} and
 * E mu = Z^T f.  u_m1 may be NULL (u_{-1} = 0).  work: 2n + 4k doubles. */
static void adef2_start(const oracle_t *o, const double *f, const double *u_m1, double *u0,
                        double *work) {
    int64_t n = o->n;
    int32_t k = o->k;
    double *ku = work, *zero = work + n, *b1 = work + 2 * n, *lam = b1 + k, *b2 = lam + k,
           *mu = b2 + k;
    if (k == 0) {
        for (int64_t i = 0; i < n; i++) u0[i] = u_m1 ? u_m1[i] : 0.0;
        return;
    }
    if (u_m1) {
        spmv(o, u_m1, ku);
        zt_times(o, ku, b1);
    } else {
        for (int32_t j = 0; j < k; j++) b1[j] = 0.0;
    }
    coarse_solve(o, b1, lam);
    zt_times(o, f, b2);
    coarse_solve(o, b2, mu);
    for (int32_t j = 0; j < k; j++) mu[j] -= lam[j];
    for (int64_t i = 0; i < n; i++) zero[i] = u_m1 ? u_m1[i] : 0.0;
    x_plus_z_times(o, zero, mu, u0);
}

/* Algorithm 3: z = A-DEF2(r).  work: n + 4k doubles. */
static void adef2_apply(const oracle_t *o, const double *r, double *z, double *y,
                        double *work) {
    int32_t k = o->k;
    bj_apply(o, r, y);
    if (k == 0) {
        memcpy(z, y, sizeof(double) * (size_t)o->n);
        return;
    }
    double *ky = work, *b1 = work + o->n, *mu = b1 + k, *b2 = mu + k, *lam = b2 + k;
    spmv(o, y, ky);
    zt_times(o, ky, b1);
    coarse_solve(o, b1, mu);
    zt_times(o, r, b2);
    coarse_solve(o, b2, lam);
    for (int32_t j = 0; j < k; j++) lam[j] -= mu[j];
    x_plus_z_times(o, y, lam, z);
}

static int all_finite(int64_t n, const double *v) {
    for (int64_t i = 0; i < n; i++)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Algorithm 1 preconditioned by Algorithm 3, started from Algorithm 2.
 * u: in (u_{-1} when use_initial_guess) / out (solution).  history (nullable)
 * receives ||r_i||/||f|| for i = 0..iterations.  Returns a status code. */
int oracle_solve(const oracle_t *o, const double *f, double *u, double tol, int32_t max_iter,
                 int32_t use_initial_guess, int32_t *iterations, double *rel_res,
                 double *rel_res_true, double *history, int64_t *bad) {
    int64_t n = o->n;
    int32_t k = o->k;
    *iterations = 0;
    *rel_res = 0.0;
    *rel_res_true = 0.0;
    *bad = -1;
    if (!all_finite(n, f) || (use_initial_guess && !all_finite(n, u))) return OR_ENONFINITE;
    double fnorm = sqrt(dot(n, f, f));
    if (fnorm == 0.0) {
        memset(u, 0, sizeof(double) * (size_t)n);
        if (history) history[0] = 0.0;
        return OR_OK;
    }
    size_t wn = (size_t)(7 * n + 8 * (int64_t)k + 8);
    double *w = (double *)malloc(sizeof(double) * wn);
    double *r = w, *z = r + n, *p = z + n, *q = p + n, *y = q + n, *tmp = y + n;
    double *u_m1 = NULL;
    if (use_initial_guess) {
        u_m1 = (double *)xdup(u, sizeof(double) * (size_t)n);
    }
    adef2_start(o, f, u_m1, u, tmp);
    free(u_m1);
    spmv(o, u, q);
    for (int64_t i = 0; i < n; i++) r[i] = f[i] - q[i];
    double rnorm = sqrt(dot(n, r, r));
    if (history) history[0] = rnorm / fnorm;
    int status = OR_NOT_CONVERGED;
    int32_t it = 0;
    if (rnorm <= tol * fnorm) {
        status = OR_OK;
    } else {
        adef2_apply(o, r, z, y, tmp);
        memcpy(p, z, sizeof(double) * (size_t)n);
        double rho = dot(n, r, z);
        for (int32_t i = 0; i < max_iter; i++) {
            spmv(o, p, q);
            double pq = dot(n, p, q);
            double alpha = rho / pq;
            if (!(pq > 0.0) || !isfinite(pq) || !isfinite(alpha)) {
                status = OR_EBREAKDOWN;
                *bad = i;
                break;
            }
            for (int64_t j = 0; j < n; j++) u[j] += alpha * p[j];
            for (int64_t j = 0; j < n; j++) r[j] -= alpha * q[j];
            it = i + 1;
            rnorm = sqrt(dot(n, r, r));
            if (history) history[it] = rnorm / fnorm;
            if (rnorm <= tol * fnorm) {
                status = OR_OK;
                break;
            }
            adef2_apply(o, r, z, y, tmp);
            double rho_new = dot(n, r, z);
            if (!isfinite(rho_new)) {
                status = OR_EBREAKDOWN;
                *bad = i;
                break;
            }
            double beta = rho_new / rho;
            for (int64_t j = 0; j < n; j++) p[j] = z[j] + beta * p[j];
            rho = rho_new;
        }
    }
    *iterations = it;
    *rel_res = rnorm / fnorm;
    spmv(o, u, q);
    for (int64_t i = 0; i < n; i++) q[i] = f[i] - q[i];
    *rel_res_true = sqrt(dot(n, q, q)) / fnorm;
    free(w);
    return status;
}

/* ---------------------------------------------------------------- pieces, for tests */

void oracle_spmv(const oracle_t *o, const double *x, double *y) { spmv(o, x, y); }

void oracle_bj_apply(const oracle_t *o, const double *r, double *y) { bj_apply(o, r, y); }

/* z = A-DEF2(r) (Algorithm 3); y receives M^{-1} r. */
void oracle_adef2_apply(const oracle_t *o, const double *r, double *z, double *y) {
    double *w = (double *)malloc(sizeof(double) * (size_t)(o->n + 4 * (int64_t)o->k + 4));
    adef2_apply(o, r, z, y, w);
    free(w);
}

/* u0 from Algorithm 2 (u_m1 nullable) and r0 = f - K u0. */
void oracle_start(const oracle_t *o, const double *f, const double *u_m1, double *u0, double *r0) {
    double *w = (double *)malloc(sizeof(double) * (size_t)(2 * o->n + 4 * (int64_t)o->k + 4));
    adef2_start(o, f, u_m1, u0, w);
    spmv(o, u0, r0);
    for (int64_t i = 0; i < o->n; i++) r0[i] = f[i] - r0[i];
    free(w);
}

/* x = E^{-1} b. */
void oracle_coarse_solve(const oracle_t *o, const double *b, double *x) { coarse_solve(o, b, x); }

/* Copies E = Z^T K Z (k x k, symmetrised) into out. */
void oracle_coarse_matrix(const oracle_t *o, double *out) {
    if (o->k > 0) memcpy(out, o->ework, sizeof(double) * (size_t)o->k * (size_t)o->k);
}

int32_t oracle_k(const oracle_t *o) { return o->k; }

/* Threads the OpenMP loops use. */
int32_t oracle_threads(void) {
    int32_t t = 1;
#pragma omp parallel
    {
#pragma omp single
        t = (int32_t)omp_get_num_threads();
    }
    return t;
}

/* b = Z^T x (k-vector). */
void oracle_zt_times(const oracle_t *o, const double *x, double *b) { zt_times(o, x, b); }

/* y = x + Z c (x nullable: 0). */
void oracle_x_plus_z_times(const oracle_t *o, const double *x, const double *c, double *y) {
    if (x) {
        x_plus_z_times(o, x, c, y);
    } else {
        double *zero = (double *)calloc((size_t)o->n, sizeof(double));
        x_plus_z_times(o, zero, c, y);
        free(zero);
    }
}
