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
 *   - the coarse-space correction Q = Z E^{-1} Z^T and the deflation projection
 *     P = I - K Q (Sec. 3.2),
 *   - the A-DEF2 initial solution u_0 = Q f + P^T u_{-1} (Sec. 3.2, Algorithm 2),
 *   - the A-DEF2 preconditioner M_A-DEF2 = P^T M^{-1} + Q (Sec. 3.2, Algorithm 3):
 *     z = P^T y + Q r with y = M^{-1} r, i.e. y - Q(K y) + Q r, each Q applied by
 *     its own coarse Cholesky solve and the product K y formed explicitly,
 *   - preconditioned CG (Algorithm 1, Fletcher-Reeves beta), stopped when
 *     ||r_i||_2 <= tol ||f||_2 for the recursively updated residual (Sec. 4:
 *     relative tolerance 1e-8), tested after each residual update and once on r_0.
 *
 * A second, "fast" mode computes the same iterates (up to rounding) with the exact
 * rewrites the GPU library uses, so that the CPU baseline is not slowed by
 * redundant work: K Z is formed once at setup and Z^T K y is taken as (K Z)^T y
 * (K = K^T); the two coarse solves of the preconditioner are merged into one,
 * delta = E^{-1} (Z^T r - (K Z)^T y), z = y + Z delta (linearity of E^{-1}); and
 * E^{-1} is formed explicitly from the Cholesky factor (E^{-1} = L^{-T} L^{-1}), so
 * a coarse solve is one dense matrix-vector product.  The start vector is
 * u_0 = u_{-1} + Z E^{-1} (Z^T f - (K Z)^T u_{-1}).  The literal mode remains the
 * reference; the fast mode is pinned to it by the tests.
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
    /* fast mode, built on its first use (oracle_prepare_fast) */
    int fast_ready;
    int64_t *ztp; int32_t *ztc; double *ztv; /* Z^T, CSR k x n */
    int64_t *kztp; int32_t *kztc; double *kztv; /* (K Z)^T, CSR k x n */
    double *einv;                            /* E^{-1}, dense k x k */
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

/* y = x + Z c (x nullable: 0). */
static void x_plus_z_times(const oracle_t *o, const double *x, const double *c, double *y) {
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < o->n; i++) {
        double s = 0.0;
        for (int64_t e = o->zp[i]; e < o->zp[i + 1]; e++) s += o->zv[e] * c[o->zc[e]];
        y[i] = x ? x[i] + s : s;
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
    free(o->ztp); free(o->ztc); free(o->ztv);
    free(o->kztp); free(o->kztc); free(o->kztv); free(o->einv);
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

/* out = Q x = Z E^{-1} Z^T x, the coarse-space correction of Sec. 3.2, applied by a
 * Cholesky solve with E.  work: 2k doubles. */
static void apply_Q(const oracle_t *o, const double *x, double *out, double *work) {
    double *b = work, *c = work + o->k;
    zt_times(o, x, b);
    coarse_solve(o, b, c);
    x_plus_z_times(o, NULL, c, out);
}

/* Literal start (Sec. 3.2, Algorithm 2): u_0 = Q f + P^T u_{-1}, with
 * P^T u_{-1} = u_{-1} - Q K u_{-1} (P = I - K Q, K and Q symmetric).
 * u_m1 may be NULL (u_{-1} = 0).  work: 3n + 2k doubles. */
static void adef2_start(const oracle_t *o, const double *f, const double *u_m1, double *u0,
                        double *work) {
    int64_t n = o->n;
    if (o->k == 0) {
        for (int64_t i = 0; i < n; i++) u0[i] = u_m1 ? u_m1[i] : 0.0;
        return;
    }
    double *qf = work, *ku = work + n, *qku = work + 2 * n, *cw = work + 3 * n;
    apply_Q(o, f, qf, cw);
    if (u_m1) {
        spmv(o, u_m1, ku);
        apply_Q(o, ku, qku, cw);
        for (int64_t i = 0; i < n; i++) u0[i] = qf[i] + (u_m1[i] - qku[i]);
    } else {
        for (int64_t i = 0; i < n; i++) u0[i] = qf[i];
    }
}

/* Literal preconditioner (Sec. 3.2, Algorithm 3): z = M_A-DEF2 r = P^T M^{-1} r + Q r
 * = y - Q(K y) + Q r with y = M^{-1} r.  work: 3n + 2k doubles. */
static void adef2_apply(const oracle_t *o, const double *r, double *z, double *y,
                        double *work) {
    int64_t n = o->n;
    bj_apply(o, r, y);
    if (o->k == 0) {
        memcpy(z, y, sizeof(double) * (size_t)n);
        return;
    }
    double *ky = work, *qky = work + n, *qr = work + 2 * n, *cw = work + 3 * n;
    spmv(o, y, ky);
    apply_Q(o, ky, qky, cw);
    apply_Q(o, r, qr, cw);
    for (int64_t i = 0; i < n; i++) z[i] = (y[i] - qky[i]) + qr[i];
}

/* ---------------------------------------------------------------- fast mode */

/* Transpose of a CSR m x c matrix into a CSR c x m matrix (rows of each column in
 * increasing order). */
static void csr_transpose(int64_t m, int32_t c, const int64_t *p, const int32_t *ci, const double *v,
                          int64_t **tp, int32_t **tc, double **tv) {
    int64_t nnz = p[m];
    int64_t *q = (int64_t *)calloc((size_t)c + 1, sizeof(int64_t));
    for (int64_t e = 0; e < nnz; e++) q[ci[e] + 1]++;
    for (int32_t j = 0; j < c; j++) q[j + 1] += q[j];
    int64_t *fill = (int64_t *)xdup(q, sizeof(int64_t) * (size_t)c);
    int32_t *cc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
    double *vv = (double *)malloc(sizeof(double) * (size_t)(nnz ? nnz : 1));
    for (int64_t i = 0; i < m; i++)
        for (int64_t e = p[i]; e < p[i + 1]; e++) {
            int64_t d = fill[ci[e]]++;
            cc[d] = (int32_t)i;
            vv[d] = v[e];
        }
    free(fill);
    *tp = q; *tc = cc; *tv = vv;
}

/* Builds Z^T, (K Z)^T and E^{-1} for the fast mode (once per oracle). */
int oracle_prepare_fast(oracle_t *o) {
    if (o->fast_ready) return OR_OK;
    int64_t n = o->n;
    int32_t k = o->k;
    if (k > 0) {
        csr_transpose(n, k, o->zp, o->zc, o->zv, &o->ztp, &o->ztc, &o->ztv);
        /* K Z row by row: (K Z)[r, j] = sum_e K[r, c_e] Z[c_e, j], columns sorted */
        int64_t *kzp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
        int64_t r;
#pragma omp parallel
        {
            char *mark = (char *)calloc((size_t)k, 1);
#pragma omp for schedule(static)
            for (r = 0; r < n; r++) {
                int64_t cnt = 0;
                for (int64_t e = o->kp[r]; e < o->kp[r + 1]; e++)
                    for (int64_t f = o->zp[o->kc[e]]; f < o->zp[o->kc[e] + 1]; f++)
                        if (!mark[o->zc[f]]) { mark[o->zc[f]] = 1; cnt++; }
                for (int64_t e = o->kp[r]; e < o->kp[r + 1]; e++)
                    for (int64_t f = o->zp[o->kc[e]]; f < o->zp[o->kc[e] + 1]; f++) mark[o->zc[f]] = 0;
                kzp[r + 1] = cnt;
            }
            free(mark);
        }
        for (r = 0; r < n; r++) kzp[r + 1] += kzp[r];
        int32_t *kzc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(kzp[n] ? kzp[n] : 1));
        double *kzv = (double *)malloc(sizeof(double) * (size_t)(kzp[n] ? kzp[n] : 1));
#pragma omp parallel
        {
            double *acc = (double *)calloc((size_t)k, sizeof(double));
            char *mark = (char *)calloc((size_t)k, 1);
#pragma omp for schedule(static)
            for (r = 0; r < n; r++) {
                int64_t d = kzp[r];
                for (int64_t e = o->kp[r]; e < o->kp[r + 1]; e++)
                    for (int64_t f = o->zp[o->kc[e]]; f < o->zp[o->kc[e] + 1]; f++) {
                        int32_t j = o->zc[f];
                        if (!mark[j]) { mark[j] = 1; kzc[d++] = j; }
                        acc[j] += o->kv[e] * o->zv[f];
                    }
                /* sort the row's columns (insertion sort: rows hold a few dozen) */
                for (int64_t a = kzp[r] + 1; a < kzp[r + 1]; a++) {
                    int32_t t = kzc[a];
                    int64_t b = a - 1;
                    while (b >= kzp[r] && kzc[b] > t) { kzc[b + 1] = kzc[b]; b--; }
                    kzc[b + 1] = t;
                }
                for (int64_t a = kzp[r]; a < kzp[r + 1]; a++) {
                    kzv[a] = acc[kzc[a]];
                    acc[kzc[a]] = 0.0;
                    mark[kzc[a]] = 0;
                }
            }
            free(acc);
            free(mark);
        }
        csr_transpose(n, k, kzp, kzc, kzv, &o->kztp, &o->kztc, &o->kztv);
        free(kzp); free(kzc); free(kzv);
        /* E^{-1} = L^{-T} L^{-1}: X row j = column j of L^{-1} (forward substitution
         * from row j on), then (E^{-1})_{ab} = sum_{c >= max(a, b)} X[a][c] X[b][c] */
        const double *L = o->le;
        double *X = (double *)calloc((size_t)k * (size_t)k, sizeof(double));
        int32_t j;
#pragma omp parallel for schedule(dynamic, 8)
        for (j = 0; j < k; j++) {
            double *x = X + (int64_t)j * k;
            for (int64_t i = j; i < k; i++) {
                double s = (i == j) ? 1.0 : 0.0;
                for (int64_t p = j; p < i; p++) s -= L[i * k + p] * x[p];
                x[i] = s / L[i * k + i];
            }
        }
        o->einv = (double *)malloc(sizeof(double) * (size_t)k * (size_t)k);
        int32_t a;
#pragma omp parallel for schedule(dynamic, 8)
        for (a = 0; a < k; a++) {
            const double *xa = X + (int64_t)a * k;
            for (int32_t b = 0; b <= a; b++) {
                const double *xb = X + (int64_t)b * k;
                double s = 0.0;
                for (int64_t c = a; c < k; c++) s += xa[c] * xb[c];
                o->einv[(int64_t)a * k + b] = s;
            }
        }
        for (a = 0; a < k; a++)
            for (int32_t b = a + 1; b < k; b++) o->einv[(int64_t)a * k + b] = o->einv[(int64_t)b * k + a];
        free(X);
    }
    o->fast_ready = 1;
    return OR_OK;
}

/* g = Z^T a - (K Z)^T b (b nullable: 0); one k-row of each transpose per entry, summed
 * in increasing row order. */
static void fast_restrict(const oracle_t *o, const double *a, const double *b, double *g) {
    int32_t j;
#pragma omp parallel for schedule(static)
    for (j = 0; j < o->k; j++) {
        double s = 0.0, t = 0.0;
        for (int64_t e = o->ztp[j]; e < o->ztp[j + 1]; e++) s += o->ztv[e] * a[o->ztc[e]];
        if (b)
            for (int64_t e = o->kztp[j]; e < o->kztp[j + 1]; e++) t += o->kztv[e] * b[o->kztc[e]];
        g[j] = s - t;
    }
}

/* delta = E^{-1} g (dense product, each row summed in column order). */
static void fast_coarse(const oracle_t *o, const double *g, double *delta) {
    int32_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < o->k; i++) {
        const double *row = o->einv + (int64_t)i * o->k;
        double s = 0.0;
        for (int32_t j = 0; j < o->k; j++) s += row[j] * g[j];
        delta[i] = s;
    }
}

/* Fast start: u_0 = u_{-1} + Z E^{-1} (Z^T f - (K Z)^T u_{-1}).  work: 2k doubles. */
static void fast_start(const oracle_t *o, const double *f, const double *u_m1, double *u0, double *work) {
    int64_t n = o->n;
    if (o->k == 0) {
        for (int64_t i = 0; i < n; i++) u0[i] = u_m1 ? u_m1[i] : 0.0;
        return;
    }
    double *g = work, *d = work + o->k;
    fast_restrict(o, f, u_m1, g);
    fast_coarse(o, g, d);
    x_plus_z_times(o, u_m1, d, u0);
}

/* Fast preconditioner: z = y + Z E^{-1} (Z^T r - (K Z)^T y), y = M^{-1} r.  work: 2k. */
static void fast_apply(const oracle_t *o, const double *r, double *z, double *y, double *work) {
    bj_apply(o, r, y);
    if (o->k == 0) {
        memcpy(z, y, sizeof(double) * (size_t)o->n);
        return;
    }
    double *g = work, *d = work + o->k;
    fast_restrict(o, r, y, g);
    fast_coarse(o, g, d);
    x_plus_z_times(o, y, d, z);
}

static int all_finite(int64_t n, const double *v) {
    for (int64_t i = 0; i < n; i++)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Algorithm 1 preconditioned by Algorithm 3, started from Algorithm 2.
 * u: in (u_{-1} when use_initial_guess) / out (solution).  history (nullable)
 * receives ||r_i||/||f|| for i = 0..iterations.  fast = 0: the literal operators;
 * fast = 1: the fast mode (oracle_prepare_fast first).  Returns a status code. */
int oracle_solve(oracle_t *o, const double *f, double *u, double tol, int32_t max_iter,
                 int32_t use_initial_guess, int32_t fast, int32_t *iterations, double *rel_res,
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
    if (fast) oracle_prepare_fast(o);
    size_t wn = (size_t)(8 * n + 8 * (int64_t)k + 8);
    double *w = (double *)malloc(sizeof(double) * wn);
    double *r = w, *z = r + n, *p = z + n, *q = p + n, *y = q + n, *tmp = y + n;
    double *u_m1 = NULL;
    if (use_initial_guess) {
        u_m1 = (double *)xdup(u, sizeof(double) * (size_t)n);
    }
    if (fast)
        fast_start(o, f, u_m1, u, tmp);
    else
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
        if (fast)
            fast_apply(o, r, z, y, tmp);
        else
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
            if (fast)
                fast_apply(o, r, z, y, tmp);
            else
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

/* z = A-DEF2(r) (Algorithm 3); y receives M^{-1} r.  fast selects the mode. */
void oracle_adef2_apply(oracle_t *o, const double *r, double *z, double *y, int32_t fast) {
    double *w = (double *)malloc(sizeof(double) * (size_t)(3 * o->n + 4 * (int64_t)o->k + 4));
    if (fast) {
        oracle_prepare_fast(o);
        fast_apply(o, r, z, y, w);
    } else {
        adef2_apply(o, r, z, y, w);
    }
    free(w);
}

/* u0 from Algorithm 2 (u_m1 nullable) and r0 = f - K u0.  fast selects the mode. */
void oracle_start(oracle_t *o, const double *f, const double *u_m1, double *u0, double *r0, int32_t fast) {
    double *w = (double *)malloc(sizeof(double) * (size_t)(3 * o->n + 4 * (int64_t)o->k + 4));
    if (fast) {
        oracle_prepare_fast(o);
        fast_start(o, f, u_m1, u0, w);
    } else {
        adef2_start(o, f, u_m1, u0, w);
    }
    spmv(o, u0, r0);
    for (int64_t i = 0; i < o->n; i++) r0[i] = f[i] - r0[i];
    free(w);
}

/* Copies the fast mode's explicit E^{-1} (k x k) into out. */
void oracle_coarse_inverse(oracle_t *o, double *out) {
    oracle_prepare_fast(o);
    if (o->k > 0) memcpy(out, o->einv, sizeof(double) * (size_t)o->k * (size_t)o->k);
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
    x_plus_z_times(o, x, c, y);
}
