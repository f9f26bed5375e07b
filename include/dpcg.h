/*
 * dpcg.h - C ABI of the MI355X (gfx950) deflated block-Jacobi conjugate gradient
 * library: CG (Algorithm 1) preconditioned by the adapted-deflation operator
 * A-DEF2 (Sec. 3.2, Algorithms 2 and 3) combined multiplicatively with a
 * block-Jacobi preconditioner over small dense blocks (Sec. 3.4), for the SPD
 * systems K u = f of XFEM/GFEM discretisations of cracked elastic bodies
 * (Sec. 2.4, eq. linear_system).
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers (HBM of the current HIP device)
 *     unless stated otherwise; scalars and the option/info structs are host.
 *   - Floating point is IEEE binary64 throughout.
 *   - Work is ordered on the HIP stream given to dpcg_setup.  Every call returns
 *     to the host only once its results are final (a solve must learn on the host
 *     whether it converged), so outputs may be read right after the call.
 *   - A handle is not re-entrant: calls on one handle must not overlap.  Distinct
 *     handles are independent.
 *   - Return values are status codes (DPCG_OK = 0, positive = finished but not
 *     converged, negative = error).  On error, outputs are unspecified unless the
 *     entry point says otherwise, and info->bad_index names the offending item
 *     when there is one.
 */
#ifndef DPCG_H
#define DPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DPCG_OK = 0,
    DPCG_NOT_CONVERGED = 1,   /* max_iter reached; output holds the last iterate   */
    DPCG_EINVAL = -1,         /* bad sizes, indices, ordering or partition         */
    DPCG_ENOTSYM = -2,        /* |K - K^T| > 1e-12 max|K| (K must be SPD, Sec. 3.2) */
    DPCG_EBLOCK_NOT_SPD = -3, /* a diagonal block K_BB is not SPD; bad_index=block */
    DPCG_ECOARSE_NOT_SPD = -4,/* E = Z^T K Z not SPD: Z not of full column rank     */
    DPCG_EBREAKDOWN = -5,     /* p^T K p <= 0 or non-finite alpha, beta, residual  */
    DPCG_EHIP = -6,           /* HIP runtime or device allocation failure           */
    DPCG_ENONFINITE = -7,     /* NaN or Inf in an input vector                      */
    DPCG_ETOOBIG = -8         /* the problem exceeds dpcg_solve_noalloc's fixed scratch */
};

typedef struct dpcg_ctx *dpcg_handle;

enum {
    DPCG_PREC_FP64 = 0,        /* every step in binary64                                 */
    DPCG_PREC_MIXED = 1        /* FP32-stored K and block inverses inside FP64 refinement */
};

typedef struct {
    int32_t max_iter;          /* iteration cap (K p products); default 20000            */
    int32_t check_every;       /* iterations enqueued between host polls; default 16     */
    int32_t use_initial_guess; /* 1: u (or lambda) holds u_{-1} of Algorithm 2 on entry */
    int32_t record_history;    /* 1: keep ||r_i||/||f|| for i = 0..iterations            */
    int32_t precision;         /* DPCG_PREC_FP64 (default) or DPCG_PREC_MIXED            */
    int32_t max_refinements;   /* mixed: cap on refinement cycles; default 50            */
    double inner_tol;          /* mixed: each inner solve reduces its residual by this
                                  factor (0 < inner_tol < 1); default 1e-4               */
    double switch_tol;         /* mixed: the binary32 refinement stops once the true
                                  residual is <= switch_tol ||f||, and FP64 CG started
                                  from that iterate (Algorithm 2's u_{-1}) finishes the
                                  solve to tol; switch_tol <= tol: refinement only.
                                  Default 1e-6                                           */
} dpcg_options;

typedef struct {
    int32_t status;            /* same value the call returned                          */
    int32_t iterations;        /* number of K p products of Algorithm 1                 */
    double rel_res_recursive;  /* ||r_i||_2 / ||f||_2 of the recursively updated r_i    */
    double rel_res_true;       /* ||f - K u||_2 / ||f||_2 recomputed at exit            */
    double setup_ms;           /* wall time of dpcg_setup                               */
    double solve_ms;           /* wall time of the last solve                           */
    int64_t bad_index;         /* offending block / row / iteration, or -1              */
    int32_t refinements;       /* mixed: refinement cycles (inner solves); FP64: 0      */
    int32_t iterations_fp64;   /* mixed: K p products of the final FP64 phase (included
                                  in iterations); FP64: equal to iterations              */
} dpcg_info;

typedef struct {
    int64_t n;                 /* unknowns                                              */
    int64_t nnz;               /* scalar nonzeros of K                                  */
    int64_t nnzb;              /* 3x3 blocks of the internal block-CSR copy of K        */
    int64_t k;                 /* deflation vectors (columns of Z)                      */
    int64_t nnz_z;             /* nonzeros of Z                                         */
    int64_t nnz_kz;            /* nonzeros of K Z                                       */
    int64_t nblocks;           /* block-Jacobi blocks                                   */
    int64_t bj_values;         /* sum of squared sizes of the blocks of <= 18 unknowns  */
    int64_t device_bytes;      /* device memory held by the handle                      */
    int64_t dense_blocks;      /* blocks of more than 18 unknowns                       */
    int64_t dense_values;      /* entries of their stored inverses (sum of ld^2)        */
    int64_t spmv_col_bytes;    /* bytes per block column the iteration SpMV reads: 2 when
                                  every column fits as a 16-bit offset from its block
                                  row, else 4                                           */
} dpcg_stats;

typedef struct {
    int64_t spmv_launches;     /* launches of the iteration's SpMV kernel timed so far  */
    double spmv_ms;            /* their summed durations (HIP events on the stream)     */
} dpcg_timing;

/* Fills *opt with the defaults above. */
void dpcg_default_options(dpcg_options *opt);

/*
 * Builds a solver for K (n x n) with deflation matrix Z (n x k) and block
 * partition block_ptr.
 *
 *   K:  CSR, full symmetric storage (both triangles), strictly increasing column
 *       indices in each row.  k_rowptr[n+1] (int64), k_col[nnz] (int32),
 *       k_val[nnz].  Unknowns are grouped in consecutive triplets (each nodal DoF
 *       group of the XFEM approximation, eq. xfem_displ, is a 3-vector), so
 *       n % 3 == 0; setup packs K into 3x3 blocks.
 *   Z:  CSR n x k, the deflation basis W of Sec. 3.2 (subdomain rigid-body and
 *       enriched modes of Sec. 3.3); k >= 0, k = 0 disables deflation (plain
 *       block-Jacobi PCG).  Z must have full column rank.
 *   block_ptr[nblocks+1] (int32): the block-Jacobi groups (eq. block_jacobi) as
 *       contiguous ranges [block_ptr[b], block_ptr[b+1]) tiling [0, n), each of
 *       1..8192 unknowns.  Blocks of up to 18 unknowns (one node's standard plus
 *       enriched DoFs, eq. block_jacobi_enr) share the fused small-block kernels.
 *       Larger blocks (the subdomain-sized blocks of Sec. 3.4: all unknowns of
 *       one subdomain, numbered consecutively) keep an explicit FP64 inverse of
 *       ld x ld entries, ld = 32 * ceil(size / 32), made by Gauss-Jordan sweeps
 *       at setup and applied by a dense matrix-vector kernel each iteration;
 *       dpcg_solve_batch and dpcg_solve_many refuse handles with such blocks
 *       (DPCG_EINVAL).
 *   stream: hipStream_t (may be NULL for the default stream) on which all of the
 *       handle's work is ordered.
 *
 * K, Z and block_ptr are device arrays here (dpcg_setup_host takes host arrays).
 * The library deep-copies what it needs; the caller may free K, Z and block_ptr
 * on return.  Setup factorises every block and the coarse matrix E = Z^T K Z
 * (Sec. 3.2; both applied at every iteration) and allocates all device memory
 * the solves need.  Errors: DPCG_EINVAL, DPCG_ENOTSYM, DPCG_EBLOCK_NOT_SPD,
 * DPCG_ECOARSE_NOT_SPD, DPCG_EHIP.  On error *h is NULL.  info may be NULL.
 */
int dpcg_setup(dpcg_handle *h, int64_t n,
               const int64_t *k_rowptr, const int32_t *k_col, const double *k_val,
               int32_t k, const int64_t *z_rowptr, const int32_t *z_col, const double *z_val,
               int32_t nblocks, const int32_t *block_ptr,
               void *stream, dpcg_info *info);

/*
 * dpcg_setup with K, Z and block_ptr in HOST memory (the same arrays, sizes and
 * checks; k_rowptr[n] and z_rowptr[n] give the entry counts).  The arrays are
 * uploaded on `stream` into library-owned device memory, set up as by dpcg_setup
 * and released once the setup has finished; the caller may free them on return.
 * info->setup_ms includes the upload.  Errors as dpcg_setup (DPCG_EINVAL also for a
 * row pointer that does not start at 0 or a negative entry count).
 */
int dpcg_setup_host(dpcg_handle *h, int64_t n,
                    const int64_t *k_rowptr, const int32_t *k_col, const double *k_val,
                    int32_t k, const int64_t *z_rowptr, const int32_t *z_col, const double *z_val,
                    int32_t nblocks, const int32_t *block_ptr,
                    void *stream, dpcg_info *info);

/*
 * Solves K u = f to ||r_i||_2 <= tol ||f||_2 (Sec. 4: relative tolerance) with
 * Algorithm 1, started from Algorithm 2 and preconditioned by Algorithm 3.
 * f[n] and u[n] are caller-owned device buffers; u is output, and also input
 * (u_{-1}) when opt->use_initial_guess.  f = 0 gives u = 0 after 0 iterations.
 * opt may be NULL (defaults).  Returns DPCG_OK, DPCG_NOT_CONVERGED (u holds the
 * last iterate), DPCG_EBREAKDOWN (bad_index = iteration), DPCG_ENONFINITE,
 * DPCG_EINVAL (tol <= 0, max_iter < 0, inner_tol outside (0, 1) or an unknown
 * precision) or DPCG_EHIP.
 *
 * precision = DPCG_PREC_MIXED (an extension beyond the paper's FP64 method), two
 * phases.  (1) Iterative refinement in FP64 around the same method run on binary32
 * copies of K's values and of the block-Jacobi inverses (vectors, E^-1 and all
 * arithmetic stay binary64): each cycle solves K d = r_j for the current FP64
 * residual r_j = f - K u_j (FP64 K) to ||r_j - K32 d|| <= max(inner_tol ||r_j||,
 * switch_tol ||f||), then sets u_{j+1} = u_j + d, until ||f - K u_j|| <=
 * max(tol, switch_tol) ||f||.  (2) When that residual is still above tol ||f||, the
 * FP64 method itself, started from that iterate (Algorithm 2 with u_{-1} = u_j),
 * finishes to tol: each
 * refinement cycle multiplies the error by the inner solve's own error-to-residual
 * ratio, so refinement alone ends with a larger error than the FP64 method at the
 * same residual; the FP64 phase removes it.  The solve stops with the FP64 phase's
 * recursive residual <= tol ||f|| (rel_res_true is recomputed; without an FP64 phase
 * both are the refinement's true residual), or with
 * DPCG_NOT_CONVERGED after max_iter iterations in total or max_refinements cycles.
 * iterations counts all K p products (binary32 inner ones and FP64 ones;
 * iterations_fp64 the latter); the history (record_history) holds
 * ||f - K u_j|| / ||f|| per cycle, j = 0..refinements, then the true residual after
 * the FP64 phase when it ran.  The FP32 copies are made on the first mixed solve of a handle
 * (9 nnzb + sum b^2 floats).
 */
int dpcg_solve(dpcg_handle h, const double *f, double *u, double tol,
               const dpcg_options *opt, dpcg_info *info);

/*
 * Solves K lambda = g with the same operator (K = K^T) and the same method as
 * dpcg_solve, in a workspace of its own, so it never disturbs a forward solve's
 * state.  This is the adjoint solve of a loss L(u): g = dL/du.
 */
int dpcg_solve_adjoint(dpcg_handle h, const double *g, double *lambda, double tol,
                       const dpcg_options *opt, dpcg_info *info);

/*
 * Solves K U = F for nrhs right-hand sides at once, 1 <= nrhs <= 32 (an extension
 * beyond the paper's single-RHS solver): the method of dpcg_solve run as nrhs
 * independent recurrences that share every pass over K, Z, (KZ)^T, E^{-1} and the
 * block inverses.  F and U are n x nrhs, row-major (column j of row d at
 * F[d * nrhs + j]), caller-owned device arrays; U is output, and input when
 * opt->use_initial_guess.  Each column runs Algorithms 1-3 with its own scalars and
 * its own stopping test ||r_j|| <= tol ||F_j||; a column that stops is frozen while
 * the others continue, so column j takes the iterates of dpcg_solve on F[:, j] up to
 * the order of floating-point sums.  A zero column gives 0 after 0 iterations.
 * infos[nrhs] (host, may be NULL) receives one record per column.  Returns DPCG_OK
 * when every column converged, else DPCG_EBREAKDOWN if some column broke down, else
 * DPCG_NOT_CONVERGED; DPCG_EINVAL for nrhs outside [1, 32], tol <= 0, max_iter < 0,
 * record_history or a precision other than DPCG_PREC_FP64; DPCG_ENONFINITE; DPCG_EHIP.
 * The first call makes the handle's multi-RHS workspace (8 n x 32 and 2 k x 32
 * doubles).  SpMV timing (dpcg_set_timing) covers the batched product kernel.
 */
int dpcg_solve_batch(dpcg_handle h, int32_t nrhs, const double *F, double *U, double tol,
                     const dpcg_options *opt, dpcg_info *infos);

/*
 * Solves count independent systems at once (1 <= count <= 64; an extension beyond the
 * paper): handles[i] (distinct handles, each from its own dpcg_setup, any sizes, same
 * device) solves K_i U[i] = F[i] (device arrays of its n_i) with the method of
 * dpcg_solve and its own stopping test.  Each phase of an iteration runs as one kernel
 * launch over the workgroups of every system still iterating, so small systems share
 * the launches instead of queueing 7 of them per iteration each.  Handles that were
 * never tuned get their SpMV lane-group size from dpcg_autotune first.  All work of the
 * call runs on handles[0]'s stream (the others are synchronised first).
 * infos[count] (host, may be NULL).  Returns DPCG_OK when every system converged, else
 * DPCG_EBREAKDOWN if one broke down, else DPCG_NOT_CONVERGED; DPCG_EINVAL (count, a
 * repeated handle, tol, max_iter, record_history or a precision other than FP64),
 * DPCG_ENONFINITE, DPCG_EHIP.
 */
int dpcg_solve_many(dpcg_handle *handles, int32_t count, const double *const *F, double *const *U,
                    double tol, const dpcg_options *opt, dpcg_info *infos);

/*
 * New values of K on the sparsity pattern of the setup (Sec. 3.4: as the crack grows,
 * only the blocks that hold enriched DoFs need new factors).  k_rowptr,
 * k_col, k_val as in dpcg_setup; the pattern (rows, columns, block structure) must be
 * the one the handle was set up with.  The block values, the symmetry test, K Z, E and
 * E^{-1} are rebuilt; the block-Jacobi inverses only of the nchanged blocks listed in
 * changed_blocks (host array of block indices), or of every block when changed_blocks
 * is NULL.  A block whose values changed but is not listed keeps its old inverse: the
 * solves stay correct (an SPD preconditioner), they may take more iterations.
 * info->setup_ms reports the update's wall time.  Errors: DPCG_EINVAL (another
 * pattern, an invalid array or block index), DPCG_ENOTSYM, DPCG_EBLOCK_NOT_SPD,
 * DPCG_ECOARSE_NOT_SPD, DPCG_EHIP; after an error the handle must be destroyed.
 */
int dpcg_update_values(dpcg_handle h, const int64_t *k_rowptr, const int32_t *k_col, const double *k_val,
                       int32_t nchanged, const int32_t *changed_blocks, dpcg_info *info);

/* Times the SpMV kernel for each lane-group size (4, 8, 16, 32 lanes per block row;
 * reps launches each, HIP events) and keeps the fastest for every later solve of the
 * handle.  Returns the chosen size, or a negative status. */
int dpcg_autotune(dpcg_handle h, int32_t reps);

/* Releases every resource of the handle (NULL is a no-op). */
void dpcg_destroy(dpcg_handle h);

/* Device memory of destroyed handles is cached by the library and reused by later
 * setups on the same device; this returns all cached memory to the HIP runtime. */
void dpcg_release_cached_memory(void);

/* Static description of a status code. */
const char *dpcg_status_string(int status);

/* Sizes of the factorised operator; *out is host memory. */
int dpcg_get_stats(dpcg_handle h, dpcg_stats *out);

/* Residual history ||r_i||/||f||, i = 0..iterations, of the last forward solve run
 * with record_history; copies up to cap values into host memory out and returns
 * how many were written (negative status on error). */
int64_t dpcg_get_history(dpcg_handle h, double *out, int64_t cap);

/* Kernel timing for roofline measurements: with on = m >= 1 every solve brackets
 * every m-th launch of the iteration's SpMV kernel (K p, the dominant kernel; m = 1:
 * each launch) with a pair of HIP events recorded by the launch on the handle's
 * stream, and accumulates the durations of the launches that did work; on = 0 stops
 * timing, on < 0 is DPCG_EINVAL.  Turning it on resets the counters.  A timed launch
 * adds about 8 us to its iteration (measured: 0.8 ms per 105-iteration solve with
 * m = 1), so sampling every 8th launch keeps the measured run close to an untimed one.
 * In a mixed-precision solve only the SpMV of the binary32 inner iterations is timed
 * (the FP64 phase that ends it runs the FP64 kernel, which the counters leave out). */
int dpcg_set_timing(dpcg_handle h, int32_t on);
int dpcg_get_timing(dpcg_handle h, dpcg_timing *out);

/*
 * Element sensitivities for the adjoint of a solve (an extension beyond the paper's
 * solver: the assembled stiffness of Sec. 2.4, eq. linear_system, is linear in each
 * element's modulus).  For K = sum_e s_e K_e with K_e element e's matrix at s_e = 1,
 * u = K^{-1} f and a loss L(u) whose adjoint lambda = K^{-1} dL/du comes from
 * dpcg_solve_adjoint, writes g[e] = dL/ds_e = -lambda_e^T K_e u_e, e < nel.
 *   elem_ptr[nel+1] (int64): element e's DoFs are elem_dof[elem_ptr[e]..elem_ptr[e+1])
 *       (int32; -1 marks a DoF removed by a Dirichlet condition, which is skipped);
 *       at most 256 DoFs per element.
 *   kmat_off[nel] (int64): K_e (m_e x m_e, row-major, in the element's DoF order)
 *       starts at kmat[kmat_off[e]]; elements may share one matrix.  kmat_len is the
 *       number of doubles in kmat.
 *   u, lambda: n; g: nel.  All device arrays, caller-owned.
 * The element data are checked on the device first (sizes, DoF and matrix ranges):
 * DPCG_EINVAL if they are inconsistent, nothing written.  K_e must be the matrices K
 * was assembled from for g to be the gradient; the call does not check that.
 */
int dpcg_element_gradient(dpcg_handle h, int64_t nel, const int64_t *elem_ptr, const int32_t *elem_dof,
                          const int64_t *kmat_off, int64_t kmat_len, const double *kmat, const double *u,
                          const double *lambda, double *g);

/*
 * For callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid allocation): dpcg_solve in FP64 with the
 * iteration's workspace (the vectors r, y, z, q, p, the k-vectors, the partial sums
 * and the device state) in a fixed device array of the library instead of the
 * handle's workspace, so the call allocates nothing (no hipMalloc, hipFree, event or
 * pinned-memory creation).  Same arguments, kernels and results as dpcg_solve.
 * Limits: precision must be DPCG_PREC_FP64 and record_history 0 (else DPCG_EINVAL);
 * the workspace must fit in dpcg_noalloc_scratch_bytes() = 96 MiB, about 57 bytes per
 * unknown (up to about 1.7M unknowns; the 80^3 configuration, 1.66M, needs 90 MiB),
 * else DPCG_ETOOBIG before any device work; kernel timing (dpcg_set_timing) is not
 * applied.  The array is one per device, held from the first call on that device
 * until the process ends; it is cleared at the start of every call.  Calls that
 * overlap on one device (any handles, any streams) share it and race: the caller
 * must order them.  The handle must have been set up on the current device.
 */
int dpcg_solve_noalloc(dpcg_handle h, const double *f, double *u, double tol,
                       const dpcg_options *opt, dpcg_info *info);

/* Size in bytes of the fixed device array dpcg_solve_noalloc uses. */
size_t dpcg_noalloc_scratch_bytes(void);

/* ---- single steps of the iteration, each the kernel the solve runs ---- */

/* y = K x (Algorithm 1's K p_i) with the block-CSR kernel.  x, y: device, n. */
int dpcg_spmv(dpcg_handle h, const double *x, double *y);

/* Y = K X for nrhs columns at once, 1 <= nrhs <= 32 (Algorithm 1's K p for every column
 * of dpcg_solve_batch), with that solve's multi-RHS product kernel.  X, Y: n x nrhs
 * row-major device arrays (column j of row d at X[d * nrhs + j]), caller-owned.  The
 * first call makes the handle's multi-RHS workspace.  Returns after the product has
 * completed.  DPCG_EINVAL for nrhs outside [1, 32], null arrays or a handle with blocks
 * of more than 18 DoFs; DPCG_EHIP. */
int dpcg_spmv_batch(dpcg_handle h, int32_t nrhs, const double *X, double *Y);

/* y = K32 x, the product the inner solves of DPCG_PREC_MIXED use: K's values
 * rounded to binary32, products and sums in binary64. */
int dpcg_spmv_fp32(dpcg_handle h, const double *x, double *y);

/* y = M32^{-1} r with the block inverses rounded to binary32 (mixed inner solves). */
int dpcg_bj_apply_fp32(dpcg_handle h, const double *r, double *y);

/* y = M^{-1} r, the block-Jacobi apply inside Algorithm 3 (eq. block_jacobi). */
int dpcg_bj_apply(dpcg_handle h, const double *r, double *y);

/* g = Z^T a - (K Z)^T b (k-vector), the merged right-hand side of Algorithm 3's
 * two coarse solves: Z^T r - Z^T K y with a = r, b = y.  b may be NULL (b = 0). */
int dpcg_restrict(dpcg_handle h, const double *a, const double *b, double *g);

/* delta = E^{-1} g, E = Z^T K Z (k-vectors). */
int dpcg_coarse_apply(dpcg_handle h, const double *g, double *delta);

/* out = base + Z delta (base may be NULL for 0). */
int dpcg_prolong(dpcg_handle h, const double *base, const double *delta, double *out);

/* z = A-DEF2 applied to r (Algorithm 3): z = y + Z E^{-1} (Z^T r - Z^T K y),
 * y = M^{-1} r. */
int dpcg_precond(dpcg_handle h, const double *r, double *z);

#ifdef __cplusplus
}
#endif

#endif /* DPCG_H */
