// HIP kernels (gfx950, wave64) of one deflated block-Jacobi CG iteration.
//
// One iteration of Algorithm 1 preconditioned by Algorithm 3 runs as five kernels:
//   spmv_p       p_i = z_i + beta p_{i-1} (formed on the fly), q = K p_i, p_i^T q partials
//   update_bj    alpha = rho_i / p^T q; u += alpha p; r -= alpha q; ||r||^2 partials;
//                y = M^{-1} r over whole blocks staged in LDS
//   restrict     convergence test; g = Z^T r - (K Z)^T y  (the two right-hand sides of
//                Algorithm 3's coarse solves, merged by linearity, with Z^T K y = (KZ)^T y)
//   coarse       delta = E^{-1} g  (both coarse solves at once: lambda - mu = delta)
//   prolong      z = y + Z delta; r^T z partials; advance the iteration counter
// Global reductions are two-stage and fixed-order (per-workgroup partials, then a
// sequential-per-thread + fixed-tree sum), so results are bitwise reproducible.  No
// floating-point atomics are used.  Convergence and breakdown are decided on the
// device; every kernel returns at once when the state flag is set.
#include <hip/hip_ext.h>

#include <algorithm>

#include "dpcg_internal.h"

namespace dpcg {

namespace {

// Sum over the workgroup; every thread receives the same value.
__device__ __forceinline__ double block_sum(double v, double *lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    return (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

// Fixed-order sum of n partials, valid in every thread.
__device__ __forceinline__ double reduce_parts(const double *parts, int n, double *lds) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) s += parts[i];
    return block_sum(s, lds);
}

// Workgroup sum over NW waves (lds >= NW entries); every thread receives the same value.
template <int NW>
__device__ __forceinline__ double block_sum_n(double v, double *lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; w += 2) s += lds[w] + lds[w + 1];
    return s;
}

// This thread's fixed-order share of sum_i parts[i] for a block of NT threads: U
// independent accumulators (entries t + NT (U j + u)), their loads issued together, then
// the tail and a fixed tree over the accumulators.
template <int NT, int U>
__device__ __forceinline__ double strided_share(const double *__restrict__ parts, int n) {
    double a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] = 0.0;
    int i = threadIdx.x;
    for (; i + (U - 1) * NT < n; i += U * NT) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = parts[i + u * NT];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] += v[u];
    }
    for (; i < n; i += NT) a[0] += parts[i];
#pragma unroll
    for (int w = 1; w < U; w <<= 1)
#pragma unroll
        for (int u = 0; u + w < U; u += 2 * w) a[u] += a[u + w];
    return a[0];
}

template <int NW>
__device__ __forceinline__ double reduce_parts_n(const double *parts, int n, double *lds) {
    return block_sum_n<NW>(strided_share<NW * 64, 16>(parts, n), lds);
}

__device__ __forceinline__ bool leader() { return blockIdx.x == 0 && threadIdx.x == 0; }

// The state flag as seen by the whole workgroup: one thread reads it and the value is
// broadcast through LDS, so every wave of the workgroup takes the same branch even when
// another workgroup of the same kernel changes the flag meanwhile.
__device__ __forceinline__ int32_t wg_flag(const State *st) {
    __shared__ int32_t f;
    if (threadIdx.x == 0) f = __atomic_load_n(&st->flag, __ATOMIC_RELAXED);
    __syncthreads();
    const int32_t v = f;
    __syncthreads();
    return v;
}

// Two workgroup sums over NW waves at once (lds >= 2 NW entries); every thread
// receives both.
template <int NW>
__device__ __forceinline__ void block_sum2_n(double &a, double &b, double *lds) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        lds[wv] = a;
        lds[NW + wv] = b;
    }
    __syncthreads();
    double x = 0.0, y = 0.0;
#pragma unroll
    for (int w = 0; w < NW; w += 2) {
        x += lds[w] + lds[w + 1];
        y += lds[NW + w] + lds[NW + w + 1];
    }
    a = x;
    b = y;
}

struct XPlain {
    const double *__restrict__ x;
    __device__ __forceinline__ double operator()(int64_t i) const { return x[i]; }
};

// q_R = sum_b K_Rb x_b for block row R, computed by a group of G lanes; the three
// sums end up in every lane of the group.  Lanes of groups without a row pass
// row = -1 and take part in the shuffles with zeros.
// V is the storage type of the block values (double, or float for the inner solves of
// mixed precision); the arithmetic is FP64 either way.
// block column of entry b of block row `row`: stored as is (int32) or as its offset from
// the row (int16, when every offset fits)
__device__ __forceinline__ int64_t col_at(const int32_t *__restrict__ bc, int b, int row) { return bc[b]; }
__device__ __forceinline__ int64_t col_at(const int16_t *__restrict__ bc, int b, int row) {
    return (int64_t)row + bc[b];
}

// The sums over the row's G lanes, scattered: the exchanges with the lanes G/2 and then
// G/4 apart (the butterfly's first two) each halve what a lane carries, a zero fourth
// value padding the three, so that lane lg keeps element e = 2 [lg & G/2] + [lg & G/4];
// the exchanges 8 .. 1 lanes apart complete it.  Every element is summed in the
// butterfly's pairing (the same bits); lane e G/4 of the group returns element e < 3.
template <int G, int OFF>
__device__ __forceinline__ void lanes_add(double &v) {
    if constexpr (OFF >= 1) {
        v += lane_xor<OFF>(v);
        lanes_add<G, OFF / 2>(v);
    }
}

template <int G>
__device__ __forceinline__ double row_scatter(int lg, double a0, double a1, double a2) {
    const bool hi = lg & (G / 2), lo = lg & (G / 4);
    const double k0 = (hi ? a2 : a0) + lane_xor<G / 2>(hi ? a0 : a2);
    const double k1 = (hi ? 0.0 : a1) + lane_xor<G / 2>(hi ? a1 : 0.0);
    double v = (lo ? k1 : k0) + lane_xor<G / 4>(lo ? k0 : k1);
    lanes_add<G, G / 8>(v);
    return v;
}

// lane lg of a row's group holds element row_elem(lg) of the row's product (3: none)
template <int G>
__device__ __forceinline__ int row_elem(int lg) {
    return lg % (G / 4) == 0 ? lg / (G / 4) : 3;
}

template <int G, class XL, class V, class CI>
__device__ __forceinline__ double block_row_span(int row, int beg, int end, int lg, const CI *__restrict__ bcol,
                                                 const V *__restrict__ bval, const XL &xl) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    if (row >= 0) {
        const int64_t m = end - beg;
        const V *rv = bval + 9 * (int64_t)beg - beg;  // plane e of block b: rv[e * m + b]
        for (int b = beg + lg; b < end; b += G) {
            const double v0 = rv[b], v1 = rv[m + b], v2 = rv[2 * m + b];
            const double v3 = rv[3 * m + b], v4 = rv[4 * m + b], v5 = rv[5 * m + b];
            const double v6 = rv[6 * m + b], v7 = rv[7 * m + b], v8 = rv[8 * m + b];
            const int64_t c = 3 * col_at(bcol, b, row);
            const double x0 = xl(c), x1 = xl(c + 1), x2 = xl(c + 2);
            a0 = fma(v0, x0, fma(v1, x1, fma(v2, x2, a0)));
            a1 = fma(v3, x0, fma(v4, x1, fma(v5, x2, a1)));
            a2 = fma(v6, x0, fma(v7, x1, fma(v8, x2, a2)));
        }
    }
    return row_scatter<G>(lg, a0, a1, a2);
}

template <int G, class XL, class V>
__device__ __forceinline__ double block_row(int row, int lg, const int32_t *__restrict__ brow_ptr,
                                            const int32_t *__restrict__ bcol, const V *__restrict__ bval,
                                            int64_t nnzb, const XL &xl) {
    int beg = 0, end = 0;
    if (row >= 0) {
        beg = brow_ptr[row];
        end = brow_ptr[row + 1];
    }
    return block_row_span<G>(row, beg, end, lg, bcol, bval, xl);
}

struct SpmvShape {
    int32_t nb;
    int32_t steps;
    int32_t nwg;
};

// The SpMV kernels run kSpmvWaves waves per workgroup; every wave handles 64 / G rows
// per step, and a workgroup normally covers exactly one step, so each wave issues all of
// its loads at once and many small workgroups in flight hide the index -> gather latency.
constexpr int kSpmvWaves = 4;
constexpr int kSpmvThreads = 64 * kSpmvWaves;

// Row steps [s0, s1) of workgroup w: one step each when the grid has a workgroup per
// step (the usual launch; workgroups past the last step get none), else an even split.
__device__ __forceinline__ void step_range(int w, const SpmvShape &sh, int &s0, int &s1) {
    if (sh.nwg >= sh.steps) {
        s0 = w;
        s1 = w < sh.steps ? w + 1 : w;
    } else {
        s0 = (int)(((int64_t)w * sh.steps) / sh.nwg);
        s1 = (int)(((int64_t)(w + 1) * sh.steps) / sh.nwg);
    }
}

// Row handled by this lane group at step s, or -1.
template <int G>
__device__ __forceinline__ int step_row(int s, int nb) {
    constexpr int kGroupsPerWave = 64 / G;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = (s * kSpmvWaves + wv) * kGroupsPerWave + lane / G;
    return row < nb ? row : -1;
}

// MODE 0: y = K x.   MODE 1: r = f - K x and ||r||^2 partials.
template <int G, int MODE, class V>
__device__ __forceinline__ void k_spmv_body(int vb, SpmvShape sh, const int32_t *__restrict__ brow_ptr,
                                                   const int32_t *__restrict__ bcol,
                                                   const V *__restrict__ bval, int64_t nnzb,
                                                   const double *__restrict__ x, const double *__restrict__ f,
                                                   double *__restrict__ y, double *__restrict__ part) {
    __shared__ double lds[kSpmvWaves];
    const int w = xcd_remap(vb, sh.nwg);
    int s0, s1;
    step_range(w, sh, s0, s1);
    const int lg = threadIdx.x % G;
    XPlain xl{x};
    double acc = 0.0;
    for (int s = s0; s < s1; ++s) {
        const int row = step_row<G>(s, sh.nb);
        const double v = block_row<G>(row, lg, brow_ptr, bcol, bval, nnzb, xl);
        const int e = row_elem<G>(lg);
        if (row >= 0 && e < 3) {
            const int64_t i = 3 * (int64_t)row + e;
            if (MODE == 0) {
                y[i] = v;
            } else {
                const double ri = f[i] - v;
                y[i] = ri;
                acc = fma(ri, ri, acc);
            }
        }
    }
    if (MODE == 1) {
        const double t = block_sum_n<kSpmvWaves>(acc, lds);
        if (threadIdx.x == 0) part[vb] = t;
    }
}

template <int G, int MODE, class V>
__global__ __launch_bounds__(kSpmvThreads) void k_spmv(SpmvShape sh, const int32_t *__restrict__ brow_ptr,
                                                   const int32_t *__restrict__ bcol,
                                                   const V *__restrict__ bval, int64_t nnzb,
                                                   const double *__restrict__ x, const double *__restrict__ f,
                                                   double *__restrict__ y, double *__restrict__ part) {
    k_spmv_body<G, MODE, V>(blockIdx.x, sh, brow_ptr, bcol, bval, nnzb, x, f, y, part);
}


// Matrix product of Algorithm 1 for iteration i = st->iter: q = K p_i (p_i in buffer
// i & 1, formed by the prolongation or the beta kernel) and partials of p_i^T q.  Only
// single-workgroup kernels and workgroup 0 of later kernels change the flag, so it is
// stable while this kernel runs.  The first step's row pointers are loaded before the
// state, so that the two round trips overlap.
template <int G, class V, class CI = int32_t>
__device__ __forceinline__ void k_spmv_p_body(int vb, SpmvShape sh, const int32_t *__restrict__ brow_ptr,
                                                         const CI *__restrict__ bcol,
                                                         const V *__restrict__ bval, int64_t nnzb,
                                                         const double *p0, const double *p1,
                                                         double *__restrict__ q, double *__restrict__ part_pq,
                                                         const State *st) {
    __shared__ double lds[kSpmvWaves];
    const int w = xcd_remap(vb, sh.nwg);
    int s0, s1;
    step_range(w, sh, s0, s1);
    const int lg = threadIdx.x % G;
    int row = s0 < s1 ? step_row<G>(s0, sh.nb) : -1;
    int beg = 0, end = 0;
    if (row >= 0) {
        beg = brow_ptr[row];
        end = brow_ptr[row + 1];
    }
    if (st->flag != kRunning) return;
    const double *__restrict__ p = (st->iter & 1) ? p1 : p0;
    XPlain xl{p};
    double acc = 0.0;
    for (int s = s0; s < s1; ++s) {
        if (s > s0) {
            row = step_row<G>(s, sh.nb);
            if (row >= 0) {
                beg = brow_ptr[row];
                end = brow_ptr[row + 1];
            }
        }
        const double v = block_row_span<G>(row, beg, end, lg, bcol, bval, xl);
        const int e = row_elem<G>(lg);
        if (row >= 0 && e < 3) {
            const int64_t i = 3 * (int64_t)row + e;
            q[i] = v;
            acc = fma(p[i], v, acc);
        }
    }
    const double t = block_sum_n<kSpmvWaves>(acc, lds);
    if (threadIdx.x == 0) part_pq[vb] = t;
}

template <int G, class V, class CI>
__global__ __launch_bounds__(kSpmvThreads) void k_spmv_p(SpmvShape sh, const int32_t *__restrict__ brow_ptr,
                                                         const CI *__restrict__ bcol,
                                                         const V *__restrict__ bval, int64_t nnzb,
                                                         const double *p0, const double *p1,
                                                         double *__restrict__ q, double *__restrict__ part_pq,
                                                         const State *st) {
    k_spmv_p_body<G, V, CI>(blockIdx.x, sh, brow_ptr, bcol, bval, nnzb, p0, p1, q, part_pq, st);
}


// First stage of p_i^T q_i: workgroup a of kAlphaParts sums its contiguous share of the
// SpMV's per-workgroup partials (one load per thread, fixed order) into part2[a]; the
// update kernel adds the kAlphaParts sums and forms alpha_i itself.
__device__ __forceinline__ void k_alpha_body(int a, const double *__restrict__ part_pq, int n,
                                             double *__restrict__ part2, const State *st) {
    __shared__ double lds[16];
    if (st->flag != kRunning) return;
    const int per = (n + kAlphaParts - 1) / kAlphaParts;
    const int i0 = min(n, a * per), i1 = min(n, i0 + per);
    const double s = block_sum_n<16>(strided_share<1024, 4>(part_pq + i0, i1 - i0), lds);
    if (threadIdx.x == 0) part2[a] = s;
}

__global__ __launch_bounds__(1024) void k_alpha(const double *__restrict__ part_pq, int n, double *__restrict__ part2,
                                                const State *st) {
    k_alpha_body(blockIdx.x, part_pq, n, part2, st);
}

// rho_i = r_i^T z_i from the prolongation partials (every workgroup reduces them in
// the same fixed order, so all hold the same bits), beta_{i-1} = rho_i / rho_{i-1} and
// the search direction p_i = z_i + beta_{i-1} p_{i-1} (p_0 = z_0) into buffer i & 1 over
// the workgroup's DoF range.  Workgroup 0 stores rho_i in slot i & 1 (rho_{i-1} in the
// other slot stays valid for the others) and tests it for breakdown.
__device__ __forceinline__ void k_beta_p_body(int vb, const double *__restrict__ part_rho, int nparts, int64_t n,
                                                     int32_t nwg, const double *__restrict__ z, double *p0,
                                                     double *p1, State *st) {
    __shared__ double lds[4];
    if (wg_flag(st) != kRunning) return;
    const int it = st->iter;
    const double rho = reduce_parts_n<4>(part_rho, nparts, lds);
    const bool bad = it > 0 && !isfinite(rho);
    const double beta = it > 0 ? rho / st->rho[(it + 1) & 1] : 0.0;
    if ((vb == 0 && threadIdx.x == 0)) {
        if (bad) {
            st->flag = kBreakdown;
            st->bad = it - 1;
            st->iters_done = it;
        } else {
            st->beta = beta;
            st->rho[it & 1] = rho;
        }
    }
    if (bad) return;
    double *__restrict__ pc = (it & 1) ? p1 : p0;
    const double *__restrict__ pp = (it & 1) ? p0 : p1;
    const int w = xcd_remap(vb, nwg);
    const int64_t per = (n + nwg - 1) / nwg;
    const int64_t d1 = min(n, (int64_t)(w + 1) * per);
    for (int64_t d = (int64_t)w * per + threadIdx.x; d < d1; d += kThreads) pc[d] = it == 0 ? z[d] : fma(beta, pp[d], z[d]);
}

__global__ __launch_bounds__(kThreads) void k_beta_p(const double *__restrict__ part_rho, int nparts, int64_t n,
                                                     int32_t nwg, const double *__restrict__ z, double *p0,
                                                     double *p1, State *st) {
    k_beta_p_body(blockIdx.x, part_rho, nparts, n, nwg, z, p0, p1, st);
}


// y_d = sum_j Minv_B[d - s_B, j] r_{s_B + j} for the DoFs of this tile (whole blocks),
// given row d's inverse row m and its packed size and position in the block.
template <class M>
__device__ __forceinline__ double bj_row_at(int t, const double *tile, const M *__restrict__ m, int meta) {
    const int size = meta >> 8, loc = meta & 255;
    const double *rt = tile + (t - loc);
    double s = 0.0;
    for (int j0 = 0; j0 < size; j0 += 6) {  // six entries' loads issued together, added in order
        double v[6];
#pragma unroll
        for (int u = 0; u < 6; ++u) v[u] = j0 + u < size ? (double)m[j0 + u] : 0.0;
#pragma unroll
        for (int u = 0; u < 6; ++u)
            if (j0 + u < size) s = fma(v[u], rt[j0 + u], s);
    }
    return s;
}

// sum_e z_val[e] delta[z_col[e]] over e in [e0, e1) in index order, four entries per step
// with their column, value and delta loads issued together (clamped as above).
__device__ __forceinline__ double z_row_dot(int e0, int e1, const int32_t *__restrict__ z_col,
                                            const double *__restrict__ z_val, const double *__restrict__ delta) {
    double c = 0.0;
    for (int e = e0; e < e1; e += 4) {
        const int i1 = min(e + 1, e1 - 1), i2 = min(e + 2, e1 - 1), i3 = min(e + 3, e1 - 1);
        const int32_t c0 = z_col[e], c1 = z_col[i1], c2 = z_col[i2], c3 = z_col[i3];
        const double v0 = z_val[e], v1 = z_val[i1], v2 = z_val[i2], v3 = z_val[i3];
        const double d0 = delta[c0], d1 = delta[c1], d2 = delta[c2], d3 = delta[c3];
        c = fma(v0, d0, c);
        if (e + 1 < e1) c = fma(v1, d1, c);
        if (e + 2 < e1) c = fma(v2, d2, c);
        if (e + 3 < e1) c = fma(v3, d3, c);
    }
    return c;
}

template <class M>
__device__ __forceinline__ double bj_row(int t, int64_t d, const double *tile, const M *__restrict__ minv,
                                         const int32_t *__restrict__ bj_rowoff,
                                         const int32_t *__restrict__ bj_meta) {
    return bj_row_at(t, tile, minv + bj_rowoff[d], bj_meta[d]);
}

// Step length, solution and residual updates of Algorithm 1 with the residual norm
// partials, then the block-Jacobi apply y = M^{-1} r that opens Algorithm 3.
template <class M>
__device__ __forceinline__ void k_update_bj_body(int vb, 
    int32_t ntiles, int32_t nwg, const int32_t *__restrict__ tile_start, double *__restrict__ u,
    double *__restrict__ r, double *__restrict__ y, const double *__restrict__ q, const double *p0,
    const double *p1, const M *__restrict__ minv, const int32_t *__restrict__ bj_rowoff,
    const int32_t *__restrict__ bj_meta, double *__restrict__ part_rr, double *__restrict__ part_ry,
    const double *__restrict__ part_pq2, State *st) {
    __shared__ double lds[2 * (kThreads / 64)];
    __shared__ double tile[kThreads];
    const int t = threadIdx.x;
    const int w = xcd_remap(vb, nwg);
    int t0, t1;
    if ((uint64_t)ntiles * (uint64_t)nwg < (1ull << 32)) {  // 32-bit quotients when they fit
        t0 = (int)(((uint32_t)w * (uint32_t)ntiles) / (uint32_t)nwg);
        t1 = (int)(((uint32_t)(w + 1) * (uint32_t)ntiles) / (uint32_t)nwg);
    } else {
        t0 = (int)(((int64_t)w * ntiles) / nwg);
        t1 = (int)(((int64_t)(w + 1) * ntiles) / nwg);
    }
    // the first tile's bounds are loaded before the state, so the two round trips overlap
    int64_t b0 = 0, b1 = 0;
    if (t0 < t1) {
        b0 = tile_start[t0];
        b1 = tile_start[t0 + 1];
    }
    if (st->flag != kRunning) return;
    // alpha_i = rho_i / p_i^T q_i: every wave adds the kAlphaParts first-stage sums with the
    // same butterfly, so all workgroups hold the same bits; a breakdown is seen by all
    const double pq = wave_sum((threadIdx.x & 63) < kAlphaParts ? part_pq2[threadIdx.x & 63] : 0.0);
    const double alpha = st->rho[st->iter & 1] / pq;
    if (!(pq > 0.0) || !isfinite(pq) || !isfinite(alpha)) {
        if (vb == 0 && threadIdx.x == 0) {
            st->flag = kBreakdown;
            st->bad = st->iter;
            st->iters_done = st->iter;
        }
        return;
    }
    const double *p = (st->iter & 1) ? p1 : p0;
    double acc = 0.0, accy = 0.0;
    for (int tt = t0; tt < t1; ++tt) {
        if (tt > t0) {
            b0 = tile_start[tt];
            b1 = tile_start[tt + 1];
        }
        const int64_t d0 = b0, d1 = b1;
        const int64_t d = d0 + t;
        double rn = 0.0;
        int meta = 0, roff = 0;  // loaded with the vectors, ahead of the barrier
        __syncthreads();
        if (d < d1) {
            meta = bj_meta[d];
            roff = bj_rowoff[d];
            u[d] = fma(alpha, p[d], u[d]);
            rn = fma(-alpha, q[d], r[d]);
            r[d] = rn;
            tile[t] = rn;
            acc = fma(rn, rn, acc);
        }
        __syncthreads();
        if (d < d1) {
            const double yd = bj_row_at(t, tile, minv + roff, meta);
            y[d] = yd;
            accy = fma(rn, yd, accy);
        }
    }
    if (part_ry) {  // r^T y partials: rho = r^T z is formed from them in the prolongation
        block_sum2_n<kThreads / 64>(acc, accy, lds);
        if (threadIdx.x == 0) {
            part_rr[vb] = acc;
            part_ry[vb] = accy;
        }
    } else {
        const double s = block_sum(acc, lds);
        if (threadIdx.x == 0) part_rr[vb] = s;
    }
}

template <class M>
__global__ __launch_bounds__(kThreads) void k_update_bj(
    int32_t ntiles, int32_t nwg, const int32_t *__restrict__ tile_start, double *__restrict__ u,
    double *__restrict__ r, double *__restrict__ y, const double *__restrict__ q, const double *p0,
    const double *p1, const M *__restrict__ minv, const int32_t *__restrict__ bj_rowoff,
    const int32_t *__restrict__ bj_meta, double *__restrict__ part_rr, double *__restrict__ part_ry,
    const double *__restrict__ part_pq2, State *st) {
    k_update_bj_body<M>(blockIdx.x, ntiles, nwg, tile_start, u, r, y, q, p0, p1, minv, bj_rowoff, bj_meta, part_rr,
                        part_ry, part_pq2, st);
}


// y = M^{-1} r only.
template <class M>
__device__ __forceinline__ void k_bj_body(int vb, int32_t ntiles, int32_t nwg, const int32_t *__restrict__ tile_start,
                                                 const double *__restrict__ r, double *__restrict__ y,
                                                 const M *__restrict__ minv,
                                                 const int32_t *__restrict__ bj_rowoff,
                                                 const int32_t *__restrict__ bj_meta, const State *st) {
    __shared__ double tile[kThreads];
    if (st && st->flag != kRunning) return;
    const int t = threadIdx.x;
    const int w = xcd_remap(vb, nwg);
    const int t0 = (int)(((int64_t)w * ntiles) / nwg), t1 = (int)(((int64_t)(w + 1) * ntiles) / nwg);
    for (int tt = t0; tt < t1; ++tt) {
        const int64_t d0 = tile_start[tt], d1 = tile_start[tt + 1];
        const int64_t d = d0 + t;
        __syncthreads();
        if (d < d1) tile[t] = r[d];
        __syncthreads();
        if (d < d1) y[d] = bj_row(t, d, tile, minv, bj_rowoff, bj_meta);
    }
}

template <class M>
__global__ __launch_bounds__(kThreads) void k_bj(int32_t ntiles, int32_t nwg, const int32_t *__restrict__ tile_start,
                                                 const double *__restrict__ r, double *__restrict__ y,
                                                 const M *__restrict__ minv,
                                                 const int32_t *__restrict__ bj_rowoff,
                                                 const int32_t *__restrict__ bj_meta, const State *st) {
    k_bj_body<M>(blockIdx.x, ntiles, nwg, tile_start, r, y, minv, bj_rowoff, bj_meta, st);
}


// y_B = M_B^-1 r_B for the blocks of more than kMaxBlock DoFs (Algorithm 3's block
// solve with the explicit inverse of a subdomain-sized block).  A workgroup owns
// kDenseRows consecutive rows of one block: r_B is staged in LDS (zero from the
// block's size up to ld), each wave takes 8 rows and every lane reads 16-byte pieces of
// all 8 rows per step, so a wave keeps 8 row streams in flight.  The row sums are
// reduced across the wave in a fixed order.
template <class M> struct DensePiece;
template <> struct DensePiece<double> { static constexpr int W = 2; using T = double2; };
template <> struct DensePiece<float> { static constexpr int W = 4; using T = float4; };

__device__ __forceinline__ double piece_dot(const double2 &a, const double *x) {
    return fma(a.y, x[1], a.x * x[0]);
}
__device__ __forceinline__ double piece_dot(const float4 &a, const double *x) {
    return fma((double)a.w, x[3], fma((double)a.z, x[2], fma((double)a.y, x[1], (double)a.x * x[0])));
}

template <class M>
__global__ __launch_bounds__(kThreads) void k_bj_dense(const DenseBlk *__restrict__ blk,
                                                       const DenseChunk *__restrict__ chunk,
                                                       const double *__restrict__ r, double *__restrict__ y,
                                                       const M *__restrict__ dinv, const State *st) {
    constexpr int W = DensePiece<M>::W;
    constexpr int R = kDenseRows / 4;  // rows per wave
    using T = typename DensePiece<M>::T;
    extern __shared__ double rb[];  // ld of the largest dense block
    if (st && st->flag != kRunning) return;
    const DenseChunk ch = chunk[xcd_remap(blockIdx.x, gridDim.x)];
    const DenseBlk B = blk[ch.dense];
    for (int j = threadIdx.x; j < B.ld; j += kThreads) rb[j] = j < B.size ? r[B.start + j] : 0.0;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i0 = ch.row0 + wave * R;
    const int nr = min(R, B.size - i0);
    if (nr <= 0) return;
    const M *base = dinv + B.off + (int64_t)i0 * B.ld;
    double acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = 0.0;
    for (int j = W * lane; j < B.ld; j += 64 * W) {
        T v[R];
#pragma unroll
        for (int q = 0; q < R; ++q)
            if (q < nr) v[q] = *reinterpret_cast<const T *>(base + (int64_t)q * B.ld + j);
#pragma unroll
        for (int q = 0; q < R; ++q)
            if (q < nr) acc[q] += piece_dot(v[q], rb + j);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        double a = acc[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
        if (lane == 0 && q < nr) y[B.start + i0 + q] = a;
    }
}

// Convergence test (workgroup 0 only) and g_j = Z^T a - (K Z)^T b, one column per
// workgroup of kRestrictThreads threads; each thread takes every T-th entry of the
// column's two lists, kRestrictDepth entries (index, value, then the gathered vector
// entry) at a time, so that one or two rounds of dependent loads cover a column.  h (when
// given) receives Z^T a and workgroup 0 also sums the r^T y partials into st->ry; advance
// (iteration launches whose iterate continues) moves the state to the next iteration
// after the test.
constexpr int kRestrictWaves = 8;
constexpr int kRestrictThreads = 64 * kRestrictWaves;
constexpr int kRestrictDepth = 8;  // entries per thread whose loads are in flight together
static_assert(kRestrictThreads * kRestrictDepth == kRestrictRound, "restriction round");

__device__ __forceinline__ void k_restrict_body(int vb, int vg,
    int32_t k, const int32_t *__restrict__ zt_ptr, const int32_t *__restrict__ zt_idx,
    const double *__restrict__ zt_val, const int32_t *__restrict__ kzt_ptr, const int32_t *__restrict__ kzt_idx,
    const double *__restrict__ kzt_val, const double *__restrict__ a, const double *__restrict__ b,
    double *__restrict__ g, double *__restrict__ h, State *st, const double *__restrict__ part_rr,
    const double *__restrict__ part_ry, int n_rr, int iter_offset, int max_iter, double *__restrict__ hist,
    int advance, const int32_t *__restrict__ order = nullptr) {
    __shared__ double lds[2 * kRestrictWaves];
    if (st) {
        if (wg_flag(st) != kRunning) return;
        if (vb == 0 && n_rr > 0) {
            double rr = strided_share<kRestrictThreads, 8>(part_rr, n_rr);
            double ry = part_ry ? strided_share<kRestrictThreads, 8>(part_ry, n_rr) : 0.0;
            block_sum2_n<kRestrictWaves>(rr, ry, lds);
            if (threadIdx.x == 0) {
                const int done = st->iter + iter_offset;
                st->rr = rr;
                st->ry = ry;
                const double rn = sqrt(rr);
                if (hist) hist[done] = rn;
                if (!isfinite(rr)) {
                    st->flag = kBreakdown;
                    st->bad = st->iter;
                    st->iters_done = done;
                } else if (rn <= st->thr) {
                    st->flag = kConverged;
                    st->iters_done = done;
                } else if (done >= max_iter) {
                    st->flag = kMaxIter;
                    st->iters_done = done;
                } else if (advance) {
                    st->iter = st->iter + 1;
                }
            }
        }
    }
    constexpr int T = kRestrictThreads;
    for (int jj = xcd_remap(vb, vg); jj < k; jj += vg) {
        const int j = order ? order[jj] : jj;  // columns with more rounds of loads first (a
                                               // shorter tail); each column's sum is unchanged
        // the column's Z^T entries, then its (K Z)^T entries (when b is given), as one list:
        // each thread loads kRestrictDepth entries and their gathers at a time
        const int zb = zt_ptr[j], nz = zt_ptr[j + 1] - zb;
        const int kb0 = b ? kzt_ptr[j] : 0, nt = nz + (b ? kzt_ptr[j + 1] - kb0 : 0);
        double za = 0.0, kb = 0.0;  // Z^T a and -(K Z)^T b
        for (int e0 = threadIdx.x; e0 < nt; e0 += kRestrictDepth * T) {
            int32_t idx[kRestrictDepth];
            double v[kRestrictDepth], x[kRestrictDepth];
            // one load of each kind per entry: the lane picks the list (and vector) by address
#pragma unroll
            for (int u = 0; u < kRestrictDepth; ++u) {
                const int e = e0 + u * T;
                const bool inz = e < nz;
                const int o = inz ? zb + e : kb0 + e - nz;
                const int32_t *ip = inz ? zt_idx : kzt_idx;
                const double *vp = inz ? zt_val : kzt_val;
                idx[u] = 0;
                v[u] = 0.0;
                if (e < nt) {
                    idx[u] = ip[o];
                    v[u] = vp[o];
                }
            }
#pragma unroll
            for (int u = 0; u < kRestrictDepth; ++u) {
                const int e = e0 + u * T;
                const double *xp = e < nz ? a : b;
                x[u] = e < nt ? xp[idx[u]] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kRestrictDepth; ++u) {
                const bool inz = e0 + u * T < nz;
                za = fma(inz ? v[u] : 0.0, x[u], za);
                kb = fma(inz ? 0.0 : -v[u], x[u], kb);
            }
        }
        block_sum2_n<kRestrictWaves>(za, kb, lds);
        if (threadIdx.x == 0) {
            g[j] = za + kb;
            if (h) h[j] = za;
        }
    }
}

__global__ __launch_bounds__(kRestrictThreads) void k_restrict(
    int32_t k, const int32_t *__restrict__ zt_ptr, const int32_t *__restrict__ zt_idx,
    const double *__restrict__ zt_val, const int32_t *__restrict__ kzt_ptr, const int32_t *__restrict__ kzt_idx,
    const double *__restrict__ kzt_val, const double *__restrict__ a, const double *__restrict__ b,
    double *__restrict__ g, State *st, const double *__restrict__ part_rr, int n_rr, int iter_offset,
    int max_iter, double *__restrict__ hist, double *__restrict__ h, const double *__restrict__ part_ry,
    int advance, const int32_t *__restrict__ order) {
    k_restrict_body(blockIdx.x, gridDim.x, k, zt_ptr, zt_idx, zt_val, kzt_ptr, kzt_idx, kzt_val, a, b, g, h, st,
                    part_rr, part_ry, n_rr, iter_offset, max_iter, hist, advance, order);
}


// The coarse product delta = E^-1 g on the stored lower triangle of the symmetric E^-1
// (kCoarseTile^2 tiles, tile row X = entries X T .. X T + T - 1), in two launches.
// Stage 1, one workgroup per stored tile (I, J): the tile's rows against g_J are the
// contribution of the tile pair (I, J) to delta_I, and for I > J its columns against
// g_I are the contribution of the mirrored tile (J, I) to delta_J; each goes to
// cpart[(X nt + Y) T ..] for its pair (X, Y).  Every stored value is read once.
// Stage 2, one workgroup per tile row X: delta_X = sum over Y = 0..nt-1 of the pair
// contributions in that order; with h given, also hdp[X] = sum of h_j delta_j over the
// row's entries (the fused prolongation forms rho = r^T y + h^T delta from them).
__device__ __forceinline__ void k_coarse_tiles_body(int vb, int32_t k, int32_t nt, const double *__restrict__ tiles,
                                                    const double *__restrict__ g, double *__restrict__ cpart,
                                                    const State *st) {
    constexpr int T = kCoarseTile;
    __shared__ double gi[T], gj[T];
    __shared__ double X[T][T + 1];
    __shared__ double part[2][4][T];
    if (st && st->flag != kRunning) return;
    const int64_t tid = vb;
    int I = (int)((sqrt(8.0 * (double)tid + 1.0) - 1.0) * 0.5);
    while ((int64_t)(I + 1) * (I + 2) / 2 <= tid) ++I;
    while ((int64_t)I * (I + 1) / 2 > tid) --I;
    const int J = (int)(tid - (int64_t)I * (I + 1) / 2);
    const double *__restrict__ A = tiles + tid * T * T;
    const int t = threadIdx.x, b = t & 63, rq = t >> 6;
    // the thread's column strip: rows 16 rq .. 16 rq + 15 of column b (each load
    // instruction of a wave reads one whole 512-byte tile row)
    double v[16];
#pragma unroll
    for (int a = 0; a < 16; ++a) v[a] = A[(16 * rq + a) * T + b];
    if (t < T) {
        gj[t] = J * T + t < k ? g[J * T + t] : 0.0;
        gi[t] = I * T + t < k ? g[I * T + t] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 16; ++a) X[16 * rq + a][b] = v[a] * gj[b];
    if (I != J) {
        double cs = 0.0;
#pragma unroll
        for (int a = 0; a < 16; ++a) cs = fma(v[a], gi[16 * rq + a], cs);
        part[1][rq][b] = cs;
    }
    __syncthreads();
    // row a = b of the tile, quarter rq of its columns
    {
        double rs = 0.0;
#pragma unroll
        for (int i = 0; i < 16; ++i) rs += X[b][16 * rq + i];
        part[0][rq][b] = rs;
    }
    __syncthreads();
    if (t < T) {
        cpart[((int64_t)I * nt + J) * T + t] = (part[0][0][t] + part[0][1][t]) + (part[0][2][t] + part[0][3][t]);
        if (I != J)
            cpart[((int64_t)J * nt + I) * T + t] =
                (part[1][0][t] + part[1][1][t]) + (part[1][2][t] + part[1][3][t]);
    }
}

__device__ __forceinline__ void k_coarse_sum_body(int vb, int32_t k, int32_t nt, const double *__restrict__ cpart,
                                                  double *__restrict__ delta, const double *__restrict__ h,
                                                  double *__restrict__ hdp, const State *st) {
    constexpr int T = kCoarseTile;
    __shared__ double ps[4][T];
    if (st && st->flag != kRunning) return;
    const int Xr = vb;
    const int a = threadIdx.x & 63, yq = threadIdx.x >> 6;
    const int y0 = (nt * yq) / 4, y1 = (nt * (yq + 1)) / 4;
    const double *__restrict__ src = cpart + (int64_t)Xr * nt * T + a;
    double s = 0.0;
    int y = y0;
    for (; y + 5 < y1; y += 6) {  // six loads in flight, added in order
        double v[6];
#pragma unroll
        for (int u = 0; u < 6; ++u) v[u] = src[(int64_t)(y + u) * T];
#pragma unroll
        for (int u = 0; u < 6; ++u) s += v[u];
    }
    for (; y < y1; ++y) s += src[(int64_t)y * T];
    ps[yq][a] = s;
    __syncthreads();
    if (threadIdx.x < T) {  // wave 0
        const double dv = (ps[0][a] + ps[1][a]) + (ps[2][a] + ps[3][a]);
        const int row = Xr * T + a;
        double hv = 0.0;
        if (row < k) {
            delta[row] = dv;
            if (h) hv = h[row] * dv;
        }
        if (h) {
            hv = wave_sum(hv);
            if (a == 0) hdp[Xr] = hv;
        }
    }
}

__global__ __launch_bounds__(256) void k_coarse_tiles(int32_t k, int32_t nt, const double *__restrict__ tiles,
                                                      const double *__restrict__ g, double *__restrict__ cpart,
                                                      const State *st) {
    k_coarse_tiles_body(blockIdx.x, k, nt, tiles, g, cpart, st);
}

__global__ __launch_bounds__(256) void k_coarse_sum(int32_t k, int32_t nt, const double *__restrict__ cpart,
                                                    double *__restrict__ delta, const double *__restrict__ h,
                                                    double *__restrict__ hdp, const State *st) {
    k_coarse_sum_body(blockIdx.x, k, nt, cpart, delta, h, hdp, st);
}

// out = base + Z delta; optional partials of rdot^T out; optionally advance the iteration.
__device__ __forceinline__ void k_prolong_body(int vb, int64_t n, int32_t nwg, const int32_t *__restrict__ z_ptr,
                                                      const int32_t *__restrict__ z_col,
                                                      const double *__restrict__ z_val,
                                                      const double *__restrict__ delta,
                                                      const double *base, double *out,
                                                      const double *__restrict__ rdot, double *__restrict__ part,
                                                      State *st, int advance) {
    __shared__ double lds[4];
    if (st && st->flag != kRunning) return;
    const int w = xcd_remap(vb, nwg);
    const int64_t per = (n + nwg - 1) / nwg;
    const int64_t d0 = (int64_t)w * per, d1 = min(n, d0 + per);
    double acc = 0.0;
    for (int64_t d = d0 + threadIdx.x; d < d1; d += kThreads) {
        double s = base ? base[d] : 0.0;
        const double c = z_row_dot(z_ptr[d], z_ptr[d + 1], z_col, z_val, delta);
        s += c;
        out[d] = s;
        if (rdot) acc = fma(rdot[d], s, acc);
    }
    if (rdot) {
        const double t = block_sum(acc, lds);
        if (threadIdx.x == 0) part[vb] = t;
    }
    if (advance && (vb == 0 && threadIdx.x == 0)) st->iter = st->iter + 1;
}

__global__ __launch_bounds__(kThreads) void k_prolong(int64_t n, int32_t nwg, const int32_t *__restrict__ z_ptr,
                                                      const int32_t *__restrict__ z_col,
                                                      const double *__restrict__ z_val,
                                                      const double *__restrict__ delta,
                                                      const double *base, double *out,
                                                      const double *__restrict__ rdot, double *__restrict__ part,
                                                      State *st, int advance) {
    k_prolong_body(blockIdx.x, n, nwg, z_ptr, z_col, z_val, delta, base, out, rdot, part, st, advance);
}


// The prolongation of Algorithm 3 fused with beta and the new search direction of
// Algorithm 1.  With h = Z^T r from the restriction, r^T z = r^T y + h^T delta exactly, so
// rho_i is r^T y (summed by the restriction) plus the fixed-order sum of the k entries
// (several systems per launch) or tile-row sums (single system) of h_j delta_j left by
// the coarse product: every workgroup forms the same bits of rho_i
// and of beta_{i-1} = rho_i / rho_{i-1} and writes p_i = y + Z delta + beta_{i-1} p_{i-1}
// into buffer i & 1 directly (z itself is never stored).  The restriction has already
// advanced the iteration.  Workgroup 0 stores rho_i in slot i & 1 and tests it.
__device__ __forceinline__ void k_prolong_p_body(int vb, int64_t n, int32_t nwg, const int32_t *__restrict__ z_ptr,
                                                 const int32_t *__restrict__ z_col, const double *__restrict__ z_val,
                                                 const double *__restrict__ delta, const double *__restrict__ y,
                                                 const double *__restrict__ hparts, int32_t nhp, double *p0,
                                                 double *p1, State *st) {
    __shared__ double lds[4];
    if (wg_flag(st) != kRunning) return;
    const int it = st->iter;
    double *__restrict__ pc = (it & 1) ? p1 : p0;
    const double *__restrict__ pp = (it & 1) ? p0 : p1;
    const int w = xcd_remap(vb, nwg);
    const int64_t per = (n + nwg - 1) / nwg;
    const int64_t d1 = min(n, (int64_t)(w + 1) * per);
    // the thread's first two rows (the grid gives each thread two or more), y + Z delta and the
    // old p, before beta is known: these loads overlap the reduction below
    int64_t d = (int64_t)w * per + threadIdx.x;
    const int64_t d2 = d + kThreads;
    double v = 0.0, pold = 0.0, v2 = 0.0, pold2 = 0.0;
    if (d < d1) {
        const double c = z_row_dot(z_ptr[d], z_ptr[d + 1], z_col, z_val, delta);
        v = y[d] + c;
        pold = pp[d];
    }
    if (d2 < d1) {
        const double c = z_row_dot(z_ptr[d2], z_ptr[d2 + 1], z_col, z_val, delta);
        v2 = y[d2] + c;
        pold2 = pp[d2];
    }
    const double rho = st->ry + block_sum(strided_share<kThreads, 8>(hparts, nhp), lds);
    const bool bad = !isfinite(rho);
    const double beta = rho / st->rho[(it + 1) & 1];
    if (vb == 0 && threadIdx.x == 0) {
        if (bad) {
            st->flag = kBreakdown;
            st->bad = it - 1;
            st->iters_done = it;
        } else {
            st->beta = beta;
            st->rho[it & 1] = rho;
        }
    }
    if (bad) return;
    if (d < d1) pc[d] = fma(beta, pold, v);
    if (d2 < d1) pc[d2] = fma(beta, pold2, v2);
    for (d += 2 * kThreads; d < d1; d += kThreads) {
        const double c = z_row_dot(z_ptr[d], z_ptr[d + 1], z_col, z_val, delta);
        pc[d] = fma(beta, pp[d], y[d] + c);
    }
}

__global__ __launch_bounds__(kThreads) void k_prolong_p(int64_t n, int32_t nwg, const int32_t *__restrict__ z_ptr,
                                                        const int32_t *__restrict__ z_col,
                                                        const double *__restrict__ z_val,
                                                        const double *__restrict__ delta,
                                                        const double *__restrict__ y,
                                                        const double *__restrict__ hparts, int32_t nhp, double *p0,
                                                        double *p1, State *st) {
    k_prolong_p_body(blockIdx.x, n, nwg, z_ptr, z_col, z_val, delta, y, hparts, nhp, p0, p1, st);
}

// ||a||^2 partials and a count of non-finite entries of a and b (b may be null).
__global__ __launch_bounds__(kThreads) void k_norm_finite(int64_t n, int32_t nwg, const double *__restrict__ a,
                                                          const double *__restrict__ b, double *__restrict__ part_sq,
                                                          double *__restrict__ part_bad) {
    __shared__ double lds[4];
    const int64_t per = (n + nwg - 1) / nwg;
    const int64_t d0 = (int64_t)blockIdx.x * per, d1 = min(n, d0 + per);
    double acc = 0.0, bad = 0.0;
    for (int64_t d = d0 + threadIdx.x; d < d1; d += kThreads) {
        const double v = a[d];
        if (!isfinite(v)) bad += 1.0;
        acc = fma(v, v, acc);
        if (b && !isfinite(b[d])) bad += 1.0;
    }
    const double s = block_sum(acc, lds);
    const double c = block_sum(bad, lds);
    if (threadIdx.x == 0) {
        part_sq[blockIdx.x] = s;
        part_bad[blockIdx.x] = c;
    }
}

// st->aux = sum of n partials of part_a; st->nonfinite = (sum of part_b > 0) when part_b given.
__global__ __launch_bounds__(kThreads) void k_reduce_aux(const double *__restrict__ part_a,
                                                         const double *__restrict__ part_b, int n, State *st) {
    __shared__ double lds[4];
    const double s = reduce_parts(part_a, n, lds);
    const double c = part_b ? reduce_parts(part_b, n, lds) : 0.0;
    if (threadIdx.x == 0) {
        st->aux = s;
        st->nonfinite = c > 0.0 ? 1 : 0;
    }
}

template <int G>
hipError_t spmv_p_g(const dpcg_ctx *c, Workspace &w, hipEvent_t ev0, hipEvent_t ev1) {
    SpmvShape sh{c->nb, c->spmv.steps, c->spmv.nwg};
    // the events (when given) take the kernel's own start and end timestamps; block
    // columns as 16-bit row offsets when the handle has them
    const int16_t *b16 = c->bcol16;
    if (c->inner32 && b16)
        hipExtLaunchKernelGGL((k_spmv_p<G, float, int16_t>), dim3(c->spmv.nwg), dim3(kSpmvThreads), 0, c->stream, ev0,
                              ev1, 0, sh, c->brow_ptr, b16, (const float *)c->bval32, c->nnzb,
                              (const double *)w.p[0], (const double *)w.p[1], w.q, w.part_a, (const State *)w.st);
    else if (c->inner32)
        hipExtLaunchKernelGGL((k_spmv_p<G, float, int32_t>), dim3(c->spmv.nwg), dim3(kSpmvThreads), 0, c->stream, ev0,
                              ev1, 0, sh, c->brow_ptr, (const int32_t *)c->bcol, (const float *)c->bval32, c->nnzb,
                              (const double *)w.p[0], (const double *)w.p[1], w.q, w.part_a, (const State *)w.st);
    else if (b16)
        hipExtLaunchKernelGGL((k_spmv_p<G, double, int16_t>), dim3(c->spmv.nwg), dim3(kSpmvThreads), 0, c->stream,
                              ev0, ev1, 0, sh, c->brow_ptr, b16, (const double *)c->bval, c->nnzb,
                              (const double *)w.p[0], (const double *)w.p[1], w.q, w.part_a, (const State *)w.st);
    else
        hipExtLaunchKernelGGL((k_spmv_p<G, double, int32_t>), dim3(c->spmv.nwg), dim3(kSpmvThreads), 0, c->stream,
                              ev0, ev1, 0, sh, c->brow_ptr, (const int32_t *)c->bcol, (const double *)c->bval,
                              c->nnzb, (const double *)w.p[0], (const double *)w.p[1], w.q, w.part_a,
                              (const State *)w.st);
    return hipGetLastError();
}

template <int G, int MODE>
hipError_t spmv_g(const dpcg_ctx *c, const double *x, const double *f, double *y, double *part) {
    SpmvShape sh{c->nb, c->spmv.steps, c->spmv.nwg};
    if (c->inner32)
        hipLaunchKernelGGL((k_spmv<G, MODE, float>), dim3(c->spmv.nwg), dim3(kSpmvThreads), 0, c->stream, sh,
                           c->brow_ptr, c->bcol, (const float *)c->bval32, c->nnzb, x, f, y, part);
    else
        hipLaunchKernelGGL((k_spmv<G, MODE, double>), dim3(c->spmv.nwg), dim3(kSpmvThreads), 0, c->stream, sh,
                           c->brow_ptr, c->bcol, (const double *)c->bval, c->nnzb, x, f, y, part);
    return hipGetLastError();
}

__global__ void k_to_f32(const double *__restrict__ src, int64_t count, float *__restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

__global__ void k_add(int64_t n, const double *__restrict__ x, double *__restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += x[i];
}

// ---------------------------------------------------------------- several systems per launch
// Each phase of an iteration of several independent systems runs as one launch whose
// workgroups are the systems' own, concatenated: a workgroup finds its system and its
// index within that system in the phase's offset table (each system's count is a
// multiple of 8 where the kernel remaps workgroups over the XCDs, so the mapping holds), and
// then runs the single-system body on that system's operator, vectors and state.
__device__ __forceinline__ int ms_find(const MsTable *__restrict__ tab, int phase, int bid) {
    int lo = 0, hi = tab->nsys;  // last s with off[phase][s] <= bid
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tab->off[phase][mid] <= bid) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <int MODE>
__global__ __launch_bounds__(kSpmvThreads) void k_ms_spmv(const MsTable *__restrict__ tab,
                                                          const MsSys *__restrict__ sys) {
    const int s = ms_find(tab, kMsSpmv, blockIdx.x);
    const MsSys &S = sys[s];
    const int vb = blockIdx.x - tab->off[kMsSpmv][s];
    const SpmvShape sh{S.nb, S.steps, S.spmv_nwg};
    if (MODE == 0) {
        switch (S.group) {
            case 4: k_spmv_p_body<4, double>(vb, sh, S.brow_ptr, S.bcol, S.bval, S.nnzb, S.p0, S.p1, S.q, S.part_a, S.st); break;
            case 8: k_spmv_p_body<8, double>(vb, sh, S.brow_ptr, S.bcol, S.bval, S.nnzb, S.p0, S.p1, S.q, S.part_a, S.st); break;
            case 16: k_spmv_p_body<16, double>(vb, sh, S.brow_ptr, S.bcol, S.bval, S.nnzb, S.p0, S.p1, S.q, S.part_a, S.st); break;
            default: k_spmv_p_body<32, double>(vb, sh, S.brow_ptr, S.bcol, S.bval, S.nnzb, S.p0, S.p1, S.q, S.part_a, S.st); break;
        }
    } else {
        if (S.st->flag != kRunning) return;
        switch (S.group) {
            case 4: k_spmv_body<4, 1, double>(vb, sh, S.brow_ptr, S.bcol, S.bval, S.nnzb, S.u, S.f, S.r, S.part_b); break;
            case 8: k_spmv_body<8, 1, double>(vb, sh, S.brow_ptr, S.bcol, S.bval, S.nnzb, S.u, S.f, S.r, S.part_b); break;
            case 16: k_spmv_body<16, 1, double>(vb, sh, S.brow_ptr, S.bcol, S.bval, S.nnzb, S.u, S.f, S.r, S.part_b); break;
            default: k_spmv_body<32, 1, double>(vb, sh, S.brow_ptr, S.bcol, S.bval, S.nnzb, S.u, S.f, S.r, S.part_b); break;
        }
    }
}

// first stage of p^T q for system blockIdx.x / kAlphaParts (as k_alpha)
__global__ __launch_bounds__(1024) void k_ms_alpha(const MsSys *__restrict__ sys) {
    const MsSys &S = sys[blockIdx.x / kAlphaParts];
    k_alpha_body(blockIdx.x % kAlphaParts, S.part_a, S.spmv_nwg, S.part_d, S.st);
}

__global__ __launch_bounds__(kThreads) void k_ms_update_bj(const MsTable *__restrict__ tab,
                                                           const MsSys *__restrict__ sys) {
    const int s = ms_find(tab, kMsBj, blockIdx.x);
    const MsSys &S = sys[s];
    k_update_bj_body<double>(blockIdx.x - tab->off[kMsBj][s], S.bj_ntiles, S.bj_nwg, S.bj_wg_start, S.u, S.r, S.y,
                             S.q, S.p0, S.p1, S.minv, S.bj_rowoff, S.bj_meta, S.part_b, S.part_c, S.part_d, S.st);
}

__global__ __launch_bounds__(kThreads) void k_ms_bj(const MsTable *__restrict__ tab, const MsSys *__restrict__ sys) {
    const int s = ms_find(tab, kMsBj, blockIdx.x);
    const MsSys &S = sys[s];
    k_bj_body<double>(blockIdx.x - tab->off[kMsBj][s], S.bj_ntiles, S.bj_nwg, S.bj_wg_start, S.r, S.y, S.minv,
                      S.bj_rowoff, S.bj_meta, S.st);
}

// mode 0: g = Z^T f - (KZ)^T u_{-1} (no state); mode 1: g = Z^T r - (KZ)^T y with the
// convergence test when check.
__global__ __launch_bounds__(kRestrictThreads) void k_ms_restrict(const MsTable *__restrict__ tab,
                                                                  const MsSys *__restrict__ sys, int mode, int check,
                                                                  int iter_offset, int max_iter) {
    const int s = ms_find(tab, kMsRestrict, blockIdx.x);
    const MsSys &S = sys[s];
    const int vb = blockIdx.x - tab->off[kMsRestrict][s];
    const int vg = tab->off[kMsRestrict][s + 1] - tab->off[kMsRestrict][s];
    if (mode == 0) {
        if (S.st->flag != kRunning) return;
        k_restrict_body(vb, vg, S.k, S.zt_ptr, S.zt_idx, S.zt_val, S.kzt_ptr, S.kzt_idx, S.kzt_val, S.f,
                        S.guess ? S.u : nullptr, S.g, nullptr, nullptr, nullptr, nullptr, 0, 0, 0, nullptr, 0);
    } else {
        // iterations (iter_offset 1) take the fused prolongation: h = Z^T r and the advance
        k_restrict_body(vb, vg, S.k, S.zt_ptr, S.zt_idx, S.zt_val, S.kzt_ptr, S.kzt_idx, S.kzt_val, S.r, S.y, S.g,
                        iter_offset ? S.h : nullptr, S.st, S.part_b, iter_offset ? S.part_c : nullptr,
                        check ? (iter_offset ? S.bj_nwg : S.spmv_nwg) : 0, iter_offset, max_iter, nullptr,
                        iter_offset);
    }
}

// the coarse product's two stages (as launch_coarse); with_state 0: the start (no
// state), 1: with the state, 2: also the tile-row sums of h_j delta_j for the prolongation
__global__ __launch_bounds__(kThreads) void k_ms_coarse(const MsTable *__restrict__ tab, const MsSys *__restrict__ sys,
                                                        int with_state) {
    const int s = ms_find(tab, kMsCoarse, blockIdx.x);
    const MsSys &S = sys[s];
    if (!with_state && S.st->flag != kRunning) return;
    k_coarse_tiles_body(blockIdx.x - tab->off[kMsCoarse][s], S.k, S.coarse_nt, S.einv_tiles, S.g, S.cpart,
                        with_state ? S.st : nullptr);
}

__global__ __launch_bounds__(kThreads) void k_ms_coarse_sum(const MsTable *__restrict__ tab,
                                                            const MsSys *__restrict__ sys, int with_state) {
    const int s = ms_find(tab, kMsCoarseSum, blockIdx.x);
    const MsSys &S = sys[s];
    if (!with_state && S.st->flag != kRunning) return;
    k_coarse_sum_body(blockIdx.x - tab->off[kMsCoarseSum][s], S.k, S.coarse_nt, S.cpart, S.delta,
                      with_state == 2 ? S.h : nullptr, S.hdp, with_state ? S.st : nullptr);
}

// mode 0: u = u_{-1} + Z delta (no state); mode 1: z = y + Z delta with r^T z partials;
// mode 2: the fused prolongation, beta and search direction of an iteration
__global__ __launch_bounds__(kThreads) void k_ms_prolong(const MsTable *__restrict__ tab,
                                                         const MsSys *__restrict__ sys, int mode, int advance) {
    const int s = ms_find(tab, kMsVec, blockIdx.x);
    const MsSys &S = sys[s];
    const int vb = blockIdx.x - tab->off[kMsVec][s];
    if (mode == 0) {
        if (S.st->flag != kRunning) return;
        if (S.k > 0)
            k_prolong_body(vb, S.n, S.vec_nwg, S.z_ptr, S.z_col, S.z_val, S.delta, S.guess ? S.u : nullptr, S.u,
                           nullptr, nullptr, nullptr, 0);
        else if (!S.guess)
            k_prolong_body(vb, S.n, S.vec_nwg, S.z_ptr, S.z_col, S.z_val, S.delta, nullptr, S.u, nullptr, nullptr,
                           nullptr, 0);
    } else if (mode == 1) {
        k_prolong_body(vb, S.n, S.vec_nwg, S.z_ptr, S.z_col, S.z_val, S.delta, S.y, S.z, S.r, S.part_c, S.st,
                       advance);
    } else {
        k_prolong_p_body(vb, S.n, S.vec_nwg, S.z_ptr, S.z_col, S.z_val, S.delta, S.y, S.hdp, max(1, S.coarse_nt),
                         S.p0, S.p1, S.st);
    }
}

__global__ __launch_bounds__(kThreads) void k_ms_beta_p(const MsTable *__restrict__ tab,
                                                        const MsSys *__restrict__ sys) {
    const int s = ms_find(tab, kMsVec, blockIdx.x);
    const MsSys &S = sys[s];
    k_beta_p_body(blockIdx.x - tab->off[kMsVec][s], S.part_c, S.vec_nwg, S.n, S.vec_nwg, S.z, S.p0, S.p1, S.st);
}

}  // namespace

hipError_t launch_to_f32(const dpcg_ctx *c, const double *src, int64_t count, float *dst) {
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(8192, (count + kThreads - 1) / kThreads));
    hipLaunchKernelGGL(k_to_f32, dim3(grid), dim3(kThreads), 0, c->stream, src, count, dst);
    return hipGetLastError();
}

hipError_t launch_add(const dpcg_ctx *c, const double *x, double *y) {
    hipLaunchKernelGGL(k_add, dim3(c->vec_nwg), dim3(kThreads), 0, c->stream, c->n, x, y);
    return hipGetLastError();
}

hipError_t launch_spmv_p(const dpcg_ctx *c, Workspace &w, hipEvent_t ev0, hipEvent_t ev1) {
    switch (c->spmv.group) {
        case 4: return spmv_p_g<4>(c, w, ev0, ev1);
        case 8: return spmv_p_g<8>(c, w, ev0, ev1);
        case 32: return spmv_p_g<32>(c, w, ev0, ev1);
        default: return spmv_p_g<16>(c, w, ev0, ev1);
    }
}

hipError_t launch_spmv_plain(const dpcg_ctx *c, const double *x, double *y) {
    switch (c->spmv.group) {
        case 4: return spmv_g<4, 0>(c, x, nullptr, y, nullptr);
        case 8: return spmv_g<8, 0>(c, x, nullptr, y, nullptr);
        case 32: return spmv_g<32, 0>(c, x, nullptr, y, nullptr);
        default: return spmv_g<16, 0>(c, x, nullptr, y, nullptr);
    }
}

hipError_t launch_spmv_residual(const dpcg_ctx *c, const double *x, const double *f, double *r, double *part,
                                Workspace &w, int check) {
    (void)w;
    (void)check;
    switch (c->spmv.group) {
        case 4: return spmv_g<4, 1>(c, x, f, r, part);
        case 8: return spmv_g<8, 1>(c, x, f, r, part);
        case 32: return spmv_g<32, 1>(c, x, f, r, part);
        default: return spmv_g<16, 1>(c, x, f, r, part);
    }
}

hipError_t launch_update_bj(const dpcg_ctx *c, double *u, Workspace &w, bool fused) {
    hipLaunchKernelGGL(k_alpha, dim3(kAlphaParts), dim3(1024), 0, c->stream, (const double *)w.part_a, c->spmv.nwg,
                       w.part_d, (const State *)w.st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (c->inner32)
        hipLaunchKernelGGL(k_update_bj<float>, dim3(c->bj_nwg), dim3(kThreads), 0, c->stream, c->bj_ntiles,
                           c->bj_nwg, c->bj_wg_start, u, w.r, w.y, (const double *)w.q, (const double *)w.p[0],
                           (const double *)w.p[1], (const float *)c->minv32, c->bj_rowoff, c->bj_meta, w.part_b,
                           fused ? w.part_c : nullptr, (const double *)w.part_d, w.st);
    else
        hipLaunchKernelGGL(k_update_bj<double>, dim3(c->bj_nwg), dim3(kThreads), 0, c->stream, c->bj_ntiles,
                           c->bj_nwg, c->bj_wg_start, u, w.r, w.y, (const double *)w.q, (const double *)w.p[0],
                           (const double *)w.p[1], (const double *)c->minv, c->bj_rowoff, c->bj_meta, w.part_b,
                           fused ? w.part_c : nullptr, (const double *)w.part_d, w.st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_bj_dense(c, w.r, w.y, w.st);
}

hipError_t launch_beta(const dpcg_ctx *c, Workspace &w) {
    hipLaunchKernelGGL(k_beta_p, dim3(c->vec_nwg), dim3(kThreads), 0, c->stream, w.part_c, c->vec_nwg, c->n,
                       c->vec_nwg, w.z, w.p[0], w.p[1], w.st);
    return hipGetLastError();
}

hipError_t launch_bj(const dpcg_ctx *c, const double *r, double *y, Workspace *w) {
    const State *st = w ? w->st : nullptr;
    if (c->inner32)
        hipLaunchKernelGGL(k_bj<float>, dim3(c->bj_nwg), dim3(kThreads), 0, c->stream, c->bj_ntiles, c->bj_nwg,
                           c->bj_wg_start, r, y, (const float *)c->minv32, c->bj_rowoff, c->bj_meta, st);
    else
        hipLaunchKernelGGL(k_bj<double>, dim3(c->bj_nwg), dim3(kThreads), 0, c->stream, c->bj_ntiles, c->bj_nwg,
                           c->bj_wg_start, r, y, (const double *)c->minv, c->bj_rowoff, c->bj_meta, st);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_bj_dense(c, r, y, st);
}

// the dense blocks' part of y = M^-1 r, after the small blocks' kernel on the same stream
hipError_t launch_bj_dense(const dpcg_ctx *c, const double *r, double *y, const State *st) {
    if (c->ndense == 0) return hipSuccess;
    const size_t lds = sizeof(double) * (size_t)c->dense_maxld;
    if (c->inner32)
        hipLaunchKernelGGL(k_bj_dense<float>, dim3(c->ndchunks), dim3(kThreads), lds, c->stream, c->dense, c->dchunk,
                           r, y, (const float *)c->dinv32, st);
    else
        hipLaunchKernelGGL(k_bj_dense<double>, dim3(c->ndchunks), dim3(kThreads), lds, c->stream, c->dense, c->dchunk,
                           r, y, (const double *)c->dinv, st);
    return hipGetLastError();
}

hipError_t launch_restrict(const dpcg_ctx *c, const double *a, const double *b, double *g, Workspace *w,
                           int check, int n_parts, int iter_offset, int max_iter, int record, bool fused) {
    // a multiple of 8 workgroups, so that the XCD-aware column mapping applies
    const int grid = c->k >= 8 ? (c->k + 7) & ~7 : std::max(1, c->k);
    hipLaunchKernelGGL(k_restrict, dim3(grid), dim3(kRestrictThreads), 0, c->stream, c->k, c->zt_ptr, c->zt_idx,
                       c->zt_val, c->kzt_ptr, c->kzt_idx, c->kzt_val, a, b, g, w ? w->st : nullptr,
                       w ? w->part_b : nullptr, check ? n_parts : 0, iter_offset, max_iter,
                       (w && record) ? w->hist : nullptr, fused ? w->h : nullptr, fused ? w->part_c : nullptr,
                       fused ? 1 : 0, (const int32_t *)c->rs_order);
    return hipGetLastError();
}

hipError_t launch_coarse(const dpcg_ctx *c, const double *g, double *delta, const State *st, double *cpart,
                         const double *h, double *hdp) {
    if (c->k == 0) return hipSuccess;
    const int nt = c->coarse_nt;
    hipLaunchKernelGGL(k_coarse_tiles, dim3((unsigned)coarse_tile_count(nt)), dim3(256), 0, c->stream, c->k, nt,
                       (const double *)c->einv_tiles, g, cpart, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_coarse_sum, dim3(nt), dim3(256), 0, c->stream, c->k, nt, (const double *)cpart, delta, h, hdp,
                       st);
    return hipGetLastError();
}

hipError_t launch_prolong(const dpcg_ctx *c, const double *base, const double *delta, double *out,
                          Workspace *w, const double *rdot, int advance) {
    hipLaunchKernelGGL(k_prolong, dim3(c->vec_nwg), dim3(kThreads), 0, c->stream, c->n, c->vec_nwg, c->z_ptr,
                       c->z_col, c->z_val, delta, base, out, rdot, w ? w->part_c : nullptr,
                       w ? w->st : nullptr, advance);
    return hipGetLastError();
}

hipError_t launch_prolong_p(const dpcg_ctx *c, Workspace &w) {
    hipLaunchKernelGGL(k_prolong_p, dim3(c->prolong_nwg), dim3(kThreads), 0, c->stream, c->n, c->prolong_nwg,
                       c->z_ptr, c->z_col, c->z_val, w.delta, w.y, (const double *)w.hdp, std::max(1, c->coarse_nt),
                       w.p[0], w.p[1], w.st);
    return hipGetLastError();
}

hipError_t launch_check_finite_norm(const dpcg_ctx *c, const double *a, const double *b, Workspace &w) {
    hipLaunchKernelGGL(k_norm_finite, dim3(c->vec_nwg), dim3(kThreads), 0, c->stream, c->n, c->vec_nwg, a, b,
                       w.part_a, w.part_b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_aux, dim3(1), dim3(kThreads), 0, c->stream, w.part_a, w.part_b, c->vec_nwg,
                       w.st);
    return hipGetLastError();
}

hipError_t launch_ms_spmv_p(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid) {
    if (ngrid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ms_spmv<0>, dim3(ngrid), dim3(kSpmvThreads), 0, s, tab, sys);
    return hipGetLastError();
}

hipError_t launch_ms_spmv_res(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid) {
    if (ngrid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ms_spmv<1>, dim3(ngrid), dim3(kSpmvThreads), 0, s, tab, sys);
    return hipGetLastError();
}

hipError_t launch_ms_alpha(hipStream_t s, const MsSys *sys, int nsys) {
    hipLaunchKernelGGL(k_ms_alpha, dim3(nsys * kAlphaParts), dim3(1024), 0, s, sys);
    return hipGetLastError();
}

hipError_t launch_ms_update_bj(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid) {
    if (ngrid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ms_update_bj, dim3(ngrid), dim3(kThreads), 0, s, tab, sys);
    return hipGetLastError();
}

hipError_t launch_ms_bj(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid) {
    if (ngrid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ms_bj, dim3(ngrid), dim3(kThreads), 0, s, tab, sys);
    return hipGetLastError();
}

hipError_t launch_ms_restrict(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid, int mode, int check,
                              int iter_offset, int max_iter) {
    if (ngrid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ms_restrict, dim3(ngrid), dim3(kRestrictThreads), 0, s, tab, sys, mode, check, iter_offset,
                       max_iter);
    return hipGetLastError();
}

hipError_t launch_ms_coarse(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid, int with_state) {
    if (ngrid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ms_coarse, dim3(ngrid), dim3(kThreads), 0, s, tab, sys, with_state);
    return hipGetLastError();
}

hipError_t launch_ms_coarse_sum(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid, int with_state) {
    if (ngrid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ms_coarse_sum, dim3(ngrid), dim3(kThreads), 0, s, tab, sys, with_state);
    return hipGetLastError();
}

hipError_t launch_ms_prolong(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid, int mode, int advance) {
    if (ngrid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ms_prolong, dim3(ngrid), dim3(kThreads), 0, s, tab, sys, mode, advance);
    return hipGetLastError();
}

hipError_t launch_ms_beta(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid) {
    if (ngrid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ms_beta_p, dim3(ngrid), dim3(kThreads), 0, s, tab, sys);
    return hipGetLastError();
}

hipError_t launch_reduce_aux(const dpcg_ctx *c, Workspace &w, int n_parts) {
    hipLaunchKernelGGL(k_reduce_aux, dim3(1), dim3(kThreads), 0, c->stream, w.part_a, nullptr, n_parts, w.st);
    return hipGetLastError();
}

}  // namespace dpcg
