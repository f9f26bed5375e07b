// Multi-RHS solves: the method of dpcg_solve (Algorithm 1 started by Algorithm 2, with
// the A-DEF2 preconditioner of Algorithm 3 around block-Jacobi) run as up to 32
// independent recurrences whose vectors are the columns of n x 32 row-major arrays, so
// that every pass over K, Z, (KZ)^T, E^-1 and the block inverses serves all of them.
// A column whose residual test passes is frozen (its u and r no longer change) while
// the others continue, so each column follows the iterates of its own single solve.
// Lane j of every 32-lane group owns column j; row accesses are 256-byte contiguous.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "dpcg_internal.h"

namespace dpcg {
namespace {

constexpr int W = kBatchCols;

// The batch's "any column running" flag as seen by the whole workgroup (one read,
// broadcast through LDS): the restriction's workgroup 0 may change it meanwhile.
__device__ __forceinline__ int32_t wg_any(const BatchState *st) {
    __shared__ int32_t a;
    if (threadIdx.x == 0) a = st->any;
    __syncthreads();
    const int32_t v = a;
    __syncthreads();
    return v;
}

// Fixed-order column sums of nparts rows of part (row-major, W columns): partial sum h
// (h < 32) adds rows h, h + 32, ..., and the 32 partial sums are then added in order.  A
// workgroup of 32 NG threads computes partial sums h = g, g + NG, ... in lane group g,
// so the result does not depend on NG.  Valid in threads j < W.
// sum of x[i stride] over i in [i0, n) with step di, added in index order, eight loads
// issued before their additions
__device__ __forceinline__ double seq_sum(const double *__restrict__ x, int64_t stride, int i0, int n, int di) {
    double s = 0.0;
    int i = i0;
    for (; i + 7 * di < n; i += 8 * di) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = x[(int64_t)(i + u * di) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; i < n; i += di) s += x[(int64_t)i * stride];
    return s;
}

template <int NG>
__device__ __forceinline__ double col_reduce(const double *__restrict__ part, int nparts, double (*lds)[W + 1]) {
    const int j = threadIdx.x & 31, g = threadIdx.x >> 5;
    for (int h = g; h < 32; h += NG) lds[h][j] = seq_sum(part + j, W, h, nparts, 32);
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x < W)
        for (int h = 0; h < 32; ++h) t += lds[h][threadIdx.x];
    return t;
}

__device__ __forceinline__ double col_reduce_1024(const double *__restrict__ part, int nparts, double (*lds)[W + 1]) {
    return col_reduce<32>(part, nparts, lds);
}

// Same over the 8 groups of a 256-thread workgroup (values v of group g, lane j).
__device__ __forceinline__ double group_sum_8(double v, double (*lds)[W]) {
    const int j = threadIdx.x & 31, g = threadIdx.x >> 5;
    lds[g][j] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x < W)
        for (int h = 0; h < 8; ++h) t += lds[h][threadIdx.x];
    return t;
}

// MODE 0: y = K x and partials of x_j^T y_j (column-major: part[j * gridDim.x + wg]).
// MODE 1: y = f - K x and partials of ||y_j||^2 (row-major: part[wg * W + j]).
// One wave per slot of two consecutive block rows (2 s, 2 s + 1).  A row's values are
// contiguous (nine planes of m values), so they are staged through wave-private LDS with
// coalesced loads (lane l loads block l of every plane) together with the column
// indices, and read back as LDS broadcasts.  Lane (bg, cq) = (lane >> 3, lane & 7) takes
// every eighth entry starting at bg (kSpmmSteps at a time) and the four columns
// col4(cq, t): each 16-byte load of an x row by the eight lanes cq covers one whole
// 128-byte half of the 256-byte row.  When both rows of a slot have at most kPairMax
// blocks (a "pair", most of the matrix), the wave walks the merged list of their block
// columns (built once per workspace by k_pair_merge) and applies every gathered x row to
// each row that has a block there: consecutive rows share about two thirds of their
// columns, so a pair gathers about a third fewer x rows than its two rows one by one,
// and the gathers bound this kernel.  Longer rows with the same block columns ("twins":
// the block rows of one enriched node, about a fifth of the blocks) walk their common
// list in chunks of 64 blocks, each gathered x row serving both.  Other slots run their
// rows one after the other in chunks of 64 blocks.  The eight block groups of a row are added by a fixed shuffle
// tree, so every result is deterministic.
__device__ __forceinline__ int col4(int cq, int t) { return (t >> 1) * 16 + 2 * cq + (t & 1); }

constexpr int kSpmmChunk = 64;
constexpr int kSpmmSteps = 2;  // entries per lane whose x rows are loaded together
constexpr int kPairMax = 64;   // blocks per row of a pair
constexpr int kPairCap = 128;  // merged columns of a pair (stride of the merged lists)
constexpr int kNoBlock = 255;  // "no block of this row at this column" in a merged entry
constexpr int kSpmmWaves = 4;  // waves (slots) per workgroup

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// the lane's four columns of the three x rows of block column c
__device__ __forceinline__ void load_x3(const double *__restrict__ x, int32_t c, int cq, double (&xv)[3][4]) {
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
        const double *xr = x + (3 * (int64_t)c + jj) * W + 2 * cq;
        const double2 lo = *(const double2 *)xr, hi = *(const double2 *)(xr + 16);
        xv[jj][0] = lo.x;
        xv[jj][1] = lo.y;
        xv[jj][2] = hi.x;
        xv[jj][3] = hi.y;
    }
}

// a += block k of the staged planes sv times xv
__device__ __forceinline__ void block_fma(const double (*sv)[kSpmmChunk], int k, const double (&xv)[3][4],
                                          double (&a)[3][4]) {
#pragma unroll
    for (int jj = 0; jj < 3; ++jj)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double v = sv[3 * i + jj][k];
#pragma unroll
            for (int t = 0; t < 4; ++t) a[i][t] = fma(v, xv[jj][t], a[i][t]);
        }
}

// the row's result from the lane groups' sums: y rows (MODE), and the dot partials
template <int MODE>
__device__ __forceinline__ void finish_row(double (&a)[3][4], int row, int bg, int cq, const double *__restrict__ x,
                                           const double *__restrict__ f, double *__restrict__ y, double (&acc)[4]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            a[i][t] += lane_xor<8>(a[i][t]);
            a[i][t] += lane_xor<16>(a[i][t]);
            a[i][t] += lane_xor<32>(a[i][t]);
        }
    if (bg == 0) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int64_t o = (3 * (int64_t)row + i) * W;
            double out[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t oj = o + col4(cq, t);
                if (MODE == 0) {
                    out[t] = a[i][t];
                    acc[t] = fma(x[oj], out[t], acc[t]);
                } else {
                    out[t] = f[oj] - a[i][t];
                    acc[t] = fma(out[t], out[t], acc[t]);
                }
            }
            *(double2 *)(y + o + 2 * cq) = make_double2(out[0], out[1]);
            *(double2 *)(y + o + 16 + 2 * cq) = make_double2(out[2], out[3]);
        }
    }
}

// rows r0 and r0 + 1 finished together from their lane-group sums aa and ab: three
// exchanges between lane groups 8, 16 and 32 lanes apart (finish_row's pairings, so every
// element is the same sum) each halve what a lane carries, leaving lane group bg with row
// r0 + (bg & 1) at position t = bg >> 1 of its column quad (21 doubles exchanged per lane
// against 72 for two finish_row calls).  The dot partials keep finish_row's order: the
// row-r0 lane passes its three-term chain to the row-(r0 + 1) lane of the same column,
// which continues it; the odd lane groups return column col4(cq, bg >> 1)'s partial in
// accs (the wave's first and only rows: the chains start from zero)
template <int MODE>
__device__ __forceinline__ void finish_pair(const double (&aa)[3][4], const double (&ab)[3][4], int r0, int bg, int cq,
                                            const double *__restrict__ x, const double *__restrict__ f,
                                            double *__restrict__ y, double &accs) {
    const bool b0 = bg & 1, b1 = (bg >> 1) & 1, b2 = (bg >> 2) & 1;
    double k1[3][4];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const double keep = b0 ? ab[i][t] : aa[i][t], give = b0 ? aa[i][t] : ab[i][t];
            k1[i][t] = keep + lane_xor<8>(give);
        }
    double k2[3][2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double lo = k1[i][2 * h], hi = k1[i][2 * h + 1];
            k2[i][h] = (b1 ? hi : lo) + lane_xor<16>(b1 ? lo : hi);
        }
    const int row = r0 + b0, t = bg >> 1;
    double out[3], other[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double sum = (b2 ? k2[i][1] : k2[i][0]) + lane_xor<32>(b2 ? k2[i][0] : k2[i][1]);
        const int64_t oj = (3 * (int64_t)row + i) * W + col4(cq, t);
        if (MODE == 0) {
            out[i] = sum;
            other[i] = x[oj];
        } else {
            out[i] = f[oj] - sum;
            other[i] = out[i];
        }
        y[oj] = out[i];
    }
    double pa = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) pa = fma(other[i], out[i], pa);
    double pb = lane_xor<8>(pa);
#pragma unroll
    for (int i = 0; i < 3; ++i) pb = fma(other[i], out[i], pb);
    accs = pb;
}

// one row in chunks of 64 blocks (sv, sc: the wave's LDS)
template <int MODE>
__device__ __forceinline__ void single_row(int row, const int32_t *__restrict__ brow_ptr,
                                           const int32_t *__restrict__ bcol, const double *__restrict__ bval,
                                           const double *__restrict__ x, const double *__restrict__ f,
                                           double *__restrict__ y, double (*sv)[kSpmmChunk], int32_t *sc, int lane,
                                           double (&acc)[4]) {
    const int bg = lane >> 3, cq = lane & 7;
    const int beg = brow_ptr[row], end = brow_ptr[row + 1];
    const int64_t m = end - beg;
    const double *rv = bval + 9 * (int64_t)beg;  // plane e of block beg + i: rv[e * m + i]
    double a[3][4];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t) a[i][t] = 0.0;
    for (int c0 = 0; c0 < m; c0 += kSpmmChunk) {
        const int cnt = m - c0 < kSpmmChunk ? (int)(m - c0) : kSpmmChunk;
        if (lane < cnt) {
            double v[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) v[e] = rv[e * m + c0 + lane];
            sc[lane] = bcol[beg + c0 + lane];
#pragma unroll
            for (int e = 0; e < 9; ++e) sv[e][lane] = v[e];
        }
        wave_lds_sync();  // the wave's own LDS writes complete before its reads below
        for (int k0 = bg; k0 < cnt; k0 += 8 * kSpmmSteps) {
            double xv[kSpmmSteps][3][4];
#pragma unroll
            for (int h = 0; h < kSpmmSteps; ++h) {
                const int k = k0 + 8 * h;
                if (k < cnt) load_x3(x, sc[k], cq, xv[h]);
            }
#pragma unroll
            for (int h = 0; h < kSpmmSteps; ++h)
                if (k0 + 8 * h < cnt) block_fma(sv, k0 + 8 * h, xv[h], a);
        }
        wave_lds_sync();  // every lane is done reading this chunk before the next one is written
    }
    finish_row<MODE>(a, row, bg, cq, x, f, y, acc);
}

// rows ra and ra + 1 with the same block columns, in chunks of 64 blocks: each gathered
// x row serves both rows, and each row sums its blocks in single_row's order
template <int MODE>
__device__ __forceinline__ void twin_rows(int ra, const int32_t *__restrict__ brow_ptr,
                                          const int32_t *__restrict__ bcol, const double *__restrict__ bval,
                                          const double *__restrict__ x, const double *__restrict__ f,
                                          double *__restrict__ y, double (*sv)[9][kSpmmChunk], int32_t *sc, int lane,
                                          double &accs) {
    const int bg = lane >> 3, cq = lane & 7;
    const int ba = brow_ptr[ra], bb = brow_ptr[ra + 1];
    const int64_t m = bb - ba;  // the length of both rows
    const double *rva = bval + 9 * (int64_t)ba, *rvb = bval + 9 * (int64_t)bb;
    double aa[3][4], ab[3][4];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t) aa[i][t] = ab[i][t] = 0.0;
    for (int c0 = 0; c0 < m; c0 += kSpmmChunk) {
        const int cnt = m - c0 < kSpmmChunk ? (int)(m - c0) : kSpmmChunk;
        if (lane < cnt) {
            double v[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) v[e] = rva[e * m + c0 + lane];
            sc[lane] = bcol[ba + c0 + lane];
#pragma unroll
            for (int e = 0; e < 9; ++e) sv[0][e][lane] = v[e];
#pragma unroll
            for (int e = 0; e < 9; ++e) v[e] = rvb[e * m + c0 + lane];
#pragma unroll
            for (int e = 0; e < 9; ++e) sv[1][e][lane] = v[e];
        }
        wave_lds_sync();
        for (int k = bg; k < cnt; k += 8) {
            double xv[3][4];
            load_x3(x, sc[k], cq, xv);
            block_fma(sv[0], k, xv, aa);
            block_fma(sv[1], k, xv, ab);
        }
        wave_lds_sync();  // every lane is done reading this chunk before the next one is written
    }
    finish_pair<MODE>(aa, ab, ra, bg, cq, x, f, y, accs);
}

template <int MODE>
__global__ __launch_bounds__(64 * kSpmmWaves) __attribute__((amdgpu_waves_per_eu(4))) void k_bspmm(int32_t nb, const int32_t *__restrict__ brow_ptr,
                                               const int32_t *__restrict__ bcol, const double *__restrict__ bval,
                                               const int32_t *__restrict__ pair_len,
                                               const int32_t *__restrict__ pair_col,
                                               const uint16_t *__restrict__ pair_ab, const double *__restrict__ x,
                                               const double *__restrict__ f, double *__restrict__ y,
                                               double *__restrict__ part, const BatchState *st) {
    __shared__ double lds[kSpmmWaves][W];
    __shared__ double sv[kSpmmWaves][2][9][kSpmmChunk];
    __shared__ int32_t sc[kSpmmWaves][kPairCap];
    __shared__ uint16_t sab[kSpmmWaves][kPairCap];
    if (st && !st->any) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, bg = lane >> 3, cq = lane & 7;
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // single rows: the bg == 0 lanes' four columns
    double accs = 0.0;                      // two rows finished together: see finish_pair
    const int slot = w * kSpmmWaves + wv, ra = 2 * slot, rb = ra + 1;
    const int u = ra < nb ? pair_len[slot] : 0;  // merged columns of a pair, -1 twins, 0 otherwise
    if (u > 0) {
        const int ba = brow_ptr[ra], bb = brow_ptr[rb], eb = brow_ptr[rb + 1];
        const int ma = bb - ba, mb = eb - bb;
        const double *rva = bval + 9 * (int64_t)ba, *rvb = bval + 9 * (int64_t)bb;
        {
            double va[9], vb[9];
            int32_t c0 = 0, c1 = 0;
            uint16_t a0 = 0, a1 = 0;
#pragma unroll
            for (int e = 0; e < 9; ++e) {
                va[e] = lane < ma ? rva[e * ma + lane] : 0.0;
                vb[e] = lane < mb ? rvb[e * mb + lane] : 0.0;
            }
            const int64_t mo = (int64_t)slot * kPairCap;
            if (lane < u) {
                c0 = pair_col[mo + lane];
                a0 = pair_ab[mo + lane];
            }
            if (lane + 64 < u) {
                c1 = pair_col[mo + 64 + lane];
                a1 = pair_ab[mo + 64 + lane];
            }
#pragma unroll
            for (int e = 0; e < 9; ++e) {
                sv[wv][0][e][lane] = va[e];
                sv[wv][1][e][lane] = vb[e];
            }
            sc[wv][lane] = c0;
            sab[wv][lane] = a0;
            sc[wv][64 + lane] = c1;
            sab[wv][64 + lane] = a1;
        }
        wave_lds_sync();
        double aa[3][4], ab[3][4];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int t = 0; t < 4; ++t) aa[i][t] = ab[i][t] = 0.0;
        for (int k0 = bg; k0 < u; k0 += 8 * kSpmmSteps) {
            double xv[kSpmmSteps][3][4];
#pragma unroll
            for (int h = 0; h < kSpmmSteps; ++h) {
                const int k = k0 + 8 * h;
                if (k < u) load_x3(x, sc[wv][k], cq, xv[h]);
            }
#pragma unroll
            for (int h = 0; h < kSpmmSteps; ++h) {
                const int k = k0 + 8 * h;
                if (k < u) {
                    const int e = sab[wv][k], ia = e & 255, ib = e >> 8;
                    if (ia != kNoBlock) block_fma(sv[wv][0], ia, xv[h], aa);
                    if (ib != kNoBlock) block_fma(sv[wv][1], ib, xv[h], ab);
                }
            }
        }
        finish_pair<MODE>(aa, ab, ra, bg, cq, x, f, y, accs);
    } else if (u < 0) {
        twin_rows<MODE>(ra, brow_ptr, bcol, bval, x, f, y, sv[wv], sc[wv], lane, accs);
    } else {
        if (ra < nb) single_row<MODE>(ra, brow_ptr, bcol, bval, x, f, y, sv[wv][0], sc[wv], lane, acc);
        if (rb < nb) single_row<MODE>(rb, brow_ptr, bcol, bval, x, f, y, sv[wv][0], sc[wv], lane, acc);
    }
    if (u != 0) {
        if (bg & 1) lds[wv][col4(cq, bg >> 1)] = accs;
    } else if (bg == 0) {
#pragma unroll
        for (int t = 0; t < 4; ++t) lds[wv][col4(cq, t)] = acc[t];
    }
    __syncthreads();
    if (threadIdx.x < W) {
        double v = lds[0][threadIdx.x];
#pragma unroll
        for (int h = 1; h < kSpmmWaves; ++h) v += lds[h][threadIdx.x];
        if (MODE == 0) part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = v;
        else part[(int64_t)blockIdx.x * W + threadIdx.x] = v;
    }
}

// The merged block-column list of slot s = (rows 2 s, 2 s + 1), one wave per slot, when
// both rows have at most kPairMax blocks: the columns of either row in increasing order,
// each once, with the block's index in row 2 s (low byte) and in row 2 s + 1 (high byte),
// kNoBlock where the row has none; pair_len[s] = their number (0: not a pair).  A row's
// columns are strictly increasing (a checked input property), so the position of a
// column in the merged list is the number of distinct columns of both rows below it.
__global__ __launch_bounds__(256) void k_pair_merge(int32_t nb, const int32_t *__restrict__ brow_ptr,
                                                    const int32_t *__restrict__ bcol, int32_t nslots,
                                                    int32_t *__restrict__ pair_len, int32_t *__restrict__ pair_col,
                                                    uint16_t *__restrict__ pair_ab) {
    __shared__ int32_t ca[4][64], cb[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int s = blockIdx.x * 4 + wv;
    if (s >= nslots) return;  // no barrier below: waves leave independently
    const int ra = 2 * s, rb = ra + 1;
    int ma = 0, mb = 0, ba = 0, bb = 0;
    if (rb < nb) {
        ba = brow_ptr[ra];
        bb = brow_ptr[rb];
        ma = bb - ba;
        mb = brow_ptr[rb + 1] - bb;
    }
    if (rb >= nb) {
        if (lane == 0) pair_len[s] = 0;
        return;
    }
    if (ma > kPairMax || mb > kPairMax) {
        // twins: the same block columns (the block rows of one enriched node), -1
        bool same = ma == mb;
        for (int i0 = 0; same && i0 < ma; i0 += 64)
            same = __ballot(lane + i0 < ma && bcol[ba + i0 + lane] != bcol[bb + i0 + lane]) == 0;
        if (lane == 0) pair_len[s] = same ? -1 : 0;
        return;
    }
    const int32_t a = lane < ma ? bcol[ba + lane] : INT32_MAX;
    const int32_t b = lane < mb ? bcol[bb + lane] : INT32_MAX;
    ca[wv][lane] = a;
    cb[wv][lane] = b;
    wave_lds_sync();
    // lower bounds: lt_b = #{b_j < a}, lt_a = #{a_i < b}
    int lo = 0, hi = mb;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cb[wv][mid] < a) lo = mid + 1;
        else hi = mid;
    }
    const int lt_b = lo;
    lo = 0;
    hi = ma;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ca[wv][mid] < b) lo = mid + 1;
        else hi = mid;
    }
    const int lt_a = lo;
    const bool a_in_b = lane < ma && lt_b < mb && cb[wv][lt_b] == a;
    const bool b_in_a = lane < mb && lt_a < ma && ca[wv][lt_a] == b;
    const uint64_t dup = __ballot(b_in_a);
    auto below = [&](int n) { return n >= 64 ? __popcll(dup) : __popcll(dup & ((1ull << n) - 1)); };
    const int64_t mo = (int64_t)s * kPairCap;
    if (lane < ma) {
        const int pos = lane + lt_b - below(lt_b);
        pair_col[mo + pos] = a;
        pair_ab[mo + pos] = (uint16_t)(lane | ((a_in_b ? lt_b : kNoBlock) << 8));
    }
    if (lane < mb && !b_in_a) {
        const int pos = lt_a + lane - below(lane);
        pair_col[mo + pos] = b;
        pair_ab[mo + pos] = (uint16_t)(kNoBlock | (lane << 8));
    }
    if (lane == 0) pair_len[s] = ma + mb - __popcll(dup);
}

// Fixed-order sum of column j of column-major partials (nparts per column) by one
// 256-thread workgroup; valid in thread 0.
__device__ __forceinline__ double col_sum_cm(const double *__restrict__ part, int nparts, int j, double *lds4) {
    const double *pc = part + (int64_t)j * nparts;
    double s = seq_sum(pc, 1, threadIdx.x, nparts, 256);
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) lds4[threadIdx.x >> 6] = s;
    __syncthreads();
    return (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
}

// alpha_j = rho_j / p_j^T q_j for the running columns (breakdown test as in Algorithm 1);
// workgroup j reduces column j of the SpMM partials.
__global__ __launch_bounds__(1024) void k_balpha(const double *__restrict__ part, int nparts, BatchState *st) {
    __shared__ double lds[16];
    if (!st->any) return;
    const int j = blockIdx.x;
    double pq;
    {  // fixed-order sum of column j over 1024 threads
        const double *pc = part + (int64_t)j * nparts;
        double s = seq_sum(pc, 1, threadIdx.x, nparts, 1024);
        s = wave_sum(s);
        if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
        __syncthreads();
        pq = 0.0;
#pragma unroll
        for (int h = 0; h < 16; h += 2) pq += lds[h] + lds[h + 1];
    }
    if (threadIdx.x == 0 && st->flag[j] == kRunning) {
        const int it = st->iter;
        const double a = st->rho[it & 1][j] / pq;
        if (!(pq > 0.0) || !isfinite(pq) || !isfinite(a)) {
            st->flag[j] = kBreakdown;
            st->bad[j] = it;
            st->iters_done[j] = it;
        } else {
            st->alpha[j] = a;
        }
    }
}

// update = 1: u_j += alpha_j p_j and r_j -= alpha_j q_j for the running columns, with
// partials of ||r_j||^2; then (both modes) y = M^{-1} r over the tile's whole blocks
// from an LDS copy of r.  One workgroup per contiguous range of tiles.  A tile's block
// inverses are one contiguous range of minv (whole blocks), staged in LDS with coalesced
// loads when it fits in kBjStage entries (3 x 3 blocks: 3 per DoF), so the product reads
// broadcast LDS words instead of broadcast global loads; each DoF's row offset, block size
// and position go packed into one LDS word.
constexpr int kBjStage = 480;

__global__ __launch_bounds__(256) void k_bupdate_bj(int32_t ntiles, int32_t nwg, const int32_t *__restrict__ tile_start,
                                                    double *__restrict__ u, double *__restrict__ r,
                                                    double *__restrict__ y, const double *__restrict__ q,
                                                    const double *__restrict__ p, const double *__restrict__ minv,
                                                    const int32_t *__restrict__ bj_rowoff,
                                                    const int32_t *__restrict__ bj_meta, double *__restrict__ part,
                                                    const BatchState *st, int update) {
    __shared__ double tile[kBatchTileDofs][W];
    __shared__ double mv[kBjStage];  // also the 8 x W doubles of the final group sum
    __shared__ int32_t md[kBatchTileDofs];
    static_assert(kBjStage >= 8 * W && kBatchTileDofs * kMaxBlock < (1 << 21) && kMaxBlock < 32, "packing");
    if (!st->any) return;
    const int j = threadIdx.x & 31, g = threadIdx.x >> 5;
    const bool run = update && st->flag[j] == kRunning;
    const double alpha = run ? st->alpha[j] : 0.0;
    const int w = xcd_remap(blockIdx.x, nwg);
    const int t0 = (int)(((int64_t)w * ntiles) / nwg), t1 = (int)(((int64_t)(w + 1) * ntiles) / nwg);
    double acc = 0.0;
    for (int t = t0; t < t1; ++t) {
        const int64_t d0 = tile_start[t], d1 = tile_start[t + 1];
        if (d1 <= d0) continue;  // uniform: the last tile can be empty
        const int32_t m0 = bj_rowoff[d0], m1 = bj_rowoff[d1 - 1] + (bj_meta[d1 - 1] >> 8);
        const bool staged = m1 - m0 <= kBjStage;
        __syncthreads();
        if (staged)
            for (int e = threadIdx.x; e < m1 - m0; e += blockDim.x) mv[e] = minv[m0 + e];
        if (threadIdx.x < d1 - d0) {
            const int mt = bj_meta[d0 + threadIdx.x];
            md[threadIdx.x] = ((bj_rowoff[d0 + threadIdx.x] - m0) << 10) | ((mt >> 8) << 5) | (mt & 255);
        }
        // eight DoFs of the group at a time (a whole tile): all loads first, then the updates
        for (int64_t db = d0 + g; db < d1; db += 64) {
            double rv[8], pv[8], qv[8], uv[8];
#pragma unroll
            for (int h = 0; h < 8; ++h) {
                const int64_t d = db + 8 * h, o = d * W + j;
                rv[h] = pv[h] = qv[h] = uv[h] = 0.0;
                if (d < d1) {
                    rv[h] = r[o];
                    if (run) {
                        pv[h] = p[o];
                        qv[h] = q[o];
                        uv[h] = u[o];
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < 8; ++h) {
                const int64_t d = db + 8 * h, o = d * W + j;
                if (d >= d1) continue;
                double rn = rv[h];
                if (run) {
                    u[o] = fma(alpha, pv[h], uv[h]);
                    rn = fma(-alpha, qv[h], rn);
                    r[o] = rn;
                }
                tile[d - d0][j] = rn;
                acc = fma(rn, rn, acc);
            }
        }
        __syncthreads();
        for (int64_t db = d0 + g; db < d1; db += 32) {
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int64_t d = db + 8 * h;
                if (d >= d1) continue;
                const int mt = md[d - d0], size = (mt >> 5) & 31, ro = mt >> 10;
                const int base = (int)(d - d0) - (mt & 31);
                double s = 0.0;
                if (staged)
                    for (int kk = 0; kk < size; ++kk) s = fma(mv[ro + kk], tile[base + kk][j], s);
                else
                    for (int kk = 0; kk < size; ++kk) s = fma(minv[m0 + ro + kk], tile[base + kk][j], s);
                y[d * W + j] = s;
            }
        }
    }
    __syncthreads();  // the last tile's reads of mv precede its reuse
    const double tot = group_sum_8(acc, reinterpret_cast<double(*)[W]>(mv));
    if (update && threadIdx.x < W) part[(int64_t)blockIdx.x * W + threadIdx.x] = tot;
}

// Column checks by workgroup 0 of a restriction launch (32 NG threads): ||r_j|| from the
// row-major partials against thr_j and the iteration cap, then any = some column still
// running.
template <int NG>
__device__ void column_check(BatchState *st, const double *__restrict__ part_rr, int n_rr, int iter_offset,
                             int max_iter, double (*lds)[W + 1]) {
    const int j = threadIdx.x & 31;
    const double rr = col_reduce<NG>(part_rr, n_rr, lds);
    __shared__ int32_t run_s[W];
    if (threadIdx.x < W) {
        int32_t fl = st->flag[j];
        if (fl == kRunning) {
            const int done = st->iter + iter_offset;
            st->rr[j] = rr;
            if (!isfinite(rr)) {
                fl = kBreakdown;
                st->bad[j] = st->iter;
            } else if (sqrt(rr) <= st->thr[j]) {
                fl = kConverged;
            } else if (done >= max_iter) {
                fl = kMaxIter;
            }
            if (fl != kRunning) {
                st->flag[j] = fl;
                st->iters_done[j] = done;
            }
        }
        run_s[j] = fl == kRunning;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t any = 0;
        for (int h = 0; h < W; ++h) any |= run_s[h];
        st->any = any;
    }
    __syncthreads();
}

// Workgroup 0 runs the column checks when n_rr > 0.  Then the merged right-hand side
// of Algorithm 3 in segments: segment s of deflation vector c
// sums Z^T[c, e] a[e][j] over its entries (list 0) or -(KZ)^T[c, e] b[e][j] (list 1; 0
// when b is null) into seg_part[s][j].  Group g of 32 lanes takes the chunks of 32
// entries g, g + 32, ...: lane j loads entry j of the chunk (one coalesced load of
// indices and values), the chunk's row indices are passed round by shuffles and eight
// row gathers are in flight at a time; the group sums are added in a fixed order.
__global__ __launch_bounds__(1024) void k_brestrict(const int32_t *__restrict__ seg, int32_t nseg,
                                                   const int32_t *__restrict__ zt_idx,
                                                   const double *__restrict__ zt_val,
                                                   const int32_t *__restrict__ kzt_idx,
                                                   const double *__restrict__ kzt_val, const double *__restrict__ a,
                                                   const double *__restrict__ b, double *__restrict__ seg_part,
                                                   BatchState *st, const double *__restrict__ part_rr, int n_rr,
                                                   int iter_offset, int max_iter) {
    __shared__ double lds[32][W + 1];
    const int j = threadIdx.x & 31, g = threadIdx.x >> 5;
    if (st) {
        if (wg_any(st) == 0) return;
        if (blockIdx.x == 0 && n_rr > 0) column_check<32>(st, part_rr, n_rr, iter_offset, max_iter, lds);
    }
    const int sg = xcd_remap(blockIdx.x, gridDim.x);
    if (sg >= nseg) return;
    const int list = seg[4 * sg + 1], e0 = seg[4 * sg + 2], e1 = seg[4 * sg + 3];
    const int32_t *idx = list ? kzt_idx : zt_idx;
    const double *val = list ? kzt_val : zt_val;
    const double *vec = list ? b : a;
    constexpr int kInFlight = 8;
    double s = 0.0;
    if (vec) {
        for (int c0 = e0 + 32 * g; c0 < e1; c0 += 32 * 32) {
            const int e = c0 + j;
            int col = 0;
            double v = 0.0;
            if (e < e1) {
                col = idx[e];
                v = val[e];
            }
            const int cnt = min(32, e1 - c0);  // the same for the whole group
#pragma unroll
            for (int q0 = 0; q0 < 32; q0 += kInFlight) {
                double x[kInFlight];
#pragma unroll
                for (int q = 0; q < kInFlight; ++q) {
                    const int cq = __shfl(col, q0 + q, 32);
                    x[q] = q0 + q < cnt ? vec[(int64_t)cq * W + j] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < kInFlight; ++q) {
                    const double vq = __shfl(v, q0 + q, 32);
                    if (q0 + q < cnt) s = fma(vq, x[q], s);
                }
            }
        }
    }
    __syncthreads();  // lds may still be read by the check above
    lds[g][j] = s;
    __syncthreads();
    if (threadIdx.x < W) {
        double t = 0.0;
        for (int h = 0; h < 32; ++h) t += lds[h][threadIdx.x];
        seg_part[(int64_t)sg * W + threadIdx.x] = list ? -t : t;
    }
}

// g[c][j] = sum of column c's segment partials, in segment order (8 columns per
// workgroup).
__global__ __launch_bounds__(256) void k_bsegsum(int32_t k, const int32_t *__restrict__ seg_ptr,
                                                 const double *__restrict__ seg_part, double *__restrict__ gout,
                                                 const BatchState *st) {
    if (st && !st->any) return;
    const int c = blockIdx.x * 8 + (threadIdx.x >> 5), j = threadIdx.x & 31;
    if (c >= k) return;
    double t = 0.0;
    for (int sg = seg_ptr[c]; sg < seg_ptr[c + 1]; ++sg) t += seg_part[(int64_t)sg * W + j];
    gout[(int64_t)c * W + j] = t;
}

// ---- grouped restriction on the matrix cores ----
// Runs of consecutive deflation vectors whose Z columns cover the same DoF triplets (the
// rigid-body modes of one subdomain, or those restricted to one enrichment function's
// DoFs) and whose (KZ)^T rows coincide form groups of up to kGroupCols vectors.  Z is
// kept per group as a dense kg x L block over the group's triplet rows (zeros where a
// mode has no component; column c's L values follow column c - 1's), as (KZ)^T already
// is, so
//   G[group] = Z_g^T a[rows_g] - (KZ)_g^T b[rows'_g]
// is a dense (kg x L) by (L x 32) product: every gathered row of a or b serves all kg
// vectors at once, where the per-entry kernel gathers it once per vector.
typedef double bdbl4 __attribute__((ext_vector_type(4)));
constexpr int kGroupCols = 16;    // vectors of a group (one MFMA row tile)
constexpr int kGroupRows = 128;   // rows of a group's list per segment (one wave)
constexpr int kGroupUnroll = 8;   // 4-row MFMA steps whose loads are issued together
constexpr int kGroupSeg = 7;      // ints per segment record

// flag[j] = 1 when column j of (ptr, idx) lists the same rows as column j - 1 (flag[0] =
// 0); one wave per column.
__global__ __launch_bounds__(256) void k_same_rows(int32_t k, const int32_t *__restrict__ ptr,
                                                   const int32_t *__restrict__ idx, uint8_t *__restrict__ flag) {
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (j >= k) return;
    bool same = false;
    if (j > 0) {
        const int a0 = ptr[j - 1], a1 = ptr[j], len = a1 - a0;
        same = len == ptr[j + 1] - a1;
        if (same) {
            bool mine = true;
            for (int e = lane; e < len; e += 64) mine = mine && idx[a0 + e] == idx[a1 + e];
            same = __ballot(!mine) == 0ull;
        }
    }
    if (lane == 0) flag[j] = same ? 1 : 0;
}

// One wave per segment gseg[7 s ..] = (first vector j0, vectors kg, list 0 = the dense
// group blocks of Z (rows zr, values zv) / 1 = (KZ)^T, first row-list entry of the
// segment, its first value for vector j0, rows, row-list length L): 4 rows per
// v_mfma_f64_16x16x4f64 step, a = value of vector m = l % 16 at row l / 16 of the step
// (0 for m >= kg), b = row l / 16 of the vector at columns l % 16 and 16 + l % 16 (two
// 16-column halves).  The row indices and values of kGroupUnroll steps are loaded
// before their row gathers.  Rows m < kg of the result go to seg_part[s][m][.],
// negated for list 1 (0 when b is null).  Workgroup 0 runs the column checks.
constexpr int kGroupWaves = 16;  // segments (waves) per workgroup of the grouped restriction

__global__ __launch_bounds__(64 * kGroupWaves) void k_brestrict_mfma(const int32_t *__restrict__ gseg, int32_t ngseg,
                                                        const int32_t *__restrict__ zr,
                                                        const double *__restrict__ zv,
                                                        const int32_t *__restrict__ kzt_idx,
                                                        const double *__restrict__ kzt_val,
                                                        const double *__restrict__ a, const double *__restrict__ b,
                                                        double *__restrict__ seg_part, BatchState *st,
                                                        const double *__restrict__ part_rr, int n_rr, int iter_offset,
                                                        int max_iter) {
    __shared__ double lds[32][W + 1];
    if (st) {
        if (wg_any(st) == 0) return;
        if (blockIdx.x == 0 && n_rr > 0) column_check<2 * kGroupWaves>(st, part_rr, n_rr, iter_offset, max_iter, lds);
    }
    const int sg = xcd_remap(blockIdx.x, gridDim.x) * kGroupWaves + (threadIdx.x >> 6), l = threadIdx.x & 63;
    if (sg >= ngseg) return;
    const int32_t *G = gseg + kGroupSeg * sg;
    const int kg = G[1], list = G[2], ibeg = G[3], vbeg = G[4], nrows = G[5], L = G[6];
    const int32_t *idx = list ? kzt_idx : zr;
    const double *val = list ? kzt_val : zv;
    const double *vec = list ? b : a;
    const int m = l & 15, kk = l >> 4, mm = min(m, kg - 1);
    bdbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    if (vec) {
        const int nsteps = (nrows + 3) / 4;
        for (int s0 = 0; s0 < nsteps; s0 += kGroupUnroll) {
            int32_t ri[kGroupUnroll];
            double av[kGroupUnroll];
#pragma unroll
            for (int u = 0; u < kGroupUnroll; ++u) {
                const int r = 4 * (s0 + u) + kk, rc = min(r, nrows - 1);  // past the end: the last row, masked
                ri[u] = idx[ibeg + rc];
                const double v = val[vbeg + (int64_t)mm * L + rc];
                av[u] = (r < nrows && m < kg) ? v : 0.0;
            }
            double b0[kGroupUnroll], b1[kGroupUnroll];
#pragma unroll
            for (int u = 0; u < kGroupUnroll; ++u) {
                const double *row = vec + (int64_t)ri[u] * W;
                b0[u] = row[m];
                b1[u] = row[16 + m];
            }
#pragma unroll
            for (int u = 0; u < kGroupUnroll; ++u) {
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], b0[u], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], b1[u], acc1, 0, 0, 0);
            }
        }
    }
    const double sgn = list ? -1.0 : 1.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int mo = kk + 4 * v;  // result item v of lane l: row l / 16 + 4 v, column l % 16
        if (mo < kg) {
            double *o = seg_part + ((int64_t)sg * kGroupCols + mo) * W;
            o[m] = sgn * acc0[v];
            o[16 + m] = sgn * acc1[v];
        }
    }
}

// g[c][j] = sum over the segments gcol[3c] .. gcol[3c+1]-1 of c's group of their partial
// row gcol[3c+2], in segment order (8 vectors per workgroup).
__global__ __launch_bounds__(256) void k_bgroupsum(int32_t k, const int32_t *__restrict__ gcol,
                                                   const double *__restrict__ seg_part, double *__restrict__ gout,
                                                   const BatchState *st) {
    if (st && !st->any) return;
    const int c = blockIdx.x * 8 + (threadIdx.x >> 5), j = threadIdx.x & 31;
    if (c >= k) return;
    const int s0 = gcol[3 * c], s1 = gcol[3 * c + 1], mo = gcol[3 * c + 2];
    double t = 0.0;
    for (int sg = s0; sg < s1; sg += 8) {  // eight loads in flight, added in segment order
        double x[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) x[q] = sg + q < s1 ? seg_part[((int64_t)(sg + q) * kGroupCols + mo) * W + j] : 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (sg + q < s1) t += x[q];
    }
    gout[(int64_t)c * W + j] = t;
}

// delta = E^{-1} g for all 32 columns on the matrix cores: workgroup = 16 rows of
// E^{-1}; wave w of 8 takes the w-th eighth of the contraction index c in steps of 4
// (v_mfma_f64_16x16x4f64: a = E^{-1}[row l % 16][c + l / 16], b = g[c + l / 16][col],
// two 16-column halves), then the eight partial tiles are added in wave order in LDS.
// Result item v of lane l is row l / 16 + 4 v, column l % 16 of a half.
constexpr int kCoarseWaves = 8;
__global__ __launch_bounds__(64 * kCoarseWaves) void k_bcoarse(int32_t k, int64_t ld,
                                                               const double *__restrict__ einv,
                                                               const double *__restrict__ gin,
                                                               double *__restrict__ delta, const BatchState *st) {
    __shared__ double part[kCoarseWaves][16][W + 1];
    if (st && !st->any) return;
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r0 = blockIdx.x * 16;
    const int row = r0 + (l & 15), kq = l >> 4;
    const int steps = (k + 3) / 4;
    const int s0 = (int)(((int64_t)wv * steps) / kCoarseWaves), s1 = (int)(((int64_t)(wv + 1) * steps) / kCoarseWaves);
    const double *erow = einv + (int64_t)min(row, k - 1) * ld;
    bdbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    for (int sb = s0; sb < s1; sb += 4) {  // four steps' loads in flight, then their products
        double a[4], b0[4], b1[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = 4 * (sb + u) + kq;
            const bool ok = sb + u < s1 && c < k;
            const double *gr = gin + (int64_t)min(c, k - 1) * W;
            a[u] = ok && row < k ? erow[min(c, k - 1)] : 0.0;
            b0[u] = ok ? gr[l & 15] : 0.0;
            b1[u] = ok ? gr[16 + (l & 15)] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b0[u], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b1[u], acc1, 0, 0, 0);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        part[wv][kq + 4 * v][l & 15] = acc0[v];
        part[wv][kq + 4 * v][16 + (l & 15)] = acc1[v];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 16 * W; t += 64 * kCoarseWaves) {
        const int rr = t / W, j = t % W;
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < kCoarseWaves; ++w) sum += part[w][rr][j];
        if (r0 + rr < k) delta[(int64_t)(r0 + rr) * W + j] = sum;
    }
}

// sum_e z_val[e] delta[z_col[e]][j] over the cnt entries of a row from e0, in index order:
// lane j loads entry j of each chunk of 32 (one coalesced load), the column indices are
// passed round by shuffles and up to eight delta rows are gathered at a time
__device__ __forceinline__ double zrow_dot_long(int e0, int cnt, int j, const int32_t *__restrict__ z_col,
                                                const double *__restrict__ z_val, const double *__restrict__ delta) {
    double c = 0.0;
    for (int b0 = 0; b0 < cnt; b0 += 32) {
        int col = 0;
        double v = 0.0;
        if (b0 + j < cnt) {
            col = z_col[e0 + b0 + j];
            v = z_val[e0 + b0 + j];
        }
        const int m = min(32, cnt - b0);  // the same for the whole group
        for (int q0 = 0; q0 < m; q0 += 8) {
            double x[8], vq[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int cq = __shfl(col, q0 + q, 32);
                vq[q] = __shfl(v, q0 + q, 32);
                x[q] = q0 + q < m ? delta[(int64_t)cq * W + j] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q0 + q < m) c = fma(vq[q], x[q], c);
        }
    }
    return c;
}

// out = base + Z delta (base may be null); optional partials of rdot_j^T out_j;
// optionally advance the iteration.
__global__ __launch_bounds__(256) void k_bprolong(int64_t n, int32_t nwg, const int32_t *__restrict__ z_ptr,
                                                  const int32_t *__restrict__ z_col, const double *__restrict__ z_val,
                                                  const double *__restrict__ delta, const double *base, double *out,
                                                  const double *__restrict__ rdot, double *__restrict__ part,
                                                  BatchState *st, int advance) {
    __shared__ double lds[8][W];
    if (st && !st->any) return;
    const int j = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int w = xcd_remap(blockIdx.x, nwg);
    const int64_t per = (n + nwg - 1) / nwg;
    const int64_t d1 = std::min<int64_t>(n, (int64_t)(w + 1) * per);
    double acc = 0.0;
    // rows d and d + 8 of the group per pass, their loads issued together; each row's
    // entries are added in index order (c from zero), then s = base + c
    for (int64_t d = (int64_t)w * per + g; d < d1; d += 16) {
        const int64_t db = d + 8;
        const bool hb = db < d1;
        const int64_t oa = d * W + j, ob = db * W + j;
        double sa = base ? base[oa] : 0.0, sb = base && hb ? base[ob] : 0.0;
        double ca = 0.0, cb = 0.0;
        if (delta) {
            const int ea = z_ptr[d], na = z_ptr[d + 1] - ea;
            const int eb = hb ? z_ptr[db] : 0, nb = hb ? z_ptr[db + 1] - eb : 0;
            if (na <= 32 && nb <= 32) {
                // lane j loads entry j of each row; the entries are passed round by shuffles,
                // four per row and step, and their delta rows gathered together
                int cola = 0, colb = 0;
                double va = 0.0, vb = 0.0;
                if (j < na) {
                    cola = z_col[ea + j];
                    va = z_val[ea + j];
                }
                if (j < nb) {
                    colb = z_col[eb + j];
                    vb = z_val[eb + j];
                }
                const int m = max(na, nb);  // the same for the whole group
                for (int q0 = 0; q0 < m; q0 += 4) {
                    double xa[4], xb[4], wa[4], wb[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int ka = __shfl(cola, q0 + q, 32), kb = __shfl(colb, q0 + q, 32);
                        wa[q] = __shfl(va, q0 + q, 32);
                        wb[q] = __shfl(vb, q0 + q, 32);
                        xa[q] = q0 + q < na ? delta[(int64_t)ka * W + j] : 0.0;
                        xb[q] = q0 + q < nb ? delta[(int64_t)kb * W + j] : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (q0 + q < na) ca = fma(wa[q], xa[q], ca);
                        if (q0 + q < nb) cb = fma(wb[q], xb[q], cb);
                    }
                }
            } else {
                ca = zrow_dot_long(ea, na, j, z_col, z_val, delta);
                if (hb) cb = zrow_dot_long(eb, nb, j, z_col, z_val, delta);
            }
        }
        sa += ca;
        out[oa] = sa;
        if (rdot) acc = fma(rdot[oa], sa, acc);
        if (hb) {
            sb += cb;
            out[ob] = sb;
            if (rdot) acc = fma(rdot[ob], sb, acc);
        }
    }
    if (rdot) {
        const double t = group_sum_8(acc, lds);
        if (threadIdx.x < W) part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;  // column-major
    }
    if (advance && blockIdx.x == 0 && threadIdx.x == 0) st->iter = st->iter + 1;
}

// rho_j = r_j^T z_j, beta_{i-1,j} = rho_{i,j} / rho_{i-1,j} for the running columns,
// rho kept in two parity slots; workgroup j reduces column j of the prolongation
// partials.
__global__ __launch_bounds__(256) void k_bbeta(const double *__restrict__ part, int nparts, BatchState *st) {
    __shared__ double lds[4];
    if (!st->any) return;
    const int j = blockIdx.x;
    const double rho = col_sum_cm(part, nparts, j, lds);
    if (threadIdx.x == 0 && st->flag[j] == kRunning) {
        const int it = st->iter;
        if (it > 0 && !isfinite(rho)) {
            st->flag[j] = kBreakdown;
            st->bad[j] = it - 1;
            st->iters_done[j] = it;
        } else {
            st->beta[j] = it > 0 ? rho / st->rho[(it + 1) & 1][j] : 0.0;
            st->rho[it & 1][j] = rho;
        }
    }
}

// p_j = z_j + beta_j p_j (p_0 = z_0) for the running columns; 0 for the others.
__global__ __launch_bounds__(256) void k_bpupdate(int64_t n, const double *__restrict__ z, double *__restrict__ p,
                                                  const BatchState *st) {
    if (!st->any) return;
    const int j = threadIdx.x & 31;
    const bool run = st->flag[j] == kRunning;
    const bool first = st->iter == 0;
    const double beta = st->beta[j];
    for (int64_t d = blockIdx.x * 8ll + (threadIdx.x >> 5); d < n; d += (int64_t)gridDim.x * 8) {
        const int64_t o = d * W + j;
        p[o] = run ? (first ? z[o] : fma(beta, p[o], z[o])) : 0.0;
    }
}

// dst[d][j] = src[d * nrhs + j] for j < nrhs, 0 for the padding columns.
__global__ void k_bpack(int64_t n, int32_t nrhs, const double *__restrict__ src, double *__restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * W; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = i / W;
        const int j = (int)(i % W);
        dst[i] = j < nrhs ? src[d * nrhs + j] : 0.0;
    }
}

// dst[d * nrhs + j] = src[d][j], or 0 for the columns in zero_mask.
__global__ void k_bunpack(int64_t n, int32_t nrhs, const double *__restrict__ src, double *__restrict__ dst,
                          uint32_t zero_mask) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * nrhs;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = i / nrhs;
        const int j = (int)(i % nrhs);
        dst[i] = ((zero_mask >> j) & 1u) ? 0.0 : src[d * W + j];
    }
}

// Column partials of ||a_j||^2 and of the count of non-finite entries of a and b.
__global__ __launch_bounds__(256) void k_bnorm(int64_t n, int32_t nwg, const double *__restrict__ a,
                                               const double *__restrict__ b, double *__restrict__ part,
                                               double *__restrict__ part_bad) {
    __shared__ double lds[8][W];
    const int j = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int64_t per = (n + nwg - 1) / nwg;
    const int64_t d1 = std::min<int64_t>(n, (int64_t)(blockIdx.x + 1) * per);
    double acc = 0.0, bad = 0.0;
    for (int64_t d = (int64_t)blockIdx.x * per + g; d < d1; d += 8) {
        const double v = a[d * W + j];
        acc = fma(v, v, acc);
        if (!isfinite(v)) bad += 1.0;
        if (b && !isfinite(b[d * W + j])) bad += 1.0;
    }
    const double t = group_sum_8(acc, lds);
    __syncthreads();
    const double tb = group_sum_8(bad, lds);
    if (threadIdx.x < W) {
        part[(int64_t)blockIdx.x * W + threadIdx.x] = t;
        part_bad[(int64_t)blockIdx.x * W + threadIdx.x] = tb;
    }
}

// aux[j] = column sums of part; nonfinite = 1 when the column sums of part_bad (if
// given) are not all zero.
__global__ __launch_bounds__(1024) void k_baux(const double *__restrict__ part, const double *__restrict__ part_bad,
                                               int nparts, BatchState *st) {
    __shared__ double lds[32][W + 1];
    const double s = col_reduce_1024(part, nparts, lds);
    if (threadIdx.x < W) st->aux[threadIdx.x] = s;
    if (part_bad) {
        __syncthreads();
        const double b = col_reduce_1024(part_bad, nparts, lds);
        __shared__ double bsum[W];
        if (threadIdx.x < W) bsum[threadIdx.x] = b;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int h = 0; h < W; ++h) t += bsum[h];
            st->nonfinite = t > 0.0 ? 1 : 0;
        }
    }
}

// ---------------------------------------------------------------- host side
#define BLAUNCH(...)                                         \
    do {                                                     \
        hipLaunchKernelGGL(__VA_ARGS__);                     \
        if (hipGetLastError() != hipSuccess) return DPCG_EHIP; \
    } while (0)
#define BHIP(expr)                                    \
    do {                                              \
        if ((expr) != hipSuccess) return DPCG_EHIP;   \
    } while (0)
#define BTRY(expr)                         \
    do {                                   \
        int s_ = (expr);                   \
        if (s_ != DPCG_OK) return s_;      \
    } while (0)

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int grid_rows(int64_t work, int per, int cap) {
    int g = (int)std::max<int64_t>(1, std::min<int64_t>(cap, (work + per - 1) / per));
    if (g >= 8) g = (g + 7) & ~7;
    return g;
}

template <class T>
int balloc(dpcg_ctx *c, T **p, size_t count) {
    void *q = nullptr;
    const size_t bytes = std::max<size_t>(1, count) * sizeof(T);
    BHIP(dev_alloc(&q, bytes));
    c->allocations.push_back(q);
    c->device_bytes += (int64_t)bytes;
    *p = (T *)q;
    return DPCG_OK;
}

int ensure_ws(dpcg_ctx *c) {
    if (c->bws) return DPCG_OK;
    auto *b = new BatchWorkspace();
    c->bws = b;
    const size_t nw = (size_t)c->n * W, kw = (size_t)std::max(1, c->k) * W;
    BTRY(balloc(c, &b->f, nw));
    BTRY(balloc(c, &b->u, nw));
    BTRY(balloc(c, &b->r, nw));
    BTRY(balloc(c, &b->y, nw));
    BTRY(balloc(c, &b->z, nw));
    BTRY(balloc(c, &b->q, nw));
    BTRY(balloc(c, &b->p, nw));
    BTRY(balloc(c, &b->g, kw));
    BTRY(balloc(c, &b->delta, kw));
    const int64_t nslots = (c->nb + 1) / 2;
    b->spmm_nwg = grid_rows(nslots, kSpmmWaves, 1 << 30);
    BTRY(balloc(c, &b->pair_len, (size_t)nslots));
    BTRY(balloc(c, &b->pair_col, (size_t)nslots * kPairCap));
    BTRY(balloc(c, &b->pair_ab, (size_t)nslots * kPairCap));
    BLAUNCH(k_pair_merge, dim3((unsigned)((nslots + 3) / 4)), dim3(256), 0, c->stream, c->nb, c->brow_ptr, c->bcol,
            (int32_t)nslots, b->pair_len, b->pair_col, b->pair_ab);
    b->upd_nwg = grid_rows(c->bjb_ntiles, 1, 4096);  // about one tile per workgroup at 40^3
    b->vec_nwg = grid_rows(c->n, 32, 8192);  // prolongation 44.9 -> 42.4 us at 40^3 against 4,096
    const size_t np = (size_t)std::max({b->spmm_nwg, b->upd_nwg, b->vec_nwg}) * W;
    BTRY(balloc(c, &b->part, np));
    BTRY(balloc(c, &b->part2, np));
    BTRY(balloc(c, &b->st, 1));
    BHIP(hipHostMalloc((void **)&b->snap, sizeof(BatchState), hipHostMallocDefault));
    // restriction segments from the column pointers of Z^T and (KZ)^T
    std::vector<int32_t> zp(c->k + 1, 0), kp(c->k + 1, 0), seg, sptr(c->k + 1, 0);
    if (c->k > 0) {
        BHIP(hipMemcpyAsync(zp.data(), c->zt_ptr, sizeof(int32_t) * (c->k + 1), hipMemcpyDeviceToHost, c->stream));
        BHIP(hipMemcpyAsync(kp.data(), c->kzt_ptr, sizeof(int32_t) * (c->k + 1), hipMemcpyDeviceToHost, c->stream));
        BHIP(hipStreamSynchronize(c->stream));
    }
    for (int cc = 0; cc < c->k; ++cc) {
        sptr[cc] = (int32_t)(seg.size() / 4);
        for (int list = 0; list < 2; ++list) {
            const int32_t e0 = list ? kp[cc] : zp[cc], e1 = list ? kp[cc + 1] : zp[cc + 1];
            for (int32_t e = e0; e == e0 || e < e1; e += kBatchSegEntries) {
                seg.push_back(cc);
                seg.push_back(list);
                seg.push_back(e);
                seg.push_back(std::min(e1, e + kBatchSegEntries));
            }
        }
    }
    b->nseg = (int32_t)(seg.size() / 4);
    sptr[c->k] = b->nseg;
    BTRY(balloc(c, &b->seg, std::max<size_t>(4, seg.size())));
    BTRY(balloc(c, &b->seg_ptr, (size_t)c->k + 1));
    // groups of consecutive vectors whose Z columns cover the same triplets and whose
    // (KZ)^T rows coincide; the grouped kernel is used when they hold two vectors or more
    // on average
    std::vector<int32_t> gseg, gcol(3 * (size_t)std::max(1, c->k), 0), zr;
    std::vector<double> zv;
    if (c->k > 0) {
        const int64_t nz = zp[c->k];
        std::vector<int32_t> zi(std::max<int64_t>(1, nz));
        std::vector<double> zval(std::max<int64_t>(1, nz));
        std::vector<uint8_t> fk(c->k);
        void *fl_d = nullptr;
        BHIP(dev_alloc(&fl_d, (size_t)c->k));
        hipLaunchKernelGGL(k_same_rows, dim3((c->k + 3) / 4), dim3(256), 0, c->stream, c->k, c->kzt_ptr, c->kzt_idx,
                           (uint8_t *)fl_d);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(fk.data(), fl_d, fk.size(), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && nz > 0)
            e = hipMemcpyAsync(zi.data(), c->zt_idx, sizeof(int32_t) * nz, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && nz > 0)
            e = hipMemcpyAsync(zval.data(), c->zt_val, sizeof(double) * nz, hipMemcpyDeviceToHost, c->stream);
        const hipError_t es = hipStreamSynchronize(c->stream);
        dev_release(fl_d);
        if (e != hipSuccess || es != hipSuccess) return DPCG_EHIP;
        // the triplets of column j (its rows are increasing, so equal triplets are adjacent)
        auto triplets = [&](int j, std::vector<int32_t> &t) {
            t.clear();
            for (int32_t q = zp[j]; q < zp[j + 1]; ++q)
                if (t.empty() || t.back() != zi[q] / 3) t.push_back(zi[q] / 3);
        };
        std::vector<int32_t> tprev, tcur;
        int ngroups = 0;
        for (int j0 = 0; j0 < c->k;) {
            triplets(j0, tprev);
            int j1 = j0 + 1;
            while (j1 < c->k && j1 - j0 < kGroupCols && fk[j1]) {
                triplets(j1, tcur);
                if (tcur != tprev) break;
                ++j1;
            }
            const int kg = j1 - j0, s0 = (int)(gseg.size() / kGroupSeg);
            // dense Z block of the group: rows 3t, 3t + 1, 3t + 2 of its triplets t
            const int32_t L = 3 * (int32_t)tprev.size(), r_off = (int32_t)zr.size(), v_off = (int32_t)zv.size();
            for (int32_t t : tprev)
                for (int i = 0; i < 3; ++i) zr.push_back(3 * t + i);
            zv.resize(zv.size() + (size_t)kg * L, 0.0);
            for (int m = 0; m < kg; ++m) {
                size_t ti = 0;
                for (int32_t q = zp[j0 + m]; q < zp[j0 + m + 1]; ++q) {
                    while (tprev[ti] != zi[q] / 3) ++ti;  // both increasing; every triplet is present
                    zv[v_off + (size_t)m * L + 3 * ti + zi[q] % 3] = zval[q];
                }
            }
            for (int32_t r0 = 0; r0 < L; r0 += kGroupRows) {
                const int32_t rec[kGroupSeg] = {j0, kg, 0, r_off + r0, v_off + r0, std::min(kGroupRows, L - r0), L};
                gseg.insert(gseg.end(), rec, rec + kGroupSeg);
            }
            const int32_t e0 = kp[j0], len = kp[j0 + 1] - e0;
            for (int32_t r0 = 0; r0 < len; r0 += kGroupRows) {
                const int32_t rec[kGroupSeg] = {j0, kg, 1, e0 + r0, e0 + r0, std::min(kGroupRows, len - r0), len};
                gseg.insert(gseg.end(), rec, rec + kGroupSeg);
            }
            const int s1 = (int)(gseg.size() / kGroupSeg);
            for (int cc = j0; cc < j1; ++cc) {
                gcol[3 * cc] = s0;
                gcol[3 * cc + 1] = s1;
                gcol[3 * cc + 2] = cc - j0;
            }
            ++ngroups;
            j0 = j1;
        }
        b->grouped = c->k >= 2 * ngroups && zv.size() <= (size_t)INT32_MAX;
    }
    b->ngseg = b->grouped ? (int32_t)(gseg.size() / kGroupSeg) : 0;
    if (b->grouped) {
        BTRY(balloc(c, &b->gseg, std::max<size_t>(kGroupSeg, gseg.size())));
        BTRY(balloc(c, &b->gcol, gcol.size()));
        BTRY(balloc(c, &b->zr, std::max<size_t>(1, zr.size())));
        BTRY(balloc(c, &b->zv, std::max<size_t>(1, zv.size())));
        if (!gseg.empty())
            BHIP(hipMemcpyAsync(b->gseg, gseg.data(), sizeof(int32_t) * gseg.size(), hipMemcpyHostToDevice, c->stream));
        BHIP(hipMemcpyAsync(b->gcol, gcol.data(), sizeof(int32_t) * gcol.size(), hipMemcpyHostToDevice, c->stream));
        if (!zr.empty())
            BHIP(hipMemcpyAsync(b->zr, zr.data(), sizeof(int32_t) * zr.size(), hipMemcpyHostToDevice, c->stream));
        if (!zv.empty())
            BHIP(hipMemcpyAsync(b->zv, zv.data(), sizeof(double) * zv.size(), hipMemcpyHostToDevice, c->stream));
    }
    BTRY(balloc(c, &b->seg_part,
                std::max<size_t>((size_t)std::max(1, b->nseg) * W, (size_t)b->ngseg * kGroupCols * W)));
    if (!seg.empty()) BHIP(hipMemcpyAsync(b->seg, seg.data(), sizeof(int32_t) * seg.size(), hipMemcpyHostToDevice, c->stream));
    BHIP(hipMemcpyAsync(b->seg_ptr, sptr.data(), sizeof(int32_t) * sptr.size(), hipMemcpyHostToDevice, c->stream));
    BHIP(hipStreamSynchronize(c->stream));
    return DPCG_OK;
}

int read_bstate(dpcg_ctx *c, BatchState &out) {
    BatchWorkspace *b = c->bws;
    BHIP(hipMemcpyAsync(b->snap, b->st, sizeof(BatchState), hipMemcpyDeviceToHost, c->stream));
    BHIP(hipStreamSynchronize(c->stream));
    out = *b->snap;
    return DPCG_OK;
}

int enqueue_restrict(dpcg_ctx *c, const double *a, const double *bvec, BatchState *st, const double *part_rr, int n_rr,
                     int iter_offset, int max_iter) {
    BatchWorkspace *b = c->bws;
    if (b->grouped) {
        const int grid = ((b->ngseg + kGroupWaves - 1) / kGroupWaves + 7) & ~7;  // a multiple of 8: XCD-aware mapping
        BLAUNCH(k_brestrict_mfma, dim3(grid), dim3(64 * kGroupWaves), 0, c->stream, (const int32_t *)b->gseg, b->ngseg,
                (const int32_t *)b->zr, (const double *)b->zv, c->kzt_idx, (const double *)c->kzt_val, a, bvec,
                b->seg_part, st, part_rr, n_rr, iter_offset, max_iter);
        BLAUNCH(k_bgroupsum, dim3((c->k + 7) / 8), dim3(256), 0, c->stream, c->k, (const int32_t *)b->gcol,
                (const double *)b->seg_part, b->g, (const BatchState *)st);
        return DPCG_OK;
    }
    const int grid = std::max(8, (b->nseg + 7) & ~7);
    BLAUNCH(k_brestrict, dim3(grid), dim3(1024), 0, c->stream, (const int32_t *)b->seg, b->nseg, c->zt_idx,
            (const double *)c->zt_val, c->kzt_idx, (const double *)c->kzt_val, a, bvec, b->seg_part, st, part_rr, n_rr,
            iter_offset, max_iter);
    if (c->k > 0)
        BLAUNCH(k_bsegsum, dim3((c->k + 7) / 8), dim3(256), 0, c->stream, c->k, (const int32_t *)b->seg_ptr,
                (const double *)b->seg_part, b->g, (const BatchState *)st);
    return DPCG_OK;
}

int enqueue_coarse(dpcg_ctx *c, const BatchState *st) {
    BatchWorkspace *b = c->bws;
    if (c->k == 0) return DPCG_OK;
    BLAUNCH(k_bcoarse, dim3((c->k + 15) / 16), dim3(64 * kCoarseWaves), 0, c->stream, c->k, c->einv_ld, c->einv,
            b->g, b->delta, st);
    return DPCG_OK;
}

int enqueue_prolong(dpcg_ctx *c, const double *base, double *out, const double *rdot, BatchState *st, int advance) {
    BatchWorkspace *b = c->bws;
    BLAUNCH(k_bprolong, dim3(b->vec_nwg), dim3(256), 0, c->stream, c->n, b->vec_nwg, c->z_ptr, c->z_col, c->z_val,
            c->k > 0 ? b->delta : nullptr, base, out, rdot, b->part, st, advance);
    return DPCG_OK;
}

// Algorithm 2 for every column, then Algorithm 3 on r_0 and p_0 = z_0.
int enqueue_bstart(dpcg_ctx *c, bool guess, int max_iter) {
    BatchWorkspace *b = c->bws;
    BatchState *st = b->st;
    if (c->k > 0) {
        BTRY(enqueue_restrict(c, b->f, guess ? b->u : nullptr, nullptr, nullptr, 0, 0, 0));
        BTRY(enqueue_coarse(c, nullptr));
        BTRY(enqueue_prolong(c, guess ? b->u : nullptr, b->u, nullptr, nullptr, 0));
    }
    BLAUNCH(k_bspmm<1>, dim3(b->spmm_nwg), dim3(64 * kSpmmWaves), 0, c->stream, c->nb, c->brow_ptr, c->bcol, c->bval,
            (const int32_t *)b->pair_len, (const int32_t *)b->pair_col, (const uint16_t *)b->pair_ab,
            (const double *)b->u, (const double *)b->f, b->r, b->part2, (const BatchState *)st);
    BLAUNCH(k_bupdate_bj, dim3(b->upd_nwg), dim3(256), 0, c->stream, c->bjb_ntiles, b->upd_nwg, c->bjb_start, b->u,
            b->r, b->y, (const double *)b->q, (const double *)b->p, (const double *)c->minv, c->bj_rowoff, c->bj_meta,
            b->part, (const BatchState *)st, 0);
    BTRY(enqueue_restrict(c, b->r, b->y, st, b->part2, b->spmm_nwg, 0, max_iter));
    BTRY(enqueue_coarse(c, st));
    BTRY(enqueue_prolong(c, b->y, b->z, b->r, st, 0));
    BLAUNCH(k_bbeta, dim3(W), dim3(256), 0, c->stream, (const double *)b->part, b->vec_nwg, st);
    BLAUNCH(k_bpupdate, dim3(std::min<int64_t>(8192, (c->n + 7) / 8)), dim3(256), 0, c->stream, c->n,
            (const double *)b->z, b->p, (const BatchState *)st);
    return DPCG_OK;
}

int enqueue_biteration(dpcg_ctx *c, int max_iter, std::vector<hipEvent_t> &ev, size_t &ev_used, int32_t index) {
    BatchWorkspace *b = c->bws;
    BatchState *st = b->st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing > 0 && index % c->timing == 0) {
        if (ev_used + 2 > ev.size())
            for (int i = 0; i < 32; ++i) {
                hipEvent_t e;
                BHIP(hipEventCreate(&e));
                ev.push_back(e);
            }
        e0 = ev[ev_used];
        e1 = ev[ev_used + 1];
        ev_used += 2;
    }
    hipExtLaunchKernelGGL(k_bspmm<0>, dim3(b->spmm_nwg), dim3(64 * kSpmmWaves), 0, c->stream, e0, e1, 0, c->nb, c->brow_ptr,
                          c->bcol, (const double *)c->bval, (const int32_t *)b->pair_len,
                          (const int32_t *)b->pair_col, (const uint16_t *)b->pair_ab, (const double *)b->p,
                          (const double *)nullptr, b->q, b->part, (const BatchState *)st);
    BHIP(hipGetLastError());
    BLAUNCH(k_balpha, dim3(W), dim3(1024), 0, c->stream, (const double *)b->part, b->spmm_nwg, st);
    BLAUNCH(k_bupdate_bj, dim3(b->upd_nwg), dim3(256), 0, c->stream, c->bjb_ntiles, b->upd_nwg, c->bjb_start, b->u,
            b->r, b->y, (const double *)b->q, (const double *)b->p, (const double *)c->minv, c->bj_rowoff, c->bj_meta,
            b->part2, (const BatchState *)st, 1);
    BTRY(enqueue_restrict(c, b->r, b->y, st, b->part2, b->upd_nwg, 1, max_iter));
    BTRY(enqueue_coarse(c, st));
    BTRY(enqueue_prolong(c, b->y, b->z, b->r, st, 1));
    BLAUNCH(k_bbeta, dim3(W), dim3(256), 0, c->stream, (const double *)b->part, b->vec_nwg, st);
    BLAUNCH(k_bpupdate, dim3(std::min<int64_t>(8192, (c->n + 7) / 8)), dim3(256), 0, c->stream, c->n,
            (const double *)b->z, b->p, (const BatchState *)st);
    return DPCG_OK;
}

// ||a_j||^2 into aux (and the non-finite test of a and b when asked).
int column_norms(dpcg_ctx *c, const double *a, const double *bvec, bool check, BatchState &out) {
    BatchWorkspace *b = c->bws;
    BLAUNCH(k_bnorm, dim3(b->vec_nwg), dim3(256), 0, c->stream, c->n, b->vec_nwg, a, bvec, b->part, b->part2);
    BLAUNCH(k_baux, dim3(1), dim3(1024), 0, c->stream, (const double *)b->part, check ? (const double *)b->part2 : nullptr,
            b->vec_nwg, b->st);
    return read_bstate(c, out);
}

}  // namespace

// Y = K X for nrhs <= 32 columns (n x nrhs row-major, as in solve_batch): the columns
// packed into the batch layout, the multi-RHS product of the batched iteration
// (k_bspmm, mode 0: pairs, twin rows and single rows as there), and unpacked.
int spmv_batch(dpcg_ctx *c, int32_t nrhs, const double *X, double *Y) {
    if (!c || nrhs < 1 || nrhs > W || !X || !Y || c->ndense > 0) return DPCG_EINVAL;
    BTRY(ensure_ws(c));
    BatchWorkspace *b = c->bws;
    hipStream_t s = c->stream;
    const int pgrid = (int)std::min<int64_t>(8192, (c->n * W + 255) / 256);
    BLAUNCH(k_bpack, dim3(pgrid), dim3(256), 0, s, c->n, nrhs, X, b->p);
    BLAUNCH(k_bspmm<0>, dim3(b->spmm_nwg), dim3(64 * kSpmmWaves), 0, s, c->nb, c->brow_ptr, c->bcol, c->bval,
            (const int32_t *)b->pair_len, (const int32_t *)b->pair_col, (const uint16_t *)b->pair_ab,
            (const double *)b->p, (const double *)nullptr, b->q, b->part, (const BatchState *)nullptr);
    BLAUNCH(k_bunpack, dim3(pgrid), dim3(256), 0, s, c->n, nrhs, (const double *)b->q, Y, 0u);
    BHIP(hipStreamSynchronize(s));
    return DPCG_OK;
}

int solve_batch(dpcg_ctx *c, int32_t nrhs, const double *F, double *U, double tol, const dpcg_options *opt_in,
                dpcg_info *infos) {
    const double t0 = now_ms();
    dpcg_options opt;
    dpcg_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (!c || nrhs < 1 || nrhs > W || !F || !U || !(tol > 0.0) || opt.max_iter < 0) return DPCG_EINVAL;
    if (opt.precision != DPCG_PREC_FP64 || opt.record_history || c->ndense > 0) return DPCG_EINVAL;
    if (opt.check_every <= 0) opt.check_every = 16;
    const bool guess = opt.use_initial_guess != 0;
    BTRY(ensure_ws(c));
    BatchWorkspace *b = c->bws;
    hipStream_t s = c->stream;
    const int pgrid = (int)std::min<int64_t>(8192, (c->n * W + 255) / 256);
    BLAUNCH(k_bpack, dim3(pgrid), dim3(256), 0, s, c->n, nrhs, F, b->f);
    if (guess) BLAUNCH(k_bpack, dim3(pgrid), dim3(256), 0, s, c->n, nrhs, (const double *)U, b->u);
    else BHIP(hipMemsetAsync(b->u, 0, sizeof(double) * c->n * W, s));
    BatchState nrm;
    BTRY(column_norms(c, b->f, guess ? b->u : nullptr, true, nrm));
    if (nrm.nonfinite) return DPCG_ENONFINITE;
    BatchState init{};
    init.any = 0;
    uint32_t zero_mask = 0;
    double fnorm[W];
    for (int j = 0; j < W; ++j) {
        fnorm[j] = std::sqrt(nrm.aux[j]);
        const bool live = j < nrhs && nrm.aux[j] > 0.0;
        init.flag[j] = live ? kRunning : kConverged;
        init.thr[j] = tol * fnorm[j];
        if (live) init.any = 1;
        else if (j < nrhs) zero_mask |= 1u << j;
    }
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    BatchState st = init;
    if (init.any) {
        *b->snap = init;
        BHIP(hipMemcpyAsync(b->st, b->snap, sizeof(BatchState), hipMemcpyHostToDevice, s));
        BHIP(hipStreamSynchronize(s));
        BTRY(enqueue_bstart(c, guess, opt.max_iter));
        BTRY(read_bstate(c, st));
        int32_t enq = 0;
        while (st.any && enq < opt.max_iter) {
            const int m = std::min(opt.check_every, opt.max_iter - enq);
            for (int i = 0; i < m; ++i) BTRY(enqueue_biteration(c, opt.max_iter, ev, ev_used, enq + i));
            enq += m;
            BTRY(read_bstate(c, st));
        }
        for (int j = 0; j < W; ++j)
            if (st.flag[j] == kRunning) {  // the host-side cap ended the loop (max_iter == 0)
                st.flag[j] = kMaxIter;
                st.iters_done[j] = enq;
            }
        if (c->timing) {
            int32_t real = 0;
            for (int j = 0; j < nrhs; ++j) real = std::max(real, st.iters_done[j]);
            real = (real + c->timing - 1) / c->timing;  // timed launches of working iterations
            for (size_t i = 0; i + 1 < ev_used && (int32_t)(i / 2) < real; i += 2) {
                float ms = 0.f;
                BHIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
                c->spmv_ms += ms;
                c->spmv_launches += 1;
            }
        }
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    // true residuals f_j - K u_j
    BLAUNCH(k_bspmm<1>, dim3(b->spmm_nwg), dim3(64 * kSpmmWaves), 0, s, c->nb, c->brow_ptr, c->bcol, c->bval,
            (const int32_t *)b->pair_len, (const int32_t *)b->pair_col, (const uint16_t *)b->pair_ab,
            (const double *)b->u, (const double *)b->f, b->q, b->part2, (const BatchState *)nullptr);
    BLAUNCH(k_baux, dim3(1), dim3(1024), 0, s, (const double *)b->part2, (const double *)nullptr, b->spmm_nwg, b->st);
    BatchState fin;
    BTRY(read_bstate(c, fin));
    BLAUNCH(k_bunpack, dim3(pgrid), dim3(256), 0, s, c->n, nrhs, (const double *)b->u, U, zero_mask);
    BHIP(hipStreamSynchronize(s));
    const double ms = now_ms() - t0;
    int worst = DPCG_OK;
    for (int j = 0; j < nrhs; ++j) {
        int status;
        int64_t bad = -1;
        switch (st.flag[j]) {
            case kConverged: status = DPCG_OK; break;
            case kBreakdown: status = DPCG_EBREAKDOWN; bad = st.bad[j]; break;
            default: status = DPCG_NOT_CONVERGED; break;
        }
        const bool zero = (zero_mask >> j) & 1u;
        if (status == DPCG_EBREAKDOWN) worst = DPCG_EBREAKDOWN;
        else if (status == DPCG_NOT_CONVERGED && worst == DPCG_OK) worst = DPCG_NOT_CONVERGED;
        if (infos) {
            dpcg_info &in = infos[j];
            in.status = status;
            in.iterations = zero ? 0 : st.iters_done[j];
            in.rel_res_recursive = zero ? 0.0 : std::sqrt(st.rr[j]) / fnorm[j];
            in.rel_res_true = zero ? 0.0 : std::sqrt(fin.aux[j]) / fnorm[j];
            in.setup_ms = c->setup_ms;
            in.solve_ms = ms;
            in.bad_index = bad;
            in.refinements = 0;
            in.iterations_fp64 = in.iterations;
        }
    }
    return worst;
}

void release_batch(dpcg_ctx *c) {
    if (!c || !c->bws) return;
    if (c->bws->snap) (void)hipHostFree(c->bws->snap);
    delete c->bws;  // device arrays are in c->allocations
    c->bws = nullptr;
}

}  // namespace dpcg
