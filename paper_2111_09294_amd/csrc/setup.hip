// Setup of a dpcg handle on the GPU: every factorisation the iteration applies.
//
//   validation   CSR structure of K and Z, block partition, symmetry of K
//   block-CSR    K packed into 3x3 blocks (nine value planes)
//   block-Jacobi Cholesky and explicit inverse of each block (one wave per block)
//   Z^T          transpose of Z with rows ascending in every column
//   K Z, E       per deflation vector j: K z_j on a dense window of rows (deterministic
//                gather, no atomics on values), E[j, :] = (K z_j)^T Z
//   E^-1         block Gauss-Jordan sweeps (32 x 32 pivots), SPD check on every pivot
// All sums run in a fixed order, so a setup is bitwise reproducible.
#include <algorithm>
#include <cfloat>
#include <vector>

#include "dpcg_internal.h"

namespace dpcg {

namespace {

constexpr int kTileDofs = 239;   // block-Jacobi tile window: tiles hold <= 239 + 17 = 256 DoFs
constexpr int kNb = 32;          // Gauss-Jordan pivot block

// ---------------------------------------------------------------- small helpers
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t *lds, int64_t &total) {
    // 256 threads; lds >= 4 entries.  Returns the exclusive prefix of v, total = sum.
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    __syncthreads();
    if (lane == 63) lds[wv] = x;
    __syncthreads();
    int64_t base = 0;
    for (int w = 0; w < wv; ++w) base += lds[w];
    total = lds[0] + lds[1] + lds[2] + lds[3];
    return base + x - v;
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ double bsum(double v, double *lds) {
    v = wsum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    return (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

// ---------------------------------------------------------------- scans (int64)
constexpr int kScanChunk = 2048;

__global__ __launch_bounds__(256) void k_scan_partials(const int64_t *__restrict__ a, int64_t n,
                                                       int64_t *__restrict__ part) {
    __shared__ int64_t l64[4];
    const int64_t b = (int64_t)blockIdx.x * kScanChunk;
    int64_t s = 0;
    for (int i = threadIdx.x; i < kScanChunk; i += 256)
        if (b + i < n) s += a[b + i];
    int64_t tot;
    block_exclusive_scan(s, l64, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_top(int64_t *part, int m) {
    __shared__ int64_t l64[4];
    int64_t carry = 0;
    for (int c = 0; c < m; c += 256) {
        const int i = c + threadIdx.x;
        const int64_t v = i < m ? part[i] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_scan(v, l64, tot);
        if (i < m) part[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
}

// out[i] = exclusive prefix of a (out has n+1 entries; out[n] = total).
__global__ __launch_bounds__(256) void k_scan_apply(const int64_t *__restrict__ a, int64_t n,
                                                    const int64_t *__restrict__ part, int64_t *__restrict__ out) {
    __shared__ int64_t l64[4];
    const int64_t b = (int64_t)blockIdx.x * kScanChunk;
    int64_t carry = part[blockIdx.x];
    for (int c = 0; c < kScanChunk; c += 256) {
        const int64_t i = b + c + threadIdx.x;
        const int64_t v = i < n ? a[i] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_scan(v, l64, tot);
        if (i < n) out[i] = carry + ex;
        if (i == n - 1) out[n] = carry + ex + v;
        carry += tot;
        __syncthreads();
    }
}

__global__ void k_to_i32(const int64_t *__restrict__ a, int64_t n, int32_t *__restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (int32_t)a[i];
}

// ---------------------------------------------------------------- validation
// flags[0]: first invalid row of K (or INT_MAX), flags[1]: first invalid row of Z,
// flags[2]: first invalid block, flags[3]: first asymmetric row.
// Checks of a CSR matrix: row pointer monotone and in range, columns strictly increasing
// and in range, values finite.  Pass 1 (one thread per
// row): the row pointer, and a bit at each nonempty row's first entry.  Pass 2 (one
// thread per entry): column in range, value finite, and, unless the next entry opens a
// row, a larger column in the next entry; the failing row is found by bisection of the
// row pointer.  Optionally the per-workgroup maxima of |value| (for the symmetry
// tolerance) go to mxpart.
__global__ __launch_bounds__(256) void k_csr_rows(int64_t rows, const int64_t *__restrict__ ptr, int64_t nnz,
                                                  uint32_t *bits, int *flag) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < rows; i += (int64_t)gridDim.x * 256) {
        const int64_t a = ptr[i], b = ptr[i + 1];
        const bool ok = (i != 0 || a == 0) && a >= 0 && a <= b && b <= nnz;
        if (!ok) atomicMin(flag, (int)i);
        else if (a < b) atomicOr(&bits[a >> 5], 1u << (a & 31));
    }
}

__global__ __launch_bounds__(256) void k_csr_entries(int64_t rows, int64_t cols, const int64_t *__restrict__ ptr,
                                                     const int32_t *__restrict__ idx,
                                                     const double *__restrict__ val, int64_t nnz,
                                                     const uint32_t *__restrict__ bits, int *flag,
                                                     double *__restrict__ mxpart) {
    __shared__ double lds[4];
    double mx = 0.0;
    for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * 256) {
        const int64_t c = idx[e];
        const double v = val[e];
        bool bad = c < 0 || c >= cols || !isfinite(v);
        const int64_t n1 = e + 1;
        if (n1 < nnz && !((bits[n1 >> 5] >> (n1 & 31)) & 1u) && idx[n1] <= c) bad = true;
        mx = fmax(mx, fabs(v));
        if (bad) {
            int64_t lo = 0, hi = rows;  // last row with ptr <= e
            while (hi - lo > 1) {
                const int64_t mid = (lo + hi) >> 1;
                if (ptr[mid] <= e) lo = mid;
                else hi = mid;
            }
            atomicMin(flag, (int)lo);
        }
    }
    if (!mxpart) return;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) mxpart[blockIdx.x] = fmax(fmax(lds[0], lds[1]), fmax(lds[2], lds[3]));
}

// flag = first invalid block; maxsize = size of the largest block
__global__ void k_check_blocks(int32_t nblocks, const int32_t *__restrict__ bp, int64_t n, int *flag, int *maxsize) {
    int big = 0;
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nblocks; b += gridDim.x * blockDim.x) {
        const int64_t s = bp[b], e = bp[b + 1];
        bool ok = (b != 0 || s == 0) && (b != nblocks - 1 || e == n) && e - s >= 1 && e - s <= kMaxDense;
        if (!ok) atomicMin(flag, b);
        else big = max(big, (int)(e - s));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) big = max(big, __shfl_xor(big, off));
    if ((threadIdx.x & 63) == 0 && big > kMaxBlock) atomicMax(maxsize, big);
}

// part[0] = max over part[0..m): one workgroup, fixed order
__global__ __launch_bounds__(256) void k_max_reduce(double *part, int m) {
    __shared__ double lds[4];
    double x = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) x = fmax(x, part[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) part[0] = fmax(fmax(lds[0], lds[1]), fmax(lds[2], lds[3]));
}

// |K_ij - K_ji| <= 1e-12 max|K| over the packed 3x3 blocks, one thread per block (R, C)
// with R = brow[b].  A diagonal block is compared with its own transpose; block (R, C),
// C > R, with the transpose of block (C, R), found by binary search in block row C (a
// missing block counts as 0).  Blocks below the diagonal are only counted: when their
// number equals the number of upper blocks whose mirror was found, every lower block is
// such a mirror and has been compared; otherwise k_check_sym_lower compares the
// unpaired ones with 0.  part[2 w], part[2 w + 1]: lower blocks, found mirrors of
// workgroup w.
__device__ __forceinline__ int64_t find_block(const int32_t *__restrict__ bcol, int64_t l, int64_t h, int32_t col) {
    while (l < h) {
        const int64_t mid = (l + h) >> 1;
        if (bcol[mid] < col) l = mid + 1;
        else h = mid;
    }
    return l;
}

__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t *lds4) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) lds4[threadIdx.x >> 6] = v;
    __syncthreads();
    return (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
}

__global__ __launch_bounds__(256) void k_check_sym(const int32_t *__restrict__ bptr, const int32_t *__restrict__ brow,
                                                   const int32_t *__restrict__ bcol, const double *__restrict__ bval,
                                                   int64_t nnzb, const double *__restrict__ maxpart, int nmax, int *flag,
                                                   int64_t *__restrict__ part) {
    __shared__ int64_t lds4[4];
    double mx = 0.0;
    for (int i = 0; i < nmax; ++i) mx = fmax(mx, maxpart[i]);
    const double tol = 1e-12 * mx;
    int64_t lower = 0, found_n = 0;
    // a contiguous range of blocks per workgroup, runs of neighbouring ranges per XCD:
    // the mirrors of neighbouring rows sit side by side in the same block rows, so they
    // share the XCD's L2 lines
    const int64_t per = ((nnzb + gridDim.x - 1) / gridDim.x + 255) / 256 * 256;
    const int64_t b0 = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * per, b1 = min(nnzb, b0 + per);
    for (int64_t b = b0 + threadIdx.x; b < b1; b += 256) {
        const int32_t R = brow[b], C = bcol[b];
        if (C < R) {
            ++lower;
            continue;
        }
        const int64_t bR = bptr[R], mR = bptr[R + 1] - bR;
        double v[9];
        for (int e = 0; e < 9; ++e) v[e] = bval[9 * bR + (int64_t)e * mR + (b - bR)];
        bool ok = true;
        if (C == R) {
            for (int i = 0; i < 3; ++i)
                for (int j = i + 1; j < 3; ++j) ok = ok && fabs(v[3 * i + j] - v[3 * j + i]) <= tol;
        } else {
            const int64_t bC = bptr[C], mC = bptr[C + 1] - bC;
            const int64_t l = find_block(bcol, bC, bC + mC, R);
            const bool found = l < bC + mC && bcol[l] == R;
            found_n += found;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    const double m = found ? bval[9 * bC + (int64_t)(3 * j + i) * mC + (l - bC)] : 0.0;
                    ok = ok && fabs(v[3 * i + j] - m) <= tol;
                }
        }
        if (!ok) atomicMin(flag + 3, 3 * R);
    }
    lower = block_sum(lower, lds4);
    __syncthreads();
    found_n = block_sum(found_n, lds4);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = lower;
        part[2 * blockIdx.x + 1] = found_n;
    }
}

// need[0] = 1 when some block below the diagonal has no mirror above it
__global__ __launch_bounds__(256) void k_sym_reduce(const int64_t *__restrict__ part, int nwg, int *need) {
    __shared__ int64_t lds4[4];
    int64_t d = 0;
    for (int w = threadIdx.x; w < nwg; w += 256) d += part[2 * w] - part[2 * w + 1];
    d = block_sum(d, lds4);
    if (threadIdx.x == 0) need[0] = d != 0;
}

__global__ __launch_bounds__(256) void k_check_sym_lower(const int32_t *__restrict__ bptr,
                                                         const int32_t *__restrict__ brow,
                                                         const int32_t *__restrict__ bcol,
                                                         const double *__restrict__ bval, int64_t nnzb,
                                                         const double *__restrict__ maxpart, int nmax, int *flag,
                                                         const int *__restrict__ need) {
    if (!need[0]) return;
    double mx = 0.0;
    for (int i = 0; i < nmax; ++i) mx = fmax(mx, maxpart[i]);
    const double tol = 1e-12 * mx;
    for (int64_t b = blockIdx.x * 256ll + threadIdx.x; b < nnzb; b += (int64_t)gridDim.x * 256) {
        const int32_t R = brow[b], C = bcol[b];
        if (C >= R) continue;
        const int64_t bC = bptr[C], mC = bptr[C + 1] - bC;
        const int64_t l = find_block(bcol, bC, bC + mC, R);
        if (l < bC + mC && bcol[l] == R) continue;
        const int64_t bR = bptr[R], mR = bptr[R + 1] - bR;
        bool ok = true;
        for (int e = 0; e < 9; ++e) ok = ok && fabs(bval[9 * bR + (int64_t)e * mR + (b - bR)]) <= tol;
        if (!ok) atomicMin(flag + 3, 3 * R);
    }
}

// ---------------------------------------------------------------- block-CSR over DoF triplets
// Block columns of block row R: the union of col/3 over scalar rows 3R..3R+2.  One
// wave per block row.  When the three rows have the same set of block columns (a K
// assembled from 3x3 nodal blocks always does), a block's position is the rank of its
// block column among the row's distinct block columns, found with ballots; otherwise
// lane 0 merges the three rows.
constexpr int kMaxDistinct = 256;

__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

// distinct block columns of one scalar row, ranks from ballots; returns the count
__device__ int row_distinct(int64_t a, int64_t e, const int32_t *__restrict__ idx, int32_t *dcol) {
    const int lane = threadIdx.x & 63;
    int count = 0;
    for (int64_t base = a; base < e; base += 64) {
        const int64_t p = base + lane;
        const bool in = p < e;
        const int32_t c = in ? idx[p] / 3 : -1;
        const bool first = in && (p == a || idx[p - 1] / 3 != c);
        const unsigned long long bal = __ballot(first);
        const int rank = count + __popcll(bal & ((1ull << lane) - 1ull));
        if (first && rank < kMaxDistinct) dcol[rank] = c;
        count += __popcll(bal);
    }
    return count;
}

// Block-CSR of K, one wave per block row R (its scalar rows 3R, 3R+1, 3R+2).  FILL false:
// the number of distinct block columns; FILL true: block columns, block rows and the nine
// value planes.  Rows of at most 128 entries each (nearly all) are read once, all three
// rows' loads in one round, and ranked from registers with ballots; longer rows are ranked
// chunk by chunk from memory.  Rows whose three scalar rows do not share one block-column
// set take the serial merge of lane 0.
template <bool FILL>
__global__ __launch_bounds__(256) void k_bsr(int32_t nb, const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                             const double *__restrict__ val, int64_t *__restrict__ cnt,
                                             const int32_t *__restrict__ bptr, int32_t *__restrict__ bcol,
                                             double *__restrict__ bval, int32_t *__restrict__ brow) {
    __shared__ int32_t dcol_s[4][3][kMaxDistinct];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int64_t R = blockIdx.x * 4ll + wv; R < nb; R += (int64_t)gridDim.x * 4) {
        int64_t a[3], e[3];
        for (int i = 0; i < 3; ++i) {
            a[i] = ptr[3 * R + i];
            e[i] = ptr[3 * R + i + 1];
        }
        const bool small = e[0] - a[0] <= 128 && e[1] - a[1] <= 128 && e[2] - a[2] <= 128;
        int dn[3];
        unsigned long long bal[3][2] = {{0ull, 0ull}, {0ull, 0ull}, {0ull, 0ull}};
        double cv[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
        int32_t ci[3][2];
        if (small) {
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int64_t p = a[i] + 64 * c + lane;
                    const bool in = p < e[i];
                    ci[i][c] = in ? idx[p] : -3;
                    if (FILL) cv[i][c] = in ? val[p] : 0.0;
                }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                int count = 0;
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int32_t cur = ci[i][c];
                    // the previous entry of the row: lane - 1 of this chunk, or lane 63 of the last
                    int32_t prev = __shfl_up(cur, 1);
                    const int32_t last = __shfl(ci[i][0], 63);
                    if (lane == 0) prev = c == 0 ? -3 : last;
                    const bool in = a[i] + 64 * c + lane < e[i];
                    const bool first = in && (prev < 0 || prev / 3 != cur / 3);
                    bal[i][c] = __ballot(first);
                    const int rank = count + __popcll(bal[i][c] & below);
                    if (first && rank < kMaxDistinct) dcol_s[wv][i][rank] = cur / 3;
                    count += __popcll(bal[i][c]);
                }
                dn[i] = count;
            }
        } else {
            for (int i = 0; i < 3; ++i) dn[i] = row_distinct(a[i], e[i], idx, dcol_s[wv][i]);
        }
        wave_sync();
        bool same = dn[0] == dn[1] && dn[1] == dn[2] && dn[0] <= kMaxDistinct;
        if (same)
            for (int t = lane; t < dn[0]; t += 64)
                if (dcol_s[wv][0][t] != dcol_s[wv][1][t] || dcol_s[wv][0][t] != dcol_s[wv][2][t]) same = false;
        same = __ballot(!same) == 0ull;
        if (same) {
            if (!FILL) {
                if (lane == 0) cnt[R] = dn[0];
            } else {
                const int64_t beg = bptr[R], m = dn[0];
                for (int t = lane; t < m; t += 64) {
                    bcol[beg + t] = dcol_s[wv][0][t];
                    brow[beg + t] = (int32_t)R;
                }
                if (small) {
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        int count = 0;
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            // rank of the entry's block column: first entries up to and including it, minus 1
                            const int rank = count + __popcll(bal[i][c] & (below | (1ull << lane))) - 1;
                            if (a[i] + 64 * c + lane < e[i])
                                bval[9 * beg + (int64_t)(3 * i + ci[i][c] % 3) * m + rank] = cv[i][c];
                            count += __popcll(bal[i][c]);
                        }
                    }
                } else {
                    for (int i = 0; i < 3; ++i) {
                        int count = 0;
                        for (int64_t base = a[i]; base < e[i]; base += 64) {
                            const int64_t p = base + lane;
                            const bool in = p < e[i];
                            const int32_t c = in ? idx[p] : 0;
                            const bool first = in && (p == a[i] || idx[p - 1] / 3 != c / 3);
                            const unsigned long long bl = __ballot(first);
                            const int rank = count + __popcll(bl & ((2ull << lane) - 1ull)) - 1;
                            if (in) bval[9 * beg + (int64_t)(3 * i + c % 3) * m + rank] = val[p];
                            count += __popcll(bl);
                        }
                    }
                }
            }
        } else if (lane == 0) {
            int64_t h[3] = {a[0], a[1], a[2]};
            const int64_t beg = FILL ? bptr[R] : 0, m = FILL ? (int64_t)bptr[R + 1] - bptr[R] : 0;
            int64_t pos = beg, count = 0;
            while (true) {
                int32_t cur = INT32_MAX;
                for (int i = 0; i < 3; ++i)
                    if (h[i] < e[i]) cur = min(cur, idx[h[i]] / 3);
                if (cur == INT32_MAX) break;
                if (FILL) {
                    bcol[pos] = cur;
                    brow[pos] = (int32_t)R;
                }
                for (int i = 0; i < 3; ++i)
                    while (h[i] < e[i] && idx[h[i]] / 3 == cur) {
                        if (FILL) bval[9 * beg + (int64_t)(3 * i + idx[h[i]] % 3) * m + (pos - beg)] = val[h[i]];
                        ++h[i];
                    }
                ++pos;
                ++count;
            }
            if (!FILL) cnt[R] = count;
        }
        wave_sync();
    }
}

// ---------------------------------------------------------------- block-Jacobi
__global__ void k_block_sq(int32_t nblocks, const int32_t *__restrict__ bp, int64_t *__restrict__ sq) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nblocks; b += gridDim.x * blockDim.x) {
        const int64_t m = bp[b + 1] - bp[b];
        sq[b] = m <= kMaxBlock ? m * m : 0;  // larger blocks keep dense inverses of their own
    }
}

// Block-Jacobi inverses: Cholesky with the pivot test m * DBL_EPSILON * |original
// diagonal entry|, then the explicit inverse L^-T L^-1, in the operation order of a
// sequential column algorithm.  Blocks of up to kSmallBlock DoFs take one thread each
// (register arrays, every index a compile-time constant); larger blocks one wave each.
constexpr int kSmallBlock = 6;

// list (may be null): factorise only the nlist blocks list[0..nlist) instead of all.
__global__ __launch_bounds__(256) void k_bj_small(int32_t nblocks, const int32_t *__restrict__ bp,
                                                  const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                                  const double *__restrict__ val, const int64_t *__restrict__ moff,
                                                  double *__restrict__ minv, int32_t *__restrict__ rowoff,
                                                  int32_t *__restrict__ meta, int *bad_block,
                                                  const int32_t *__restrict__ list, int32_t nlist) {
    constexpr int M = kSmallBlock;
    const int count = list ? nlist : nblocks;
    for (int ib = blockIdx.x * blockDim.x + threadIdx.x; ib < count; ib += gridDim.x * blockDim.x) {
        const int b = list ? list[ib] : ib;
        const int32_t s = bp[b];
        const int m = bp[b + 1] - s;
        if (m > M) continue;
        double A[M][M], Li[M][M];
#pragma unroll
        for (int i = 0; i < M; ++i) {
#pragma unroll
            for (int j = 0; j < M; ++j) A[i][j] = 0.0;
            if (i < m) {
                // first entry of the row with column >= s (columns are sorted)
                int64_t lo = ptr[s + i], hi = ptr[s + i + 1];
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (idx[mid] < s) lo = mid + 1;
                    else hi = mid;
                }
                const int64_t end = ptr[s + i + 1];
#pragma unroll
                for (int j = 0; j < M; ++j)
                    if (j < m && lo < end && idx[lo] == s + j) {
                        A[i][j] = val[lo];
                        ++lo;
                    }
            }
        }
        bool ok = true;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if (j >= m) continue;
            double d = A[j][j];
            const double fl = m * DBL_EPSILON * fabs(d);
#pragma unroll
            for (int p = 0; p < j; ++p) d -= A[j][p] * A[j][p];
            if (!(d > fl) || !isfinite(d)) ok = false;
            const double l = sqrt(d > 0.0 ? d : 1.0);
            A[j][j] = l;
#pragma unroll
            for (int i = j + 1; i < M; ++i) {
                if (i >= m) continue;
                double sacc = A[i][j];
#pragma unroll
                for (int p = 0; p < j; ++p) sacc -= A[i][p] * A[j][p];
                A[i][j] = sacc / l;
            }
        }
        if (!ok) {
            atomicMin(bad_block, b);
            continue;
        }
#pragma unroll
        for (int j = 0; j < M; ++j)
#pragma unroll
            for (int i = 0; i < M; ++i) {
                if (i < j || i >= m || j >= m) {
                    Li[i][j] = 0.0;
                    continue;
                }
                double sacc = (i == j) ? 1.0 : 0.0;
#pragma unroll
                for (int p = j; p < i; ++p) sacc -= A[i][p] * Li[p][j];
                Li[i][j] = sacc / A[i][i];
            }
        double *out = minv + moff[b];
#pragma unroll
        for (int i = 0; i < M; ++i) {
            if (i >= m) continue;
#pragma unroll
            for (int j = i; j < M; ++j) {
                if (j >= m) continue;
                double sacc = 0.0;
#pragma unroll
                for (int p = j; p < M; ++p)
                    if (p < m) sacc += Li[p][i] * Li[p][j];
                out[i * m + j] = sacc;
                out[j * m + i] = sacc;
            }
            rowoff[s + i] = (int32_t)(moff[b] + (int64_t)i * m);
            meta[s + i] = (m << 8) | i;
        }
    }
}

__global__ __launch_bounds__(64) void k_bj_factor(int32_t nblocks, const int32_t *__restrict__ bp,
                                                  const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                                  const double *__restrict__ val, const int64_t *__restrict__ moff,
                                                  double *__restrict__ minv, int32_t *__restrict__ rowoff,
                                                  int32_t *__restrict__ meta, int *bad_block,
                                                  const int32_t *__restrict__ list, int32_t nlist) {
    __shared__ double A[kMaxBlock * kMaxBlock];
    __shared__ double Li[kMaxBlock * kMaxBlock];
    __shared__ int fail;
    const int lane = threadIdx.x;
    const int count = list ? nlist : nblocks;
    for (int ib = blockIdx.x; ib < count; ib += gridDim.x) {
        const int b = list ? list[ib] : ib;
        const int32_t s = bp[b];
        const int m = bp[b + 1] - s;
        if (m <= kSmallBlock || m > kMaxBlock) continue;
        __syncthreads();
        for (int t = lane; t < m * m; t += 64) A[t] = 0.0;
        if (lane == 0) fail = 0;
        __syncthreads();
        if (lane < m) {
            // the row's entries in columns [s, s + m) follow its first column >= s
            int64_t lo = ptr[s + lane], hi = ptr[s + lane + 1];
            const int64_t end = hi;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (idx[mid] < s) lo = mid + 1;
                else hi = mid;
            }
#pragma unroll
            for (int q = 0; q < kMaxBlock; ++q) {
                const int64_t e = lo + q;
                if (q < m && e < end) {
                    const int32_t c = idx[e];
                    if (c < s + m) A[lane * m + (c - s)] = val[e];
                }
            }
        }
        __syncthreads();
        for (int j = 0; j < m; ++j) {
            if (lane == 0) {
                double d = A[j * m + j];
                const double fl = m * DBL_EPSILON * fabs(d);
                for (int p = 0; p < j; ++p) d -= A[j * m + p] * A[j * m + p];
                if (!(d > fl) || !isfinite(d)) fail = 1;
                else A[j * m + j] = sqrt(d);
            }
            __syncthreads();
            if (fail) break;
            const double l = A[j * m + j];
            if (lane > j && lane < m) {
                double sacc = A[lane * m + j];
                for (int p = 0; p < j; ++p) sacc -= A[lane * m + p] * A[j * m + p];
                A[lane * m + j] = sacc / l;
            }
            __syncthreads();
        }
        if (fail) {
            if (lane == 0) atomicMin(bad_block, b);
            continue;
        }
        // column j of L^-1 (lane j), rows i >= j
        if (lane < m) {
            const int j = lane;
            for (int i = 0; i < m; ++i) {
                if (i < j) {
                    Li[i * m + j] = 0.0;
                    continue;
                }
                double sacc = (i == j) ? 1.0 : 0.0;
                for (int p = j; p < i; ++p) sacc -= A[i * m + p] * Li[p * m + j];
                Li[i * m + j] = sacc / A[i * m + i];
            }
        }
        __syncthreads();
        double *out = minv + moff[b];
        if (lane < m) {
            const int i = lane;
            for (int j = i; j < m; ++j) {
                double sacc = 0.0;
                for (int p = j; p < m; ++p) sacc += Li[p * m + i] * Li[p * m + j];
                out[i * m + j] = sacc;
                out[j * m + i] = sacc;
            }
            rowoff[s + i] = (int32_t)(moff[b] + (int64_t)i * m);
            meta[s + i] = (m << 8) | i;
        }
    }
}

// tile t = blocks starting in [t * window, (t+1) * window); start = first such block,
// or t * window itself when that DoF lies inside a block of more than kMaxBlock DoFs
// (their rows need no neighbours in the tile), so a tile holds < window + kMaxBlock DoFs.
// One thread per block b <= nblocks (bp[nblocks] = n): the targets t * window in
// (bp[b-1], bp[b]] have b as their first block starting at or after the target, so b
// writes those tiles (usually none or one) and no thread searches.
__global__ void k_tiles(int32_t ntiles, int32_t nblocks, const int32_t *__restrict__ bp, int64_t n,
                        int32_t window, int32_t *__restrict__ tile_start) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= nblocks; b += gridDim.x * blockDim.x) {
        const int64_t hi = bp[b];
        const int64_t t0 = b == 0 ? 0 : (int64_t)bp[b - 1] / window + 1;
        const int64_t t1 = min<int64_t>(ntiles - 1, hi / window);
        const bool split = b > 0 && hi - bp[b - 1] > kMaxBlock;  // the target lies inside block b - 1
        for (int64_t t = t0; t <= t1; ++t) tile_start[t] = split ? (int32_t)(t * window) : (int32_t)hi;
        if (b == nblocks) tile_start[ntiles] = (int32_t)n;
    }
}

// Block columns as offsets from their block row in 16 bits (the iteration SpMV reads 2
// bytes per block instead of 4); *bad becomes 1 when an offset does not fit.
__global__ void k_bcol16(int64_t nnzb, const int32_t *__restrict__ brow, const int32_t *__restrict__ bcol,
                         int16_t *__restrict__ out, int *bad) {
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nnzb; b += (int64_t)gridDim.x * blockDim.x) {
        const int32_t d = bcol[b] - brow[b];
        const bool fits = d >= INT16_MIN && d <= INT16_MAX;
        out[b] = fits ? (int16_t)d : (int16_t)0;
        if (!fits) *bad = 1;
    }
}

// ---------------------------------------------------------------- Z^T
// Z^T by a stable counting sort over chunks of Z's entries in row-major order.  Pass 1
// counts each chunk's entries per column into cnt[c * nch + w]; an exclusive scan in
// (column, chunk) order gives every (column, chunk) pair its first slot; pass 2 walks a
// chunk's entries in order with one wave and places them, so every column of Z^T lists
// its rows in increasing order without atomics on global memory.  Columns go in ranges
// of kZtCols (LDS tables), one grid row per range.
constexpr int kZtCols = 8192;

__global__ void k_entry_rows(int64_t rows, const int64_t *__restrict__ ptr, int32_t *__restrict__ erow) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x)
        for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) erow[e] = (int32_t)r;
}

__global__ __launch_bounds__(256) void k_zt_count(int64_t nnz, int64_t per, int nch, int32_t k,
                                                  const int32_t *__restrict__ idx, int64_t *__restrict__ cnt) {
    extern __shared__ int32_t hist[];
    const int w = blockIdx.x;
    const int32_t c0 = blockIdx.y * kZtCols, nc = min(kZtCols, k - c0);
    for (int t = threadIdx.x; t < nc; t += 256) hist[t] = 0;
    __syncthreads();
    const int64_t e0 = (int64_t)w * per, e1 = min(nnz, e0 + per);
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
        const int32_t c = idx[e] - c0;
        if (c >= 0 && c < nc) atomicAdd(&hist[c], 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nc; t += 256) cnt[(int64_t)(c0 + t) * nch + w] = hist[t];
}

__global__ void k_zt_ptr(int32_t k, int nch, const int64_t *__restrict__ off, int64_t *__restrict__ ztp) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c <= k; c += (int64_t)gridDim.x * blockDim.x)
        ztp[c] = off[c * nch];
}

__global__ __launch_bounds__(64) void k_zt_place(int64_t nnz, int64_t per, int nch, int32_t k,
                                                 const int32_t *__restrict__ idx, const double *__restrict__ val,
                                                 const int32_t *__restrict__ erow, const int64_t *__restrict__ off,
                                                 int32_t *__restrict__ zti, double *__restrict__ ztv) {
    extern __shared__ int64_t run[];
    const int w = blockIdx.x, lane = threadIdx.x;
    const int32_t c0 = blockIdx.y * kZtCols, nc = min(kZtCols, k - c0);
    for (int t = lane; t < nc; t += 64) run[t] = off[(int64_t)(c0 + t) * nch + w];
    __syncthreads();
    const int64_t e0 = (int64_t)w * per, e1 = min(nnz, e0 + per);
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int64_t base = e0; base < e1; base += 64) {
        const int64_t e = base + lane;
        const int32_t c = e < e1 ? idx[e] - c0 : -1;
        const bool mine = c >= 0 && c < nc;
        unsigned long long todo = __ballot(mine);
        // one distinct column per step: its lanes take consecutive slots in lane order
        while (todo) {
            const int leader = __builtin_ctzll(todo);
            const int32_t cl = __shfl(c, leader);
            const unsigned long long grp = __ballot(mine && c == cl);
            const int64_t b = run[cl];
            if (mine && c == cl) {
                const int64_t q = b + __popcll(grp & lt);
                zti[q] = erow[e];
                ztv[q] = val[e];
            }
            if (lane == leader) run[cl] = b + __popcll(grp);
            todo &= ~grp;
        }
    }
}

// ---------------------------------------------------------------- K Z and E
// Row window of K z_j: [first column of K over the rows of z_j, last column].
__global__ __launch_bounds__(256) void k_kz_window(int32_t k, const int64_t *__restrict__ ztp,
                                                   const int32_t *__restrict__ zti, const int64_t *__restrict__ kp,
                                                   const int32_t *__restrict__ kc, int64_t *__restrict__ wlo,
                                                   int64_t *__restrict__ wsize) {
    __shared__ int64_t lo_s[4], hi_s[4];
    const int j = blockIdx.x;
    if (j >= k) return;
    int64_t lo = INT64_MAX, hi = -1;
    for (int64_t e = ztp[j] + threadIdx.x; e < ztp[j + 1]; e += 256) {
        const int64_t r = zti[e];
        if (kp[r + 1] > kp[r]) {
            lo = min<int64_t>(lo, kc[kp[r]]);
            hi = max<int64_t>(hi, kc[kp[r + 1] - 1]);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = min<int64_t>(lo, __shfl_xor(lo, off));
        hi = max<int64_t>(hi, __shfl_xor(hi, off));
    }
    if ((threadIdx.x & 63) == 0) {
        lo_s[threadIdx.x >> 6] = lo;
        hi_s[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        lo = min(min(lo_s[0], lo_s[1]), min(lo_s[2], lo_s[3]));
        hi = max(max(hi_s[0], hi_s[1]), max(hi_s[2], hi_s[3]));
        wlo[j] = hi >= lo ? lo : 0;
        wsize[j] = hi >= lo ? hi - lo + 1 : 0;
    }
}

// ---- K Z and E in batches of kBatch consecutive deflation vectors ----
// A batch owns the union window of its vectors' rows in whole DoF triplets
// [lo3, lo3 + w3).  Per scalar row t of the window (t = row - 3 lo3): zd[t][b] =
// Z[row, j0+b] and kd[t][b] = (K z_{j0+b})_row.  Per triplet T: rb[T] = vectors with a
// nonzero in triplet lo3 + T, mk[T] = vectors whose K z_j has that triplet in its block
// structure (coupled by a 3x3 block of K to a triplet of z_j).  K z_j is evaluated on
// the packed 3x3 blocks; a structure triplet contributes its three rows.  Windows are
// processed in slices of kSlice triplets, one workgroup per (slice, batch).
constexpr int kBatch = 16;
constexpr int kSlice = 1024;
constexpr int kTouchLds = 2048;  // LDS words of the touched-vector bitmap (k <= 65536)

struct KzBatch {
    int64_t j0, ncol, lo3, w3, off3, slice0, nslice, bit0;
    int64_t moff;  // first triplet of the batch's window in the structure masks mk and rb
};

// clears the batch's touched bits and, when masks, its structure masks
__global__ __launch_bounds__(256) void k_kzb_init(const KzBatch *__restrict__ bt, int words, uint32_t *__restrict__ mk,
                                                  uint32_t *__restrict__ rb, uint32_t *__restrict__ touched,
                                                  int masks) {
    const KzBatch B = bt[blockIdx.y];
    if (blockIdx.x >= B.nslice) return;
    const int64_t t0 = (int64_t)blockIdx.x * kSlice, t1 = min<int64_t>(B.w3, t0 + kSlice);
    for (int64_t t = t0 + threadIdx.x; t < t1; t += 256) {
        if (masks) {
            mk[B.moff + t] = 0u;
            rb[B.moff + t] = 0u;
        }
    }
    if (blockIdx.x == 0)
        for (int t = threadIdx.x; t < words; t += 256) touched[B.bit0 + t] = 0u;
}

// one workgroup per (vector, batch): scatter z_j and flag its triplets.  The three rows
// of each flagged triplet are cleared first (column b belongs to this workgroup), so zd
// holds z_j exactly where rb flags vector b and is never read elsewhere.
__global__ __launch_bounds__(256) void k_kzb_scatter(const KzBatch *__restrict__ bt, const int64_t *__restrict__ ztp,
                                                     const int32_t *__restrict__ zti, const double *__restrict__ ztv,
                                                     double *__restrict__ zd, uint32_t *rb) {
    const KzBatch B = bt[blockIdx.y];
    const int b = blockIdx.x;
    if (b >= B.ncol) return;
    const int64_t j = B.j0 + b;
    for (int64_t e = ztp[j] + threadIdx.x; e < ztp[j + 1]; e += 256) {
        const int64_t t = (int64_t)zti[e] - 3 * B.lo3;
        if (t < 0 || t >= 3 * B.w3) continue;
        const int64_t t3 = 3 * (t / 3);
        for (int r = 0; r < 3; ++r) zd[(3 * B.off3 + t3 + r) * kBatch + b] = 0.0;
    }
    __syncthreads();
    for (int64_t e = ztp[j] + threadIdx.x; e < ztp[j + 1]; e += 256) {
        const int64_t t = (int64_t)zti[e] - 3 * B.lo3;
        if (t < 0 || t >= 3 * B.w3) continue;
        zd[(3 * B.off3 + t) * kBatch + b] = ztv[e];
        atomicOr(&rb[B.moff + t / 3], 1u << b);
    }
}

// block structure of K z_j: every block column of the block rows of z_j's triplets.  A
// workgroup ORs the bits of its slice's block rows into an LDS window of the columns
// around the slice (kMarkHalo triplets on either side) and then ORs each nonzero window
// word into mk once; a column outside the window goes to mk directly.  Slices without a
// flagged triplet return at once.
constexpr int kMarkHalo = 7680;
constexpr int kMarkWindow = kSlice + 2 * kMarkHalo;  // 16384 words, 64 KB of LDS
constexpr int kMarkRun = 16;  // block columns of a row loaded together

__global__ __launch_bounds__(256) void k_kzb_mark(const KzBatch *__restrict__ bt, const int32_t *__restrict__ bptr,
                                                  const int32_t *__restrict__ bcol, const uint32_t *__restrict__ rb,
                                                  uint32_t *mk) {
    __shared__ uint32_t win[kMarkWindow];
    const KzBatch B = bt[blockIdx.y];
    if (blockIdx.x >= B.nslice) return;
    const int64_t t0 = (int64_t)blockIdx.x * kSlice, t1 = min<int64_t>(B.w3, t0 + kSlice);
    bool any = false;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += 256) any = any || rb[B.moff + t] != 0u;
    if (!__syncthreads_or(any)) return;
    for (int i = threadIdx.x; i < kMarkWindow; i += 256) win[i] = 0u;
    __syncthreads();
    const int64_t w0 = t0 - kMarkHalo;  // window column of win[0] (may be negative)
    for (int64_t t = t0 + threadIdx.x; t < t1; t += 256) {
        const uint32_t bits = rb[B.moff + t];
        if (!bits) continue;
        const int64_t R = B.lo3 + t;
        const int64_t q0 = bptr[R], q1 = bptr[R + 1];
        for (int64_t q = q0; q < q1; q += kMarkRun) {
            // a run of block columns loaded together, then their marks
            int32_t cr[kMarkRun];
#pragma unroll
            for (int u = 0; u < kMarkRun; ++u) cr[u] = q + u < q1 ? bcol[q + u] : -1;
#pragma unroll
            for (int u = 0; u < kMarkRun; ++u) {
                if (cr[u] < 0) continue;
                const int64_t c = (int64_t)cr[u] - B.lo3;
                if (c < 0 || c >= B.w3) continue;
                const int64_t l = c - w0;
                if (l >= 0 && l < kMarkWindow) atomicOr(&win[l], bits);
                else atomicOr(&mk[B.moff + c], bits);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kMarkWindow; i += 256) {
        const uint32_t v = win[i];
        const int64_t c = w0 + i;
        if (v && c >= 0 && c < B.w3) atomicOr(&mk[B.moff + c], v);
    }
}

// per (slice, vector) counts of structure rows (three per structure triplet), and per
// slice the number of structure triplets (work items)
__global__ __launch_bounds__(256) void k_kzb_count(const KzBatch *__restrict__ bt, const uint32_t *__restrict__ mk,
                                                   int32_t *__restrict__ cnt, int32_t *__restrict__ tcnt) {
    __shared__ int32_t c_s[kBatch + 1];
    const KzBatch B = bt[blockIdx.y];
    if (blockIdx.x >= B.nslice) return;
    if (threadIdx.x <= kBatch) c_s[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kSlice, t1 = min<int64_t>(B.w3, t0 + kSlice);
    int32_t mine[kBatch + 1];
    for (int b = 0; b <= kBatch; ++b) mine[b] = 0;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += 256) {
        const uint32_t m = mk[B.moff + t];
        for (int b = 0; b < kBatch; ++b) mine[b] += 3 * ((m >> b) & 1u);
        mine[kBatch] += m != 0u;
    }
    for (int b = 0; b <= kBatch; ++b)
        if (mine[b]) atomicAdd(&c_s[b], mine[b]);
    __syncthreads();
    if (threadIdx.x < kBatch) cnt[(B.slice0 + blockIdx.x) * kBatch + threadIdx.x] = c_s[threadIdx.x];
    if (threadIdx.x == kBatch) tcnt[B.slice0 + blockIdx.x] = c_s[kBatch];
}

// Per batch (kBatch + 1 threads): thread b < ncol forms the slice offsets within vector
// b's structure and the vector's total; thread kBatch forms each slice's first work item
// (exclusive prefix of the triplet counts) and the batch's number of items.
__global__ void k_kzb_offsets(const KzBatch *__restrict__ bt, int nbat, const int32_t *__restrict__ cnt,
                              const int32_t *__restrict__ tcnt, int32_t *__restrict__ soff,
                              int64_t *__restrict__ kzcnt, int32_t *__restrict__ icnt, int64_t *__restrict__ nitems) {
    const int bi = blockIdx.x;
    if (bi >= nbat) return;
    const KzBatch B = bt[bi];
    const int b = threadIdx.x;
    int64_t run = 0;
    if (b == kBatch) {
        for (int64_t sl = 0; sl < B.nslice; ++sl) {
            icnt[B.slice0 + sl] = (int32_t)run;
            run += tcnt[B.slice0 + sl];
        }
        nitems[bi] = run;
        return;
    }
    if (b >= B.ncol) return;
    for (int64_t sl = 0; sl < B.nslice; ++sl) {
        soff[(B.slice0 + sl) * kBatch + b] = (int32_t)run;
        run += cnt[(B.slice0 + sl) * kBatch + b];
    }
    kzcnt[B.j0 + b] = run;
}

// Rank pass: every structure triplet of the slice gets a work item (its triplet, its
// mask of vectors, and for each vector its output position in (KZ)^T), stored densely
// per batch in slice order.
struct KzItem {
    int32_t t, mask;
    int32_t pos[kBatch];
};

__global__ __launch_bounds__(256) void k_kzb_rank(const KzBatch *__restrict__ bt, const uint32_t *__restrict__ mk,
                                                  const int32_t *__restrict__ soff, const int32_t *__restrict__ icnt,
                                                  const int64_t *__restrict__ kzp, KzItem *__restrict__ items) {
    __shared__ int32_t wave_cnt[4][kBatch + 1];
    __shared__ int32_t carry[kBatch + 1];
    const KzBatch B = bt[blockIdx.y];
    if (blockIdx.x >= B.nslice) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x <= kBatch) carry[threadIdx.x] = 0;
    __syncthreads();
    // items of this slice start after the items of the batch's earlier slices
    const int64_t item0 = B.off3 + icnt[B.slice0 + blockIdx.x];
    const int64_t t0 = (int64_t)blockIdx.x * kSlice, t1 = min<int64_t>(B.w3, t0 + kSlice);
    for (int64_t c0 = t0; c0 < t1; c0 += 256) {
        const int64_t t = c0 + threadIdx.x;
        const uint32_t m = t < t1 ? mk[B.moff + t] : 0u;
        int32_t rank[kBatch + 1];
        for (int b = 0; b <= kBatch; ++b) {
            const bool f = b < kBatch ? ((m >> b) & 1u) : (m != 0u);
            const unsigned long long bal = __ballot(f);
            rank[b] = __popcll(bal & ((1ull << lane) - 1ull));
            if (lane == 0) wave_cnt[wv][b] = __popcll(bal);
        }
        __syncthreads();
        if (m) {
            int32_t before[kBatch + 1];
            for (int b = 0; b <= kBatch; ++b) {
                before[b] = carry[b];
                for (int w2 = 0; w2 < wv; ++w2) before[b] += wave_cnt[w2][b];
            }
            KzItem it;
            it.t = (int32_t)t;
            it.mask = (int32_t)m;
            for (int b = 0; b < kBatch; ++b)
                it.pos[b] = (b < B.ncol && ((m >> b) & 1u))
                                ? (int32_t)(kzp[B.j0 + b] + soff[(B.slice0 + blockIdx.x) * kBatch + b] +
                                            3 * (before[b] + rank[b]))
                                : -1;
            items[item0 + before[kBatch] + rank[kBatch]] = it;
        }
        __syncthreads();
        if (threadIdx.x <= kBatch)
            carry[threadIdx.x] += wave_cnt[0][threadIdx.x] + wave_cnt[1][threadIdx.x] + wave_cnt[2][threadIdx.x] +
                                  wave_cnt[3][threadIdx.x];
        __syncthreads();
    }
}

// Compute pass: (K z_j) on the three rows of each structure triplet from the packed 3x3
// blocks.  Sixteen lanes per work item: lane bits 0-1 pick four of the batch's vectors,
// bits 2-3 a quarter of the block row's blocks; the quarters are combined by a fixed
// shuffle tree.  Writes (KZ)^T at the ranked positions, the dense kd, and flags the
// deflation vectors with a nonzero in a structure row as touched.
__global__ __launch_bounds__(256) void k_kzb_values(const KzBatch *__restrict__ bt, const int64_t *__restrict__ nitems,
                                                    const KzItem *__restrict__ items, const int32_t *__restrict__ bptr,
                                                    const int32_t *__restrict__ bcol, const double *__restrict__ bval,
                                                    const double *__restrict__ zd, const uint32_t *__restrict__ rb,
                                                    const int64_t *__restrict__ zp,
                                                    const int32_t *__restrict__ zc, int32_t *__restrict__ kzi,
                                                    double *__restrict__ kzv, double *__restrict__ kd,
                                                    int words, uint32_t *touched) {
    __shared__ uint32_t tw[kTouchLds];
    const KzBatch B = bt[blockIdx.y];
    const int64_t n_it = nitems[blockIdx.y];
    const int sub = threadIdx.x & 3, part = (threadIdx.x >> 2) & 3;
    const bool lds_bits = words <= kTouchLds;
    if (lds_bits)
        for (int t = threadIdx.x; t < words; t += 256) tw[t] = 0u;
    __syncthreads();
    uint32_t *tb = lds_bits ? tw : touched + B.bit0;
    // a contiguous run of items per workgroup (neighbouring triplets, few deflation
    // vectors); the loop bound is uniform over the workgroup, so the shuffles stay in step
    const int64_t per = ((n_it + gridDim.x - 1) / gridDim.x + 15) / 16 * 16;
    const int64_t x0 = (int64_t)blockIdx.x * per, x1 = min(n_it, x0 + per);
    for (int64_t x = x0 + (threadIdx.x >> 4); x - (threadIdx.x >> 4) < x1; x += 16) {
        const bool live = x < x1;
        double acc[3][4];
        for (int i = 0; i < 3; ++i)
            for (int b = 0; b < 4; ++b) acc[i][b] = 0.0;
        int64_t t = 0, R = 0;
        if (live) {
            t = items[B.off3 + x].t;
            R = B.lo3 + t;
            const int64_t beg = bptr[R], mR = bptr[R + 1] - beg;
            const double *rv = bval + 9 * beg;
            for (int64_t q = beg + part; q < beg + mR; q += 4) {
                const int64_t c = (int64_t)bcol[q] - B.lo3;
                if (c < 0 || c >= B.w3) continue;
                const uint32_t zb = rb[B.moff + c] >> (4 * sub);
                if (!(zb & 15u)) continue;  // none of this lane's vectors has support on triplet c
                double v[9];
                for (int e = 0; e < 9; ++e) v[e] = rv[e * mR + (q - beg)];
                const double *z = zd + (3 * (B.off3 + c)) * kBatch + 4 * sub;
                for (int jj = 0; jj < 3; ++jj)
                    for (int b = 0; b < 4; ++b) {
                        const double zz = ((zb >> b) & 1u) ? z[jj * kBatch + b] : 0.0;
                        acc[0][b] = fma(v[jj], zz, acc[0][b]);
                        acc[1][b] = fma(v[3 + jj], zz, acc[1][b]);
                        acc[2][b] = fma(v[6 + jj], zz, acc[2][b]);
                    }
            }
        }
        for (int i = 0; i < 3; ++i)
            for (int b = 0; b < 4; ++b) {
                double v = acc[i][b];
                v += __shfl_xor(v, 4);
                v += __shfl_xor(v, 8);
                acc[i][b] = v;
            }
        if (!live || part != 0) continue;
        double *o = kd + (3 * (B.off3 + t)) * kBatch + 4 * sub;
        for (int i = 0; i < 3; ++i)
            for (int b = 0; b < 4; ++b) o[i * kBatch + b] = acc[i][b];
        for (int b = 0; b < 4; ++b) {
            const int32_t pos = items[B.off3 + x].pos[4 * sub + b];
            if (pos < 0) continue;
            for (int i = 0; i < 3; ++i) {
                kzi[pos + i] = (int32_t)(3 * R + i);
                kzv[pos + i] = acc[i][b];
            }
        }
        if (sub == 0)
            for (int i = 0; i < 3; ++i)
                for (int64_t e = zp[3 * R + i]; e < zp[3 * R + i + 1]; ++e) {
                    const int32_t col = zc[e];
                    atomicOr(&tb[col / 32], 1u << (col % 32));
                }
    }
    if (!lds_bits) return;
    __syncthreads();
    for (int t = threadIdx.x; t < words; t += 256)
        if (tw[t]) atomicOr(&touched[B.bit0 + t], tw[t]);
}

// E_raw[j0+b, i] = sum over the structure rows t of the batch in the rows of z_i of
// Z[t, i] (K z_{j0+b})_t, for the vectors i flagged as touched.  One wave per (i,
// batch); lanes stride over the rows of z_i inside the window, then a fixed-order
// wave reduction.
// First index in [a, e) whose entry is >= key (e if none), for an increasing array, by
// the whole wave: each round tests 64 evenly spaced entries and keeps the one gap that
// holds the answer, so a range of L entries takes about log_64 L rounds of one load.
__device__ __forceinline__ int64_t wave_lower_bound(const int32_t *__restrict__ v, int64_t a, int64_t e,
                                                    int64_t key) {
    const int lane = threadIdx.x & 63;
    int64_t lo = a, hi = e;  // the answer lies in [lo, hi]
    while (lo < hi) {
        const int64_t step = (hi - lo + 63) / 64;
        const int64_t idx = lo + lane * step;
        const bool below = idx < hi && (int64_t)v[idx] < key;
        const int nless = __popcll(__ballot(below));  // the samples below key form a prefix
        if (nless == 0) {
            hi = lo;
        } else {
            const int64_t nlo = lo + (int64_t)(nless - 1) * step + 1;
            hi = min(hi, lo + (int64_t)nless * step);
            lo = nlo;
        }
    }
    return lo;
}

constexpr int kErowRun = 4;  // entries per lane whose rows and masks are loaded together

__global__ __launch_bounds__(256) void k_kzb_erows(const KzBatch *__restrict__ bt, int32_t k,
                                                   const int64_t *__restrict__ ztp, const int32_t *__restrict__ zti,
                                                   const double *__restrict__ ztv, const double *__restrict__ kd,
                                                   const uint32_t *__restrict__ mk, const uint32_t *__restrict__ touched,
                                                   double *__restrict__ eraw, int64_t ld) {
    const KzBatch B = bt[blockIdx.y];
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= k || B.w3 == 0) return;
    if (!((touched[B.bit0 + i / 32] >> (i % 32)) & 1u)) return;
    const int64_t lo = 3 * B.lo3, w = 3 * B.w3;
    int64_t a = ztp[i], e = ztp[i + 1];
    if (a == e || zti[e - 1] < lo || zti[a] >= lo + w) return;
    // the entries of z_i with rows in the window: [first row >= lo, first row >= lo + w)
    e = wave_lower_bound(zti, a, e, lo + w);
    a = wave_lower_bound(zti, a, e, lo);
    double acc[kBatch];
    for (int b = 0; b < kBatch; ++b) acc[b] = 0.0;
    for (int64_t q0 = a + lane; q0 < e; q0 += 64 * kErowRun) {
        // a run of the lane's entries: rows, then their structure masks, loaded together
        int64_t tr[kErowRun];
        bool on[kErowRun];
#pragma unroll
        for (int u = 0; u < kErowRun; ++u) tr[u] = q0 + 64 * u < e ? (int64_t)zti[q0 + 64 * u] - lo : -1;
#pragma unroll
        for (int u = 0; u < kErowRun; ++u) on[u] = tr[u] >= 0 && mk[B.moff + tr[u] / 3] != 0u;
        for (int u = 0; u < kErowRun; ++u) {
            if (!on[u]) continue;  // (K z_j)_t is structurally zero for every vector of the batch
            const double z = ztv[q0 + 64 * u];
            const double *kdr = kd + (3 * B.off3 + tr[u]) * kBatch;
            for (int b = 0; b < kBatch; ++b) acc[b] = fma(z, kdr[b], acc[b]);
        }
    }
    for (int b = 0; b < kBatch; ++b) {
        double v = acc[b];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        acc[b] = v;
    }
    if (lane == 0)
        for (int b = 0; b < kBatch; ++b)
            if (b < B.ncol) eraw[(B.j0 + b) * ld + i] = acc[b];
}

// A = S (E + E^T)/2 S with S = diag(1 / sqrt(E_ii)), padded to ld x ld with an identity
// tail; diag0 = diagonal of A; scale = the diagonal of S (1 where E_ii <= 0, whose
// pivot then fails the SPD test).  Inverting the Jacobi-scaled matrix is exact
// (E^-1 = S (S E S)^-1 S) and much better conditioned when the deflation vectors' scales
// differ (rigid-body rotations against translations, enriched against standard DoFs);
// the Schur pivots scale with the diagonal, so the SPD test is the unscaled one.
__global__ void k_symmetrise(int32_t k, int64_t ld, const double *__restrict__ eraw, double *__restrict__ A,
                             double *__restrict__ diag0, double *__restrict__ scale) {
    const int64_t total = ld * ld;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / ld, j = t % ld;
        double v;
        if (i < k && j < k) {
            const double di = eraw[i * ld + i], dj = eraw[j * ld + j];
            const double si = di > 0.0 ? 1.0 / sqrt(di) : 1.0, sj = dj > 0.0 ? 1.0 / sqrt(dj) : 1.0;
            v = (0.5 * (eraw[i * ld + j] + eraw[j * ld + i]) * si) * sj;
            if (i == j) scale[i] = si;
        } else {
            v = (i == j) ? 1.0 : 0.0;
        }
        A[t] = v;
        if (i == j) diag0[i] = v;
    }
}

// ---------------------------------------------------------------- block Gauss-Jordan
// P = S^-1 for the symmetric positive definite 32 x 32 pivot block S (LDS) by in-place
// Gauss-Jordan elimination without pivoting (on an SPD matrix its pivots are the Schur
// complement pivots of the Cholesky factorisation).  Step k, pivot p = a_kk:
//   a_rc -= a_rk a_kc / p (r, c != k),  a_kc /= p,  a_rk = -a_rk / p,  a_kk = 1 / p.
// Thread (ty, tx) of the 256 keeps a[ty + 8q][tx], q < 4, in registers; only row k and
// column k travel through LDS (W, ping-pong by step parity), one barrier per step.
// Every pivot is tested against kdim * DBL_EPSILON times the original diagonal entry;
// a failure sets *fail to 1 (failval < 0) or lowers it to failval.
__device__ void pivot_inverse(const double *S, int lds, double *W, const double *diag0, int64_t gcol0, int32_t kdim,
                              double *P, int *fail, int failval) {
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    double *rowk = W, *colk = W + 2 * kNb;  // [parity][32] each
    // thread j tests pivot j; its floor is loaded before the first barrier
    const int64_t gmine = gcol0 + threadIdx.x;
    const double myfl = ((int)threadIdx.x < kNb && gmine < kdim) ? (double)kdim * DBL_EPSILON * fabs(diag0[gmine]) : 0.0;
    double a[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = ty + 8 * q;
        a[q] = S[r * lds + tx];
        if (r == 0) rowk[tx] = a[q];
        if (tx == 0) colk[r] = a[q];
    }
    bool bad = false;
    __syncthreads();
    // unrolled by 8 only: fully unrolled it needs ~150 VGPRs, which would cap the occupancy
    // of every sweep workgroup at 3 waves per SIMD (this routine is inlined into the sweeps)
#pragma unroll 8
    for (int k = 0; k < kNb; ++k) {
        // all LDS reads of the step first (one wait), then selects instead of branches
        const int cb = k & 1, nb = cb ^ 1;
        const double p = rowk[cb * kNb + k];
        const double kc = rowk[cb * kNb + tx];
        double rk[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) rk[q] = colk[cb * kNb + ty + 8 * q];
        if ((int)threadIdx.x == k && (!(p > myfl) || !isfinite(p))) bad = true;
        // 1/p: hardware reciprocal refined by two Newton steps
        double ip = __builtin_amdgcn_rcp(p);
        ip = fma(ip, fma(-p, ip, 1.0), ip);
        ip = fma(ip, fma(-p, ip, 1.0), ip);
        const double kcip = kc * ip;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = ty + 8 * q;
            const double m = -rk[q] * ip;
            double v = fma(m, kc, a[q]);
            v = (tx == k) ? m : v;
            v = (r == k) ? ((tx == k) ? ip : kcip) : v;
            a[q] = v;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = ty + 8 * q;
            if (r == k + 1) rowk[nb * kNb + tx] = a[q];
            if (tx == k + 1) colk[nb * kNb + r] = a[q];
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) P[(ty + 8 * q) * kNb + tx] = a[q];
    if (bad) {
        if (failval < 0) atomicOr(fail, 1);
        else atomicMin(fail, failval);
    }
}

// The 32 x 32 tile products of the sweeps on the matrix cores: wave w of the 256 threads
// computes the 16 x 16 quarter (w / 2, w % 2) of X Y (X, Y in LDS, row stride kLd) as
// eight v_mfma_f64_16x16x4f64 steps.  Operand lanes: a = X[row l % 16][k-step col l / 16],
// b = Y[k-step row l / 16][col l % 16]; result item v of lane l is element
// (l / 16 + 4 v, l % 16) of the quarter.  The stride 33 spreads a column's 16 rows over
// distinct LDS banks.
constexpr int kLd = kNb + 1;
typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dbl4 tile_mfma(const double *X, const double *Y) {
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = (wv >> 1) * 16 + (l & 15), c = (wv & 1) * 16 + (l & 15), kq = l >> 4;
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s4 = 0; s4 < kNb; s4 += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(X[r * kLd + s4 + kq], Y[(s4 + kq) * kLd + c], acc, 0, 0, 0);
    return acc;
}

// row and column (within the 32 x 32 tile) of result item v of this thread
__device__ __forceinline__ int tile_row(int v) {
    return ((threadIdx.x >> 6) >> 1) * 16 + ((threadIdx.x & 63) >> 4) + 4 * v;
}
__device__ __forceinline__ int tile_col() { return ((threadIdx.x >> 6) & 1) * 16 + (threadIdx.x & 15); }

// One sweep with pivot block p of the dense block-Jacobi blocks' inversion: B = sweep(A).
// Tile (I, J) of 32 x 32:
//   I = J = p: P;  I = p: P A_pJ;  J = p: -A_Ip P;  else A_IJ - A_Ip (P A_pJ).
// Every tile is computed from its own formula (the coarse matrix, Jacobi-scaled, uses
// the symmetric 64-wide sweeps below instead).  All global loads of a tile are issued
// before the first LDS store, and P A_pJ reuses the LDS of A_pJ.  The workgroup of tile
// (p+1, p+1) also inverts the next pivot block.
__device__ __forceinline__ void gj_sweep_tile(int p, int nt, int I, int J, const double *__restrict__ A,
                                              double *__restrict__ B, int64_t ld, int32_t kdim,
                                              const double *__restrict__ Pcur, double *__restrict__ Pnext,
                                              const double *__restrict__ diag0, int *fail, int failval) {
    __shared__ double Ps[kNb * kLd], X[kNb * kLd], Y[kNb * kLd];
    const int64_t r0 = (int64_t)I * kNb, c0 = (int64_t)J * kNb, q0 = (int64_t)p * kNb;
    const bool piv = I == p && J == p, rowp = !piv && I == p, colp = !piv && J == p;
    const bool gen = !piv && !rowp && !colp;
    const bool use_x = colp || gen, use_y = rowp || gen;  // X = A_Ip, Y = A_pJ
    const int cc = tile_col();
    double pr[4], xr[4], yr[4], sr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int t = threadIdx.x + 256 * q, a = t / kNb, b = t % kNb;
        pr[q] = Pcur[t];
        xr[q] = use_x ? A[(r0 + a) * ld + q0 + b] : 0.0;
        yr[q] = use_y ? A[(q0 + a) * ld + c0 + b] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) sr[v] = gen ? A[(r0 + tile_row(v)) * ld + c0 + cc] : 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int t = threadIdx.x + 256 * q, a = t / kNb, b = t % kNb;
        Ps[a * kLd + b] = pr[q];
        if (use_x) X[a * kLd + b] = xr[q];
        if (use_y) Y[a * kLd + b] = yr[q];
    }
    __syncthreads();
    dbl4 d;
    if (piv) {
#pragma unroll
        for (int v = 0; v < 4; ++v) d[v] = Ps[tile_row(v) * kLd + cc];
    } else if (rowp) {
        d = tile_mfma(Ps, Y);
    } else if (colp) {
        const dbl4 x4 = tile_mfma(X, Ps);
#pragma unroll
        for (int v = 0; v < 4; ++v) d[v] = -x4[v];
    } else {
        const dbl4 t4 = tile_mfma(Ps, Y);  // P A_pJ, into Y once every wave has read Y
        __syncthreads();
#pragma unroll
        for (int v = 0; v < 4; ++v) Y[tile_row(v) * kLd + cc] = t4[v];
        __syncthreads();
        const dbl4 x4 = tile_mfma(X, Y);
#pragma unroll
        for (int v = 0; v < 4; ++v) d[v] = sr[v] - x4[v];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) B[(r0 + tile_row(v)) * ld + c0 + cc] = d[v];
    if (I == p + 1 && J == p + 1) {
        __syncthreads();  // every wave is done with Y
#pragma unroll
        for (int v = 0; v < 4; ++v) Y[tile_row(v) * kLd + cc] = d[v];
        __syncthreads();
        pivot_inverse(Y, kLd, X, diag0, (int64_t)(p + 1) * kNb, kdim, Pnext, fail, failval);
    }
}

// ---------------------------------------------------------------- E^-1: symmetric sweeps
// The coarse matrix is symmetric positive definite, so its block Gauss-Jordan inverse is
// run as the symmetric sweep operator on the lower triangle of 64 x 64 tiles only.  After
// the sweeps over pivot blocks 0 .. p-1 the working matrix is symmetric up to signs: its
// entry (i, j) equals sigma_i sigma_j times entry (j, i), sigma = -1 on the rows of the
// pivot blocks already swept and +1 on the others, so every tile above the diagonal is a
// signed transpose of one below it, and a diagonal tile is symmetric (its upper half is
// always taken from its lower half).  Sweep p, with P = A_pp^-1 (symmetrised):
//   new row p:        T_J  = P A_pJ                       (panel kernel, every J)
//   new column p:     B_Ip = -A_Ip P = -T_I^T   (I > p)
//   new pivot tile:   B_pp = P
//   every other tile: B_IJ = A_IJ - A_Ip T_J
// so each lower tile costs one 64 x 64 x 64 product on the matrix cores, and a sweep
// reads and writes the lower triangle once: a quarter of the work of the full 32-wide
// sweeps over every tile.  The panel kernel stores T and the column panel C_I = A_Ip in
// buffers of their own, so the sweep updates the matrix in place.  In a numpy model on
// the Jacobi-scaled coarse matrices of the 40^3 and 80^3 workloads this form leaves
// max |I - E E^-1| at the level of the full 32-wide sweeps (80^3: 2.6e-3 against 2.9e-3).
constexpr int kCb = 64;
constexpr int kCbLd = kCb + 1;  // LDS row stride: a column's 16 rows in distinct banks

// P = S^-1 (symmetrised, in place) for the 64 x 64 SPD pivot block S in LDS (row stride
// kCbLd) by Gauss-Jordan elimination without pivoting, as pivot_inverse, in its
// symmetric form: during the in-place elimination of a symmetric matrix, entry (k, c)
// equals sigma_c times entry (c, k), sigma_c = -1 for the columns already pivoted and +1
// for the others, so step k reads only column k and takes row k from it.  Thread
// (ty, tx) = (t / 64, t % 64) keeps rows 16 ty + q, q < 16, of column tx in registers;
// the lane that owns column k + 1 writes it to W (2 kCb doubles, ping-pong by step
// parity), one barrier per step.  Pivot j is tested against kdim * DBL_EPSILON times the
// original diagonal entry gcol0 + j; returns whether one failed (in every thread).
__device__ __forceinline__ bool pivot_inverse64(double *S, double *W, const double *__restrict__ diag0, int64_t gcol0,
                                                int32_t kdim) {
    __shared__ int bad_s;
    const int tx = threadIdx.x & 63, r0 = (threadIdx.x >> 6) * 16;
    const int64_t gmine = gcol0 + threadIdx.x;
    const double myfl = ((int)threadIdx.x < kCb && gmine < kdim) ? (double)kdim * DBL_EPSILON * fabs(diag0[gmine]) : 0.0;
    if (threadIdx.x == 0) bad_s = 0;
    double a[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) a[q] = S[(r0 + q) * kCbLd + tx];
    if ((int)threadIdx.x < kCb) W[threadIdx.x] = S[threadIdx.x * kCbLd];  // column 0
    bool bad = false;
    __syncthreads();
#pragma unroll 1
    for (int k = 0; k < kCb; ++k) {
        const double *col = W + (k & 1) * kCb;
        double *nxt = W + ((k & 1) ^ 1) * kCb;
        // all LDS reads of the step first (one wait)
        const double p = col[k];
        const double ck = col[tx];
        double rk[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) rk[q] = col[r0 + q];
        const double kc = tx < k ? -ck : ck;  // entry (k, tx)
        if ((int)threadIdx.x == k && (!(p > myfl) || !isfinite(p))) bad = true;
        // 1/p: hardware reciprocal refined by two Newton steps
        double ip = __builtin_amdgcn_rcp(p);
        ip = fma(ip, fma(-p, ip, 1.0), ip);
        ip = fma(ip, fma(-p, ip, 1.0), ip);
        const double kcip = kc * ip;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const double m = -rk[q] * ip;
            const double v = fma(m, kc, a[q]);
            a[q] = (tx == k) ? m : v;
        }
        if (k >= r0 && k < r0 + 16) {  // row k lies in this wave: a uniform branch
#pragma unroll
            for (int q = 0; q < 16; ++q)
                if (r0 + q == k) a[q] = (tx == k) ? ip : kcip;
        }
        if (tx == k + 1) {
#pragma unroll
            for (int q = 0; q < 16; ++q) nxt[r0 + q] = a[q];
        }
        __syncthreads();
    }
    if (bad) atomicOr(&bad_s, 1);
#pragma unroll
    for (int q = 0; q < 16; ++q) S[(r0 + q) * kCbLd + tx] = a[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) a[q] = 0.5 * (S[(r0 + q) * kCbLd + tx] + S[tx * kCbLd + r0 + q]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) S[(r0 + q) * kCbLd + tx] = a[q];
    __syncthreads();
    return bad_s != 0;
}

// X Y for 64 x 64 tiles X, Y in LDS (row stride kCbLd) on the matrix cores: wave w of the
// 256 threads computes the 32 x 32 quadrant (w / 2, w % 2) as 2 x 2 blocks of 16 x 16,
// sixteen v_mfma_f64_16x16x4f64 steps each.  Result item v of block b = 2 bi + bj of lane
// l is element (cb_row(b, v), cb_col(b)) of the product.
__device__ __forceinline__ int cb_row(int b, int v) {
    return ((threadIdx.x >> 6) >> 1) * 32 + (b >> 1) * 16 + ((threadIdx.x & 63) >> 4) + 4 * v;
}
__device__ __forceinline__ int cb_col(int b) { return ((threadIdx.x >> 6) & 1) * 32 + (b & 1) * 16 + (threadIdx.x & 15); }

__device__ __forceinline__ void cb_mfma(const double *X, const double *Y, dbl4 (&acc)[4]) {
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, kq = l >> 4;
    const int r0 = (wv >> 1) * 32 + (l & 15), c0 = (wv & 1) * 32 + (l & 15);
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int s4 = 0; s4 < kCb; s4 += 4) {
        const double x0 = X[r0 * kCbLd + s4 + kq], x1 = X[(r0 + 16) * kCbLd + s4 + kq];
        const double y0 = Y[(s4 + kq) * kCbLd + c0], y1 = Y[(s4 + kq) * kCbLd + c0 + 16];
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y0, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y1, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y0, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y1, acc[3], 0, 0, 0);
    }
}

// entry (a, b) of diagonal tile (I, I) (first row r0) of the row-major ld x ld array A,
// from its lower half
__device__ __forceinline__ double diag_tile_at(const double *__restrict__ A, int64_t ld, int64_t r0, int a, int b) {
    return a >= b ? A[(r0 + a) * ld + r0 + b] : A[(r0 + b) * ld + r0 + a];
}

// P_0 = A_00^-1 (symmetrised) from the first diagonal tile's lower half.
__global__ __launch_bounds__(256) void k_cgj_first_pivot(const double *__restrict__ A, int64_t ld, int32_t kdim,
                                                         const double *__restrict__ diag0, double *__restrict__ P,
                                                         int *fail) {
    __shared__ double S[kCb * kCbLd], W[4 * kCb];
    const int tb = threadIdx.x & 63, ta = threadIdx.x >> 6;  // element (ta + 4 q, tb)
    double sv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) sv[q] = A[(ta + 4 * q) * ld + tb];
#pragma unroll
    for (int q = 0; q < 16; ++q) S[(ta + 4 * q) * kCbLd + tb] = sv[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int a = ta + 4 * q;
        sv[q] = a >= tb ? S[a * kCbLd + tb] : S[tb * kCbLd + a];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) S[(ta + 4 * q) * kCbLd + tb] = sv[q];
    __syncthreads();
    const bool bad = pivot_inverse64(S, W, diag0, 0, kdim);
#pragma unroll
    for (int q = 0; q < 16; ++q) P[(ta + 4 * q) * kCb + tb] = S[(ta + 4 * q) * kCbLd + tb];
    if (bad && threadIdx.x == 0) atomicOr(fail, 1);
}

// Panel of sweep p, workgroup J != p: the tile A_pJ (stored below the diagonal for J < p;
// for J > p the transpose of the stored (J, p), sign +1), T_J = P A_pJ into tbuf[J], and
// the column tile A_Jp = s A_pJ^T into cbuf[J] (s = +1 for J > p, -1 for J < p: block row
// J is swept, block row p not yet).  Both buffers hold nt tiles of 64 x 64, row-major.
__global__ __launch_bounds__(256) void k_cgj_panel(int p, const double *__restrict__ A, int64_t ld,
                                                   const double *__restrict__ P, double *__restrict__ cbuf,
                                                   double *__restrict__ tbuf) {
    __shared__ double S[kCb * kCbLd], Y[kCb * kCbLd];
    const int J = blockIdx.x;
    if (J == p) return;
    const int64_t rp = (int64_t)p * kCb, cj = (int64_t)J * kCb;
    // all loads (coalesced, row-major) before the first LDS store: P, and the stored
    // tile (p, J) for J < p or (J, p) for J > p, which is A_pJ transposed
    const int tb = threadIdx.x & 63, ta = threadIdx.x >> 6;  // element (ta + 4 q, tb)
    const int64_t yo = J < p ? rp * ld + cj : cj * ld + rp;
    double pv[16], yv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int a = ta + 4 * q;
        pv[q] = P[a * kCb + tb];
        yv[q] = A[yo + (int64_t)a * ld + tb];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int a = ta + 4 * q;
        S[a * kCbLd + tb] = pv[q];
        if (J < p) Y[a * kCbLd + tb] = yv[q];
        else Y[tb * kCbLd + a] = yv[q];
    }
    __syncthreads();
    const double s = J > p ? 1.0 : -1.0;
    double *cj_out = cbuf + (int64_t)J * kCb * kCb;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int a = ta + 4 * q;
        cj_out[a * kCb + tb] = s * Y[tb * kCbLd + a];
    }
    dbl4 acc[4];
    cb_mfma(S, Y, acc);
    double *tj = tbuf + (int64_t)J * kCb * kCb;
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) tj[cb_row(b, v) * kCb + cb_col(b)] = acc[b][v];
}

// Sweep p over the lower tiles (I, J), I >= J, in place (tiles numbered row by row,
// I (I + 1) / 2 + J).  The tiles are rotated so that the next pivot tile (p + 1, p + 1)
// is dispatched first: its workgroup also inverts it into Pnext (the critical path of
// the sweep, overlapped with the other tiles).  P and Pnext are distinct buffers.
__global__ __launch_bounds__(256) void k_cgj_sweep(int p, int nt, double *__restrict__ A, int64_t ld, int32_t kdim,
                                                   const double *__restrict__ P, double *__restrict__ Pnext,
                                                   const double *__restrict__ cbuf, const double *__restrict__ tbuf,
                                                   const double *__restrict__ diag0, int *fail) {
    __shared__ double X[kCb * kCbLd], Y[kCb * kCbLd], W[4 * kCb];
    const int64_t ntl = (int64_t)nt * (nt + 1) / 2;
    const int64_t first = p + 1 < nt ? (int64_t)(p + 1) * (p + 2) / 2 + (p + 1) : 0;
    const int64_t tid = (blockIdx.x + first) % ntl;
    int I = (int)((sqrt(8.0 * (double)tid + 1.0) - 1.0) * 0.5);
    while ((int64_t)(I + 1) * (I + 2) / 2 <= tid) ++I;
    while ((int64_t)I * (I + 1) / 2 > tid) --I;
    const int J = (int)(tid - (int64_t)I * (I + 1) / 2);
    const int64_t r0 = (int64_t)I * kCb, c0 = (int64_t)J * kCb;
    const int tb = threadIdx.x & 63, ta = threadIdx.x >> 6;  // element (ta + 4 q, tb)
    if (I == p || J == p) {
        // pivot tile P; row p: T_J; column p: -T_I^T (transposed through LDS)
        const double *src = I == p && J == p ? P : tbuf + (int64_t)(I == p ? J : I) * kCb * kCb;
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = src[(ta + 4 * q) * kCb + tb];
        if (J == p && I != p) {
#pragma unroll
            for (int q = 0; q < 16; ++q) X[(ta + 4 * q) * kCbLd + tb] = v[q];
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = -X[tb * kCbLd + ta + 4 * q];
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) A[(r0 + ta + 4 * q) * ld + c0 + tb] = v[q];
        return;
    }
    // all loads before the first LDS store
    const double *xi = cbuf + (int64_t)I * kCb * kCb, *yj = tbuf + (int64_t)J * kCb * kCb;
    double sr[16], xr[16], yr[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        xr[q] = xi[(ta + 4 * q) * kCb + tb];
        yr[q] = yj[(ta + 4 * q) * kCb + tb];
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int a = cb_row(b, v), c = cb_col(b);
            sr[4 * b + v] = I == J ? diag_tile_at(A, ld, r0, a, c) : A[(r0 + a) * ld + c0 + c];
        }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        X[(ta + 4 * q) * kCbLd + tb] = xr[q];
        Y[(ta + 4 * q) * kCbLd + tb] = yr[q];
    }
    __syncthreads();
    dbl4 acc[4];
    cb_mfma(X, Y, acc);
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            sr[4 * b + v] -= acc[b][v];
            A[(r0 + cb_row(b, v)) * ld + c0 + cb_col(b)] = sr[4 * b + v];
        }
    if (I == p + 1 && J == p + 1) {
        __syncthreads();  // every wave is done with X
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) X[cb_row(b, v) * kCbLd + cb_col(b)] = sr[4 * b + v];
        __syncthreads();
        // the symmetric block from the lower half
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int a = ta + 4 * q;
            Y[a * kCbLd + tb] = a >= tb ? X[a * kCbLd + tb] : X[tb * kCbLd + a];
        }
        __syncthreads();
        const bool bad = pivot_inverse64(Y, W, diag0, r0, kdim);
#pragma unroll
        for (int q = 0; q < 16; ++q) Pnext[(ta + 4 * q) * kCb + tb] = Y[(ta + 4 * q) * kCbLd + tb];
        if (bad && threadIdx.x == 0) atomicOr(fail, 1);
    }
}

// The final E^-1 from the lower tiles of the inverse X of the scaled matrix: F = S X S,
// entry (i, j) from X's entry (max(i, j), min(i, j)), written to the dense array (both
// triangles) and as the packed lower-triangle tiles of the solve; one workgroup per
// lower tile of kCoarseTile^2.  The two scale factors are applied in index order, so the
// dense result is exactly symmetric.
__global__ __launch_bounds__(256) void k_einv_from_lower(int32_t k, int64_t ld, const double *__restrict__ scale,
                                                         const double *__restrict__ X, double *__restrict__ einv,
                                                         double *__restrict__ tiles) {
    constexpr int T = kCoarseTile;
    __shared__ double F[T][T + 1];
    const int64_t tid = blockIdx.x;
    int I = (int)((sqrt(8.0 * (double)tid + 1.0) - 1.0) * 0.5);
    while ((int64_t)(I + 1) * (I + 2) / 2 <= tid) ++I;
    while ((int64_t)I * (I + 1) / 2 > tid) --I;
    const int J = (int)(tid - (int64_t)I * (I + 1) / 2);
    double *out = tiles + tid * T * T;
    for (int e = threadIdx.x; e < T * T; e += 256) {
        const int a = e / T, b = e % T;
        const int ra = I * T + a, cb = J * T + b;
        double f = 0.0;
        if (ra < k && cb < k) {
            const int hi = max(ra, cb), lo = min(ra, cb);
            f = (X[(int64_t)hi * ld + lo] * scale[lo]) * scale[hi];
            einv[(int64_t)ra * ld + cb] = f;
        }
        out[e] = f;
        F[a][b] = f;
    }
    if (I != J) {  // the mirrored tile (J, I) of the dense array, written row by row
        __syncthreads();
        for (int e = threadIdx.x; e < T * T; e += 256) {
            const int a = e / T, b = e % T;
            const int rb = J * T + a, ca = I * T + b;
            if (rb < k && ca < k) einv[(int64_t)rb * ld + ca] = F[b][a];
        }
    }
}

// ---------------------------------------------------------------- dense blocks
// Block-Jacobi blocks of more than kMaxBlock DoFs (subdomain-sized blocks).  K_BB is
// gathered from the block's lower triangle (mirrored), padded to ld = 32 * ceil(m / 32)
// with the identity, and inverted by the Gauss-Jordan sweeps above, batched over the
// blocks: the table is sorted by ld, largest first, so the blocks that still have a
// pivot tile p form a prefix, and sweep p runs the tiles of that prefix in one launch.
// A failed pivot lowers the flag to the block's index.
struct GjMat {
    int64_t off;    // first entry of its ld x ld matrix in the work buffers (= in dinv)
    int64_t tile0;  // first workgroup of its tiles in a sweep (prefix of nt^2)
    int64_t dg;     // first entry of its original diagonal in diag0 (prefix of ld)
    int32_t ld, size, start, block;
};

__device__ __forceinline__ int gj_find(const GjMat *__restrict__ m, int count, int64_t wg) {
    int lo = 0, hi = count - 1;  // last matrix with tile0 <= wg
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (m[mid].tile0 <= wg) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// rows of matrix blockIdx.y (grid-stride): the lower-triangle entries of K_BB to both
// (i, c) and (c, i), the original diagonal to diag0, the identity beyond the block's
// size.  A and diag0 are zero on entry.
__global__ __launch_bounds__(256) void k_dense_gather(const GjMat *__restrict__ mats, int count,
                                                      const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                                      const double *__restrict__ val, double *__restrict__ A,
                                                      double *__restrict__ diag0) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int mi = blockIdx.y; mi < count; mi += gridDim.y) {
        const GjMat G = mats[mi];
        double *a = A + G.off;
        for (int i = blockIdx.x * 4 + wave; i < G.ld; i += gridDim.x * 4) {
            if (i >= G.size) {
                if (lane == 0) {
                    a[(int64_t)i * G.ld + i] = 1.0;
                    diag0[G.dg + i] = 1.0;
                }
                continue;
            }
            const int64_t g = (int64_t)G.start + i;
            for (int64_t e = ptr[g] + lane; e < ptr[g + 1]; e += 64) {
                const int64_t c = (int64_t)idx[e] - G.start;
                if (c < 0 || c > i) continue;
                const double v = val[e];
                a[(int64_t)i * G.ld + c] = v;
                a[c * G.ld + i] = v;
                if (c == i) diag0[G.dg + i] = v;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_gjb_first_pivot(const GjMat *__restrict__ mats, int count,
                                                         const double *__restrict__ A,
                                                         const double *__restrict__ diag0, double *__restrict__ P,
                                                         int *fail) {
    __shared__ double S[kNb * kNb], W[kNb * kNb];
    for (int mi = blockIdx.x; mi < count; mi += gridDim.x) {
        const GjMat G = mats[mi];
        __syncthreads();
        for (int t = threadIdx.x; t < kNb * kNb; t += 256) S[t] = A[G.off + (t / kNb) * (int64_t)G.ld + (t % kNb)];
        __syncthreads();
        pivot_inverse(S, kNb, W, diag0 + G.dg, 0, G.size, P + (int64_t)mi * 2 * kNb * kNb, fail, G.block);
    }
}

// sweep p over the first count matrices (those with more than p pivot tiles)
__global__ __launch_bounds__(256) void k_gjb_sweep(int p, const GjMat *__restrict__ mats, int count,
                                                   const double *__restrict__ A, double *__restrict__ B,
                                                   double *__restrict__ P, const double *__restrict__ diag0,
                                                   int *fail) {
    const int mi = gj_find(mats, count, blockIdx.x);
    const GjMat G = mats[mi];
    const int nt = G.ld / kNb;
    const int64_t t = blockIdx.x - G.tile0;
    double *pv = P + (int64_t)mi * 2 * kNb * kNb;
    gj_sweep_tile(p, nt, (int)(t / nt), (int)(t % nt), A + G.off, B + G.off, G.ld, G.size, pv + (p & 1) * kNb * kNb,
                  pv + ((p + 1) & 1) * kNb * kNb, diag0 + G.dg, fail, G.block);
}

__global__ __launch_bounds__(256) void k_gjb_zero(const GjMat *__restrict__ mats, int count, double *__restrict__ A) {
    for (int mi = blockIdx.y; mi < count; mi += gridDim.y) {
        const GjMat G = mats[mi];
        const int64_t len = (int64_t)G.ld * G.ld;
        for (int64_t t = blockIdx.x * 256ll + threadIdx.x; t < len; t += (int64_t)gridDim.x * 256) A[G.off + t] = 0.0;
    }
}

// matrices with an even number of pivot tiles end their sweeps in the work buffer
__global__ __launch_bounds__(256) void k_gjb_copy_even(const GjMat *__restrict__ mats, int count,
                                                       const double *__restrict__ src, double *__restrict__ dst) {
    for (int mi = blockIdx.y; mi < count; mi += gridDim.y) {
        const GjMat G = mats[mi];
        if ((G.ld / kNb) % 2 != 0) continue;
        const int64_t len = (int64_t)G.ld * G.ld;
        for (int64_t t = blockIdx.x * 256ll + threadIdx.x; t < len; t += (int64_t)gridDim.x * 256)
            dst[G.off + t] = src[G.off + t];
    }
}

// ---------------------------------------------------------------- value updates
__global__ void k_to_i64(const int32_t *__restrict__ a, int64_t n, int64_t *__restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a[i];
}

__global__ void k_to_f32_s(const double *__restrict__ a, int64_t n, float *__restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)a[i];
}

// flag = first block row whose block count differs from the stored row pointer
__global__ void k_cmp_counts(int32_t nb, const int64_t *__restrict__ cnt, const int32_t *__restrict__ bptr,
                             int *flag) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nb; r += (int64_t)gridDim.x * blockDim.x)
        if (cnt[r] != (int64_t)(bptr[r + 1] - bptr[r])) atomicMin(flag, (int)r);
}

// flag = 0 when a[i] != b[i] for some i
__global__ void k_cmp_i32(int64_t n, const int32_t *__restrict__ a, const int32_t *__restrict__ b, int *flag) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (a[i] != b[i]) atomicMin(flag, 0);
}

// ---------------------------------------------------------------- host helpers
// Scratch of one setup call; released (to the cache) once the stream is idle.
struct Pool {
    dpcg_ctx *c;
    std::vector<void *> scratch;
    std::vector<void *> pinned;  // host read-back buffers (pinned, so the copies stay asynchronous)
    // work enqueued on the side stream after fork() runs beside the main stream from that
    // point on; join() makes the main stream wait for all of it
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool pending = false;
    ~Pool() {
        if (pending) (void)hipStreamSynchronize(side);
        (void)hipStreamSynchronize(c->stream);
        for (void *p : scratch) dev_release(p);
        for (void *p : pinned) host_release(p);
        sync_event_give(ev_fork);
        sync_event_give(ev_join);
    }
    hipError_t fork(hipStream_t *sb) {
        hipError_t e = side_stream(&side);
        if (e == hipSuccess && !ev_fork) e = sync_event_take(&ev_fork);
        if (e == hipSuccess && !ev_join) e = sync_event_take(&ev_join);
        if (e == hipSuccess) e = hipEventRecord(ev_fork, c->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(side, ev_fork, 0);
        if (e != hipSuccess) return e;
        pending = true;
        *sb = side;
        return hipSuccess;
    }
    hipError_t join() {
        if (!pending) return hipSuccess;
        hipError_t e = hipEventRecord(ev_join, side);
        if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, ev_join, 0);
        if (e == hipSuccess) pending = false;
        return e;
    }
    template <class T>
    hipError_t host(T **p, size_t count) {
        void *q = nullptr;
        hipError_t e = host_alloc(&q, std::max<size_t>(1, count) * sizeof(T));
        if (e == hipSuccess) pinned.push_back(q);
        *p = (T *)q;
        return e;
    }
    template <class T>
    hipError_t tmp(T **p, size_t count) {
        void *q = nullptr;
        hipError_t e = dev_alloc(&q, std::max<size_t>(1, count) * sizeof(T));
        if (e == hipSuccess) scratch.push_back(q);
        *p = (T *)q;
        return e;
    }
};

template <class T>
hipError_t keep(dpcg_ctx *c, T **p, size_t count) {
    void *q = nullptr;
    const size_t bytes = std::max<size_t>(1, count) * sizeof(T);
    hipError_t e = dev_alloc(&q, bytes);
    if (e == hipSuccess) {
        c->allocations.push_back(q);
        c->device_bytes += (int64_t)bytes;
    }
    *p = (T *)q;
    return e;
}

int grid_for(int64_t work, int per = 256, int cap = 8192) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (work + per - 1) / per));
}

// Checks a CSR matrix (rows x cols, nnz entries) into *flag; with mx, also max |value|
// into (*mx)[0] (scratch from the pool).
hipError_t check_csr(hipStream_t s, Pool &pool, int64_t rows, int64_t cols, const int64_t *ptr, const int32_t *idx,
                     const double *val, int64_t nnz, int *flag, double **mx) {
    uint32_t *bits = nullptr;
    hipError_t e = pool.tmp(&bits, nnz / 32 + 1);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(bits, 0, sizeof(uint32_t) * (size_t)(nnz / 32 + 1), s);
    if (e != hipSuccess) return e;
    const int ge = grid_for(nnz, 256, 4096);
    double *part = nullptr;
    if (mx) {
        e = pool.tmp(&part, ge);
        if (e != hipSuccess) return e;
        *mx = part;
    }
    hipLaunchKernelGGL(k_csr_rows, dim3(grid_for(rows, 256, 4096)), dim3(256), 0, s, rows, ptr, nnz, bits, flag);
    hipLaunchKernelGGL(k_csr_entries, dim3(ge), dim3(256), 0, s, rows, cols, ptr, idx, val, nnz,
                       (const uint32_t *)bits, flag, part);
    if (mx) hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, s, part, ge);
    return hipGetLastError();
}

// out[0..n] = exclusive scan of a[0..n); tmp holds the chunk partials.
hipError_t scan(hipStream_t s, const int64_t *a, int64_t n, int64_t *out, int64_t *part) {
    const int chunks = (int)std::max<int64_t>(1, (n + kScanChunk - 1) / kScanChunk);
    hipLaunchKernelGGL(k_scan_partials, dim3(chunks), dim3(256), 0, s, a, n, part);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, part, chunks);
    hipLaunchKernelGGL(k_scan_apply, dim3(chunks), dim3(256), 0, s, a, n, part, out);
    return hipGetLastError();
}

#define HT(expr)                                       \
    do {                                               \
        if ((expr) != hipSuccess) return DPCG_EHIP;    \
    } while (0)

// K Z (as (KZ)^T) and E = Z^T K Z in batches of kBatch deflation vectors, then E^-1 by
// blocked Gauss-Jordan sweeps.  Inputs: Z (int64 row pointer), Z^T (int64 pointer), the
// row windows of K z_j (wlo on the device, ws on the host).  reuse: the arrays of a
// previous build are overwritten (same structure) instead of allocated.
int coarse_operator(dpcg_ctx *c, Pool &pool, int32_t k, const int64_t *zp, const int32_t *zc, const int64_t *ztp,
                    const int32_t *zti, const double *ztv, const int64_t *wl, const int64_t *ws, int64_t *part,
                    int *flags, int64_t *bad, bool reuse) {
    hipStream_t s = c->stream;
    int *fl = nullptr;  // pinned read-backs: fl[0..4), nkz, cf
    int64_t *nkzp = nullptr;
    HT(pool.host(&fl, 5));
    HT(pool.host(&nkzp, 1));
    {
        // ---- K Z and E, in batches of kBatch vectors; batch groups bound the scratch ----
        // (wl, ws: host copies of the row windows of K z_j)
        const int nbat = (k + kBatch - 1) / kBatch;
        const int words = (k + 31) / 32;
        std::vector<KzBatch> bt(nbat);
        int64_t slices = 0;
        for (int bi = 0; bi < nbat; ++bi) {
            KzBatch &B = bt[bi];
            B.j0 = (int64_t)bi * kBatch;
            B.ncol = std::min<int64_t>(kBatch, k - B.j0);
            int64_t lo = INT64_MAX, hi = -1;
            for (int64_t j = B.j0; j < B.j0 + B.ncol; ++j)
                if (ws[j] > 0) {
                    lo = std::min(lo, wl[j]);
                    hi = std::max(hi, wl[j] + ws[j]);
                }
            B.lo3 = hi > 0 ? lo / 3 : 0;
            B.w3 = hi > 0 ? (hi + 2) / 3 - B.lo3 : 0;
            B.nslice = std::max<int64_t>(1, (B.w3 + kSlice - 1) / kSlice);
            B.slice0 = slices;
            slices += B.nslice;
        }
        // group consecutive batches so that a group's scratch (the dense z and K z of its
        // windows) stays under the budget: 8 GB, under 3% of the device's memory, so that
        // a large system takes few groups, whose launches fill the device better (at 80^3
        // two groups instead of sixteen with 1 GB: 4.7 against 7.7 ms of these kernels)
        const int64_t per_triplet = 2 * 3 * kBatch * sizeof(double) + 2 * sizeof(uint32_t);
        const int64_t budget = int64_t(8) << 30;
        std::vector<int> gcut{0};
        int64_t acc_w = 0, max_group_w = 0, total_w = 0;
        int max_group_nb = 0;
        for (int bi = 0; bi < nbat; ++bi) {
            if (acc_w > 0 && (acc_w + bt[bi].w3) * per_triplet > budget) {
                gcut.push_back(bi);
                acc_w = 0;
            }
            bt[bi].off3 = acc_w;
            bt[bi].moff = total_w;
            total_w += bt[bi].w3;
            bt[bi].bit0 = (int64_t)(bi - gcut.back()) * words;
            acc_w += bt[bi].w3;
            max_group_w = std::max(max_group_w, acc_w);
            max_group_nb = std::max(max_group_nb, bi - gcut.back() + 1);
        }
        gcut.push_back(nbat);
        KzBatch *bt_d = nullptr;
        int32_t *scnt = nullptr, *soff = nullptr, *tcnt = nullptr;
        int64_t *kzcnt = nullptr, *kzp = nullptr;
        double *zd = nullptr, *kd = nullptr;
        uint32_t *mk = nullptr, *rbits = nullptr, *touched = nullptr;
        HT(pool.tmp(&bt_d, nbat));
        HT(hipMemcpyAsync(bt_d, bt.data(), sizeof(KzBatch) * nbat, hipMemcpyHostToDevice, s));
        HT(pool.tmp(&scnt, slices * kBatch));
        HT(pool.tmp(&tcnt, slices));
        HT(pool.tmp(&soff, slices * kBatch));
        HT(pool.tmp(&kzcnt, k));
        HT(pool.tmp(&kzp, k + 1));
        HT(pool.tmp(&zd, 3 * max_group_w * kBatch));
        HT(pool.tmp(&kd, 3 * max_group_w * kBatch));
        // the structure masks of every batch at once (4 bytes per window triplet each):
        // the values pass of a call with several groups then needs no second marking
        HT(pool.tmp(&mk, std::max<int64_t>(1, total_w)));
        HT(pool.tmp(&rbits, std::max<int64_t>(1, total_w)));
        HT(pool.tmp(&touched, (int64_t)max_group_nb * words));
        int32_t *icnt = nullptr;
        int64_t *nitems = nullptr;
        KzItem *items = nullptr;
        HT(pool.tmp(&icnt, slices));
        HT(pool.tmp(&nitems, nbat));
        HT(pool.tmp(&items, max_group_w));
        auto max_slices = [&](int g0, int g1) {
            int64_t m = 1;
            for (int bi = g0; bi < g1; ++bi) m = std::max(m, bt[bi].nslice);
            return (int)m;
        };
        // full: the count pass (masks cleared, z scattered, structure marked); otherwise the
        // values pass of a later group, which only needs its z rows again (the scatter's
        // bits are already in rbits) and clear touched bits
        auto prepare = [&](int g0, int g1, bool full) {
            const dim3 gs(max_slices(g0, g1), g1 - g0);
            hipLaunchKernelGGL(k_kzb_init, gs, dim3(256), 0, s, bt_d + g0, words, mk, rbits, touched, full ? 1 : 0);
            hipLaunchKernelGGL(k_kzb_scatter, dim3(kBatch, g1 - g0), dim3(256), 0, s, bt_d + g0, ztp, zti, ztv, zd,
                               rbits);
            if (full) hipLaunchKernelGGL(k_kzb_mark, gs, dim3(256), 0, s, bt_d + g0, c->brow_ptr, c->bcol, rbits, mk);
        };
        for (size_t g = 0; g + 1 < gcut.size(); ++g) {
            prepare(gcut[g], gcut[g + 1], true);
            hipLaunchKernelGGL(k_kzb_count, dim3(max_slices(gcut[g], gcut[g + 1]), gcut[g + 1] - gcut[g]), dim3(256),
                               0, s, bt_d + gcut[g], mk, scnt, tcnt);
        }
        hipLaunchKernelGGL(k_kzb_offsets, dim3(nbat), dim3(kBatch + 1), 0, s, bt_d, nbat, scnt, tcnt, soff, kzcnt,
                           icnt, nitems);
        HT(scan(s, kzcnt, k, kzp, part));
        HT(hipMemcpyAsync(nkzp, kzp + k, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        int64_t *zp_h = nullptr, *kp_h = nullptr;  // list lengths for the restriction's column order
        if (!reuse) {
            HT(pool.host(&zp_h, k + 1));
            HT(pool.host(&kp_h, k + 1));
            HT(hipMemcpyAsync(zp_h, ztp, sizeof(int64_t) * (k + 1), hipMemcpyDeviceToHost, s));
            HT(hipMemcpyAsync(kp_h, kzp, sizeof(int64_t) * (k + 1), hipMemcpyDeviceToHost, s));
        }
        HT(pool.join());  // the symmetry and block flags are read here
        HT(hipMemcpyAsync(fl, flags, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
        HT(hipStreamSynchronize(s));
        const int64_t nkz = *nkzp;
        if (fl[3] != INT32_MAX) return DPCG_ENOTSYM;
        if (fl[1] != INT32_MAX) {
            *bad = fl[1];
            return DPCG_EBLOCK_NOT_SPD;
        }
        if (nkz > (int64_t)INT32_MAX) return DPCG_EINVAL;
        if (reuse && nkz != c->nnz_kz) return DPCG_EINVAL;  // the structure of K Z must not change
        c->nnz_kz = nkz;
        if (!reuse) {
            // the restriction's column order: columns needing more rounds of its loads first,
            // launch order kept within each class (neighbouring columns share their gathers)
            // (a counting sort: classes of 0 .. 63 rounds and one of 64 or more)
            constexpr int kCls = 64;
            std::vector<int32_t> cls(k), start(kCls + 2, 0);
            for (int32_t j = 0; j < k; ++j) {
                const int64_t len = zp_h[j + 1] - zp_h[j] + kp_h[j + 1] - kp_h[j];
                const int64_t r = std::min<int64_t>((len + kRestrictRound - 1) / kRestrictRound, kCls);
                cls[j] = kCls - (int32_t)r;  // more rounds, earlier class
                ++start[cls[j] + 1];
            }
            for (int q = 0; q <= kCls; ++q) start[q + 1] += start[q];
            c->rs_order_h.resize(k);
            for (int32_t j = 0; j < k; ++j) c->rs_order_h[start[cls[j]]++] = j;
        }
        if (!reuse) {
            HT(keep(c, &c->kzt_idx, nkz));
            HT(keep(c, &c->kzt_val, nkz));
        }
        const int64_t ld = ((int64_t)k + kCb - 1) / kCb * kCb;
        c->einv_ld = ld;
        double *eraw = nullptr, *ga = nullptr, *diag0 = nullptr, *pv = nullptr;
        HT(pool.tmp(&eraw, ld * ld));
        HT(hipMemsetAsync(eraw, 0, sizeof(double) * ld * ld, s));
        for (size_t g = 0; g + 1 < gcut.size(); ++g) {
            const int g0 = gcut[g], g1 = gcut[g + 1];
            if (gcut.size() > 2) prepare(g0, g1, false);  // one group: the count pass left it ready
            hipLaunchKernelGGL(k_kzb_rank, dim3(max_slices(g0, g1), g1 - g0), dim3(256), 0, s, bt_d + g0, mk, soff,
                               icnt, kzp, items);
            hipLaunchKernelGGL(k_kzb_values, dim3(512, g1 - g0), dim3(256),
                               0, s, bt_d + g0, nitems + g0, items, c->brow_ptr, c->bcol, c->bval, zd, rbits, zp, zc,
                               c->kzt_idx, c->kzt_val, kd, words, touched);
            hipLaunchKernelGGL(k_kzb_erows, dim3((k + 3) / 4, g1 - g0), dim3(256), 0, s, bt_d + g0, k, ztp, zti, ztv,
                               kd, mk, touched, eraw, ld);
        }
        HT(hipGetLastError());
        // ---- E^-1 ----
        HT(pool.tmp(&ga, ld * ld));
        if (!reuse) HT(keep(c, &c->einv, ld * ld));
        double *esc = nullptr;
        HT(pool.tmp(&diag0, ld));
        HT(pool.tmp(&esc, ld));
        HT(pool.tmp(&pv, 2 * kCb * kCb));
        hipLaunchKernelGGL(k_symmetrise, dim3(grid_for(ld * ld)), dim3(256), 0, s, k, ld, eraw, ga, diag0, esc);
        int *cfail = flags + 2;
        HT(hipMemsetAsync(cfail, 0, sizeof(int), s));
        const int nt = (int)(ld / kCb);
        double *cbuf = nullptr, *tbuf = nullptr;
        HT(pool.tmp(&cbuf, ld * kCb));
        HT(pool.tmp(&tbuf, ld * kCb));
        hipLaunchKernelGGL(k_cgj_first_pivot, dim3(1), dim3(256), 0, s, (const double *)ga, ld, k, diag0, pv, cfail);
        for (int p = 0; p < nt; ++p) {
            const double *pc = pv + (p & 1) * kCb * kCb;
            hipLaunchKernelGGL(k_cgj_panel, dim3(nt), dim3(256), 0, s, p, (const double *)ga, ld, pc, cbuf, tbuf);
            hipLaunchKernelGGL(k_cgj_sweep, dim3((unsigned)coarse_tile_count(nt)), dim3(256), 0, s, p, nt, ga, ld, k, pc,
                               pv + ((p + 1) & 1) * kCb * kCb, (const double *)cbuf, (const double *)tbuf, diag0,
                               cfail);
        }
        // E^-1 from the lower tiles, and its lower-triangle tiles for the solve's coarse product
        const int32_t cnt = (int32_t)((k + kCoarseTile - 1) / kCoarseTile);
        c->coarse_nt = cnt;
        if (!reuse) HT(keep(c, &c->einv_tiles, coarse_tile_count(cnt) * kCoarseTile * kCoarseTile));
        hipLaunchKernelGGL(k_einv_from_lower, dim3((unsigned)coarse_tile_count(cnt)), dim3(256), 0, s, k, ld,
                           (const double *)esc, (const double *)ga, c->einv, c->einv_tiles);
        HT(hipGetLastError());
        if (!reuse) {
            HT(keep(c, &c->kzt_ptr, k + 1));
            hipLaunchKernelGGL(k_to_i32, dim3(grid_for(k + 1)), dim3(256), 0, s, kzp, (int64_t)k + 1, c->kzt_ptr);
            HT(keep(c, &c->rs_order, k));
            HT(hipMemcpyAsync(c->rs_order, c->rs_order_h.data(), sizeof(int32_t) * k, hipMemcpyHostToDevice, s));
        }
        HT(hipMemcpyAsync(fl + 4, cfail, sizeof(int), hipMemcpyDeviceToHost, s));
        HT(hipStreamSynchronize(s));
        if (fl[4]) return DPCG_ECOARSE_NOT_SPD;
        return DPCG_OK;
    }
}

// Inverses of the dense blocks which[] (indices into c->dense_h), written to c->dinv.
// A block that is not SPD to working precision lowers *bad_flag to its block index.
int dense_inverses(dpcg_ctx *c, Pool &pool, const int64_t *kp, const int32_t *kc, const double *kv,
                   const std::vector<int32_t> &which, int *bad_flag) {
    hipStream_t s = c->stream;
    const int count = (int)which.size();
    if (count == 0) return DPCG_OK;
    std::vector<GjMat> m(count);
    for (int i = 0; i < count; ++i) {
        const DenseBlk &D = c->dense_h[which[i]];
        m[i] = GjMat{D.off, 0, 0, D.ld, D.size, D.start, D.block};
    }
    std::stable_sort(m.begin(), m.end(), [](const GjMat &a, const GjMat &b) { return a.ld > b.ld; });
    std::vector<int64_t> tiles(count + 1, 0);
    int64_t dg = 0;
    for (int i = 0; i < count; ++i) {
        const int64_t nt = m[i].ld / kNb;
        m[i].tile0 = tiles[i];
        tiles[i + 1] = tiles[i] + nt * nt;
        m[i].dg = dg;
        dg += m[i].ld;
    }
    GjMat *md = nullptr;
    double *X0 = nullptr, *diag0 = nullptr, *pv = nullptr;
    HT(pool.tmp(&md, count));
    HT(pool.tmp(&X0, c->dinv_len));
    HT(pool.tmp(&diag0, dg));
    HT(pool.tmp(&pv, (int64_t)count * 2 * kNb * kNb));
    HT(hipMemcpyAsync(md, m.data(), sizeof(GjMat) * count, hipMemcpyHostToDevice, s));
    HT(hipMemsetAsync(diag0, 0, sizeof(double) * dg, s));
    const int gy = std::min(count, 65535);
    const int ldmax = m[0].ld;
    hipLaunchKernelGGL(k_gjb_zero, dim3(64, gy), dim3(256), 0, s, md, count, X0);
    hipLaunchKernelGGL(k_dense_gather, dim3(std::min(1024, (ldmax + 3) / 4), gy), dim3(256), 0, s, md, count, kp, kc,
                       kv, X0, diag0);
    hipLaunchKernelGGL(k_gjb_first_pivot, dim3(gy), dim3(256), 0, s, md, count, X0, diag0, pv, bad_flag);
    int active = count;
    for (int p = 0; p < ldmax / kNb; ++p) {
        while (active > 0 && m[active - 1].ld / kNb <= p) --active;
        const double *src = (p & 1) ? c->dinv : X0;
        double *dst = (p & 1) ? X0 : c->dinv;
        hipLaunchKernelGGL(k_gjb_sweep, dim3((unsigned)tiles[active]), dim3(256), 0, s, p, md, active, src, dst, pv,
                           diag0, bad_flag);
    }
    hipLaunchKernelGGL(k_gjb_copy_even, dim3(64, gy), dim3(256), 0, s, md, count, X0, c->dinv);
    HT(hipGetLastError());
    return DPCG_OK;
}

// The dense-block tables from the host copy of the partition: extents, offsets in dinv,
// and the apply's workgroups (kDenseRows rows of one block each).
int dense_tables(dpcg_ctx *c, const int32_t *bph, int32_t nblocks) {
    hipStream_t s = c->stream;
    c->dense_h.clear();
    int64_t off = 0;
    for (int32_t b = 0; b < nblocks; ++b) {
        const int32_t m = bph[b + 1] - bph[b];
        if (m <= kMaxBlock) continue;
        const int32_t ld = (m + kNb - 1) / kNb * kNb;
        c->dense_h.push_back(DenseBlk{off, bph[b], m, ld, (int32_t)b});
        c->dense_maxld = std::max(c->dense_maxld, ld);
        off += (int64_t)ld * ld;
    }
    std::vector<DenseChunk> ch;
    for (size_t i = 0; i < c->dense_h.size(); ++i)
        for (int32_t r = 0; r < c->dense_h[i].size; r += kDenseRows) ch.push_back(DenseChunk{(int32_t)i, r});
    c->ndense = (int32_t)c->dense_h.size();
    c->ndchunks = (int32_t)ch.size();
    c->dinv_len = off;
    HT(keep(c, &c->dense, c->ndense));
    HT(keep(c, &c->dchunk, c->ndchunks));
    HT(keep(c, &c->dinv, off));
    HT(hipMemcpyAsync(c->dense, c->dense_h.data(), sizeof(DenseBlk) * c->ndense, hipMemcpyHostToDevice, s));
    HT(hipMemcpyAsync(c->dchunk, ch.data(), sizeof(DenseChunk) * c->ndchunks, hipMemcpyHostToDevice, s));
    HT(hipStreamSynchronize(s));  // ch is a host temporary
    return DPCG_OK;
}

}  // namespace

int gpu_setup(dpcg_ctx *c, int64_t n, const int64_t *kp, const int32_t *kc, const double *kv, int32_t k,
              const int64_t *zp, const int32_t *zc, const double *zv, int32_t nblocks, const int32_t *bp,
              int64_t *bad) {
    hipStream_t s = c->stream;
    Pool pool{c, {}};
    // ---- sizes ----
    int64_t *ends = nullptr;  // pinned read-backs of the setup
    int *fl = nullptr;
    int64_t *tot = nullptr;
    HT(pool.host(&ends, 4));
    HT(pool.host(&fl, 5));
    HT(pool.host(&tot, 2));
    ends[2] = ends[3] = 0;
    HT(hipMemcpyAsync(&ends[0], kp, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HT(hipMemcpyAsync(&ends[1], kp + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (k > 0) {
        HT(hipMemcpyAsync(&ends[2], zp, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HT(hipMemcpyAsync(&ends[3], zp + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    }
    HT(hipStreamSynchronize(s));
    const int64_t nnz = ends[1], nnz_z = k > 0 ? ends[3] : 0;
    if (ends[0] != 0 || nnz < 0 || nnz > (int64_t)INT32_MAX || ends[2] != 0 || nnz_z < 0 ||
        nnz_z > (int64_t)INT32_MAX)
        return DPCG_EINVAL;
    c->nnz = nnz;
    c->nnz_z = nnz_z;
    // ---- validation ----
    const double *maxpart = nullptr;
    int nmaxpart = 0;
    int *flags = nullptr;
    HT(pool.tmp(&flags, 5));
    const int init_flags[5] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX, 0};  // [4]: largest block above kMaxBlock
    HT(hipMemcpyAsync(flags, init_flags, sizeof(init_flags), hipMemcpyHostToDevice, s));
    double *mxk = nullptr;
    HT(check_csr(s, pool, n, n, kp, kc, kv, nnz, flags, &mxk));
    if (k > 0) HT(check_csr(s, pool, n, (int64_t)k, zp, zc, zv, nnz_z, flags + 1, nullptr));
    hipLaunchKernelGGL(k_check_blocks, dim3(grid_for(nblocks)), dim3(256), 0, s, nblocks, bp, n, flags + 2,
                       flags + 4);
    HT(hipGetLastError());
    HT(hipMemcpyAsync(fl, flags, sizeof(int) * 5, hipMemcpyDeviceToHost, s));
    HT(hipStreamSynchronize(s));
    if (fl[2] != INT32_MAX) *bad = fl[2];
    if (fl[0] != INT32_MAX || fl[1] != INT32_MAX || fl[2] != INT32_MAX) return DPCG_EINVAL;
    if (fl[4] > kMaxBlock) {
        int32_t *bph = nullptr;
        HT(pool.host(&bph, nblocks + 1));
        HT(hipMemcpyAsync(bph, bp, sizeof(int32_t) * (nblocks + 1), hipMemcpyDeviceToHost, s));
        HT(hipStreamSynchronize(s));
        const int st = dense_tables(c, bph, nblocks);
        if (st != DPCG_OK) return st;
    }
    maxpart = mxk;
    nmaxpart = 1;  // the maximum of |K| over all entries, in mxk[0]
    // ---- block-CSR counts, block-Jacobi offsets, Z^T, windows ----
    const int32_t nb = c->nb;
    int64_t *cnt = nullptr, *bptr64 = nullptr, *part = nullptr;
    const int64_t scan_parts = std::max<int64_t>({nb, nblocks, (int64_t)k, 1}) / kScanChunk + 2;
    HT(pool.tmp(&cnt, std::max<int64_t>({nb, nblocks, (int64_t)k}) + 1));
    HT(pool.tmp(&bptr64, nb + 1));
    HT(pool.tmp(&part, scan_parts));
    hipLaunchKernelGGL((k_bsr<false>), dim3(grid_for(nb, 4)), dim3(256), 0, s, nb, kp, kc, kv, cnt, nullptr, nullptr,
                       nullptr, nullptr);
    HT(scan(s, cnt, nb, bptr64, part));
    int64_t *moff = nullptr, *sq = nullptr;
    HT(pool.tmp(&moff, nblocks + 1));
    HT(pool.tmp(&sq, nblocks));
    hipLaunchKernelGGL(k_block_sq, dim3(grid_for(nblocks)), dim3(256), 0, s, nblocks, bp, sq);
    int64_t *part2 = nullptr;
    HT(pool.tmp(&part2, scan_parts));
    HT(scan(s, sq, nblocks, moff, part2));
    int64_t *ztp = nullptr, *wlo = nullptr, *wsize = nullptr;
    int32_t *zti = nullptr;
    double *ztv = nullptr;
    if (k > 0) {
        // chunks of Z's entries: at most 1024, and at most 4M (column, chunk) pairs
        const int64_t nch_cap = std::max<int64_t>(1, std::min<int64_t>(1024, ((int64_t)1 << 22) / k));
        const int64_t per = std::max<int64_t>(256, (nnz_z + nch_cap - 1) / nch_cap);
        const int nch = (int)std::max<int64_t>(1, (nnz_z + per - 1) / per);
        const int nranges = (int)((k + kZtCols - 1) / kZtCols);
        const int64_t pairs = (int64_t)k * nch;
        int64_t *cnt = nullptr, *off = nullptr, *part3 = nullptr;
        int32_t *erow = nullptr;
        HT(pool.tmp(&cnt, pairs));
        HT(pool.tmp(&off, pairs + 1));
        HT(pool.tmp(&part3, pairs / kScanChunk + 2));
        HT(pool.tmp(&erow, nnz_z));
        HT(pool.tmp(&ztp, k + 1));
        HT(keep(c, &c->zt_idx, nnz_z));
        HT(keep(c, &c->zt_val, nnz_z));
        zti = c->zt_idx;
        ztv = c->zt_val;
        const int cols_lds = std::min<int>(k, kZtCols);
        hipLaunchKernelGGL(k_entry_rows, dim3(grid_for(n)), dim3(256), 0, s, n, zp, erow);
        hipLaunchKernelGGL(k_zt_count, dim3(nch, nranges), dim3(256), sizeof(int32_t) * cols_lds, s, nnz_z, per, nch,
                           k, zc, cnt);
        HT(scan(s, cnt, pairs, off, part3));
        hipLaunchKernelGGL(k_zt_ptr, dim3(grid_for(k + 1)), dim3(256), 0, s, k, nch, off, ztp);
        hipLaunchKernelGGL(k_zt_place, dim3(nch, nranges), dim3(64), sizeof(int64_t) * cols_lds, s, nnz_z, per, nch, k,
                           zc, zv, erow, off, zti, ztv);
        HT(pool.tmp(&wlo, k));
        HT(pool.tmp(&wsize, k));
        hipLaunchKernelGGL(k_kz_window, dim3(k), dim3(256), 0, s, k, ztp, zti, kp, kc, wlo, wsize);
        HT(hipGetLastError());
    }
    int64_t *ws = nullptr, *wl = nullptr;
    HT(pool.host(&ws, k));
    HT(pool.host(&wl, k));
    HT(hipMemcpyAsync(&tot[0], bptr64 + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HT(hipMemcpyAsync(&tot[1], moff + nblocks, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HT(hipMemcpyAsync(fl, flags, sizeof(int) * 5, hipMemcpyDeviceToHost, s));
    if (k > 0) {
        HT(hipMemcpyAsync(ws, wsize, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s));
        HT(hipMemcpyAsync(wl, wlo, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s));
    }
    HT(hipStreamSynchronize(s));
    const int64_t nnzb = tot[0];
    if (nnzb > (int64_t)INT32_MAX || tot[1] > (int64_t)INT32_MAX) return DPCG_EINVAL;
    c->nnzb = nnzb;
    c->bj_values = tot[1];
    // ---- block-CSR, block-Jacobi, tiles ----
    HT(keep(c, &c->brow_ptr, nb + 1));
    hipLaunchKernelGGL(k_to_i32, dim3(grid_for(nb + 1)), dim3(256), 0, s, bptr64, (int64_t)nb + 1, c->brow_ptr);
    HT(keep(c, &c->bcol, nnzb));
    HT(keep(c, &c->bval, 9 * (size_t)nnzb));
    HT(hipMemsetAsync(c->bval, 0, sizeof(double) * 9 * (size_t)nnzb, s));
    int32_t *brow = nullptr;
    HT(pool.tmp(&brow, nnzb));
    hipLaunchKernelGGL((k_bsr<true>), dim3(grid_for(nb, 4)), dim3(256), 0, s, nb, kp, kc, kv, nullptr, c->brow_ptr,
                       c->bcol, c->bval, brow);
    // block columns as 16-bit offsets from their row for the iteration SpMV (kept when
    // every offset fits: read back at the end of setup)
    int *b16bad = nullptr;
    HT(pool.tmp(&b16bad, 1));
    HT(keep(c, &c->bcol16, nnzb));
    HT(hipMemsetAsync(b16bad, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_bcol16, dim3(grid_for(nnzb)), dim3(256), 0, s, nnzb, (const int32_t *)brow,
                       (const int32_t *)c->bcol, c->bcol16, b16bad);
    // The symmetry test and the small block-Jacobi inverses do not feed K Z, E or E^-1:
    // they run on the side stream beside that chain (whose kernels are latency bound and
    // leave most of the chip idle), joined before their flags are read.  Dense blocks
    // keep one stream.
    hipStream_t sb = s;
    if (c->ndense == 0) HT(pool.fork(&sb));
    const int gsym = (grid_for(nnzb, 256, 16384) + 7) / 8 * 8;
    int64_t *sympart = nullptr;
    int *need = nullptr;
    HT(pool.tmp(&sympart, 2 * (int64_t)gsym));
    HT(pool.tmp(&need, 1));
    HT(keep(c, &c->minv, tot[1]));
    HT(keep(c, &c->bj_rowoff, n));
    HT(keep(c, &c->bj_meta, n));
    hipLaunchKernelGGL(k_check_sym, dim3(gsym), dim3(256), 0, sb, c->brow_ptr, brow, c->bcol, c->bval, nnzb, maxpart,
                       nmaxpart, flags, sympart);
    hipLaunchKernelGGL(k_sym_reduce, dim3(1), dim3(256), 0, sb, sympart, gsym, need);
    hipLaunchKernelGGL(k_check_sym_lower, dim3(gsym), dim3(256), 0, sb, c->brow_ptr, brow, c->bcol, c->bval, nnzb,
                       maxpart, nmaxpart, flags, need);
    int *bjbad = flags + 1;  // reuse: Z's flag is known to be clear
    if (c->ndense > 0) {  // the DoFs of dense blocks take no part in the small-block kernels
        HT(hipMemsetAsync(c->bj_meta, 0, sizeof(int32_t) * n, s));
        HT(hipMemsetAsync(c->bj_rowoff, 0, sizeof(int32_t) * n, s));
    }
    hipLaunchKernelGGL(k_bj_small, dim3(grid_for(nblocks)), dim3(256), 0, sb, nblocks, bp, kp, kc, kv, moff, c->minv,
                       c->bj_rowoff, c->bj_meta, bjbad, (const int32_t *)nullptr, 0);
    hipLaunchKernelGGL(k_bj_factor, dim3(std::min<int32_t>(nblocks, 4096)), dim3(64), 0, sb, nblocks, bp, kp, kc, kv,
                       moff, c->minv, c->bj_rowoff, c->bj_meta, bjbad, (const int32_t *)nullptr, 0);
    HT(hipGetLastError());
    if (c->ndense > 0) {
        std::vector<int32_t> all(c->ndense);
        for (int32_t i = 0; i < c->ndense; ++i) all[i] = i;
        const int st = dense_inverses(c, pool, kp, kc, kv, all, bjbad);
        if (st != DPCG_OK) return st;
    }
    // kept for value updates: the partition and each block's offset in minv
    HT(keep(c, &c->block_ptr, nblocks + 1));
    HT(keep(c, &c->bj_moff, nblocks + 1));
    HT(hipMemcpyAsync(c->block_ptr, bp, sizeof(int32_t) * (nblocks + 1), hipMemcpyDeviceToDevice, s));
    HT(hipMemcpyAsync(c->bj_moff, moff, sizeof(int64_t) * (nblocks + 1), hipMemcpyDeviceToDevice, s));
    c->bj_ntiles = (int32_t)((n + kTileDofs - 1) / kTileDofs);
    HT(keep(c, &c->bj_wg_start, c->bj_ntiles + 1));
    hipLaunchKernelGGL(k_tiles, dim3(grid_for((int64_t)nblocks + 1)), dim3(256), 0, s, c->bj_ntiles, nblocks, bp, n,
                       kTileDofs, c->bj_wg_start);
    // the multi-RHS kernels stage tiles of <= kBatchTileDofs DoFs times 32 columns
    c->bjb_ntiles = (int32_t)((n + kBatchTileWindow - 1) / kBatchTileWindow);
    HT(keep(c, &c->bjb_start, c->bjb_ntiles + 1));
    hipLaunchKernelGGL(k_tiles, dim3(grid_for((int64_t)nblocks + 1)), dim3(256), 0, s, c->bjb_ntiles, nblocks, bp, n,
                       kBatchTileWindow, c->bjb_start);
    // Z by rows (int32 row pointer) for the prolongation
    HT(keep(c, &c->z_ptr, n + 1));
    if (k > 0) {
        hipLaunchKernelGGL(k_to_i32, dim3(grid_for(n + 1)), dim3(256), 0, s, zp, n + 1, c->z_ptr);
        HT(keep(c, &c->z_col, nnz_z));
        HT(keep(c, &c->z_val, nnz_z));
        HT(hipMemcpyAsync(c->z_col, zc, sizeof(int32_t) * nnz_z, hipMemcpyDeviceToDevice, s));
        HT(hipMemcpyAsync(c->z_val, zv, sizeof(double) * nnz_z, hipMemcpyDeviceToDevice, s));
    } else {
        HT(hipMemsetAsync(c->z_ptr, 0, sizeof(int32_t) * (n + 1), s));
    }
    HT(hipGetLastError());
    if (k > 0) {
        const int st = coarse_operator(c, pool, k, zp, zc, ztp, zti, ztv, wl, ws, part, flags, bad, false);
        if (st != DPCG_OK) return st;
        // transposed pointers as int32
        HT(keep(c, &c->zt_ptr, k + 1));
        hipLaunchKernelGGL(k_to_i32, dim3(grid_for(k + 1)), dim3(256), 0, s, ztp, (int64_t)k + 1, c->zt_ptr);
        HT(hipStreamSynchronize(s));
    } else {
        HT(pool.join());
        HT(hipMemcpyAsync(fl, flags, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
        HT(hipStreamSynchronize(s));
        if (fl[3] != INT32_MAX) return DPCG_ENOTSYM;
        if (fl[1] != INT32_MAX) {
            *bad = fl[1];
            return DPCG_EBLOCK_NOT_SPD;
        }
    }
    int b16 = 0;
    HT(hipMemcpy(&b16, b16bad, sizeof(int), hipMemcpyDeviceToHost));
    if (b16) c->bcol16 = nullptr;  // an offset does not fit: the SpMV reads the int32 columns
    return DPCG_OK;
}

// New values of K on the same sparsity pattern: block values, the symmetry test, the
// inverses of the listed blocks (all when list is null), K Z, E and E^-1 again.
int gpu_update_values(dpcg_ctx *c, const int64_t *kp, const int32_t *kc, const double *kv, int32_t nlist,
                      const int32_t *list_host, int64_t *bad) {
    hipStream_t s = c->stream;
    Pool pool{c, {}};
    const int64_t n = c->n;
    const int32_t nb = c->nb, k = c->k, nblocks = c->nblocks;
    if (list_host)
        for (int32_t i = 0; i < nlist; ++i)
            if (list_host[i] < 0 || list_host[i] >= nblocks) return DPCG_EINVAL;
    int64_t *ends = nullptr;  // pinned read-backs
    int *fl = nullptr;
    HT(pool.host(&ends, 2));
    HT(pool.host(&fl, 4));
    HT(hipMemcpyAsync(&ends[0], kp, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HT(hipMemcpyAsync(&ends[1], kp + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HT(hipStreamSynchronize(s));
    if (ends[0] != 0 || ends[1] != c->nnz) return DPCG_EINVAL;
    const int64_t nnz = c->nnz, nnzb = c->nnzb;
    int *flags = nullptr;
    HT(pool.tmp(&flags, 4));
    const int init_flags[4] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
    HT(hipMemcpyAsync(flags, init_flags, sizeof(init_flags), hipMemcpyHostToDevice, s));
    double *mxp = nullptr;
    HT(check_csr(s, pool, n, n, kp, kc, kv, nnz, flags, &mxp));
    HT(hipMemcpyAsync(fl, flags, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
    HT(hipStreamSynchronize(s));
    if (fl[0] != INT32_MAX) return DPCG_EINVAL;
    // the CSR arrays are valid: the block structure must be the stored one
    int64_t *cnt = nullptr;
    HT(pool.tmp(&cnt, nb));
    hipLaunchKernelGGL((k_bsr<false>), dim3(grid_for(nb, 4)), dim3(256), 0, s, nb, kp, kc, kv, cnt, nullptr, nullptr,
                       nullptr, nullptr);
    hipLaunchKernelGGL(k_cmp_counts, dim3(grid_for(nb)), dim3(256), 0, s, nb, cnt, c->brow_ptr, flags + 2);
    HT(hipMemcpyAsync(fl, flags, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
    HT(hipStreamSynchronize(s));
    if (fl[2] != INT32_MAX) return DPCG_EINVAL;
    // max |K| for the symmetry tolerance: mxp[0], from the checks above
    // block values; the block columns must be the stored ones
    int32_t *bcol2 = nullptr, *brow = nullptr;
    HT(pool.tmp(&bcol2, nnzb));
    HT(pool.tmp(&brow, nnzb));
    HT(hipMemsetAsync(c->bval, 0, sizeof(double) * 9 * (size_t)nnzb, s));
    hipLaunchKernelGGL((k_bsr<true>), dim3(grid_for(nb, 4)), dim3(256), 0, s, nb, kp, kc, kv, nullptr, c->brow_ptr,
                       bcol2, c->bval, brow);
    hipLaunchKernelGGL(k_cmp_i32, dim3(grid_for(nnzb)), dim3(256), 0, s, nnzb, bcol2, c->bcol, flags + 2);
    {
        const int gsym = (grid_for(nnzb, 256, 16384) + 7) / 8 * 8;
        int64_t *sympart = nullptr;
        int *need = nullptr;
        HT(pool.tmp(&sympart, 2 * (int64_t)gsym));
        HT(pool.tmp(&need, 1));
        hipLaunchKernelGGL(k_check_sym, dim3(gsym), dim3(256), 0, s, c->brow_ptr, brow, c->bcol, c->bval, nnzb, mxp,
                           1, flags, sympart);
        hipLaunchKernelGGL(k_sym_reduce, dim3(1), dim3(256), 0, s, sympart, gsym, need);
        hipLaunchKernelGGL(k_check_sym_lower, dim3(gsym), dim3(256), 0, s, c->brow_ptr, brow, c->bcol, c->bval, nnzb,
                           mxp, 1, flags, need);
    }
    // block-Jacobi inverses of the listed blocks
    int32_t *list_d = nullptr;
    if (list_host && nlist > 0) {
        HT(pool.tmp(&list_d, nlist));
        HT(hipMemcpyAsync(list_d, list_host, sizeof(int32_t) * nlist, hipMemcpyHostToDevice, s));
    }
    if (!list_host || nlist > 0) {
        const int32_t count = list_host ? nlist : nblocks;
        hipLaunchKernelGGL(k_bj_small, dim3(grid_for(count)), dim3(256), 0, s, nblocks, c->block_ptr, kp, kc, kv,
                           c->bj_moff, c->minv, c->bj_rowoff, c->bj_meta, flags + 1, (const int32_t *)list_d, nlist);
        hipLaunchKernelGGL(k_bj_factor, dim3(std::min<int32_t>(std::max(count, 1), 4096)), dim3(64), 0, s, nblocks,
                           c->block_ptr, kp, kc, kv, c->bj_moff, c->minv, c->bj_rowoff, c->bj_meta, flags + 1,
                           (const int32_t *)list_d, nlist);
    }
    if (c->ndense > 0) {  // the listed dense blocks (all without a list)
        std::vector<int32_t> which;
        if (!list_host) {
            for (int32_t i = 0; i < c->ndense; ++i) which.push_back(i);
        } else {
            std::vector<char> seen(c->ndense, 0);
            for (int32_t i = 0; i < nlist; ++i) {
                auto it = std::lower_bound(c->dense_h.begin(), c->dense_h.end(), list_host[i],
                                           [](const DenseBlk &d, int32_t b) { return d.block < b; });
                if (it != c->dense_h.end() && it->block == list_host[i] && !seen[it - c->dense_h.begin()]) {
                    seen[it - c->dense_h.begin()] = 1;
                    which.push_back((int32_t)(it - c->dense_h.begin()));
                }
            }
        }
        const int st = dense_inverses(c, pool, kp, kc, kv, which, flags + 1);
        if (st != DPCG_OK) return st;
    }
    HT(hipGetLastError());
    HT(hipMemcpyAsync(fl, flags, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
    HT(hipStreamSynchronize(s));
    if (fl[2] != INT32_MAX) return DPCG_EINVAL;
    if (k > 0) {
        int64_t *ztp = nullptr, *zp = nullptr, *wlo = nullptr, *wsize = nullptr, *part = nullptr;
        HT(pool.tmp(&ztp, k + 1));
        HT(pool.tmp(&zp, n + 1));
        HT(pool.tmp(&wlo, k));
        HT(pool.tmp(&wsize, k));
        HT(pool.tmp(&part, (int64_t)k / kScanChunk + 2));
        hipLaunchKernelGGL(k_to_i64, dim3(grid_for(k + 1)), dim3(256), 0, s, c->zt_ptr, (int64_t)k + 1, ztp);
        hipLaunchKernelGGL(k_to_i64, dim3(grid_for(n + 1)), dim3(256), 0, s, c->z_ptr, n + 1, zp);
        hipLaunchKernelGGL(k_kz_window, dim3(k), dim3(256), 0, s, k, ztp, c->zt_idx, kp, kc, wlo, wsize);
        int64_t *ws = nullptr, *wl = nullptr;
        HT(pool.host(&ws, k));
        HT(pool.host(&wl, k));
        HT(hipMemcpyAsync(ws, wsize, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s));
        HT(hipMemcpyAsync(wl, wlo, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s));
        HT(hipStreamSynchronize(s));
        const int st = coarse_operator(c, pool, k, zp, c->z_col, ztp, c->zt_idx, c->zt_val, wl, ws, part, flags, bad,
                                       true);
        if (st != DPCG_OK) return st;
    } else {
        if (fl[3] != INT32_MAX) return DPCG_ENOTSYM;
        if (fl[1] != INT32_MAX) {
            *bad = fl[1];
            return DPCG_EBLOCK_NOT_SPD;
        }
    }
    // binary32 copies of a handle that has run mixed solves
    if (c->bval32) {
        hipLaunchKernelGGL(k_to_f32_s, dim3(grid_for(9 * nnzb, 256, 8192)), dim3(256), 0, s, c->bval, 9 * nnzb, c->bval32);
        hipLaunchKernelGGL(k_to_f32_s, dim3(grid_for(c->bj_values, 256, 8192)), dim3(256), 0, s, c->minv,
                           c->bj_values, c->minv32);
        if (c->ndense > 0)
            hipLaunchKernelGGL(k_to_f32_s, dim3(grid_for(c->dinv_len, 256, 8192)), dim3(256), 0, s, c->dinv,
                               c->dinv_len, c->dinv32);
    }
    HT(hipGetLastError());
    HT(hipStreamSynchronize(s));
    return DPCG_OK;
}

}  // namespace dpcg
