// Internal data layout of a dpcg handle and the kernel launchers.
//
// Device layout (all in HBM, FP64 values, int32 indices):
//   K   block-CSR over DoF triplets: brow_ptr[nb+1], bcol[nnzb], and the nine
//       entries of each 3x3 block stored row by row as nine planes: the values of
//       block row R (blocks beg..end-1, m = end - beg) occupy bval[9 beg, 9 end) and
//       entry e = 3*i + j of block b sits at bval[9 beg + e*m + (b - beg)], so the
//       lanes working on consecutive blocks of a row read consecutive words and a
//       row's values form one contiguous stretch.
//   M^-1 explicit inverse of each block-Jacobi block of up to kMaxBlock DoFs,
//       row-major, concatenated; per DoF d: bj_rowoff[d] = offset of d's row,
//       bj_meta[d] = size<<8 | (d - block start), 0 for the DoFs of larger blocks.
//       Tile w of the update kernel, [bj_wg_start[w], bj_wg_start[w+1]), holds whole
//       small blocks (a tile may cut a large block).  Blocks of kMaxBlock+1 ..
//       kMaxDense DoFs ("dense blocks", subdomain-sized) keep their inverse in dinv:
//       ld x ld row-major, ld = 32 * ceil(size / 32), zero beyond size.
//   Z   CSR by rows (prolongation), Z^T and (KZ)^T as CSR with k rows
//       (restriction), E^-1 dense row-major with leading dimension einv_ld.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/dpcg.h"

namespace dpcg {

constexpr int kThreads = 256;     // threads per workgroup everywhere
constexpr int kMaxBlock = 18;     // largest block-Jacobi block of the fused (nodal) path
constexpr int kMaxDense = 8192;   // largest block-Jacobi block (dense path above kMaxBlock)
constexpr int kDenseRows = 32;    // rows of a dense block per workgroup of its apply
constexpr int kMaxElemDofs = 256; // largest element (DoFs) of dpcg_element_gradient
constexpr int kCoarseTile = 64;   // E^-1 kept as the lower-triangle tiles of this size
constexpr int kAlphaParts = 64;   // workgroups of the first stage of p^T q
constexpr int kRestrictRound = 4096;  // list entries per round of the restriction's loads (threads x depth)

// tile (I, J), I >= J, of the lower triangle of a matrix of nt x nt tiles: index I (I + 1) / 2 + J
__host__ __device__ inline int64_t coarse_tile_count(int32_t nt) { return (int64_t)nt * (nt + 1) / 2; }
constexpr int kBatchCols = 32;    // columns of the multi-RHS workspace (right-hand sides per batch)
constexpr int kBatchSegEntries = 2048;  // entries per multi-RHS restriction segment
constexpr int kBatchTileWindow = 47;                         // block starts per multi-RHS tile
constexpr int kBatchTileDofs = kBatchTileWindow + kMaxBlock - 1;  // <= 64 DoFs per tile

// The hardware spreads consecutive workgroups round-robin over the 8 XCDs.  The remap
// gives each XCD runs of kXcdChunk consecutive logical workgroups (neighbouring rows,
// whose gathers share that XCD's L2) and deals the runs round-robin over the XCDs, so
// that every XCD gets an even share of any region of the matrix: the crack's enriched
// rows are several times longer than the others and sit in one band of the numbering,
// which one contiguous eighth of the rows per XCD would hand to a single XCD.  The
// last partial group of 8 kXcdChunk workgroups keeps launch order.
constexpr int kXcdChunk = 16;

__device__ __forceinline__ int xcd_remap(int w, int nwg) {
    const int full = nwg / (8 * kXcdChunk) * (8 * kXcdChunk);
    if (w >= full) return w;
    const int i = w >> 3;  // position of w among its XCD's workgroups
    return (i / kXcdChunk) * (8 * kXcdChunk) + (w & 7) * kXcdChunk + (i % kXcdChunk);
}

// v from lane (lane ^ OFF) of the wave, every lane active: OFF 1, 2, 8 as one DPP move per
// 32-bit half (quad permutations, rotation by 8 within a row of 16 lanes), 4 as two (the
// half-row mirror, lane ^ 7, then the quad reversal, ^ 3), 16 as a bit-mode swizzle
// within 32-lane halves, 32 as a permute through the LDS crossbar
template <int OFF>
__device__ __forceinline__ int lane_xor_b32(int v) {
    static_assert(OFF == 1 || OFF == 2 || OFF == 4 || OFF == 8 || OFF == 16 || OFF == 32, "lane offset");
    if constexpr (OFF == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
    else if constexpr (OFF == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
    else if constexpr (OFF == 4)
        return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false), 0x1B, 0xF, 0xF, false);
    else if constexpr (OFF == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);
    else if constexpr (OFF == 16) return __builtin_amdgcn_ds_swizzle(v, 0x401F);
    else return __shfl_xor(v, 32);
}

template <int OFF>
__device__ __forceinline__ double lane_xor(double v) {
    const int lo = lane_xor_b32<OFF>(__double2loint(v)), hi = lane_xor_b32<OFF>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Sum over the wave (every lane active), valid in every lane: exchanges 32, 16, .. 1 lanes apart
__device__ __forceinline__ double wave_sum(double v) {
    v += lane_xor<32>(v);
    v += lane_xor<16>(v);
    v += lane_xor<8>(v);
    v += lane_xor<4>(v);
    v += lane_xor<2>(v);
    v += lane_xor<1>(v);
    return v;
}

// Solver state shared by the kernels of one solve; lives in device memory.  Every
// field is written by exactly one thread of one kernel, and read only by kernels
// that run after that one in stream order.
struct State {
    int32_t flag;        // kRunning, kConverged, kMaxIter, kBreakdown
    int32_t iter;        // index i of the iteration in flight (advanced by the restriction when
                         // the prolongation is fused with beta, else by the prolongation)
    int32_t iters_done;  // final iteration count, set together with the flag
    int32_t bad;         // iteration of a breakdown
    double thr;          // tol * ||f||_2
    double rho[2];       // rho_i = r_i^T z_i in slot i & 1 (beta kernel or fused prolongation),
                         // so rho_{i-1} stays readable
    double alpha;        // alpha_i (k_alpha)
    double beta;         // beta_{i-1} (as rho; 0 at i = 0)
    double rr;           // ||r||^2 of the last check
    double aux;          // scratch scalar for one-off reductions
    double ry;           // r_i^T y_i (the fused restriction, from the update's partials)
    int32_t nonfinite;   // set by the input check
    int32_t pad;
};

enum : int32_t { kRunning = 0, kConverged = 1, kMaxIter = 2, kBreakdown = 3 };

struct Workspace {
    double *r = nullptr, *y = nullptr, *z = nullptr, *q = nullptr, *p[2] = {nullptr, nullptr};
    double *g = nullptr, *delta = nullptr, *tmp = nullptr;
    double *h = nullptr;        // Z^T r for the fused prolongation
    double *cpart = nullptr;    // coarse product: contribution of tile pair (X, Y) to delta_X,
                                // nt x nt x kCoarseTile
    double *hdp = nullptr;      // per tile row X of delta: sum of h_j delta_j over its entries
    double *part_a = nullptr;   // partial sums (p^T q, r^T r, r^T z); sized max grid
    double *part_b = nullptr;
    double *part_c = nullptr;
    double *part_d = nullptr;   // kAlphaParts first-stage sums of p^T q
    double *rout = nullptr;     // mixed precision: FP64 residual f - K u of the refinement
    double *dcor = nullptr;     // mixed precision: correction of one inner solve
    State *st = nullptr;        // device
    State *snap = nullptr;      // pinned host mirror
    double *hist = nullptr;     // device, ||r_i|| per iteration
    int64_t hist_cap = 0;
    std::vector<double> host_hist;
    int32_t hist_len = 0;
};

// Device state of a multi-RHS solve: one recurrence per column, as State.
struct BatchState {
    int32_t any;                 // 1 while some column runs (set by the restriction's check)
    int32_t iter;                // iteration in flight
    int32_t flag[kBatchCols];    // kRunning, kConverged, kMaxIter, kBreakdown per column
    int32_t iters_done[kBatchCols];
    int32_t bad[kBatchCols];
    int32_t pad;
    double thr[kBatchCols];
    double rho[2][kBatchCols];
    double alpha[kBatchCols];
    double beta[kBatchCols];
    double rr[kBatchCols];
    double aux[kBatchCols];      // per-column scratch (norms)
    int32_t nonfinite;
    int32_t pad2;
};

// n x kBatchCols row-major vectors (entry (d, j) at d * kBatchCols + j).
struct BatchWorkspace {
    double *f = nullptr, *u = nullptr, *r = nullptr, *y = nullptr, *z = nullptr, *q = nullptr, *p = nullptr;
    double *g = nullptr, *delta = nullptr;        // k x kBatchCols
    double *part = nullptr, *part2 = nullptr;     // per-workgroup column partials
    BatchState *st = nullptr;                     // device
    BatchState *snap = nullptr;                   // pinned host mirror
    int32_t spmm_nwg = 0, upd_nwg = 0, vec_nwg = 0;
    // the SpMM's slots of two consecutive block rows: pair_len[s] merged block columns
    // when both rows of slot s are short (0 otherwise), the merged columns and each
    // one's block indices in the two rows at pair_col / pair_ab[s * 128 ..]
    int32_t *pair_len = nullptr, *pair_col = nullptr;
    uint16_t *pair_ab = nullptr;
    // restriction segments: seg[4 s .. 4 s + 3] = (column, list 0 = Z^T / 1 = (KZ)^T, begin,
    // end), at most kBatchSegEntries entries each; column c owns segments
    // seg_ptr[c] .. seg_ptr[c + 1] - 1, whose partial sums are added in that order
    int32_t *seg = nullptr, *seg_ptr = nullptr;
    double *seg_part = nullptr;
    int32_t nseg = 0;
    // grouped restriction on the matrix cores, used when runs of vectors share their
    // triplets: gseg[7 s ..] = (first vector, vectors, list, first row entry, first value,
    // rows, row-list length); vector c adds partial row gcol[3c+2] of segments gcol[3c] ..
    // gcol[3c+1]-1; zr, zv: the groups' rows and dense blocks of Z
    int32_t *gseg = nullptr, *gcol = nullptr, *zr = nullptr;
    double *zv = nullptr;
    int32_t ngseg = 0;
    bool grouped = false;
};

// A block-Jacobi block of more than kMaxBlock DoFs and a workgroup of its apply.
struct DenseBlk {
    int64_t off;                    // first entry of its inverse in dinv
    int32_t start, size, ld, block; // first DoF, DoFs, leading dimension, block index
};
struct DenseChunk {
    int32_t dense, row0;            // index in the dense table, first row
};

// Several systems per launch: one descriptor per system (its operator, its forward
// workspace and its state) and, per phase, the prefix offsets of the systems'
// workgroups in the launch grid.
constexpr int kMaxSystems = 64;
enum MsPhase { kMsSpmv = 0, kMsAlpha, kMsBj, kMsRestrict, kMsCoarse, kMsCoarseSum, kMsVec, kMsPhases };

struct MsSys {
    int32_t nb, steps, spmv_nwg, group;
    int32_t k, bj_ntiles, bj_nwg, vec_nwg;
    int32_t guess, pad;
    int64_t n, nnzb, einv_ld;
    const int32_t *brow_ptr, *bcol;
    const double *bval;
    const double *minv;
    const int32_t *bj_rowoff, *bj_meta, *bj_wg_start;
    const int32_t *zt_ptr, *zt_idx;
    const double *zt_val;
    const int32_t *kzt_ptr, *kzt_idx;
    const double *kzt_val;
    const double *einv;
    const int32_t *z_ptr, *z_col;
    const double *z_val;
    const double *f;
    double *u, *r, *y, *z, *q, *p0, *p1, *g, *delta, *part_a, *part_b, *part_c, *part_d, *h;
    const double *einv_tiles;   // the coarse product's packed E^-1 and its workspace
    int32_t coarse_nt, pad2;
    double *cpart, *hdp;
    State *st;
};

struct MsTable {
    int32_t nsys;
    int32_t off[kMsPhases][kMaxSystems + 1];  // off[phase][s]: first workgroup of system s
};

struct SpmvPlan {
    int group = 16;          // lanes per block row
    int nwg = 0;             // workgroups
    int steps = 0;           // row steps in total (rows per step = 4 * 64 / group)
};

}  // namespace dpcg

struct dpcg_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t n = 0, nnz = 0, nnzb = 0, nnz_z = 0, nnz_kz = 0, bj_values = 0, device_bytes = 0;
    int32_t nb = 0, k = 0, nblocks = 0;
    // K
    int32_t *brow_ptr = nullptr, *bcol = nullptr;
    int16_t *bcol16 = nullptr;  // block columns as offsets from their row (null: an offset exceeds 16 bits)
    double *bval = nullptr;
    // FP32 copies (same layouts) for the inner solves of mixed precision; made on the
    // first mixed solve.  inner32 selects them in the launchers while an inner solve runs.
    float *bval32 = nullptr, *minv32 = nullptr;
    bool inner32 = false;
    // block-Jacobi
    double *minv = nullptr;
    int32_t *bj_rowoff = nullptr, *bj_meta = nullptr, *bj_wg_start = nullptr;
    int32_t bj_nwg = 0, bj_ntiles = 0;
    int32_t *bjb_start = nullptr;   // tiles of whole blocks, <= kBatchTileDofs DoFs (multi-RHS)
    int32_t *block_ptr = nullptr;   // the block partition (nblocks + 1), kept for value updates
    int64_t *bj_moff = nullptr;     // offset of each block's inverse in minv (nblocks + 1)
    int32_t bjb_ntiles = 0;
    // dense (subdomain-sized) blocks, in increasing block order
    int32_t ndense = 0, ndchunks = 0, dense_maxld = 0;
    std::vector<dpcg::DenseBlk> dense_h;
    dpcg::DenseBlk *dense = nullptr;
    dpcg::DenseChunk *dchunk = nullptr;
    double *dinv = nullptr;
    float *dinv32 = nullptr;
    int64_t dinv_len = 0;
    dpcg::BatchWorkspace *bws = nullptr;  // multi-RHS workspace, made on the first batched solve
    // deflation
    int32_t *z_ptr = nullptr, *z_col = nullptr;
    double *z_val = nullptr;
    int32_t *zt_ptr = nullptr, *zt_idx = nullptr;
    double *zt_val = nullptr;
    int32_t *kzt_ptr = nullptr, *kzt_idx = nullptr;
    double *kzt_val = nullptr;
    int32_t *rs_order = nullptr;  // the restriction's column order (longer columns first), k entries
    std::vector<int32_t> rs_order_h;  // its host copy (the source of the upload)
    double *einv = nullptr;
    int64_t einv_ld = 0;       // leading dimension of E^-1 (k rounded up to 64)
    double *einv_tiles = nullptr;  // the lower triangle of E^-1 as kCoarseTile^2 row-major tiles,
                                   // zero beyond k (symmetric diagonal tiles stored whole)
    int32_t coarse_nt = 0;         // tiles per side: ceil(k / kCoarseTile)
    int32_t prolong_nwg = 0;       // grid of the fused prolongation (one DoF per thread)
    // launch shapes
    dpcg::SpmvPlan spmv;
    int32_t vec_nwg = 0;       // grid of the elementwise kernels (one DoF per thread)
    dpcg::Workspace ws[2];     // [0] forward solves, [1] adjoint solves
    int32_t part_cap = 0;      // entries of each workspace partial-sum array
    bool tuned = false;        // SpMV lane-group size chosen by measurement (dpcg_autotune)
    std::vector<void *> allocations;
    double setup_ms = 0.0;
    // optional event timing of the SpMV kernel
    int32_t timing = 0;               // time every timing-th SpMV launch (0: off)
    std::vector<hipEvent_t> events;   // pairs (start, stop), reused per solve
    int32_t events_used = 0;
    int64_t spmv_launches = 0;
    double spmv_ms = 0.0;
};

namespace dpcg {

// ---- launchers (kernels.hip); all enqueue on ctx->stream and return hipError_t ----
hipError_t launch_check_finite_norm(const dpcg_ctx *c, const double *a, const double *b, Workspace &w);
hipError_t launch_spmv_plain(const dpcg_ctx *c, const double *x, double *y);
hipError_t launch_spmv_residual(const dpcg_ctx *c, const double *x, const double *f, double *r,
                                double *part, Workspace &w, int check);
// ev0, ev1 (may be null): events that record the kernel's start and end
hipError_t launch_spmv_p(const dpcg_ctx *c, Workspace &w, hipEvent_t ev0, hipEvent_t ev1);
// fused: also the r^T y partials (part_c) for the fused prolongation (no dense blocks)
hipError_t launch_update_bj(const dpcg_ctx *c, double *u, Workspace &w, bool fused = false);
hipError_t launch_beta(const dpcg_ctx *c, Workspace &w);
hipError_t launch_bj(const dpcg_ctx *c, const double *r, double *y, Workspace *w);
hipError_t launch_bj_dense(const dpcg_ctx *c, const double *r, double *y, const State *st);
hipError_t launch_restrict(const dpcg_ctx *c, const double *a, const double *b, double *g, Workspace *w,
                           int check, int n_parts, int iter_offset, int max_iter, int record, bool fused = false);
// delta = E^-1 g on the packed tiles (cpart: the pair contributions, nt^2 T); with h
// given also the tile-row sums hdp of h_j delta_j; st may be null (no state check)
hipError_t launch_coarse(const dpcg_ctx *c, const double *g, double *delta, const State *st, double *cpart,
                         const double *h = nullptr, double *hdp = nullptr);
// z = y + Z delta, rho = r^T y + h^T delta, beta and p in one kernel (after the fused
// update, restriction and coarse product)
hipError_t launch_prolong_p(const dpcg_ctx *c, Workspace &w);
hipError_t launch_prolong(const dpcg_ctx *c, const double *base, const double *delta, double *out,
                          Workspace *w, const double *rdot, int advance);
hipError_t launch_reduce_aux(const dpcg_ctx *c, Workspace &w, int n_parts);
// several systems per launch (tab, sys: device copies); mode 0: start of Algorithm 2
// (restriction of f and of the guess), 1: the merged right-hand side of Algorithm 3
hipError_t launch_ms_spmv_p(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid);
hipError_t launch_ms_spmv_res(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid);
hipError_t launch_ms_alpha(hipStream_t s, const MsSys *sys, int nsys);
hipError_t launch_ms_update_bj(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid);
hipError_t launch_ms_bj(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid);
hipError_t launch_ms_restrict(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid, int mode, int check,
                              int iter_offset, int max_iter);
hipError_t launch_ms_coarse(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid, int with_state);
hipError_t launch_ms_coarse_sum(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid, int with_state);
hipError_t launch_ms_prolong(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid, int mode, int advance);
hipError_t launch_ms_beta(hipStream_t s, const MsTable *tab, const MsSys *sys, int ngrid);
// dst[i] = (float) src[i]
hipError_t launch_to_f32(const dpcg_ctx *c, const double *src, int64_t count, float *dst);
// y += x
hipError_t launch_add(const dpcg_ctx *c, const double *x, double *y);

// dpcg.cpp: the solve workspace (vectors, k-vectors, partial sums, State) as one block
// of workspace_bytes(c) bytes carved by carve_workspace, and a solve on a given one
size_t workspace_bytes(const dpcg_ctx *c);
void carve_workspace(dpcg_ctx *c, Workspace &w, char *base);
int solve_on_workspace(dpcg_ctx *c, Workspace &w, const double *f, double *u, double tol, const dpcg_options *opt,
                       dpcg_info *info);

// setup.hip: new values of K on the same pattern (see dpcg_update_values)
int gpu_update_values(dpcg_ctx *c, const int64_t *kp, const int32_t *kc, const double *kv, int32_t nlist,
                      const int32_t *list_host, int64_t *bad);

// batch.hip: multi-RHS solve (nrhs <= kBatchCols columns, caller arrays n x nrhs
// row-major); returns a DPCG_* status and fills infos[nrhs] when given.
int solve_batch(dpcg_ctx *c, int32_t nrhs, const double *F, double *U, double tol, const dpcg_options *opt,
                dpcg_info *infos);
// Y = K X for nrhs <= kBatchCols columns (n x nrhs row-major) with the multi-RHS product.
int spmv_batch(dpcg_ctx *c, int32_t nrhs, const double *X, double *Y);
void release_batch(dpcg_ctx *c);

// adjoint.hip: g[e] = -lam_e^T K_e u_e after a device-side check of the element data;
// returns a DPCG_* status.
int element_gradient(dpcg_ctx *c, int64_t nel, const int64_t *ep, const int32_t *ed, const int64_t *ko,
                     int64_t kmat_len, const double *km, const double *u, const double *lam, double *g);

// devmem.cpp: cached device allocations (release only after the using stream is idle).
hipError_t dev_alloc(void **p, size_t bytes);
void dev_release(void *p);
hipError_t host_alloc(void **p, size_t bytes);  // pinned host memory, same cache
void host_release(void *p);
void dev_trim();
// a second stream of the current device for setup work beside the main chain, and
// pooled synchronisation events (without timing) of the current device
hipError_t side_stream(hipStream_t *s);
hipError_t sync_event_take(hipEvent_t *ev);
void sync_event_give(hipEvent_t ev);

// setup.hip: all setup factorisations on the GPU; returns a DPCG_* status.
int gpu_setup(dpcg_ctx *c, int64_t n, const int64_t *kp, const int32_t *kc, const double *kv, int32_t k,
              const int64_t *zp, const int32_t *zc, const double *zv, int32_t nblocks, const int32_t *bp,
              int64_t *bad);

}  // namespace dpcg
