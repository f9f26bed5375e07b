// Host side of the dpcg C ABI: argument checks, handle and workspace management, launch
// shapes, and the solve driver that enqueues the iteration kernels and polls the device
// flag.  The setup factorisations run on the GPU (setup.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include <mutex>

#include "dpcg_internal.h"

using namespace dpcg;

namespace dpcg {

namespace {
size_t up256(size_t bytes) { return (bytes + 255) & ~size_t(255); }
// entries of each partial-sum array: the largest SpMV grid any lane-group size can
// choose (autotuner) and the other kernels' grids
size_t partial_count(const dpcg_ctx *c) {
    const int spmv_max = (int)((c->nb + 7) / 8) + 8;
    return (size_t)std::max({spmv_max, c->spmv.nwg, c->bj_nwg, c->vec_nwg, 1});
}
}  // namespace

size_t workspace_bytes(const dpcg_ctx *c) {
    const size_t n = (size_t)c->n, kk = (size_t)std::max(1, c->k), np = partial_count(c);
    const size_t nt = (size_t)std::max(1, c->coarse_nt);
    return 7 * up256(8 * n) + 3 * up256(8 * kk) + 3 * up256(8 * np) + up256(8 * kAlphaParts) +
           up256(8 * nt * nt * kCoarseTile) + up256(8 * nt) + up256(sizeof(State));
}

void carve_workspace(dpcg_ctx *c, Workspace &w, char *base) {
    const size_t n = (size_t)c->n, kk = (size_t)std::max(1, c->k), np = partial_count(c);
    c->part_cap = (int32_t)np;
    double **vec[] = {&w.r, &w.y, &w.z, &w.q, &w.p[0], &w.p[1], &w.tmp};
    double **kv[] = {&w.g, &w.delta, &w.h};
    double **pv[] = {&w.part_a, &w.part_b, &w.part_c};
    size_t off = 0;
    for (double **d : vec) { *d = (double *)(base + off); off += up256(8 * n); }
    for (double **d : kv) { *d = (double *)(base + off); off += up256(8 * kk); }
    for (double **d : pv) { *d = (double *)(base + off); off += up256(8 * np); }
    w.part_d = (double *)(base + off);
    off += up256(8 * kAlphaParts);
    const size_t nt = (size_t)std::max(1, c->coarse_nt);
    w.cpart = (double *)(base + off);
    off += up256(8 * nt * nt * kCoarseTile);
    w.hdp = (double *)(base + off);
    off += up256(8 * nt);
    w.st = (State *)(base + off);
}

}  // namespace dpcg

namespace {

// Pinned state mirrors and timing events are kept in process-wide free lists: creating
// and releasing them costs milliseconds, and handles come and go once per system.
std::mutex g_pool_mutex;
std::vector<State *> g_pinned_states;
std::vector<hipEvent_t> g_events;

State *take_pinned_state() {
    {
        std::lock_guard<std::mutex> lk(g_pool_mutex);
        if (!g_pinned_states.empty()) {
            State *s = g_pinned_states.back();
            g_pinned_states.pop_back();
            return s;
        }
    }
    State *s = nullptr;
    if (hipHostMalloc((void **)&s, sizeof(State), hipHostMallocDefault) != hipSuccess) return nullptr;
    return s;
}

void give_pinned_state(State *s) {
    if (!s) return;
    std::lock_guard<std::mutex> lk(g_pool_mutex);
    g_pinned_states.push_back(s);
}

hipError_t take_event(hipEvent_t *e) {
    {
        std::lock_guard<std::mutex> lk(g_pool_mutex);
        if (!g_events.empty()) {
            *e = g_events.back();
            g_events.pop_back();
            return hipSuccess;
        }
    }
    return hipEventCreate(e);
}

void give_events(std::vector<hipEvent_t> &ev) {
    std::lock_guard<std::mutex> lk(g_pool_mutex);
    g_events.insert(g_events.end(), ev.begin(), ev.end());
    ev.clear();
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return DPCG_EHIP;         \
    } while (0)

template <class T>
int alloc(dpcg_ctx *c, T **dst, size_t count) {
    const size_t bytes = std::max<size_t>(1, count) * sizeof(T);
    void *p = nullptr;
    HIP_TRY(dev_alloc(&p, bytes));
    HIP_TRY(hipMemsetAsync(p, 0, bytes, c->stream));
    c->allocations.push_back(p);
    c->device_bytes += (int64_t)bytes;
    *dst = (T *)p;
    return DPCG_OK;
}

#define TRY(expr)                         \
    do {                                  \
        int s_ = (expr);                  \
        if (s_ != DPCG_OK) return s_;     \
    } while (0)

int alloc_workspace(dpcg_ctx *c, Workspace &w) {
    // one allocation (one zero fill) carved into 256-byte aligned arrays
    char *base = nullptr;
    TRY(alloc(c, &base, workspace_bytes(c)));
    carve_workspace(c, w, base);
    w.snap = take_pinned_state();
    if (!w.snap) return DPCG_EHIP;
    return DPCG_OK;
}

int round_grid(int want) {
    if (want >= 8) want &= ~7;
    return std::max(1, want);
}

void set_spmv_group(dpcg_ctx *c, int g) {
    c->spmv.group = g;
    const int rows_per_step = 4 * 64 / g;  // 4 waves per SpMV workgroup
    c->spmv.steps = (int)((c->nb + rows_per_step - 1) / rows_per_step);
    c->spmv.nwg = c->spmv.steps;  // one row step per workgroup (more per workgroup measured slower)
    if (c->spmv.nwg >= 8) c->spmv.nwg = (c->spmv.nwg + 7) & ~7;
}

void choose_shapes(dpcg_ctx *c) {
    const double avg = c->nb ? (double)c->nnzb / c->nb : 1.0;
    // lanes per block row: one pass over a typical row (measured on gfx950: 32 lanes for
    // rows of ~30 blocks beat 16 lanes with two passes); dpcg_autotune measures instead
    int g = 32;
    if (avg <= 6) g = 4;
    else if (avg <= 12) g = 8;
    else if (avg <= 20) g = 16;
    c->spmv.group = g;
    const int rows_per_step = 4 * 64 / g;  // 4 waves per SpMV workgroup
    c->spmv.steps = (int)((c->nb + rows_per_step - 1) / rows_per_step);
    // one step per workgroup, rounded up to a multiple of 8 (XCD-aware mapping); the
    // extra workgroups find an empty step range
    c->spmv.nwg = c->spmv.steps;  // one row step per workgroup (more per workgroup measured slower)
    if (c->spmv.nwg >= 8) c->spmv.nwg = (c->spmv.nwg + 7) & ~7;
    c->vec_nwg = round_grid((int)std::min<int64_t>((c->n + kThreads - 1) / kThreads, 1024));
    // two rows per thread: half the workgroups, each forming rho once (four measured slower)
    c->prolong_nwg = round_grid((int)std::min<int64_t>((c->n + 2 * kThreads - 1) / (2 * kThreads), 16384));
    c->bj_nwg = round_grid(std::min(c->bj_ntiles, 65536));  // one tile each (partials reduced by one workgroup)
}

int setup_impl(dpcg_ctx *c, int64_t n, const int64_t *k_rowptr, const int32_t *k_col, const double *k_val,
               int32_t k, const int64_t *z_rowptr, const int32_t *z_col, const double *z_val, int32_t nblocks,
               const int32_t *block_ptr, int64_t *bad) {
    if (n <= 0 || n % 3 != 0 || n > (int64_t)INT32_MAX / 2 || k < 0 || nblocks <= 0 || nblocks > n)
        return DPCG_EINVAL;
    if (!k_rowptr || !k_col || !k_val || !block_ptr || (k > 0 && (!z_rowptr || !z_col || !z_val)))
        return DPCG_EINVAL;
    c->n = n;
    c->k = k;
    c->nb = (int32_t)(n / 3);
    c->nblocks = nblocks;
    TRY(gpu_setup(c, n, k_rowptr, k_col, k_val, k, z_rowptr, z_col, z_val, nblocks, block_ptr, bad));
    choose_shapes(c);
    TRY(alloc_workspace(c, c->ws[0]));  // the adjoint workspace is made on the first adjoint solve
    HIP_TRY(hipStreamSynchronize(c->stream));
    return DPCG_OK;
}

void release(dpcg_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    give_events(c->events);
    release_batch(c);
    for (void *p : c->allocations) dev_release(p);
    for (auto &w : c->ws) {
        give_pinned_state(w.snap);
        if (w.hist) (void)hipFree(w.hist);
    }
    delete c;
}

void fill_info(dpcg_info *info, int status, int32_t iters, double rr, double rt, double setup_ms, double solve_ms,
               int64_t bad) {
    if (!info) return;
    info->status = status;
    info->iterations = iters;
    info->rel_res_recursive = rr;
    info->rel_res_true = rt;
    info->setup_ms = setup_ms;
    info->solve_ms = solve_ms;
    info->bad_index = bad;
    info->refinements = 0;
    info->iterations_fp64 = iters;
}

int ensure_history(dpcg_ctx *c, Workspace &w, int64_t need) {
    if (w.hist_cap >= need) return DPCG_OK;
    if (w.hist) HIP_TRY(hipFree(w.hist));
    w.hist = nullptr;
    HIP_TRY(hipMalloc((void **)&w.hist, sizeof(double) * need));
    w.hist_cap = need;
    return DPCG_OK;
}

int read_state(dpcg_ctx *c, Workspace &w, State &out) {
    HIP_TRY(hipMemcpyAsync(w.snap, w.st, sizeof(State), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    out = *w.snap;
    return DPCG_OK;
}

#define LAUNCH(expr)                                      \
    do {                                                  \
        if ((expr) != hipSuccess) return DPCG_EHIP;       \
    } while (0)

// A-DEF2 start and the first preconditioned residual (Algorithm 2, then Algorithm 3 on r_0).
int enqueue_start(dpcg_ctx *c, Workspace &w, const double *f, double *u, bool guess, int max_iter, int record) {
    const double *um1 = guess ? u : nullptr;
    if (c->k > 0) {
        LAUNCH(launch_restrict(c, f, um1, w.g, nullptr, 0, 0, 0, 0, 0));
        LAUNCH(launch_coarse(c, w.g, w.delta, nullptr, w.cpart));
        LAUNCH(launch_prolong(c, um1, w.delta, u, nullptr, nullptr, 0));
    } else if (!guess) {
        HIP_TRY(hipMemsetAsync(u, 0, sizeof(double) * c->n, c->stream));
    }
    LAUNCH(launch_spmv_residual(c, u, f, w.r, w.part_b, w, 1));
    LAUNCH(launch_bj(c, w.r, w.y, &w));
    LAUNCH(launch_restrict(c, w.r, w.y, w.g, &w, 1, c->spmv.nwg, 0, max_iter, record));
    LAUNCH(launch_coarse(c, w.g, w.delta, w.st, w.cpart));
    LAUNCH(launch_prolong(c, w.y, w.delta, w.z, &w, w.r, 0));
    LAUNCH(launch_beta(c, w));
    return DPCG_OK;
}

int next_event_pair(dpcg_ctx *c, hipEvent_t *a, hipEvent_t *b) {
    if ((size_t)c->events_used + 2 > c->events.size()) {
        for (int i = 0; i < 64; ++i) {
            hipEvent_t e;
            HIP_TRY(take_event(&e));
            c->events.push_back(e);
        }
    }
    *a = c->events[c->events_used];
    *b = c->events[c->events_used + 1];
    c->events_used += 2;
    return DPCG_OK;
}

// Adds the durations of the first `real` event pairs of this solve (the SpMV launches of
// iterations that did work; later ones returned at once) and resets the pool.
int collect_events(dpcg_ctx *c, int32_t real) {
    for (int32_t i = 0; i + 1 < c->events_used && i / 2 < real; i += 2) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c->events[i], c->events[i + 1]));
        c->spmv_ms += ms;
        c->spmv_launches += 1;
    }
    c->events_used = 0;
    return DPCG_OK;
}

// index: the iteration's position in this run (timing samples every c->timing-th one)
int enqueue_iteration(dpcg_ctx *c, Workspace &w, double *u, int max_iter, int record, int32_t index) {
    if (c->timing > 0 && index % c->timing == 0) {
        hipEvent_t a, b;
        TRY(next_event_pair(c, &a, &b));
        LAUNCH(launch_spmv_p(c, w, a, b));
    } else {
        LAUNCH(launch_spmv_p(c, w, nullptr, nullptr));
    }
    if (c->ndense == 0) {
        // y comes whole from the update kernel, so its r^T y partials and h = Z^T r give
        // rho = r^T z without z: the prolongation forms beta and p itself
        LAUNCH(launch_update_bj(c, u, w, true));
        LAUNCH(launch_restrict(c, w.r, w.y, w.g, &w, 1, c->bj_nwg, 1, max_iter, record, true));
        LAUNCH(launch_coarse(c, w.g, w.delta, w.st, w.cpart, w.h, w.hdp));
        LAUNCH(launch_prolong_p(c, w));
        return DPCG_OK;
    }
    LAUNCH(launch_update_bj(c, u, w));
    LAUNCH(launch_restrict(c, w.r, w.y, w.g, &w, 1, c->bj_nwg, 1, max_iter, record));
    LAUNCH(launch_coarse(c, w.g, w.delta, w.st, w.cpart));
    LAUNCH(launch_prolong(c, w.y, w.delta, w.z, &w, w.r, 1));
    LAUNCH(launch_beta(c, w));
    return DPCG_OK;
}

// Algorithm 1 from the start of Algorithm 2 on workspace w until the device flag leaves
// kRunning (thr: absolute threshold on ||r_i||).  st receives the final state, with
// iters_done set also when the loop ended by the host-side cap (max_iter == 0).
int run_cg(dpcg_ctx *c, Workspace &w, const double *f, double *u, double thr, bool guess, int max_iter,
           int check_every, int record, State &st) {
    State init{};
    init.flag = kRunning;
    init.thr = thr;
    *w.snap = init;
    HIP_TRY(hipMemcpyAsync(w.st, w.snap, sizeof(State), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->events_used = 0;
    TRY(enqueue_start(c, w, f, u, guess, max_iter, record));
    TRY(read_state(c, w, st));
    int32_t enq = 0;
    while (st.flag == kRunning && enq < max_iter) {
        const int m = std::min(check_every, max_iter - enq);
        for (int i = 0; i < m; ++i) TRY(enqueue_iteration(c, w, u, max_iter, record, enq + i));
        enq += m;
        TRY(read_state(c, w, st));
    }
    if (st.flag == kRunning) st.iters_done = enq;
    if (c->timing > 0) TRY(collect_events(c, (st.iters_done + c->timing - 1) / c->timing));
    return DPCG_OK;
}

// r = f - K u with FP64 K; *rn = ||r||_2.
int true_residual(dpcg_ctx *c, Workspace &w, const double *f, const double *u, double *r, double *rn) {
    LAUNCH(launch_spmv_residual(c, u, f, r, w.part_a, w, 0));
    LAUNCH(launch_reduce_aux(c, w, c->spmv.nwg));
    State fin;
    TRY(read_state(c, w, fin));
    *rn = std::sqrt(fin.aux);
    return DPCG_OK;
}

// binary32 copies of K's block values and of the block inverses (same layouts)
int ensure_fp32(dpcg_ctx *c) {
    if (c->bval32) return DPCG_OK;
    float *bv = nullptr, *mi = nullptr, *di = nullptr;
    TRY(alloc(c, &bv, 9 * (size_t)c->nnzb));
    TRY(alloc(c, &mi, (size_t)std::max<int64_t>(1, c->bj_values)));
    if (c->ndense > 0) {
        TRY(alloc(c, &di, (size_t)c->dinv_len));
        LAUNCH(launch_to_f32(c, c->dinv, c->dinv_len, di));
    }
    LAUNCH(launch_to_f32(c, c->bval, 9 * c->nnzb, bv));
    LAUNCH(launch_to_f32(c, c->minv, c->bj_values, mi));
    c->bval32 = bv;
    c->minv32 = mi;
    c->dinv32 = di;
    return DPCG_OK;
}

// Mixed precision in two phases.  (1) Iterative refinement: FP64 residuals
// r_j = f - K u_j, inner solves K32 d = r_j by the same method on the binary32 copies,
// u_{j+1} = u_j + d, down to max(tol, switch_tol) ||f||.  (2) When switch_tol > tol, the
// FP64 method started from that iterate (Algorithm 2 with u_{-1} = u_j) to tol: each
// refinement cycle multiplies the error by its inner solve's error-to-residual ratio, so
// refinement alone stops at the residual tolerance with a larger error than the FP64
// method reaches there; the FP64 phase takes the error down to the FP64 method's own.
int solve_mixed(dpcg_ctx *c, Workspace &w, const double *f, double *u, double tol, const dpcg_options &opt,
                double fnorm, double t0, dpcg_info *info) {
    TRY(ensure_fp32(c));
    if (!w.rout) {
        TRY(alloc(c, &w.rout, (size_t)c->n));
        TRY(alloc(c, &w.dcor, (size_t)c->n));
    }
    if (!opt.use_initial_guess) HIP_TRY(hipMemsetAsync(u, 0, sizeof(double) * c->n, c->stream));
    const double stop = std::max(tol, opt.switch_tol);
    double rn = 0.0;
    TRY(true_residual(c, w, f, u, w.rout, &rn));
    std::vector<double> hist(1, rn / fnorm);
    int32_t total = 0, cycles = 0, fp64_its = 0;
    int status = DPCG_NOT_CONVERGED;
    int64_t bad = -1;
    while (true) {
        if (!std::isfinite(rn)) {
            status = DPCG_EBREAKDOWN;
            bad = total;
            break;
        }
        if (rn <= stop * fnorm) {
            status = DPCG_OK;
            break;
        }
        if (total >= opt.max_iter || cycles >= opt.max_refinements) break;
        State st;
        // the last cycle aims below the switch point (half of it) so that rounding in
        // K32 - K does not leave the true residual just above it
        const double thr = std::max(opt.inner_tol * rn, 0.5 * opt.switch_tol * fnorm);
        c->inner32 = true;
        const int e = run_cg(c, w, w.rout, w.dcor, thr, false, opt.max_iter - total, opt.check_every, 0, st);
        c->inner32 = false;
        TRY(e);
        total += st.iters_done;
        ++cycles;
        if (st.flag == kBreakdown) {
            status = DPCG_EBREAKDOWN;
            bad = total;
            break;
        }
        LAUNCH(launch_add(c, w.dcor, u));
        TRY(true_residual(c, w, f, u, w.rout, &rn));
        hist.push_back(rn / fnorm);
    }
    double rr = rn / fnorm;
    if (status == DPCG_OK && opt.switch_tol > tol && rn > tol * fnorm) {
        State st;
        c->inner32 = false;
        // the SpMV timing counts the binary32 kernel only: none for the FP64 phase
        const int32_t timing = c->timing;
        c->timing = 0;
        const int e = run_cg(c, w, f, u, tol * fnorm, true, opt.max_iter - total, opt.check_every, 0, st);
        c->timing = timing;
        TRY(e);
        fp64_its = st.iters_done;
        total += st.iters_done;
        switch (st.flag) {
            case kConverged: status = DPCG_OK; break;
            case kBreakdown: status = DPCG_EBREAKDOWN; bad = total; break;
            default: status = DPCG_NOT_CONVERGED; break;
        }
        rr = std::sqrt(st.rr) / fnorm;
        TRY(true_residual(c, w, f, u, w.tmp, &rn));
        hist.push_back(rn / fnorm);
    }
    if (opt.record_history) {
        w.host_hist = hist;
        w.hist_len = (int32_t)hist.size();
    }
    fill_info(info, status, total, rr, rn / fnorm, c->setup_ms, now_ms() - t0, bad);
    if (info) {
        info->refinements = cycles;
        info->iterations_fp64 = fp64_its;
    }
    return status;
}

int solve_impl(dpcg_ctx *c, Workspace &w, const double *f, double *u, double tol, const dpcg_options *opt_in,
               dpcg_info *info) {
    const double t0 = now_ms();
    dpcg_options opt;
    dpcg_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (!c || !f || !u || !(tol > 0.0) || opt.max_iter < 0) return DPCG_EINVAL;
    const bool mixed = opt.precision == DPCG_PREC_MIXED;
    if (!mixed && opt.precision != DPCG_PREC_FP64) return DPCG_EINVAL;
    if (mixed && (!(opt.inner_tol > 0.0 && opt.inner_tol < 1.0) || opt.max_refinements < 0 ||
                  !(opt.switch_tol >= 0.0 && opt.switch_tol < 1.0)))
        return DPCG_EINVAL;
    if (opt.check_every <= 0) opt.check_every = 16;
    const bool guess = opt.use_initial_guess != 0;
    const int record = opt.record_history != 0;
    if (record && !mixed) TRY(ensure_history(c, w, (int64_t)opt.max_iter + 1));
    w.hist_len = 0;
    c->events_used = 0;
    c->inner32 = false;
    // ||f||^2 and the finiteness of the inputs
    LAUNCH(launch_check_finite_norm(c, f, guess ? u : nullptr, w));
    State s0;
    TRY(read_state(c, w, s0));
    if (s0.nonfinite) return DPCG_ENONFINITE;
    const double ff = s0.aux;
    if (ff == 0.0) {
        HIP_TRY(hipMemsetAsync(u, 0, sizeof(double) * c->n, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        if (record) w.host_hist.assign(1, 0.0), w.hist_len = 1;
        fill_info(info, DPCG_OK, 0, 0.0, 0.0, c->setup_ms, now_ms() - t0, -1);
        return DPCG_OK;
    }
    const double fnorm = std::sqrt(ff);
    if (mixed) return solve_mixed(c, w, f, u, tol, opt, fnorm, t0, info);
    State st;
    TRY(run_cg(c, w, f, u, tol * fnorm, guess, opt.max_iter, opt.check_every, record, st));
    int status;
    int64_t bad = -1;
    switch (st.flag) {
        case kConverged: status = DPCG_OK; break;
        case kBreakdown: status = DPCG_EBREAKDOWN; bad = st.bad; break;
        default: status = DPCG_NOT_CONVERGED; break;  // cap reached (on the device or by the host)
    }
    // true residual ||f - K u|| / ||f||
    double rt = 0.0;
    TRY(true_residual(c, w, f, u, w.tmp, &rt));
    if (record) {
        const int64_t len = (int64_t)st.iters_done + 1;
        w.host_hist.resize(len);
        HIP_TRY(hipMemcpy(w.host_hist.data(), w.hist, sizeof(double) * len, hipMemcpyDeviceToHost));
        for (auto &v : w.host_hist) v /= fnorm;
        w.hist_len = (int32_t)len;
    }
    fill_info(info, status, st.iters_done, std::sqrt(st.rr) / fnorm, rt / fnorm, c->setup_ms, now_ms() - t0, bad);
    return status;
}

}  // namespace

namespace dpcg {
int solve_on_workspace(dpcg_ctx *c, Workspace &w, const double *f, double *u, double tol, const dpcg_options *opt,
                       dpcg_info *info) {
    return solve_impl(c, w, f, u, tol, opt, info);
}
}  // namespace dpcg

namespace {

// ---------------------------------------------------------------- several systems
// Measures the SpMV for each lane-group size whose grid fits the workspace and keeps the
// fastest; returns the chosen size.
int autotune_spmv(dpcg_ctx *c, int reps) {
    Workspace &w = c->ws[0];
    const int cand[4] = {4, 8, 16, 32};
    hipEvent_t e0, e1;
    HIP_TRY(take_event(&e0));
    HIP_TRY(take_event(&e1));
    std::vector<hipEvent_t> evs{e0, e1};
    const SpmvPlan keep = c->spmv;
    int best = keep.group;
    float best_ms = 1e30f;
    c->inner32 = false;
    HIP_TRY(hipMemsetAsync(w.p[0], 0, sizeof(double) * c->n, c->stream));
    for (int g : cand) {
        set_spmv_group(c, g);
        if (c->spmv.nwg > c->part_cap) continue;
        LAUNCH(launch_spmv_plain(c, w.p[0], w.q));  // warm-up
        HIP_TRY(hipEventRecord(e0, c->stream));
        for (int i = 0; i < reps; ++i) LAUNCH(launch_spmv_plain(c, w.p[0], w.q));
        HIP_TRY(hipEventRecord(e1, c->stream));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            best = g;
        }
    }
    give_events(evs);
    set_spmv_group(c, best);
    if (c->spmv.nwg > c->part_cap) c->spmv = keep;
    c->tuned = true;
    return c->spmv.group;
}

int round8(int v) { return v >= 8 ? (v + 7) & ~7 : v; }

int solve_many_impl(dpcg_handle *hs, int32_t count, const double *const *F, double *const *U, double tol,
                    const dpcg_options *opt_in, dpcg_info *infos) {
    const double t0 = now_ms();
    dpcg_options opt;
    dpcg_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (!hs || count < 1 || count > kMaxSystems || !F || !U || !(tol > 0.0) || opt.max_iter < 0) return DPCG_EINVAL;
    if (opt.precision != DPCG_PREC_FP64 || opt.record_history) return DPCG_EINVAL;
    if (opt.check_every <= 0) opt.check_every = 16;
    const bool guess = opt.use_initial_guess != 0;
    for (int i = 0; i < count; ++i) {
        if (!hs[i] || !F[i] || !U[i] || hs[i]->device != hs[0]->device || hs[i]->ndense > 0) return DPCG_EINVAL;
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return DPCG_EINVAL;  // one workspace per system
    }
    // all work of the call goes to the first handle's stream
    hipStream_t S = hs[0]->stream;
    std::vector<hipStream_t> own(count);
    for (int i = 0; i < count; ++i) {
        HIP_TRY(hipStreamSynchronize(hs[i]->stream));
        own[i] = hs[i]->stream;
        hs[i]->stream = S;
        hs[i]->inner32 = false;
    }
    struct Restore {
        dpcg_handle *hs;
        std::vector<hipStream_t> &own;
        ~Restore() {
            for (size_t i = 0; i < own.size(); ++i) hs[i]->stream = own[i];
        }
    } restore{hs, own};
    for (int i = 0; i < count; ++i)
        if (!hs[i]->tuned) autotune_spmv(hs[i], 5);
    // norms and finiteness of every right-hand side (and guess)
    std::vector<double> fnorm(count);
    for (int i = 0; i < count; ++i) {
        LAUNCH(launch_check_finite_norm(hs[i], F[i], guess ? U[i] : nullptr, hs[i]->ws[0]));
    }
    HIP_TRY(hipStreamSynchronize(S));
    std::vector<State> st(count);
    for (int i = 0; i < count; ++i) {
        HIP_TRY(hipMemcpyAsync(hs[i]->ws[0].snap, hs[i]->ws[0].st, sizeof(State), hipMemcpyDeviceToHost, S));
    }
    HIP_TRY(hipStreamSynchronize(S));
    for (int i = 0; i < count; ++i) {
        const State &s0 = *hs[i]->ws[0].snap;
        if (s0.nonfinite) return DPCG_ENONFINITE;
        fnorm[i] = std::sqrt(s0.aux);
    }
    // states: zero right-hand sides are done (u = 0) before the first iteration
    for (int i = 0; i < count; ++i) {
        State init{};
        init.flag = fnorm[i] > 0.0 ? kRunning : kConverged;
        init.thr = tol * fnorm[i];
        *hs[i]->ws[0].snap = init;
        HIP_TRY(hipMemcpyAsync(hs[i]->ws[0].st, hs[i]->ws[0].snap, sizeof(State), hipMemcpyHostToDevice, S));
        if (fnorm[i] == 0.0) HIP_TRY(hipMemsetAsync(U[i], 0, sizeof(double) * hs[i]->n, S));
    }
    HIP_TRY(hipStreamSynchronize(S));
    // descriptors and phase offsets
    std::vector<MsSys> sys(count);
    MsTable tab{};
    tab.nsys = count;
    int tot[kMsPhases] = {};
    for (int i = 0; i < count; ++i) {
        dpcg_ctx *c = hs[i];
        Workspace &w = c->ws[0];
        MsSys &d = sys[i];
        d.nb = c->nb;
        d.steps = c->spmv.steps;
        d.spmv_nwg = c->spmv.nwg;
        d.group = c->spmv.group;
        d.k = c->k;
        d.bj_ntiles = c->bj_ntiles;
        d.bj_nwg = c->bj_nwg;
        d.vec_nwg = c->vec_nwg;
        d.guess = guess ? 1 : 0;
        d.pad = 0;
        d.n = c->n;
        d.nnzb = c->nnzb;
        d.einv_ld = c->einv_ld;
        d.brow_ptr = c->brow_ptr;
        d.bcol = c->bcol;
        d.bval = c->bval;
        d.minv = c->minv;
        d.bj_rowoff = c->bj_rowoff;
        d.bj_meta = c->bj_meta;
        d.bj_wg_start = c->bj_wg_start;
        d.zt_ptr = c->zt_ptr;
        d.zt_idx = c->zt_idx;
        d.zt_val = c->zt_val;
        d.kzt_ptr = c->kzt_ptr;
        d.kzt_idx = c->kzt_idx;
        d.kzt_val = c->kzt_val;
        d.einv = c->einv;
        d.z_ptr = c->z_ptr;
        d.z_col = c->z_col;
        d.z_val = c->z_val;
        d.f = F[i];
        d.u = U[i];
        d.r = w.r;
        d.y = w.y;
        d.z = w.z;
        d.q = w.q;
        d.p0 = w.p[0];
        d.p1 = w.p[1];
        d.g = w.g;
        d.delta = w.delta;
        d.part_a = w.part_a;
        d.part_b = w.part_b;
        d.part_c = w.part_c;
        d.part_d = w.part_d;
        d.h = w.h;
        d.einv_tiles = c->einv_tiles;
        d.coarse_nt = c->coarse_nt;
        d.pad2 = 0;
        d.cpart = w.cpart;
        d.hdp = w.hdp;
        d.st = w.st;
        const int n_ph[kMsPhases] = {round8(c->spmv.nwg), 1, round8(c->bj_nwg), std::max(1, c->k),
                                     c->k > 0 ? (int)coarse_tile_count(c->coarse_nt) : 0, c->coarse_nt,
                                     round8(c->vec_nwg)};
        for (int ph = 0; ph < kMsPhases; ++ph) {
            tab.off[ph][i] = tot[ph];
            tot[ph] += n_ph[ph];
        }
    }
    for (int ph = 0; ph < kMsPhases; ++ph) tab.off[ph][count] = tot[ph];
    void *dtab = nullptr, *dsys = nullptr;
    HIP_TRY(dev_alloc(&dtab, sizeof(MsTable)));
    if (dev_alloc(&dsys, sizeof(MsSys) * count) != hipSuccess) {
        dev_release(dtab);
        return DPCG_EHIP;
    }
    struct Release {
        void *a, *b;
        hipStream_t s;
        ~Release() {
            (void)hipStreamSynchronize(s);
            dev_release(a);
            dev_release(b);
        }
    } rel{dtab, dsys, S};
    HIP_TRY(hipMemcpyAsync(dtab, &tab, sizeof(MsTable), hipMemcpyHostToDevice, S));
    HIP_TRY(hipMemcpyAsync(dsys, sys.data(), sizeof(MsSys) * count, hipMemcpyHostToDevice, S));
    const MsTable *T = (const MsTable *)dtab;
    const MsSys *Y = (const MsSys *)dsys;
    const int max_iter = opt.max_iter;
    // Algorithm 2 and the first preconditioned residual, every system at once
    LAUNCH(launch_ms_restrict(S, T, Y, tot[kMsRestrict], 0, 0, 0, 0));
    LAUNCH(launch_ms_coarse(S, T, Y, tot[kMsCoarse], 0));
    LAUNCH(launch_ms_coarse_sum(S, T, Y, tot[kMsCoarseSum], 0));
    LAUNCH(launch_ms_prolong(S, T, Y, tot[kMsVec], 0, 0));
    LAUNCH(launch_ms_spmv_res(S, T, Y, tot[kMsSpmv]));
    LAUNCH(launch_ms_bj(S, T, Y, tot[kMsBj]));
    LAUNCH(launch_ms_restrict(S, T, Y, tot[kMsRestrict], 1, 1, 0, max_iter));
    LAUNCH(launch_ms_coarse(S, T, Y, tot[kMsCoarse], 1));
    LAUNCH(launch_ms_coarse_sum(S, T, Y, tot[kMsCoarseSum], 1));
    LAUNCH(launch_ms_prolong(S, T, Y, tot[kMsVec], 1, 0));
    LAUNCH(launch_ms_beta(S, T, Y, tot[kMsVec]));
    auto read_all = [&]() -> int {
        for (int i = 0; i < count; ++i)
            HIP_TRY(hipMemcpyAsync(hs[i]->ws[0].snap, hs[i]->ws[0].st, sizeof(State), hipMemcpyDeviceToHost, S));
        HIP_TRY(hipStreamSynchronize(S));
        for (int i = 0; i < count; ++i) st[i] = *hs[i]->ws[0].snap;
        return DPCG_OK;
    };
    TRY(read_all());
    int32_t enq = 0;
    auto any_running = [&]() {
        for (int i = 0; i < count; ++i)
            if (st[i].flag == kRunning) return true;
        return false;
    };
    while (any_running() && enq < max_iter) {
        const int m = std::min(opt.check_every, max_iter - enq);
        for (int it = 0; it < m; ++it) {
            LAUNCH(launch_ms_spmv_p(S, T, Y, tot[kMsSpmv]));
            LAUNCH(launch_ms_alpha(S, Y, count));
            LAUNCH(launch_ms_update_bj(S, T, Y, tot[kMsBj]));
            LAUNCH(launch_ms_restrict(S, T, Y, tot[kMsRestrict], 1, 1, 1, max_iter));
            LAUNCH(launch_ms_coarse(S, T, Y, tot[kMsCoarse], 2));
            LAUNCH(launch_ms_coarse_sum(S, T, Y, tot[kMsCoarseSum], 2));
            LAUNCH(launch_ms_prolong(S, T, Y, tot[kMsVec], 2, 0));
        }
        enq += m;
        TRY(read_all());
    }
    int worst = DPCG_OK;
    const double ms = now_ms() - t0;
    for (int i = 0; i < count; ++i) {
        dpcg_ctx *c = hs[i];
        int status;
        int64_t bad = -1;
        switch (st[i].flag) {
            case kConverged: status = DPCG_OK; break;
            case kBreakdown: status = DPCG_EBREAKDOWN; bad = st[i].bad; break;
            default: status = DPCG_NOT_CONVERGED; break;
        }
        if (st[i].flag == kRunning) st[i].iters_done = enq;
        if (status == DPCG_EBREAKDOWN) worst = DPCG_EBREAKDOWN;
        else if (status == DPCG_NOT_CONVERGED && worst == DPCG_OK) worst = DPCG_NOT_CONVERGED;
        double rt = 0.0;
        if (fnorm[i] > 0.0) TRY(true_residual(c, c->ws[0], F[i], U[i], c->ws[0].tmp, &rt));
        if (infos) {
            fill_info(&infos[i], status, fnorm[i] > 0.0 ? st[i].iters_done : 0,
                      fnorm[i] > 0.0 ? std::sqrt(st[i].rr) / fnorm[i] : 0.0, fnorm[i] > 0.0 ? rt / fnorm[i] : 0.0,
                      c->setup_ms, ms, bad);
        }
    }
    return worst;
}

}  // namespace

extern "C" {

void dpcg_default_options(dpcg_options *opt) {
    if (!opt) return;
    opt->max_iter = 20000;
    opt->check_every = 16;
    opt->use_initial_guess = 0;
    opt->record_history = 0;
    opt->precision = DPCG_PREC_FP64;
    opt->max_refinements = 50;
    opt->inner_tol = 1e-4;
    opt->switch_tol = 1e-6;
}

int dpcg_setup(dpcg_handle *h, int64_t n, const int64_t *k_rowptr, const int32_t *k_col, const double *k_val,
               int32_t k, const int64_t *z_rowptr, const int32_t *z_col, const double *z_val, int32_t nblocks,
               const int32_t *block_ptr, void *stream, dpcg_info *info) {
    const double t0 = now_ms();
    if (!h) return DPCG_EINVAL;
    *h = nullptr;
    auto *c = new dpcg_ctx();
    c->stream = (hipStream_t)stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        fill_info(info, DPCG_EHIP, 0, 0, 0, 0, 0, -1);
        return DPCG_EHIP;
    }
    int64_t bad = -1;
    int st = setup_impl(c, n, k_rowptr, k_col, k_val, k, z_rowptr, z_col, z_val, nblocks, block_ptr, &bad);
    c->setup_ms = now_ms() - t0;
    fill_info(info, st, 0, 0.0, 0.0, c->setup_ms, 0.0, bad);
    if (st != DPCG_OK) {
        release(c);
        return st;
    }
    *h = c;
    return DPCG_OK;
}

int dpcg_setup_host(dpcg_handle *h, int64_t n, const int64_t *k_rowptr, const int32_t *k_col, const double *k_val,
                    int32_t k, const int64_t *z_rowptr, const int32_t *z_col, const double *z_val, int32_t nblocks,
                    const int32_t *block_ptr, void *stream, dpcg_info *info) {
    const double t0 = now_ms();
    if (!h) return DPCG_EINVAL;
    *h = nullptr;
    if (n <= 0 || k < 0 || nblocks <= 0 || !k_rowptr || !k_col || !k_val || !block_ptr ||
        (k > 0 && (!z_rowptr || !z_col || !z_val))) {
        fill_info(info, DPCG_EINVAL, 0, 0, 0, 0, 0, -1);
        return DPCG_EINVAL;
    }
    const int64_t nnz = k_rowptr[n], nnz_z = k > 0 ? z_rowptr[n] : 0;
    if (nnz < 0 || nnz_z < 0 || k_rowptr[0] != 0 || (k > 0 && z_rowptr[0] != 0)) {
        fill_info(info, DPCG_EINVAL, 0, 0, 0, 0, 0, -1);
        return DPCG_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    // device copies of the inputs (the setup copies what it keeps, so they go back to
    // the allocation cache once it has finished)
    struct Up {
        void *p = nullptr;
        ~Up() { if (p) dev_release(p); }
    } kp, kc, kv, zp, zc, zv, bp;
    auto up = [&](Up &d, const void *src, size_t bytes) -> bool {
        if (dev_alloc(&d.p, std::max<size_t>(bytes, 1)) != hipSuccess) return false;
        return bytes == 0 || hipMemcpyAsync(d.p, src, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
    };
    bool ok = up(kp, k_rowptr, sizeof(int64_t) * (n + 1)) && up(kc, k_col, sizeof(int32_t) * nnz) &&
              up(kv, k_val, sizeof(double) * nnz) && up(bp, block_ptr, sizeof(int32_t) * (nblocks + 1));
    if (ok && k > 0)
        ok = up(zp, z_rowptr, sizeof(int64_t) * (n + 1)) && up(zc, z_col, sizeof(int32_t) * nnz_z) &&
             up(zv, z_val, sizeof(double) * nnz_z);
    if (!ok) {
        (void)hipStreamSynchronize(s);
        fill_info(info, DPCG_EHIP, 0, 0, 0, 0, 0, -1);
        return DPCG_EHIP;
    }
    const int st = dpcg_setup(h, n, (const int64_t *)kp.p, (const int32_t *)kc.p, (const double *)kv.p, k,
                              (const int64_t *)zp.p, (const int32_t *)zc.p, (const double *)zv.p, nblocks,
                              (const int32_t *)bp.p, stream, info);
    (void)hipStreamSynchronize(s);  // the uploads are released only once the stream is past them
    if (st == DPCG_OK) (*h)->setup_ms = now_ms() - t0;
    if (info) info->setup_ms = now_ms() - t0;
    return st;
}

int dpcg_solve(dpcg_handle h, const double *f, double *u, double tol, const dpcg_options *opt, dpcg_info *info) {
    if (!h) return DPCG_EINVAL;
    const int st = solve_impl(h, h->ws[0], f, u, tol, opt, info);
    if (st < 0 && info) info->status = st;
    return st;
}

int dpcg_solve_many(dpcg_handle *handles, int32_t count, const double *const *F, double *const *U, double tol,
                    const dpcg_options *opt, dpcg_info *infos) {
    return solve_many_impl(handles, count, F, U, tol, opt, infos);
}

int dpcg_update_values(dpcg_handle h, const int64_t *k_rowptr, const int32_t *k_col, const double *k_val,
                       int32_t nchanged, const int32_t *changed_blocks, dpcg_info *info) {
    const double t0 = now_ms();
    if (!h || !k_rowptr || !k_col || !k_val || (changed_blocks && nchanged < 0)) return DPCG_EINVAL;
    int64_t bad = -1;
    h->inner32 = false;
    const int st = gpu_update_values(h, k_rowptr, k_col, k_val, changed_blocks ? nchanged : 0, changed_blocks, &bad);
    h->setup_ms = now_ms() - t0;
    fill_info(info, st, 0, 0.0, 0.0, h->setup_ms, 0.0, bad);
    return st;
}

int dpcg_autotune(dpcg_handle h, int32_t reps) {
    if (!h || reps < 1) return DPCG_EINVAL;
    const int g = autotune_spmv(h, reps);
    return g > 0 ? g : DPCG_EHIP;
}

int dpcg_solve_batch(dpcg_handle h, int32_t nrhs, const double *F, double *U, double tol, const dpcg_options *opt,
                     dpcg_info *infos) {
    if (!h) return DPCG_EINVAL;
    h->inner32 = false;
    return solve_batch(h, nrhs, F, U, tol, opt, infos);
}

int dpcg_solve_adjoint(dpcg_handle h, const double *g, double *lambda, double tol, const dpcg_options *opt,
                       dpcg_info *info) {
    if (!h) return DPCG_EINVAL;
    if (!h->ws[1].st) {
        const int e = alloc_workspace(h, h->ws[1]);
        if (e != DPCG_OK) {
            if (info) info->status = e;
            return e;
        }
    }
    const int st = solve_impl(h, h->ws[1], g, lambda, tol, opt, info);
    if (st < 0 && info) info->status = st;
    return st;
}

void dpcg_destroy(dpcg_handle h) { release(h); }

void dpcg_release_cached_memory(void) { dev_trim(); }

const char *dpcg_status_string(int status) {
    switch (status) {
        case DPCG_OK: return "converged";
        case DPCG_NOT_CONVERGED: return "iteration limit reached before the tolerance";
        case DPCG_EINVAL: return "invalid argument (sizes, indices, ordering or block partition)";
        case DPCG_ENOTSYM: return "matrix is not symmetric";
        case DPCG_EBLOCK_NOT_SPD: return "a block-Jacobi block is not symmetric positive definite";
        case DPCG_ECOARSE_NOT_SPD: return "coarse matrix Z^T K Z is not SPD (Z rank deficient)";
        case DPCG_EBREAKDOWN: return "CG breakdown (p^T K p <= 0 or non-finite scalar)";
        case DPCG_EHIP: return "HIP runtime or allocation failure";
        case DPCG_ENONFINITE: return "non-finite value in an input vector";
        case DPCG_ETOOBIG: return "problem too large for the fixed scratch of the allocation-free solve";
        default: return "unknown status";
    }
}

int dpcg_get_stats(dpcg_handle h, dpcg_stats *out) {
    if (!h || !out) return DPCG_EINVAL;
    out->n = h->n;
    out->nnz = h->nnz;
    out->nnzb = h->nnzb;
    out->k = h->k;
    out->nnz_z = h->nnz_z;
    out->nnz_kz = h->nnz_kz;
    out->nblocks = h->nblocks;
    out->bj_values = h->bj_values;
    out->device_bytes = h->device_bytes;
    out->dense_blocks = h->ndense;
    out->dense_values = h->dinv_len;
    out->spmv_col_bytes = h->bcol16 ? 2 : 4;
    return DPCG_OK;
}

int64_t dpcg_get_history(dpcg_handle h, double *out, int64_t cap) {
    if (!h || (!out && cap > 0)) return DPCG_EINVAL;
    const auto &w = h->ws[0];
    const int64_t m = std::min<int64_t>(cap, w.hist_len);
    if (m > 0) std::memcpy(out, w.host_hist.data(), sizeof(double) * m);
    return m;
}

int dpcg_set_timing(dpcg_handle h, int32_t on) {
    if (!h || on < 0) return DPCG_EINVAL;
    h->timing = on;
    h->events_used = 0;
    if (h->timing) {
        h->spmv_launches = 0;
        h->spmv_ms = 0.0;
    }
    return DPCG_OK;
}

int dpcg_get_timing(dpcg_handle h, dpcg_timing *out) {
    if (!h || !out) return DPCG_EINVAL;
    out->spmv_launches = h->spmv_launches;
    out->spmv_ms = h->spmv_ms;
    return DPCG_OK;
}

#define SYNC_RET(expr)                                               \
    do {                                                             \
        if ((expr) != hipSuccess) return DPCG_EHIP;                  \
        if (hipStreamSynchronize(h->stream) != hipSuccess) return DPCG_EHIP; \
        return DPCG_OK;                                              \
    } while (0)

int dpcg_spmv(dpcg_handle h, const double *x, double *y) {
    if (!h || !x || !y) return DPCG_EINVAL;
    SYNC_RET(launch_spmv_plain(h, x, y));
}

int dpcg_spmv_batch(dpcg_handle h, int32_t nrhs, const double *X, double *Y) {
    if (!h) return DPCG_EINVAL;
    return spmv_batch(h, nrhs, X, Y);
}

int dpcg_spmv_fp32(dpcg_handle h, const double *x, double *y) {
    if (!h || !x || !y) return DPCG_EINVAL;
    const int e = ensure_fp32(h);
    if (e != DPCG_OK) return e;
    h->inner32 = true;
    const hipError_t he = launch_spmv_plain(h, x, y);
    h->inner32 = false;
    SYNC_RET(he);
}

int dpcg_bj_apply_fp32(dpcg_handle h, const double *r, double *y) {
    if (!h || !r || !y) return DPCG_EINVAL;
    const int e = ensure_fp32(h);
    if (e != DPCG_OK) return e;
    h->inner32 = true;
    const hipError_t he = launch_bj(h, r, y, nullptr);
    h->inner32 = false;
    SYNC_RET(he);
}

int dpcg_element_gradient(dpcg_handle h, int64_t nel, const int64_t *elem_ptr, const int32_t *elem_dof,
                          const int64_t *kmat_off, int64_t kmat_len, const double *kmat, const double *u,
                          const double *lambda, double *g) {
    if (!h || nel < 0 || kmat_len < 0) return DPCG_EINVAL;
    if (nel > 0 && (!elem_ptr || !elem_dof || !kmat_off || !kmat || !u || !lambda || !g)) return DPCG_EINVAL;
    return element_gradient(h, nel, elem_ptr, elem_dof, kmat_off, kmat_len, kmat, u, lambda, g);
}

int dpcg_bj_apply(dpcg_handle h, const double *r, double *y) {
    if (!h || !r || !y) return DPCG_EINVAL;
    SYNC_RET(launch_bj(h, r, y, nullptr));
}

int dpcg_restrict(dpcg_handle h, const double *a, const double *b, double *g) {
    if (!h || !a || !g) return DPCG_EINVAL;
    if (h->k == 0) return DPCG_OK;
    SYNC_RET(launch_restrict(h, a, b, g, nullptr, 0, 0, 0, 0, 0));
}

int dpcg_coarse_apply(dpcg_handle h, const double *g, double *delta) {
    if (!h || !g || !delta) return DPCG_EINVAL;
    if (h->k == 0) return DPCG_OK;
    SYNC_RET(launch_coarse(h, g, delta, nullptr, h->ws[0].cpart));
}

int dpcg_prolong(dpcg_handle h, const double *base, const double *delta, double *out) {
    if (!h || !out || (h->k > 0 && !delta)) return DPCG_EINVAL;
    SYNC_RET(launch_prolong(h, base, delta, out, nullptr, nullptr, 0));
}

int dpcg_precond(dpcg_handle h, const double *r, double *z) {
    if (!h || !r || !z) return DPCG_EINVAL;
    Workspace &w = h->ws[0];
    if (launch_bj(h, r, w.y, nullptr) != hipSuccess) return DPCG_EHIP;
    if (h->k == 0) {
        if (hipMemcpyAsync(z, w.y, sizeof(double) * h->n, hipMemcpyDeviceToDevice, h->stream) != hipSuccess)
            return DPCG_EHIP;
        return hipStreamSynchronize(h->stream) == hipSuccess ? DPCG_OK : DPCG_EHIP;
    }
    if (launch_restrict(h, r, w.y, w.g, nullptr, 0, 0, 0, 0, 0) != hipSuccess) return DPCG_EHIP;
    if (launch_coarse(h, w.g, w.delta, nullptr, w.cpart) != hipSuccess) return DPCG_EHIP;
    SYNC_RET(launch_prolong(h, w.y, w.delta, z, nullptr, nullptr, 0));
}

}  // extern "C"
