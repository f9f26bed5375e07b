// Host side of the dpcg C ABI: input validation, the one-off factorisations of
// setup (block-Jacobi inverses, K Z, E = Z^T K Z and E^-1), device upload, and the
// solve driver that enqueues the iteration kernels and polls the device flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <thread>
#include <vector>

#include "dpcg_internal.h"

using namespace dpcg;

namespace {

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Runs fn(begin, end) over [0, n) split in contiguous chunks across host threads.
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &fn, int64_t min_chunk = 1024) {
    int nt = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
    if (n < 2 * min_chunk) nt = 1;
    nt = (int)std::min<int64_t>(nt, std::max<int64_t>(1, n / min_chunk));
    if (nt <= 1) {
        fn(0, n);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) {
        const int64_t b = n * t / nt, e = n * (t + 1) / nt;
        th.emplace_back([=, &fn] { fn(b, e); });
    }
    for (auto &x : th) x.join();
}

struct Csr {
    int64_t rows = 0, cols = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> idx;
    std::vector<double> val;
};

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return DPCG_EHIP;         \
    } while (0)

int download(const void *dev, void *host, size_t bytes, hipStream_t s) {
    if (bytes == 0) return DPCG_OK;
    if (!dev) return DPCG_EINVAL;
    HIP_TRY(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
    return DPCG_OK;
}

// Structural checks of a CSR matrix: monotone row pointer, columns in range and
// strictly increasing per row, finite values.
bool valid_csr(const Csr &A) {
    if (A.ptr.size() != (size_t)A.rows + 1 || A.ptr[0] != 0) return false;
    for (int64_t i = 0; i < A.rows; ++i)
        if (A.ptr[i + 1] < A.ptr[i]) return false;
    if ((size_t)A.ptr[A.rows] != A.idx.size()) return false;
    std::atomic<bool> ok{true};
    parallel_for(A.rows, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e && ok; ++i) {
            int64_t prev = -1;
            for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
                const int64_t c = A.idx[p];
                if (c <= prev || c >= A.cols || !std::isfinite(A.val[p])) {
                    ok = false;
                    break;
                }
                prev = c;
            }
        }
    });
    return ok;
}

// |K_ij - K_ji| <= 1e-12 max|K| for every stored entry (a missing mirror counts as 0).
bool symmetric(const Csr &K) {
    double mx = 0.0;
    for (double v : K.val) mx = std::max(mx, std::fabs(v));
    const double tol = 1e-12 * mx;
    std::atomic<bool> ok{true};
    parallel_for(K.rows, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e && ok; ++i)
            for (int64_t p = K.ptr[i]; p < K.ptr[i + 1]; ++p) {
                const int64_t j = K.idx[p];
                const int32_t *lo = K.idx.data() + K.ptr[j], *hi = K.idx.data() + K.ptr[j + 1];
                const int32_t *f = std::lower_bound(lo, hi, (int32_t)i);
                const double m = (f != hi && *f == i) ? K.val[f - K.idx.data()] : 0.0;
                if (std::fabs(K.val[p] - m) > tol) {
                    ok = false;
                    break;
                }
            }
    });
    return ok;
}

// In-place Cholesky of a dense row-major m x m matrix (lower triangle); the pivot
// test: a pivot must exceed m * DBL_EPSILON times its own diagonal entry (not SPD to
// working precision otherwise).
bool chol_small(double *A, int m) {
    for (int j = 0; j < m; ++j) {
        double d = A[j * m + j];
        const double fl = m * DBL_EPSILON * std::fabs(d);
        for (int p = 0; p < j; ++p) d -= A[j * m + p] * A[j * m + p];
        if (!(d > fl) || !std::isfinite(d)) return false;
        const double l = std::sqrt(d);
        A[j * m + j] = l;
        for (int i = j + 1; i < m; ++i) {
            double s = A[i * m + j];
            for (int p = 0; p < j; ++p) s -= A[i * m + p] * A[j * m + p];
            A[i * m + j] = s / l;
        }
    }
    return true;
}

// inv = (L L^T)^{-1} from the lower factor L (m x m); inv is full and symmetric.
void inverse_from_chol(const double *L, int m, double *inv) {
    double Li[kMaxBlock * kMaxBlock];
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
            if (i < j) {
                Li[i * m + j] = 0.0;
                continue;
            }
            double s = (i == j) ? 1.0 : 0.0;
            for (int p = j; p < i; ++p) s -= L[i * m + p] * Li[p * m + j];
            Li[i * m + j] = s / L[i * m + i];
        }
    for (int i = 0; i < m; ++i)
        for (int j = i; j < m; ++j) {
            double s = 0.0;
            for (int p = j; p < m; ++p) s += Li[p * m + i] * Li[p * m + j];
            inv[i * m + j] = s;
            inv[j * m + i] = s;
        }
}

// Blocked right-looking Cholesky of the dense k x k matrix A (row-major, lower); the
// pivot floor is taken against the original diagonal entry.
bool chol_dense(std::vector<double> &A, int64_t k) {
    const int64_t nbk = 64;
    std::vector<double> diag0(k);
    for (int64_t j = 0; j < k; ++j) diag0[j] = A[j * k + j];
    for (int64_t j0 = 0; j0 < k; j0 += nbk) {
        const int64_t j1 = std::min(k, j0 + nbk);
        for (int64_t j = j0; j < j1; ++j) {
            double d = A[j * k + j];
            const double fl = (double)k * DBL_EPSILON * std::fabs(diag0[j]);
            for (int64_t p = j0; p < j; ++p) d -= A[j * k + p] * A[j * k + p];
            if (!(d > fl) || !std::isfinite(d)) return false;
            const double l = std::sqrt(d);
            A[j * k + j] = l;
            for (int64_t i = j + 1; i < j1; ++i) {
                double s = A[i * k + j];
                for (int64_t p = j0; p < j; ++p) s -= A[i * k + p] * A[j * k + p];
                A[i * k + j] = s / l;
            }
        }
        // panel below the diagonal tile: L21 = A21 L11^{-T}
        parallel_for(k - j1, [&](int64_t b, int64_t e) {
            for (int64_t i = j1 + b; i < j1 + e; ++i)
                for (int64_t j = j0; j < j1; ++j) {
                    double s = A[i * k + j];
                    for (int64_t p = j0; p < j; ++p) s -= A[i * k + p] * A[j * k + p];
                    A[i * k + j] = s / A[j * k + j];
                }
        }, 16);
        // trailing update of the lower triangle: A22 -= L21 L21^T
        parallel_for(k - j1, [&](int64_t b, int64_t e) {
            for (int64_t i = j1 + b; i < j1 + e; ++i) {
                const double *li = &A[i * k + j0];
                for (int64_t j = j1; j <= i; ++j) {
                    const double *lj = &A[j * k + j0];
                    double s = 0.0;
                    for (int64_t p = 0; p < j1 - j0; ++p) s += li[p] * lj[p];
                    A[i * k + j] -= s;
                }
            }
        }, 16);
    }
    return true;
}

// E^{-1} = L^{-T} L^{-1} from the lower factor in A (dense, full symmetric output).
void inverse_dense(const std::vector<double> &L, int64_t k, std::vector<double> &inv) {
    // column j of L^{-1} stored as row j of Lt (Lt[j][i] = Linv[i][j], i >= j)
    std::vector<double> Lt((size_t)k * k, 0.0);
    parallel_for(k, [&](int64_t b, int64_t e) {
        for (int64_t j = b; j < e; ++j) {
            double *x = &Lt[j * k];
            for (int64_t i = j; i < k; ++i) {
                double s = (i == j) ? 1.0 : 0.0;
                const double *li = &L[i * k];
                for (int64_t p = j; p < i; ++p) s -= li[p] * x[p];
                x[i] = s / li[i];
            }
        }
    }, 8);
    inv.assign((size_t)k * k, 0.0);
    // inv[i][j] = sum_{p >= max(i,j)} Linv[p][i] Linv[p][j] = sum_p Lt[i][p] Lt[j][p]
    parallel_for(k, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i)
            for (int64_t j = i; j < k; ++j) {
                const double *a = &Lt[i * k], *c = &Lt[j * k];
                double s = 0.0;
                for (int64_t p = j; p < k; ++p) s += a[p] * c[p];
                inv[i * k + j] = s;
            }
    }, 8);
    for (int64_t i = 0; i < k; ++i)
        for (int64_t j = 0; j < i; ++j) inv[i * k + j] = inv[j * k + i];
}

Csr transpose(const Csr &A) {
    Csr T;
    T.rows = A.cols;
    T.cols = A.rows;
    T.ptr.assign(T.rows + 1, 0);
    for (int32_t c : A.idx) T.ptr[c + 1]++;
    for (int64_t i = 0; i < T.rows; ++i) T.ptr[i + 1] += T.ptr[i];
    T.idx.resize(A.idx.size());
    T.val.resize(A.val.size());
    std::vector<int64_t> pos(T.ptr.begin(), T.ptr.end() - 1);
    for (int64_t r = 0; r < A.rows; ++r)
        for (int64_t p = A.ptr[r]; p < A.ptr[r + 1]; ++p) {
            const int64_t q = pos[A.idx[p]]++;
            T.idx[q] = (int32_t)r;
            T.val[q] = A.val[p];
        }
    return T;
}

// K Z row by row (Gustavson) with a dense accumulator per host thread.
Csr multiply(const Csr &K, const Csr &Z) {
    const int64_t n = K.rows, k = Z.cols;
    std::vector<std::vector<int32_t>> cols(n);
    std::vector<std::vector<double>> vals(n);
    parallel_for(n, [&](int64_t b, int64_t e) {
        std::vector<double> acc(k, 0.0);
        std::vector<char> mark(k, 0);
        std::vector<int32_t> touched;
        for (int64_t r = b; r < e; ++r) {
            touched.clear();
            for (int64_t p = K.ptr[r]; p < K.ptr[r + 1]; ++p) {
                const int64_t c = K.idx[p];
                const double kv = K.val[p];
                for (int64_t q = Z.ptr[c]; q < Z.ptr[c + 1]; ++q) {
                    const int32_t j = Z.idx[q];
                    if (!mark[j]) {
                        mark[j] = 1;
                        touched.push_back(j);
                    }
                    acc[j] += kv * Z.val[q];
                }
            }
            std::sort(touched.begin(), touched.end());
            cols[r] = touched;
            vals[r].resize(touched.size());
            for (size_t t = 0; t < touched.size(); ++t) {
                vals[r][t] = acc[touched[t]];
                acc[touched[t]] = 0.0;
                mark[touched[t]] = 0;
            }
        }
    }, 256);
    Csr P;
    P.rows = n;
    P.cols = k;
    P.ptr.assign(n + 1, 0);
    for (int64_t r = 0; r < n; ++r) P.ptr[r + 1] = P.ptr[r] + (int64_t)cols[r].size();
    P.idx.resize(P.ptr[n]);
    P.val.resize(P.ptr[n]);
    for (int64_t r = 0; r < n; ++r) {
        std::copy(cols[r].begin(), cols[r].end(), P.idx.begin() + P.ptr[r]);
        std::copy(vals[r].begin(), vals[r].end(), P.val.begin() + P.ptr[r]);
    }
    return P;
}

template <class T>
int upload(dpcg_ctx *c, T **dst, const T *src, size_t count) {
    const size_t bytes = std::max<size_t>(1, count) * sizeof(T);
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, bytes));
    c->allocations.push_back(p);
    c->device_bytes += (int64_t)bytes;
    if (count) HIP_TRY(hipMemcpyAsync(p, src, count * sizeof(T), hipMemcpyHostToDevice, c->stream));
    *dst = (T *)p;
    return DPCG_OK;
}

template <class T>
int alloc(dpcg_ctx *c, T **dst, size_t count) {
    const size_t bytes = std::max<size_t>(1, count) * sizeof(T);
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, bytes));
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
    const size_t n = (size_t)c->n;
    TRY(alloc(c, &w.r, n));
    TRY(alloc(c, &w.y, n));
    TRY(alloc(c, &w.z, n));
    TRY(alloc(c, &w.q, n));
    TRY(alloc(c, &w.p[0], n));
    TRY(alloc(c, &w.p[1], n));
    TRY(alloc(c, &w.tmp, n));
    TRY(alloc(c, &w.g, (size_t)std::max(1, c->k)));
    TRY(alloc(c, &w.delta, (size_t)std::max(1, c->k)));
    const size_t np = (size_t)std::max({c->spmv.nwg, c->bj_nwg, c->vec_nwg, 1});
    TRY(alloc(c, &w.part_a, np));
    TRY(alloc(c, &w.part_b, np));
    TRY(alloc(c, &w.part_c, np));
    TRY(alloc(c, &w.st, 1));
    HIP_TRY(hipHostMalloc((void **)&w.snap, sizeof(State), hipHostMallocDefault));
    return DPCG_OK;
}

int round_grid(int want) {
    if (want >= 8) want &= ~7;
    return std::max(1, want);
}

void choose_shapes(dpcg_ctx *c) {
    const double avg = c->nb ? (double)c->nnzb / c->nb : 1.0;
    int g = 16;
    if (avg <= 6) g = 4;
    else if (avg <= 14) g = 8;
    else if (avg > 48) g = 32;
    c->spmv.group = g;
    const int rows_per_step = 4 * 64 / g;
    c->spmv.steps = (int)((c->nb + rows_per_step - 1) / rows_per_step);
    c->spmv.nwg = round_grid(std::min(c->spmv.steps, 2048));
    c->vec_nwg = round_grid((int)std::min<int64_t>((c->n + kThreads - 1) / kThreads, 1024));
    c->bj_nwg = round_grid(std::min(c->bj_ntiles, 1024));
}

int setup_impl(dpcg_ctx *c, int64_t n, const int64_t *k_rowptr, const int32_t *k_col, const double *k_val,
               int32_t k, const int64_t *z_rowptr, const int32_t *z_col, const double *z_val, int32_t nblocks,
               const int32_t *block_ptr, int64_t *bad) {
    if (n <= 0 || n % 3 != 0 || n > (int64_t)INT32_MAX / 2 || k < 0 || nblocks <= 0 || nblocks > n)
        return DPCG_EINVAL;
    if (!k_rowptr || !k_col || !k_val || !block_ptr || (k > 0 && (!z_rowptr || !z_col || !z_val)))
        return DPCG_EINVAL;
    hipStream_t s = c->stream;
    c->n = n;
    c->k = k;
    c->nb = (int32_t)(n / 3);
    c->nblocks = nblocks;
    // ---- inputs to host ----
    Csr K;
    K.rows = K.cols = n;
    K.ptr.resize(n + 1);
    TRY(download(k_rowptr, K.ptr.data(), sizeof(int64_t) * (n + 1), s));
    HIP_TRY(hipStreamSynchronize(s));
    if (K.ptr[0] != 0 || K.ptr[n] < 0 || K.ptr[n] > (int64_t)INT32_MAX) return DPCG_EINVAL;
    const int64_t nnz = K.ptr[n];
    K.idx.resize(nnz);
    K.val.resize(nnz);
    TRY(download(k_col, K.idx.data(), sizeof(int32_t) * nnz, s));
    TRY(download(k_val, K.val.data(), sizeof(double) * nnz, s));
    Csr Z;
    Z.rows = n;
    Z.cols = k;
    Z.ptr.assign(n + 1, 0);
    if (k > 0) {
        TRY(download(z_rowptr, Z.ptr.data(), sizeof(int64_t) * (n + 1), s));
        HIP_TRY(hipStreamSynchronize(s));
        if (Z.ptr[0] != 0 || Z.ptr[n] < 0 || Z.ptr[n] > (int64_t)INT32_MAX) return DPCG_EINVAL;
        Z.idx.resize(Z.ptr[n]);
        Z.val.resize(Z.ptr[n]);
        TRY(download(z_col, Z.idx.data(), sizeof(int32_t) * Z.ptr[n], s));
        TRY(download(z_val, Z.val.data(), sizeof(double) * Z.ptr[n], s));
    }
    std::vector<int32_t> bp(nblocks + 1);
    TRY(download(block_ptr, bp.data(), sizeof(int32_t) * (nblocks + 1), s));
    HIP_TRY(hipStreamSynchronize(s));
    // ---- validation ----
    if (!valid_csr(K) || !valid_csr(Z)) return DPCG_EINVAL;
    if (bp[0] != 0 || bp[nblocks] != n) return DPCG_EINVAL;
    for (int32_t b = 0; b < nblocks; ++b) {
        const int32_t m = bp[b + 1] - bp[b];
        if (m < 1 || m > kMaxBlock) {
            *bad = b;
            return DPCG_EINVAL;
        }
    }
    if (!symmetric(K)) return DPCG_ENOTSYM;
    c->nnz = nnz;
    c->nnz_z = (int64_t)Z.idx.size();
    // ---- block-CSR over DoF triplets ----
    const int32_t nb = c->nb;
    std::vector<int32_t> bptr(nb + 1, 0);
    std::vector<std::vector<int32_t>> bcols(nb);
    parallel_for(nb, [&](int64_t b0, int64_t b1) {
        for (int64_t R = b0; R < b1; ++R) {
            auto &v = bcols[R];
            for (int i = 0; i < 3; ++i)
                for (int64_t p = K.ptr[3 * R + i]; p < K.ptr[3 * R + i + 1]; ++p) v.push_back(K.idx[p] / 3);
            std::sort(v.begin(), v.end());
            v.erase(std::unique(v.begin(), v.end()), v.end());
        }
    });
    for (int32_t R = 0; R < nb; ++R) bptr[R + 1] = bptr[R] + (int32_t)bcols[R].size();
    const int64_t nnzb = bptr[nb];
    c->nnzb = nnzb;
    std::vector<int32_t> bcol(nnzb);
    std::vector<double> bval(9 * (size_t)nnzb, 0.0);
    parallel_for(nb, [&](int64_t b0, int64_t b1) {
        for (int64_t R = b0; R < b1; ++R) {
            const auto &v = bcols[R];
            std::copy(v.begin(), v.end(), bcol.begin() + bptr[R]);
            for (int i = 0; i < 3; ++i)
                for (int64_t p = K.ptr[3 * R + i]; p < K.ptr[3 * R + i + 1]; ++p) {
                    const int32_t C = K.idx[p] / 3, j = K.idx[p] % 3;
                    const int64_t pos = bptr[R] + (std::lower_bound(v.begin(), v.end(), C) - v.begin());
                    bval[(size_t)(3 * i + j) * nnzb + pos] = K.val[p];
                }
        }
    });
    bcols.clear();
    bcols.shrink_to_fit();
    // ---- block-Jacobi inverses ----
    std::vector<int64_t> moff(nblocks + 1, 0);
    for (int32_t b = 0; b < nblocks; ++b) moff[b + 1] = moff[b] + (int64_t)(bp[b + 1] - bp[b]) * (bp[b + 1] - bp[b]);
    if (moff[nblocks] > (int64_t)INT32_MAX) return DPCG_EINVAL;
    c->bj_values = moff[nblocks];
    std::vector<double> minv(moff[nblocks]);
    std::vector<int32_t> rowoff(n), meta(n);
    std::atomic<int64_t> first_bad{INT64_MAX};
    parallel_for(nblocks, [&](int64_t b0, int64_t b1) {
        double A[kMaxBlock * kMaxBlock];
        for (int64_t b = b0; b < b1; ++b) {
            const int32_t s0 = bp[b], m = bp[b + 1] - bp[b];
            std::fill(A, A + m * m, 0.0);
            for (int i = 0; i < m; ++i)
                for (int64_t p = K.ptr[s0 + i]; p < K.ptr[s0 + i + 1]; ++p) {
                    const int32_t cc = K.idx[p];
                    if (cc >= s0 && cc < s0 + m) A[i * m + (cc - s0)] = K.val[p];
                }
            if (!chol_small(A, m)) {
                int64_t cur = first_bad.load();
                while (b < cur && !first_bad.compare_exchange_weak(cur, b)) {
                }
                continue;
            }
            inverse_from_chol(A, m, &minv[moff[b]]);
            for (int i = 0; i < m; ++i) {
                rowoff[s0 + i] = (int32_t)(moff[b] + (int64_t)i * m);
                meta[s0 + i] = (m << 8) | i;
            }
        }
    }, 64);
    if (first_bad.load() != INT64_MAX) {
        *bad = first_bad.load();
        return DPCG_EBLOCK_NOT_SPD;
    }
    // tiles of at most kThreads DoFs made of whole blocks
    std::vector<int32_t> tiles{0};
    for (int32_t b = 0; b < nblocks; ++b) {
        if (bp[b + 1] - tiles.back() > kThreads) tiles.push_back(bp[b]);
    }
    tiles.push_back((int32_t)n);
    c->bj_ntiles = (int32_t)tiles.size() - 1;
    // ---- coarse operator ----
    Csr Zt, KZt;
    std::vector<double> einv;
    if (k > 0) {
        Csr KZ = multiply(K, Z);
        c->nnz_kz = (int64_t)KZ.idx.size();
        Zt = transpose(Z);
        std::vector<double> E((size_t)k * k, 0.0);
        parallel_for(k, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) {
                double *Ei = &E[i * k];
                for (int64_t p = Zt.ptr[i]; p < Zt.ptr[i + 1]; ++p) {
                    const int64_t r = Zt.idx[p];
                    const double zr = Zt.val[p];
                    for (int64_t q = KZ.ptr[r]; q < KZ.ptr[r + 1]; ++q) Ei[KZ.idx[q]] += zr * KZ.val[q];
                }
            }
        }, 4);
        for (int64_t i = 0; i < k; ++i)
            for (int64_t j = i + 1; j < k; ++j) {
                const double v = 0.5 * (E[i * k + j] + E[j * k + i]);
                E[i * k + j] = v;
                E[j * k + i] = v;
            }
        KZt = transpose(KZ);
        if (!chol_dense(E, k)) return DPCG_ECOARSE_NOT_SPD;
        inverse_dense(E, k, einv);
        if (Zt.idx.size() > (size_t)INT32_MAX || KZt.idx.size() > (size_t)INT32_MAX) return DPCG_EINVAL;
    }
    // ---- launch shapes and upload ----
    choose_shapes(c);
    TRY(upload(c, &c->brow_ptr, bptr.data(), bptr.size()));
    TRY(upload(c, &c->bcol, bcol.data(), bcol.size()));
    TRY(upload(c, &c->bval, bval.data(), bval.size()));
    TRY(upload(c, &c->minv, minv.data(), minv.size()));
    TRY(upload(c, &c->bj_rowoff, rowoff.data(), rowoff.size()));
    TRY(upload(c, &c->bj_meta, meta.data(), meta.size()));
    TRY(upload(c, &c->bj_wg_start, tiles.data(), tiles.size()));
    std::vector<int32_t> zptr32(n + 1);
    for (int64_t i = 0; i <= n; ++i) zptr32[i] = (int32_t)Z.ptr[i];
    TRY(upload(c, &c->z_ptr, zptr32.data(), zptr32.size()));
    TRY(upload(c, &c->z_col, Z.idx.data(), Z.idx.size()));
    TRY(upload(c, &c->z_val, Z.val.data(), Z.val.size()));
    if (k > 0) {
        std::vector<int32_t> p32(k + 1);
        for (int64_t i = 0; i <= k; ++i) p32[i] = (int32_t)Zt.ptr[i];
        TRY(upload(c, &c->zt_ptr, p32.data(), p32.size()));
        TRY(upload(c, &c->zt_idx, Zt.idx.data(), Zt.idx.size()));
        TRY(upload(c, &c->zt_val, Zt.val.data(), Zt.val.size()));
        for (int64_t i = 0; i <= k; ++i) p32[i] = (int32_t)KZt.ptr[i];
        TRY(upload(c, &c->kzt_ptr, p32.data(), p32.size()));
        TRY(upload(c, &c->kzt_idx, KZt.idx.data(), KZt.idx.size()));
        TRY(upload(c, &c->kzt_val, KZt.val.data(), KZt.val.size()));
        TRY(upload(c, &c->einv, einv.data(), einv.size()));
    }
    TRY(alloc_workspace(c, c->ws[0]));
    TRY(alloc_workspace(c, c->ws[1]));
    HIP_TRY(hipStreamSynchronize(s));
    return DPCG_OK;
}

void release(dpcg_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
    for (void *p : c->allocations) (void)hipFree(p);
    for (auto &w : c->ws) {
        if (w.snap) (void)hipHostFree(w.snap);
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
        LAUNCH(launch_coarse(c, w.g, w.delta, nullptr));
        LAUNCH(launch_prolong(c, um1, w.delta, u, nullptr, nullptr, 0));
    } else if (!guess) {
        HIP_TRY(hipMemsetAsync(u, 0, sizeof(double) * c->n, c->stream));
    }
    LAUNCH(launch_spmv_residual(c, u, f, w.r, w.part_b, w, 1));
    LAUNCH(launch_bj(c, w.r, w.y, &w));
    LAUNCH(launch_restrict(c, w.r, w.y, w.g, &w, 1, c->spmv.nwg, 0, max_iter, record));
    LAUNCH(launch_coarse(c, w.g, w.delta, &w));
    LAUNCH(launch_prolong(c, w.y, w.delta, w.z, &w, w.r, 0));
    return DPCG_OK;
}

int next_event_pair(dpcg_ctx *c, hipEvent_t *a, hipEvent_t *b) {
    if ((size_t)c->events_used + 2 > c->events.size()) {
        for (int i = 0; i < 64; ++i) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
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

int enqueue_iteration(dpcg_ctx *c, Workspace &w, double *u, int max_iter, int record) {
    if (c->timing) {
        hipEvent_t a, b;
        TRY(next_event_pair(c, &a, &b));
        HIP_TRY(hipEventRecord(a, c->stream));
        LAUNCH(launch_spmv_p(c, w));
        HIP_TRY(hipEventRecord(b, c->stream));
    } else {
        LAUNCH(launch_spmv_p(c, w));
    }
    LAUNCH(launch_update_bj(c, u, w));
    LAUNCH(launch_restrict(c, w.r, w.y, w.g, &w, 1, c->bj_nwg, 1, max_iter, record));
    LAUNCH(launch_coarse(c, w.g, w.delta, &w));
    LAUNCH(launch_prolong(c, w.y, w.delta, w.z, &w, w.r, 1));
    return DPCG_OK;
}

int solve_impl(dpcg_ctx *c, Workspace &w, const double *f, double *u, double tol, const dpcg_options *opt_in,
               dpcg_info *info) {
    const double t0 = now_ms();
    dpcg_options opt;
    dpcg_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (!c || !f || !u || !(tol > 0.0) || opt.max_iter < 0) return DPCG_EINVAL;
    if (opt.check_every <= 0) opt.check_every = 16;
    const bool guess = opt.use_initial_guess != 0;
    const int record = opt.record_history != 0;
    if (record) TRY(ensure_history(c, w, (int64_t)opt.max_iter + 1));
    w.hist_len = 0;
    c->events_used = 0;
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
    State init{};
    init.flag = kRunning;
    init.thr = tol * fnorm;
    init.rho_old = 1.0;
    *w.snap = init;
    HIP_TRY(hipMemcpyAsync(w.st, w.snap, sizeof(State), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    TRY(enqueue_start(c, w, f, u, guess, opt.max_iter, record));
    State st;
    TRY(read_state(c, w, st));
    int32_t enq = 0;
    while (st.flag == kRunning && enq < opt.max_iter) {
        const int m = std::min(opt.check_every, opt.max_iter - enq);
        for (int i = 0; i < m; ++i) TRY(enqueue_iteration(c, w, u, opt.max_iter, record));
        enq += m;
        TRY(read_state(c, w, st));
    }
    int status;
    int64_t bad = -1;
    switch (st.flag) {
        case kConverged: status = DPCG_OK; break;
        case kMaxIter: status = DPCG_NOT_CONVERGED; break;
        case kBreakdown: status = DPCG_EBREAKDOWN; bad = st.bad; break;
        default: status = DPCG_NOT_CONVERGED; st.iters_done = enq; break;  // max_iter == 0 after a failed check
    }
    if (c->timing) TRY(collect_events(c, st.iters_done));
    // true residual ||f - K u|| / ||f||
    LAUNCH(launch_spmv_residual(c, u, f, w.tmp, w.part_a, w, 0));
    LAUNCH(launch_reduce_aux(c, w, c->spmv.nwg));
    State fin;
    TRY(read_state(c, w, fin));
    if (record) {
        const int64_t len = (int64_t)st.iters_done + 1;
        w.host_hist.resize(len);
        HIP_TRY(hipMemcpy(w.host_hist.data(), w.hist, sizeof(double) * len, hipMemcpyDeviceToHost));
        for (auto &v : w.host_hist) v /= fnorm;
        w.hist_len = (int32_t)len;
    }
    fill_info(info, status, st.iters_done, std::sqrt(st.rr) / fnorm, std::sqrt(fin.aux) / fnorm, c->setup_ms,
              now_ms() - t0, bad);
    return status;
}

}  // namespace

extern "C" {

void dpcg_default_options(dpcg_options *opt) {
    if (!opt) return;
    opt->max_iter = 20000;
    opt->check_every = 16;
    opt->use_initial_guess = 0;
    opt->record_history = 0;
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

int dpcg_solve(dpcg_handle h, const double *f, double *u, double tol, const dpcg_options *opt, dpcg_info *info) {
    if (!h) return DPCG_EINVAL;
    const int st = solve_impl(h, h->ws[0], f, u, tol, opt, info);
    if (st < 0 && info) info->status = st;
    return st;
}

int dpcg_solve_adjoint(dpcg_handle h, const double *g, double *lambda, double tol, const dpcg_options *opt,
                       dpcg_info *info) {
    if (!h) return DPCG_EINVAL;
    const int st = solve_impl(h, h->ws[1], g, lambda, tol, opt, info);
    if (st < 0 && info) info->status = st;
    return st;
}

void dpcg_destroy(dpcg_handle h) { release(h); }

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
    if (!h) return DPCG_EINVAL;
    h->timing = on != 0;
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
    SYNC_RET(launch_coarse(h, g, delta, nullptr));
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
    if (launch_coarse(h, w.g, w.delta, nullptr) != hipSuccess) return DPCG_EHIP;
    SYNC_RET(launch_prolong(h, w.y, w.delta, z, nullptr, nullptr, 0));
}

}  // extern "C"
