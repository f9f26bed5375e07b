// Element sensitivities for the adjoint of a solve: for K = sum_e s_e K_e and
// u = K^{-1} f, a loss L(u) with adjoint lambda = K^{-1} dL/du has
// dL/ds_e = -lambda_e^T K_e u_e (the assembled stiffness of Sec. 2.4 is linear in each
// element's modulus; dK^{-1}/ds_e = -K^{-1} K_e K^{-1}).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "dpcg_internal.h"

namespace dpcg {
namespace {

constexpr int kWaves = 4;

// flag[0] = first invalid element (or INT_MAX): size outside [0, kMaxElemDofs], matrix
// range outside [0, kmat_len), a DoF outside [-1, n), or a decreasing pointer.
__global__ __launch_bounds__(256) void k_elem_check(int64_t nel, int64_t n, const int64_t *__restrict__ ep,
                                                    const int32_t *__restrict__ ed, const int64_t *__restrict__ ko,
                                                    int64_t kmat_len, int *flag) {
    for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < nel; e += (int64_t)gridDim.x * 256) {
        const int64_t a = ep[e], b = ep[e + 1], m = b - a, o = ko[e];
        bool ok = (e != 0 || a == 0) && m >= 0 && m <= kMaxElemDofs && o >= 0 && o <= kmat_len - m * m;
        if (ok)
            for (int64_t q = a; q < b; ++q) {
                const int32_t d = ed[q];
                ok = ok && d >= -1 && d < n;
            }
        if (!ok) atomicMin(flag, (int)std::min<int64_t>(e, INT_MAX - 1));
    }
}

// One wave per element: u_e staged in LDS, lanes over the rows of K_e, a fixed-order
// wave reduction.
__global__ __launch_bounds__(64 * kWaves) void k_elem_grad(int64_t nel, const int64_t *__restrict__ ep,
                                                           const int32_t *__restrict__ ed,
                                                           const int64_t *__restrict__ ko,
                                                           const double *__restrict__ km,
                                                           const double *__restrict__ u,
                                                           const double *__restrict__ lam, double *__restrict__ g) {
    __shared__ double ue_s[kWaves][kMaxElemDofs];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double *ue = ue_s[wv];
    for (int64_t e = blockIdx.x * (int64_t)kWaves + wv; e < nel; e += (int64_t)gridDim.x * kWaves) {
        const int64_t a = ep[e];
        const int m = (int)(ep[e + 1] - a);
        const double *K = km + ko[e];
        for (int j = lane; j < m; j += 64) {
            const int32_t d = ed[a + j];
            ue[j] = d >= 0 ? u[d] : 0.0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double acc = 0.0;
        for (int i = lane; i < m; i += 64) {
            const int32_t d = ed[a + i];
            if (d < 0) continue;
            const double *Ki = K + (int64_t)i * m;
            double s = 0.0;
            for (int j = 0; j < m; ++j) s = fma(Ki[j], ue[j], s);
            acc = fma(lam[d], s, acc);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) g[e] = -acc;
        // every lane is done with ue before the next element overwrites it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

}  // namespace

int element_gradient(dpcg_ctx *c, int64_t nel, const int64_t *ep, const int32_t *ed, const int64_t *ko,
                     int64_t kmat_len, const double *km, const double *u, const double *lam, double *g) {
    if (nel == 0) return DPCG_OK;
    hipStream_t s = c->stream;
    int *flag = nullptr;
    if (dev_alloc((void **)&flag, sizeof(int)) != hipSuccess) return DPCG_EHIP;
    const int init = INT_MAX;
    int fl = INT_MAX;
    int st = DPCG_OK;
    const int grid_check = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (nel + 255) / 256));
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(16384, (nel + kWaves - 1) / kWaves));
    if (hipMemcpyAsync(flag, &init, sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess) st = DPCG_EHIP;
    if (st == DPCG_OK) {
        hipLaunchKernelGGL(k_elem_check, dim3(grid_check), dim3(256), 0, s, nel, c->n, ep, ed, ko, kmat_len, flag);
        if (hipGetLastError() != hipSuccess || hipMemcpyAsync(&fl, flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = DPCG_EHIP;
    }
    if (st == DPCG_OK && fl != INT_MAX) st = DPCG_EINVAL;
    if (st == DPCG_OK) {
        hipLaunchKernelGGL(k_elem_grad, dim3(grid), dim3(64 * kWaves), 0, s, nel, ep, ed, ko, km, u, lam, g);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) st = DPCG_EHIP;
    }
    (void)hipStreamSynchronize(s);
    dev_release(flag);
    return st;
}

}  // namespace dpcg
