// dpcg_solve_noalloc: the FP64 solve with its iteration workspace in a fixed,
// file-scope device array instead of the handle's own workspace, for callers that
// cannot allocate device memory (code under stream capture, tight serving loops).
//
// The array `scratch` below is the library's only such buffer.  Host code never
// passes its name to a kernel or to a copy: in host code the name stands for a
// host-side shadow, not for device memory.  Its device address is taken once per
// device with hipGetSymbolAddress, with that device current, and only that address
// is used afterwards (carved into the solve's vectors, partial sums and state, which
// the kernels receive as arguments).  Each device holds its own copy of the array
// for the life of the process; calls that overlap on one device share it and race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dpcg_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(96) << 20;  // 96 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (the current device), looked up on the
// first call for that device.
hipError_t scratch_address(int dev, char **out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = (char *)g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t dpcg_noalloc_scratch_bytes(void) { return kScratchBytes; }

int dpcg_solve_noalloc(dpcg_handle h, const double *f, double *u, double tol, const dpcg_options *opt,
                       dpcg_info *info) {
    if (!h) return DPCG_EINVAL;
    dpcg_options o;
    dpcg_default_options(&o);
    if (opt) o = *opt;
    if (o.precision != DPCG_PREC_FP64 || o.record_history) {
        if (info) info->status = DPCG_EINVAL;
        return DPCG_EINVAL;
    }
    const size_t need = dpcg::workspace_bytes(h);
    if (need > kScratchBytes) {
        if (info) info->status = DPCG_ETOOBIG;
        return DPCG_ETOOBIG;
    }
    int dev = 0;
    char *base = nullptr;
    if (hipGetDevice(&dev) != hipSuccess || dev != h->device || scratch_address(dev, &base) != hipSuccess) {
        if (info) info->status = DPCG_EHIP;
        return DPCG_EHIP;
    }
    // every array starts from zero, as in a freshly allocated workspace (a previous
    // call's contents stay in the array otherwise)
    if (hipMemsetAsync(base, 0, need, h->stream) != hipSuccess) {
        if (info) info->status = DPCG_EHIP;
        return DPCG_EHIP;
    }
    dpcg::Workspace w;
    dpcg::carve_workspace(h, w, base);
    dpcg::State snap{};
    w.snap = &snap;  // pageable host mirror of the state: nothing to allocate
    // kernel timing draws events from a pool that may create some: off for this call
    const int32_t timing = h->timing;
    h->timing = 0;
    const int st = dpcg::solve_on_workspace(h, w, f, u, tol, &o, info);
    h->timing = timing;
    if (st < 0 && info) info->status = st;
    return st;
}

}  // extern "C"
