// Process-wide cache of device memory blocks.  Setting up a handle needs a few dozen
// arrays; a solver that is set up once per system (a crack-growth step) would otherwise
// pay the HIP runtime's allocation and release cost every time.  Blocks are released only
// after the stream that used them has been synchronised, so a cached block is idle and
// may be handed to any stream.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "dpcg_internal.h"

namespace dpcg {

namespace {

struct Cache {
    std::mutex m;
    // (device, rounded size) -> idle blocks
    std::map<std::pair<int, size_t>, std::vector<void *>> idle;
    std::unordered_map<void *, std::pair<int, size_t>> owner;
};

Cache &cache() {
    static Cache *c = new Cache();  // never destroyed: blocks outlive static destructors
    return *c;
}

size_t round_size(size_t bytes) {
    if (bytes <= (size_t(1) << 20)) return (bytes + 255) & ~size_t(255);
    const size_t g = size_t(2) << 20;
    return (bytes + g - 1) / g * g;
}

}  // namespace

hipError_t dev_alloc(void **p, size_t bytes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const size_t sz = round_size(bytes ? bytes : 1);
    Cache &c = cache();
    {
        std::lock_guard<std::mutex> lk(c.m);
        auto it = c.idle.find({dev, sz});
        if (it != c.idle.end() && !it->second.empty()) {
            *p = it->second.back();
            it->second.pop_back();
            return hipSuccess;
        }
    }
    e = hipMalloc(p, sz);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(c.m);
    c.owner[*p] = {dev, sz};
    return hipSuccess;
}

void dev_release(void *p) {
    if (!p) return;
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.m);
    auto it = c.owner.find(p);
    if (it == c.owner.end()) return;
    c.idle[it->second].push_back(p);
}

// Pinned host blocks for the setup's read-backs of sizes and flags: a device-to-host
// copy into pinned memory stays asynchronous, so several of them share one stream
// synchronisation.  Cached like the device blocks (device -1 in the key).
hipError_t host_alloc(void **p, size_t bytes) {
    const size_t sz = round_size(bytes ? bytes : 1);
    Cache &c = cache();
    {
        std::lock_guard<std::mutex> lk(c.m);
        auto it = c.idle.find({-1, sz});
        if (it != c.idle.end() && !it->second.empty()) {
            *p = it->second.back();
            it->second.pop_back();
            return hipSuccess;
        }
    }
    hipError_t e = hipHostMalloc(p, sz, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(c.m);
    c.owner[*p] = {-1, sz};
    return hipSuccess;
}

void host_release(void *p) { dev_release(p); }

// A second stream per device for setup work that runs beside the main chain (default
// priority, created once, kept until the process ends), and a pool of synchronisation
// events (no timing) per device for the fork and join points.  Every setup takes its own
// events, so setups of different handles on the same device may share the stream.
namespace {
struct SideCache {
    std::mutex m;
    std::unordered_map<int, hipStream_t> stream;
    std::map<int, std::vector<hipEvent_t>> events;
};
SideCache &side_cache() {
    static SideCache *c = new SideCache();
    return *c;
}
}  // namespace

hipError_t side_stream(hipStream_t *s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    SideCache &c = side_cache();
    std::lock_guard<std::mutex> lk(c.m);
    auto it = c.stream.find(dev);
    if (it != c.stream.end()) {
        *s = it->second;
        return hipSuccess;
    }
    e = hipStreamCreateWithFlags(s, hipStreamNonBlocking);
    if (e == hipSuccess) c.stream[dev] = *s;
    return e;
}

hipError_t sync_event_take(hipEvent_t *ev) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    SideCache &c = side_cache();
    {
        std::lock_guard<std::mutex> lk(c.m);
        auto &v = c.events[dev];
        if (!v.empty()) {
            *ev = v.back();
            v.pop_back();
            return hipSuccess;
        }
    }
    return hipEventCreateWithFlags(ev, hipEventDisableTiming);
}

void sync_event_give(hipEvent_t ev) {
    if (!ev) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    SideCache &c = side_cache();
    std::lock_guard<std::mutex> lk(c.m);
    c.events[dev].push_back(ev);
}

void dev_trim() {
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.m);
    for (auto &kv : c.idle)
        for (void *p : kv.second) {
            if (kv.first.first < 0) (void)hipHostFree(p);
            else (void)hipFree(p);
            c.owner.erase(p);
        }
    c.idle.clear();
}

}  // namespace dpcg
