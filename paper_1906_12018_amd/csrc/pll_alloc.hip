// Caching allocators for build workspace.
//
// A label build needs tens of temporary device buffers (distance table,
// bit-vectors, queues, label arena, ...) and a few pinned host records.
// Taking them from hipMalloc / hipHostMalloc and returning them with
// hipFree / hipHostFree on every build costs host time, and the frees can
// wait for the device; in a server that builds while it answers queries
// they stall everything else.  Here freed blocks go to per-device free
// lists instead (best fit within a factor of two of the request) and are
// handed out again; a device keeps at most a bounded number of cached bytes
// and the rest is released.  Callers return a block only once the work that
// used it has completed on the device (they synchronise their stream first),
// so a block is never handed to another stream while still in use.
#include <algorithm>
#include <map>
#include <mutex>
#include <unordered_map>

#include "pll_internal.h"

namespace {

constexpr int kMaxDevices = 64;

struct Block {
    size_t bytes;
    int device;
    bool pinned;
};

struct Pools {
    std::mutex mu;
    std::multimap<size_t, void*> dev_free[kMaxDevices];
    std::multimap<size_t, void*> host_free;
    std::unordered_map<void*, Block> blocks;
    size_t dev_cached[kMaxDevices] = {};
    size_t dev_cap[kMaxDevices] = {};
    size_t host_cached = 0;
};

Pools& pools() {
    static Pools* p = new Pools();  // never destroyed: freeing at exit could outlive the runtime
    return *p;
}

size_t size_class(size_t bytes) {
    if (bytes <= (1u << 20)) return std::max<size_t>(256, (bytes + 4095) & ~size_t(4095));
    return (bytes + (2u << 20) - 1) & ~((size_t(2) << 20) - 1);
}

// Best cached block of at least `want` bytes (and at most twice that).
void* take(std::multimap<size_t, void*>& fl, size_t want, size_t* got) {
    auto it = fl.lower_bound(want);
    if (it == fl.end() || it->first > 2 * want) return nullptr;
    void* p = it->second;
    *got = it->first;
    fl.erase(it);
    return p;
}

void release_cached_device(Pools& P, int dev) {  // mu held
    for (auto& kv : P.dev_free[dev]) {
        P.blocks.erase(kv.second);
        (void)hipFree(kv.second);
    }
    P.dev_free[dev].clear();
    P.dev_cached[dev] = 0;
}

}  // namespace

hipError_t pll_ws_alloc(void** out, size_t bytes) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    const size_t want = size_class(bytes);
    Pools& P = pools();
    {
        std::lock_guard<std::mutex> lk(P.mu);
        size_t got = 0;
        if (void* p = take(P.dev_free[dev], want, &got)) {
            P.dev_cached[dev] -= got;
            *out = p;
            return hipSuccess;
        }
    }
    void* p = nullptr;
    e = hipMalloc(&p, want);
    if (e == hipErrorOutOfMemory) {  // give the cached blocks back and try once more
        std::lock_guard<std::mutex> lk(P.mu);
        release_cached_device(P, dev);
        e = hipMalloc(&p, want);
    }
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(P.mu);
    P.blocks[p] = Block{want, dev, false};
    *out = p;
    return hipSuccess;
}

void pll_ws_free(void* p) {
    if (!p) return;
    Pools& P = pools();
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.blocks.find(p);
    if (it == P.blocks.end() || it->second.pinned) return;
    const int dev = it->second.device;
    const size_t bytes = it->second.bytes;
    if (P.dev_cap[dev] == 0) {
        size_t free_b = 0, total_b = 0;
        int cur = 0;
        if (hipGetDevice(&cur) == hipSuccess && cur == dev && hipMemGetInfo(&free_b, &total_b) == hipSuccess)
            P.dev_cap[dev] = std::min<size_t>(total_b / 16, size_t(32) << 30);
        else
            P.dev_cap[dev] = size_t(4) << 30;
    }
    if (P.dev_cached[dev] + bytes > P.dev_cap[dev]) {
        P.blocks.erase(it);
        int cur = -1;
        const bool sw = hipGetDevice(&cur) == hipSuccess && cur != dev && hipSetDevice(dev) == hipSuccess;
        (void)hipFree(p);
        if (sw) (void)hipSetDevice(cur);
        return;
    }
    P.dev_free[dev].emplace(bytes, p);
    P.dev_cached[dev] += bytes;
}

size_t pll_ws_cached(int device) {
    if (device < 0 || device >= kMaxDevices) return 0;
    Pools& P = pools();
    std::lock_guard<std::mutex> lk(P.mu);
    return P.dev_cached[device];
}

hipError_t pll_pinned_alloc(void** out, size_t bytes) {
    *out = nullptr;
    const size_t want = size_class(bytes);
    Pools& P = pools();
    {
        std::lock_guard<std::mutex> lk(P.mu);
        size_t got = 0;
        if (void* p = take(P.host_free, want, &got)) {
            P.host_cached -= got;
            *out = p;
            return hipSuccess;
        }
    }
    void* p = nullptr;
    const hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(P.mu);
    P.blocks[p] = Block{want, -1, true};
    *out = p;
    return hipSuccess;
}

void pll_pinned_free(void* p) {
    if (!p) return;
    Pools& P = pools();
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.blocks.find(p);
    if (it == P.blocks.end() || !it->second.pinned) return;
    const size_t bytes = it->second.bytes;
    if (P.host_cached + bytes > (size_t(64) << 20)) {
        P.blocks.erase(it);
        (void)hipHostFree(p);
        return;
    }
    P.host_free.emplace(bytes, p);
    P.host_cached += bytes;
}
