// Device memory cache behind DBuf.  Large hipMalloc/hipFree pairs become slow
// (tens of milliseconds each) once several multi-GB buffers are alive, and the
// setup allocates and frees such buffers at every cascade step; cached blocks
// are reused instead.  A freed block keeps hipFree's ordering guarantee: the
// device is synchronised before the block becomes reusable.
#include <map>
#include <mutex>
#include <unordered_map>

#include "cs_internal.h"

namespace cs {
namespace {

constexpr size_t CACHE_CAP = size_t(96) << 30;   // cached bytes per device

struct DevicePool {
    std::multimap<size_t, void *> cached;   // size -> block
    std::unordered_map<void *, size_t> sizes;
    size_t cached_bytes = 0;
};

std::mutex g_mu;
std::map<int, DevicePool> g_pools;
int g_users = 0;

size_t round_size(size_t b) {
    const size_t g = b <= (size_t(1) << 20) ? 4096 : (size_t(2) << 20);
    return (b + g - 1) / g * g;
}

void drop_all(int dev, DevicePool &pool) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(dev);
    for (auto &kv : pool.cached) {
        (void)hipFree(kv.second);
        pool.sizes.erase(kv.second);
    }
    pool.cached.clear();
    pool.cached_bytes = 0;
    (void)hipSetDevice(cur);
}

}  // namespace

void *pool_alloc(size_t bytes) {
    const size_t want = round_size(bytes);
    int dev = 0;
    CS_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_mu);
    DevicePool &pool = g_pools[dev];
    auto it = pool.cached.lower_bound(want);
    if (it != pool.cached.end() && it->first <= 2 * want) {
        void *p = it->second;
        pool.cached_bytes -= it->first;
        pool.cached.erase(it);
        return p;
    }
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        drop_all(dev, pool);   // give the cache back and retry once
        if (hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            fail(CS_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
        }
    }
    pool.sizes[p] = want;
    return p;
}

void pool_free(void *p) {
    if (!p) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lock(g_mu);
    DevicePool &pool = g_pools[dev];
    auto s = pool.sizes.find(p);
    if (s == pool.sizes.end()) {   // not ours (cannot happen): plain free
        (void)hipFree(p);
        return;
    }
    // work still queued on any stream may use the block: wait as hipFree would
    (void)hipDeviceSynchronize();
    if (pool.cached_bytes + s->second > CACHE_CAP) {
        (void)hipFree(p);
        pool.sizes.erase(s);
        return;
    }
    pool.cached.emplace(s->second, p);
    pool.cached_bytes += s->second;
}

void pool_user(int delta) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_users += delta;
    if (g_users == 0)
        for (auto &kv : g_pools) drop_all(kv.first, kv.second);
}

}  // namespace cs
