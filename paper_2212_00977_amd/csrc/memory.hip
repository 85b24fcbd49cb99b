// Per-device cache of device memory blocks.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <vector>

#include "spc_internal.h"

namespace spc {

namespace {

struct DeviceCache {
    std::multimap<size_t, void *> free_blocks;  // size -> block
};

std::mutex g_mu;
std::vector<DeviceCache> g_cache;

DeviceCache &cache_for_current() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if ((size_t)dev >= g_cache.size()) g_cache.resize((size_t)dev + 1);
    return g_cache[(size_t)dev];
}

void flush_locked(DeviceCache &c) {
    for (auto &kv : c.free_blocks) (void)hipFree(kv.second);
    c.free_blocks.clear();
}

}  // namespace

void *cache_alloc(size_t bytes, size_t *got) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        DeviceCache &c = cache_for_current();
        auto it = c.free_blocks.lower_bound(bytes);
        if (it != c.free_blocks.end() && it->first <= bytes + bytes / 2) {
            void *p = it->second;
            *got = it->first;
            c.free_blocks.erase(it);
            return p;
        }
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(g_mu);
            flush_locked(cache_for_current());
        }
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    *got = bytes;
    return p;
}

void cache_free(void *p, size_t bytes) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    cache_for_current().free_blocks.emplace(bytes, p);
}

void cache_flush() {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &c : g_cache) flush_locked(c);
}

}  // namespace spc
