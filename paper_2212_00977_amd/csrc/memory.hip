// Per-device cache of device memory blocks, and growable arrays on the
// virtual memory API.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "spc_internal.h"

namespace spc {

namespace {

struct DeviceCache {
    std::multimap<size_t, void *> free_blocks;  // size -> block
    size_t bytes = 0;                           // total held
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
    c.bytes = 0;
}

}  // namespace

void *cache_alloc(size_t bytes, size_t *got) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        DeviceCache &c = cache_for_current();
        auto it = c.free_blocks.lower_bound(bytes);
        if (it != c.free_blocks.end() && it->first <= bytes + bytes / 8) {
            void *p = it->second;
            *got = it->first;
            c.bytes -= it->first;
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
    DeviceCache &c = cache_for_current();
    c.free_blocks.emplace(bytes, p);
    c.bytes += bytes;
}

void cache_trim(size_t max_bytes) {
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCache &c = cache_for_current();
    while (c.bytes > max_bytes && !c.free_blocks.empty()) {
        auto it = std::prev(c.free_blocks.end());  // largest first
        (void)hipFree(it->second);
        c.bytes -= it->first;
        c.free_blocks.erase(it);
    }
}

void cache_flush() {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &c : g_cache) flush_locked(c);
}

// ---------------------------------------------------------------------------
bool vmm_supported() {
    static std::mutex mu;
    static std::vector<int> known;  // per device: -1 unknown, 0 no, 1 yes
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lk(mu);
    if ((size_t)dev >= known.size()) known.resize((size_t)dev + 1, -1);
    if (known[(size_t)dev] < 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeVirtualMemoryManagementSupported, dev) !=
            hipSuccess) {
            (void)hipGetLastError();
            v = 0;
        }
        known[(size_t)dev] = v ? 1 : 0;
    }
    return known[(size_t)dev] == 1;
}

namespace {
hipMemAllocationProp device_prop(int dev) {
    hipMemAllocationProp p{};
    p.type = hipMemAllocationTypePinned;
    p.location.type = hipMemLocationTypeDevice;
    p.location.id = dev;
    return p;
}
constexpr size_t kPieceMin = size_t(2) << 20;  // mapping piece bounds
constexpr size_t kPieceMax = size_t(2) << 30;
// pieces start and end on 2 MiB boundaries (the large-page size), whatever
// smaller granularity the runtime reports
constexpr size_t kPieceAlign = size_t(2) << 20;
}  // namespace

spc_status VArray::reserve(size_t max_bytes) {
    reset();
    if (hipGetDevice(&device_) != hipSuccess) return SPC_ERR_DEVICE;
    hipMemAllocationProp prop = device_prop(device_);
    if (hipMemGetAllocationGranularity(&gran_, &prop, hipMemAllocationGranularityRecommended) !=
            hipSuccess ||
        gran_ == 0) {
        (void)hipGetLastError();
        return SPC_ERR_DEVICE;
    }
    gran_ = (std::max(gran_, kPieceAlign) + kPieceAlign - 1) / kPieceAlign * kPieceAlign;
    size_t bytes = (std::max<size_t>(max_bytes, 1) + gran_ - 1) / gran_ * gran_;
    void *p = nullptr;
    if (hipMemAddressReserve(&p, bytes, 0, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        return SPC_ERR_OUT_OF_MEMORY;
    }
    base_ = p;
    reserved_ = bytes;
    mapped_ = 0;
    return SPC_OK;
}

spc_status VArray::ensure(size_t bytes, size_t *added) {
    *added = 0;
    if (bytes <= mapped_) return SPC_OK;
    if (!base_ || bytes > reserved_) return SPC_ERR_INVALID_ARG;
    hipMemAllocationProp prop = device_prop(device_);
    while (mapped_ < bytes) {
        // pieces grow with the array (at most an eighth of it, within
        // bounds), so an array takes few pieces and little slack
        size_t piece = std::max(bytes - mapped_, std::min(std::max(kPieceMin, mapped_ / 8), kPieceMax));
        piece = (piece + gran_ - 1) / gran_ * gran_;
        piece = std::min(piece, reserved_ - mapped_);
        hipMemGenericAllocationHandle_t h{};
        if (hipMemCreate(&h, piece, &prop, 0) != hipSuccess) {
            (void)hipGetLastError();
            cache_flush();
            if (hipMemCreate(&h, piece, &prop, 0) != hipSuccess) {
                (void)hipGetLastError();
                return SPC_ERR_OUT_OF_MEMORY;
            }
        }
        char *at = static_cast<char *>(base_) + mapped_;
        if (hipMemMap(at, piece, 0, h, 0) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipMemRelease(h);
            return SPC_ERR_DEVICE;
        }
        // access is granted over the whole mapped prefix: the runtime
        // rejects some ranges that start past the reservation's base
        hipMemAccessDesc acc{};
        acc.location = prop.location;
        acc.flags = hipMemAccessFlagsProtReadWrite;
        if (hipMemSetAccess(base_, mapped_ + piece, &acc, 1) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipMemUnmap(at, piece);
            (void)hipMemRelease(h);
            return SPC_ERR_DEVICE;
        }
        pieces_.emplace_back(h, piece);
        mapped_ += piece;
        *added += piece;
    }
    return SPC_OK;
}

void VArray::reset() {
    if (!base_) return;
    size_t off = 0;
    for (auto &pc : pieces_) {
        (void)hipMemUnmap(static_cast<char *>(base_) + off, pc.second);
        (void)hipMemRelease(pc.first);
        off += pc.second;
    }
    pieces_.clear();
    (void)hipMemAddressFree(base_, reserved_);
    base_ = nullptr;
    reserved_ = mapped_ = 0;
}

}  // namespace spc
