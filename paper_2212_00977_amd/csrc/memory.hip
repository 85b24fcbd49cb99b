// Per-device cache of device memory: a pool of physical pieces behind large
// blocks and growable arrays (virtual memory API), and hipMalloc segments
// sub-allocated (best fit, split, coalesced on free) for the smaller ones.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "spc_internal.h"
#include "suballoc.h"

namespace spc {

namespace {

using Handle = hipMemGenericAllocationHandle_t;

// hipMalloc segments of the current device for the sub-allocator (not
// mapped pieces: the runtime refuses copies from mapped ranges into pageable
// host memory, which the exports make)
struct HipSegments {
    size_t round(size_t n) const { return n; }
    void *allocate(size_t n) {
        void *p = nullptr;
        if (hipMalloc(&p, n) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void release(void *p, size_t) { (void)hipFree(p); }
};

struct DeviceCache {
    SubAlloc<HipSegments> sub;   // blocks below kPoolMin
    std::vector<Handle> pieces;  // free pieces of kPoolPiece bytes
};

// a large block: an address range with pooled pieces mapped behind it
struct Mapped {
    size_t bytes = 0;
    int dev = 0;
    std::vector<Handle> pieces;
};

std::recursive_mutex g_mu;  // guards g_cache and g_mapped
std::map<int, DeviceCache> g_cache;
std::map<void *, Mapped> g_mapped;

int current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        dev = 0;
    }
    return dev;
}

DeviceCache &cache_of(int dev) { return g_cache[dev]; }

// whole free segments back to the runtime (the device must be current)
void release_blocks_locked(DeviceCache &c) { c.sub.trim(0); }

void release_pieces_locked(DeviceCache &c) {
    for (Handle h : c.pieces) (void)hipMemRelease(h);
    c.pieces.clear();
}

hipMemAllocationProp device_prop(int dev) {
    hipMemAllocationProp p{};
    p.type = hipMemAllocationTypePinned;
    p.location.type = hipMemLocationTypeDevice;
    p.location.id = dev;
    return p;
}

hipMemAccessDesc device_access(int dev) {
    hipMemAccessDesc acc{};
    acc.location = device_prop(dev).location;
    acc.flags = hipMemAccessFlagsProtReadWrite;
    return acc;
}

// a block of n pooled pieces mapped at one address range; nullptr on failure
void *mapped_alloc(int dev, size_t n) {
    const size_t bytes = n * kPoolPiece;
    void *va = nullptr;
    if (hipMemAddressReserve(&va, bytes, 0, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::vector<Handle> hs;
    if (!pool_take(dev, n, &hs)) {
        (void)hipMemAddressFree(va, bytes);
        return nullptr;
    }
    size_t done = 0;
    bool ok = true;
    for (; done < n; done++)
        if (hipMemMap(static_cast<char *>(va) + done * kPoolPiece, kPoolPiece, 0, hs[done], 0) !=
            hipSuccess) {
            ok = false;
            break;
        }
    const hipMemAccessDesc acc = device_access(dev);
    if (ok && hipMemSetAccess(va, bytes, &acc, 1) != hipSuccess) ok = false;
    if (!ok) {
        (void)hipGetLastError();
        for (size_t i = 0; i < done; i++) (void)hipMemUnmap(static_cast<char *>(va) + i * kPoolPiece, kPoolPiece);
        (void)hipMemAddressFree(va, bytes);
        pool_give(dev, hs.data(), hs.size());
        return nullptr;
    }
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    Mapped &m = g_mapped[va];
    m.bytes = bytes;
    m.dev = dev;
    m.pieces = std::move(hs);
    return va;
}

// unmaps a large block and pools its pieces; false if p is not one
bool mapped_free(void *p) {
    Mapped m;
    {
        std::lock_guard<std::recursive_mutex> lk(g_mu);
        auto it = g_mapped.find(p);
        if (it == g_mapped.end()) return false;
        m = std::move(it->second);
        g_mapped.erase(it);
    }
    for (size_t i = 0; i < m.pieces.size(); i++)
        (void)hipMemUnmap(static_cast<char *>(p) + i * kPoolPiece, kPoolPiece);
    (void)hipMemAddressFree(p, m.bytes);
    pool_give(m.dev, m.pieces.data(), m.pieces.size());
    return true;
}

}  // namespace

bool pool_take(int dev, size_t n, std::vector<Handle> *out) {
    out->clear();
    {
        std::lock_guard<std::recursive_mutex> lk(g_mu);
        DeviceCache &c = cache_of(dev);
        while (out->size() < n && !c.pieces.empty()) {
            out->push_back(c.pieces.back());
            c.pieces.pop_back();
        }
    }
    const hipMemAllocationProp prop = device_prop(dev);
    while (out->size() < n) {
        Handle h{};
        if (hipMemCreate(&h, kPoolPiece, &prop, 0) != hipSuccess) {
            (void)hipGetLastError();
            break;
        }
        out->push_back(h);
    }
    if (out->size() < n) {
        pool_give(dev, out->data(), out->size());
        out->clear();
        return false;
    }
    return true;
}

void pool_give(int dev, const Handle *h, size_t n) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    DeviceCache &c = cache_of(dev);
    c.pieces.insert(c.pieces.end(), h, h + n);
}

static void reclaim_segments(int dev) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    cache_of(dev).sub.trim(0);  // whole free segments back to the runtime
}

void *cache_alloc(size_t bytes, size_t *got) {
    const int dev = current_device();
    if (bytes >= kPoolMin && vmm_supported()) {
        const size_t n = (bytes + kPoolPiece - 1) / kPoolPiece;
        for (int attempt = 0; attempt < 2; attempt++) {
            if (void *p = mapped_alloc(dev, n)) {
                *got = n * kPoolPiece;
                return p;
            }
            if (attempt == 0) reclaim_segments(dev);  // free segments hold memory
        }
        return nullptr;
    }
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    DeviceCache &c = cache_of(dev);
    if (void *p = c.sub.alloc(bytes, got)) return p;
    // out of memory: whole free segments and pooled pieces go back to the
    // runtime, then retry
    c.sub.trim(0);
    release_pieces_locked(c);
    return c.sub.alloc(bytes, got);
}

void cache_free(void *p, size_t) {
    if (!p) return;
    if (mapped_free(p)) return;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (cache_of(current_device()).sub.release(p)) return;
    for (auto &kv : g_cache)  // a block of another device
        if (kv.second.sub.release(p)) return;
}

// a sub-allocated block cannot go back on its own: it is freed into its
// segment, which a trim returns once it is whole
void cache_release(void *p) { cache_free(p, 0); }

void cache_trim(size_t max_bytes) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    DeviceCache &c = cache_of(current_device());
    // pooled pieces first (they back the largest blocks), then whole free
    // segments, largest first: the segments serve blocks of any size
    while (c.sub.free_bytes() + c.pieces.size() * kPoolPiece > max_bytes && !c.pieces.empty()) {
        (void)hipMemRelease(c.pieces.back());
        c.pieces.pop_back();
    }
    if (c.sub.free_bytes() > max_bytes) c.sub.trim(max_bytes);
}

void cache_flush() {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    for (auto &kv : g_cache) {
        // segments are freed with their device current
        if (have && kv.first != cur && hipSetDevice(kv.first) != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        release_blocks_locked(kv.second);
        release_pieces_locked(kv.second);
    }
    if (have) (void)hipSetDevice(cur);
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
constexpr size_t kPieceMin = size_t(2) << 20;  // mapping piece bounds
constexpr size_t kPieceMax = size_t(2) << 30;
// pieces start and end on 2 MiB boundaries (the large-page size), whatever
// smaller granularity the runtime reports
constexpr size_t kPieceAlign = size_t(2) << 20;
static_assert(kPoolPiece % kPieceAlign == 0, "pooled pieces are whole large pages");
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

// maps pieces hs[0, n) of `bytes` each behind the mapped prefix and grants
// access; on failure nothing stays mapped and the caller keeps the handles
spc_status VArray::map_pieces(const Handle *hs, size_t n, size_t bytes) {
    size_t i = 0;
    for (; i < n; i++)
        if (hipMemMap(static_cast<char *>(base_) + mapped_ + i * bytes, bytes, 0, hs[i], 0) != hipSuccess)
            break;
    // access is granted over the whole mapped prefix: the runtime rejects
    // some ranges that start past the reservation's base
    const hipMemAccessDesc acc = device_access(device_);
    if (i == n && hipMemSetAccess(base_, mapped_ + n * bytes, &acc, 1) == hipSuccess) return SPC_OK;
    (void)hipGetLastError();
    for (size_t j = 0; j < i; j++) (void)hipMemUnmap(static_cast<char *>(base_) + mapped_ + j * bytes, bytes);
    return SPC_ERR_DEVICE;
}

spc_status VArray::ensure(size_t bytes, size_t *added) {
    *added = 0;
    if (bytes <= mapped_) return SPC_OK;
    if (!base_ || bytes > reserved_) return SPC_ERR_INVALID_ARG;
    hipMemAllocationProp prop = device_prop(device_);
    while (mapped_ < bytes) {
        // pieces grow with the array (at most an eighth of it, within
        // bounds), so an array takes few pieces and little slack; from the
        // pool's piece size on, pooled pieces are mapped
        size_t piece = std::max(bytes - mapped_, std::min(std::max(kPieceMin, mapped_ / 8), kPieceMax));
        if (piece >= kPoolPiece && reserved_ - mapped_ >= kPoolPiece) {
            const size_t n = std::min((piece + kPoolPiece - 1) / kPoolPiece, (reserved_ - mapped_) / kPoolPiece);
            std::vector<Handle> hs;
            if (!pool_take(device_, n, &hs)) {
                reclaim_segments(device_);  // free segments hold memory
                if (!pool_take(device_, n, &hs)) return SPC_ERR_OUT_OF_MEMORY;
            }
            if (map_pieces(hs.data(), n, kPoolPiece) != SPC_OK) {
                pool_give(device_, hs.data(), n);
                return SPC_ERR_DEVICE;
            }
            for (size_t i = 0; i < n; i++) pieces_.push_back({hs[i], kPoolPiece, true});
            mapped_ += n * kPoolPiece;
            *added += n * kPoolPiece;
            continue;
        }
        piece = (piece + gran_ - 1) / gran_ * gran_;
        piece = std::min(piece, reserved_ - mapped_);
        Handle h{};
        if (hipMemCreate(&h, piece, &prop, 0) != hipSuccess) {
            (void)hipGetLastError();
            cache_flush();
            if (hipMemCreate(&h, piece, &prop, 0) != hipSuccess) {
                (void)hipGetLastError();
                return SPC_ERR_OUT_OF_MEMORY;
            }
        }
        if (map_pieces(&h, 1, piece) != SPC_OK) {
            (void)hipMemRelease(h);
            return SPC_ERR_DEVICE;
        }
        pieces_.push_back({h, piece, false});
        mapped_ += piece;
        *added += piece;
    }
    return SPC_OK;
}

void VArray::reset() {
    if (!base_) return;
    size_t off = 0;
    std::vector<Handle> back;
    for (auto &pc : pieces_) {
        (void)hipMemUnmap(static_cast<char *>(base_) + off, pc.bytes);
        if (pc.pooled)
            back.push_back(pc.h);
        else
            (void)hipMemRelease(pc.h);
        off += pc.bytes;
    }
    if (!back.empty()) pool_give(device_, back.data(), back.size());
    pieces_.clear();
    (void)hipMemAddressFree(base_, reserved_);
    base_ = nullptr;
    reserved_ = mapped_ = 0;
}

}  // namespace spc
