// Internal declarations of the gfx950 SPC label library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "spc.h"

namespace spc {

constexpr uint64_t kSat = 0xFFFFFFFFFFFFFFFFull;
constexpr uint32_t kEmpty32 = 0xFFFFFFFFu;
constexpr int kBlock = 256;  // threads per workgroup everywhere (4 wave64)
constexpr int kWaves = kBlock / 64;

#define SPC_TRY(expr)                          \
    do {                                       \
        spc_status _st = (expr);               \
        if (_st != SPC_OK) return _st;         \
    } while (0)
#define SPC_HIP(expr)                                \
    do {                                             \
        if ((expr) != hipSuccess) return SPC_ERR_DEVICE; \
    } while (0)
#define SPC_LAUNCHED()                                         \
    do {                                                       \
        if (hipGetLastError() != hipSuccess) return SPC_ERR_DEVICE; \
    } while (0)

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t sat_add(uint64_t a, uint64_t b) {
    uint64_t s = a + b;
    return s < a ? kSat : s;
}
__device__ __forceinline__ uint64_t sat_mul(uint64_t a, uint64_t b) {
    return __umul64hi(a, b) ? kSat : a * b;
}
__device__ __forceinline__ uint64_t lanemask_lt() {
    return (1ull << (threadIdx.x & 63)) - 1ull;
}


// inclusive scan across the 64 lanes of a wave
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T x = __shfl_up(v, o, 64);
        if (lane >= o) v += x;
    }
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// exclusive scan over the threads of a block of NW waves; `total` gets the
// block sum.  lds must hold NW values; every thread of the block must call it.
template <typename T, int NW = kWaves>
__device__ __forceinline__ T block_excl_scan(T v, T *lds, T &total) {
    T inc = wave_incl_scan(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    T pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
        T x = lds[i];
        pre += (i < w) ? x : (T)0;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return pre + inc - v;
}

// wave-scope ordering of LDS accesses (a wave's lanes exchange through LDS)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Packed label entry: hub in the high bits, distance in the low bits, so the
// packed value sorts by hub.  8-bit distances use a u32 (hub < 2^24),
// 16-bit distances a u64.
template <int DB>
struct Ent;
template <>
struct Ent<8> {
    using T = uint32_t;
    static constexpr int kShift = 8;
    static constexpr uint32_t kDistMask = 0xFFu;
    static constexpr uint32_t kMaxDist = 254;  // 255 is INF in query outputs
    static constexpr uint64_t kMaxHub = (1ull << 24) - 1;
};
template <>
struct Ent<16> {
    using T = uint64_t;
    static constexpr int kShift = 16;
    static constexpr uint32_t kDistMask = 0xFFFFu;
    static constexpr uint32_t kMaxDist = 65534;
    static constexpr uint64_t kMaxHub = 0xFFFFFFFEull;
};
template <int DB>
__device__ __host__ __forceinline__ uint32_t e_hub(typename Ent<DB>::T e) {
    return (uint32_t)(e >> Ent<DB>::kShift);
}
template <int DB>
__device__ __host__ __forceinline__ uint32_t e_dist(typename Ent<DB>::T e) {
    return (uint32_t)(e & Ent<DB>::kDistMask);
}
template <int DB>
__device__ __host__ __forceinline__ typename Ent<DB>::T e_make(uint32_t hub, uint32_t d) {
    return ((typename Ent<DB>::T)hub << Ent<DB>::kShift) | (typename Ent<DB>::T)d;
}

// first index i in [0, len) with a[i] >= key (a sorted ascending)
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t *a, uint32_t len, uint32_t key) {
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}
// same over packed entries, comparing hubs
template <int DB>
__device__ __forceinline__ uint64_t lower_bound_hub(const typename Ent<DB>::T *a, uint64_t len,
                                                    uint32_t hub) {
    uint64_t lo = 0, hi = len;
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        if (e_hub<DB>(a[mid]) < hub)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Device memory cache (memory.hip).  Physical memory that the runtime takes
// back and hands out again is cleared by the driver first, about 3 s per
// 100 GB, so freed memory is kept per device and reused:
//  * blocks of at least kPoolMin bytes are address ranges with pieces of
//    kPoolPiece bytes of physical memory mapped behind them (virtual memory
//    API); a freed block's pieces go to the device's piece pool and back
//    into any later block, whatever its size;
//  * smaller blocks are carved out of hipMalloc segments (suballoc.h: best
//    fit, split, coalesced on free), so freed memory serves requests of any
//    size.
// ---------------------------------------------------------------------------
constexpr size_t kPoolPiece = size_t(512) << 20;
constexpr size_t kPoolMin = size_t(4) << 30;
// Returns a block of at least `bytes` bytes (*got = what it holds, 256-byte
// aligned): pooled pieces for large blocks, else a block of a cached segment
// or of a new hipMalloc segment (after giving back whole free segments and
// pooled pieces if that fails).  nullptr on failure.
void *cache_alloc(size_t bytes, size_t *got);
void cache_free(void *p, size_t bytes);
// give a block straight back: a large block's pieces to the pool, a small
// block to the runtime
void cache_release(void *p);
// give every cached block and pooled piece of every device back
void cache_flush();
// give pooled pieces, then whole free segments (largest first), of the
// current device back until at most max_bytes stay cached
void cache_trim(size_t max_bytes);
// n pieces of kPoolPiece bytes for device dev (pooled ones first, then new
// ones); false, with nothing taken, when the device is out of memory
bool pool_take(int dev, size_t n, std::vector<hipMemGenericAllocationHandle_t> *out);
void pool_give(int dev, const hipMemGenericAllocationHandle_t *h, size_t n);

// Growable device array on the virtual memory API: an address range is
// reserved once and physical memory is mapped behind it piece by piece, so
// growing copies nothing and the address never moves.  The owner makes sure
// no kernel still uses the range before reset().
class VArray {
  public:
    VArray() = default;
    ~VArray() { reset(); }
    VArray(const VArray &) = delete;
    VArray &operator=(const VArray &) = delete;
    // reserve `max_bytes` of address space on the current device
    spc_status reserve(size_t max_bytes);
    // map physical memory until at least `bytes` are backed; *added = bytes
    // newly mapped
    spc_status ensure(size_t bytes, size_t *added);
    void reset();  // unmap and release everything, free the range
    void *ptr() const { return base_; }
    size_t mapped() const { return mapped_; }

  private:
    struct Piece {
        hipMemGenericAllocationHandle_t h;
        size_t bytes;
        bool pooled;  // from the piece pool (goes back there)
    };
    spc_status map_pieces(const hipMemGenericAllocationHandle_t *hs, size_t n, size_t bytes);
    void *base_ = nullptr;
    size_t reserved_ = 0, mapped_ = 0, gran_ = 0;
    int device_ = 0;
    std::vector<Piece> pieces_;
};
// whether the current device supports the virtual memory API
bool vmm_supported();

// ---------------------------------------------------------------------------
// Device memory accounting (per build): every allocation is checked against
// the caller's budget; whatever is still held when the arena dies goes back
// to the block cache unless it was handed over to the index.
// ---------------------------------------------------------------------------
class Arena {
  public:
    // blocks go back to the shared cache only after `st` has drained, so no
    // pending kernel of this arena's stream can still use them
    Arena(uint64_t budget, hipStream_t st) : budget_(budget), st_(st) {}
    ~Arena() {
        if (!sizes_.empty()) (void)hipStreamSynchronize(st_);
        for (auto &kv : sizes_) cache_free(kv.first, kv.second);
    }
    Arena(const Arena &) = delete;
    Arena &operator=(const Arena &) = delete;

    template <typename T>
    spc_status alloc(T **p, size_t count) {
        size_t bytes = count * sizeof(T);
        if (bytes == 0) bytes = 256;
        bytes = (bytes + 255) & ~size_t(255);
        if (budget_ && used_ + bytes > budget_) return SPC_ERR_OUT_OF_MEMORY;
        size_t got = 0;
        void *q = cache_alloc(bytes, &got);
        if (!q) return SPC_ERR_OUT_OF_MEMORY;
        sizes_[q] = got;
        used_ += got;
        note_peak();
        *p = static_cast<T *>(q);
        return SPC_OK;
    }
    // account for memory mapped outside the arena (VArray pieces)
    spc_status charge(uint64_t bytes) {
        if (budget_ && used_ + bytes > budget_) return SPC_ERR_OUT_OF_MEMORY;
        used_ += bytes;
        note_peak();
        return SPC_OK;
    }
    void uncharge(uint64_t bytes) { used_ -= bytes < used_ ? bytes : used_; }
    bool fits(uint64_t bytes) const { return !budget_ || used_ + bytes <= budget_; }
    // high-water mark since the last begin_window()
    void begin_window() { wpeak_ = used_; }
    uint64_t window_peak() const { return wpeak_; }
    template <typename T>
    void release(T *&p) {
        if (!p) return;
        auto it = sizes_.find((void *)p);
        if (it != sizes_.end()) {
            (void)hipStreamSynchronize(st_);
            used_ -= it->second;
            cache_free(it->first, it->second);
            sizes_.erase(it);
        }
        p = nullptr;
    }
    // give a block straight back to the runtime (large blocks that later
    // requests will not fit)
    template <typename T>
    void release_to_device(T *&p) {
        if (!p) return;
        auto it = sizes_.find((void *)p);
        if (it != sizes_.end()) {
            (void)hipStreamSynchronize(st_);
            used_ -= it->second;
            cache_release(it->first);
            sizes_.erase(it);
        }
        p = nullptr;
    }
    template <typename T>
    uint64_t size_of(const T *p) const {
        auto it = sizes_.find((void *)p);
        return it == sizes_.end() ? 0 : it->second;
    }
    // hand an allocation to the index: the arena stops tracking it
    template <typename T>
    uint64_t detach(T *p) {
        auto it = sizes_.find((void *)p);
        if (it == sizes_.end()) return 0;
        uint64_t b = it->second;
        sizes_.erase(it);
        return b;
    }
    uint64_t used() const { return used_; }
    uint64_t budget() const { return budget_; }
    uint64_t peak() const { return peak_; }

  private:
    void note_peak() {
        if (used_ > peak_) peak_ = used_;
        if (used_ > wpeak_) wpeak_ = used_;
    }
    uint64_t budget_;
    hipStream_t st_;
    uint64_t used_ = 0, peak_ = 0, wpeak_ = 0;
    std::unordered_map<void *, size_t> sizes_;
};

// ---------------------------------------------------------------------------
// Library-wide primitives (primitives.hip)
// ---------------------------------------------------------------------------
// Exclusive prefix sum: out[i] = sum in[0..i), out[n] = total.  `ws` must hold
// scan_ws_elems(n) uint64 values.
size_t scan_ws_elems(uint64_t n);
spc_status scan_u32(const uint32_t *in, uint64_t *out, uint64_t n, uint64_t *ws, hipStream_t st);
spc_status scan_u64(const uint64_t *in, uint64_t *out, uint64_t n, uint64_t *ws, hipStream_t st);

// Stable LSD radix sort of (key, value) pairs on key bits [0, bits), in
// place (ping-pong through the alt buffers; the result ends in keys/vals).
size_t radix_ws_elems(uint64_t n);
spc_status radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt,
                            uint64_t n, int bits, uint64_t *ws, hipStream_t st);

// ---------------------------------------------------------------------------
// The index
// ---------------------------------------------------------------------------
// 1-shell reduction of a union CSR (reduce.hip).  Device arrays come from
// the caller's arena.
struct ShellResult {
    uint64_t *off = nullptr;  // core CSR [N+1], core ids
    uint32_t *col = nullptr;  // [NNZ]
    uint32_t *ord = nullptr;  // the given order restricted to the core, or null
    uint64_t *tie = nullptr;  // the given tie keys restricted to the core, or null
    // per input vertex: core id of root(v), depth, parent (input id)
    uint32_t *root = nullptr, *depth = nullptr, *parent = nullptr;
    uint32_t *core_vid = nullptr;  // core id -> input id
    // neighbourhood equivalence: class size per core id; per input vertex
    // the answer for two members of its class (~0: adjacent twins (1, 1),
    // else the degree: (2, degree), or unreachable at 0)
    uint32_t *weight = nullptr, *same = nullptr;
    std::vector<uint32_t> cbase;   // core id range of each graph, k+1 entries
    uint32_t N = 0;
    uint64_t NNZ = 0, fringe = 0, twins = 0;
    uint32_t max_depth = 0;
};

struct RoundCounters {
    uint64_t raw = 0, merged = 0, kept = 0, scanned = 0;
    uint64_t staged = 0, row_bytes = 0, headers = 0;
    uint64_t filter_bytes = 0;  // membership-filter words looked up by the prune probes
    uint64_t mem_peak = 0;  // device bytes held by the build at the round's high-water mark
    double kernel_ms = 0;   // fused round kernel time of this round
};

}  // namespace spc

struct spc_index {
    int device = 0;
    uint32_t n = 0;       // all vertices (union for batches)
    uint64_t m = 0;       // undirected edges
    uint32_t dist_bits = 8;
    uint32_t rounds = 0, max_dist = 0, round_cap = 0;
    bool truncated = false;
    uint64_t entries = 0, saturated = 0;
    // final index, rank space (hub-sorted labels)
    uint64_t *lab_off = nullptr;  // [n+1]
    void *lab_hd = nullptr;       // packed (hub, dist)[entries]
    uint64_t *lab_cnt = nullptr;  // [entries]
    uint32_t *rank_of = nullptr;  // vertex -> rank (union ids)
    uint32_t *order = nullptr;    // rank -> vertex (union ids)
    // the index's device blocks and their sizes (returned to the block cache)
    std::vector<std::pair<void *, size_t>> blocks;
    // graphs of a batch: vertex/rank range [vbase[i], vbase[i] + gn[i])
    std::vector<uint32_t> vbase, gn;
    std::vector<spc::RoundCounters> round_stats;
    uint64_t index_bytes = 0, peak_build_bytes = 0;
    double ms_order = 0, ms_rounds = 0, ms_finalize = 0, ms_total = 0, ms_round_kernel = 0;
    uint64_t alg_bytes_round_kernel = 0;
    uint64_t round_kernel_launches = 0;
    uint32_t query_cfg = 0;  // query launch configuration (query.hip)
    // queries with |L(s)| + |L(t)| at most this are answered 16 lanes per
    // query by spc_query_batch_multi (0: no bucketing)
    uint32_t query_small = 256;
    // on-disk tuning cache of the index (empty: none): its path and key
    std::string tune_cache;
    uint64_t tune_key = 0;
    bool tune_cached = false;
    uint32_t *g_tab = nullptr;  // per graph (vbase, gn, obase, on), device
    // directed: label rows [0, nreal) are out-labels, [nreal, 2 nreal)
    // in-labels (0: undirected)
    uint32_t nreal = 0;
    uint32_t out_bits = 8;   // width of query dist outputs
    // SPC_REDUCE_ONE_SHELL: input vertex ranges [obase[i], obase[i] + on[i])
    // of the graphs, and per input vertex (union ids) the core id of its
    // root, its depth and its parent; core id -> input id
    bool reduced = false;
    std::vector<uint32_t> obase, on;
    uint32_t *red_root = nullptr, *red_depth = nullptr, *red_parent = nullptr;
    uint32_t *core_vid = nullptr;
    uint64_t fringe = 0;
    uint32_t fringe_depth = 0;
    // neighbourhood equivalence: class size of every hub (rank space) and
    // the same-class answer per input vertex; null otherwise
    uint32_t *hub_w = nullptr, *red_same = nullptr;
    uint64_t twins = 0;
};

namespace spc {
// build.hip
spc_status build_impl(const spc_graph *gs, uint32_t k, const spc_build_opts *opts, hipStream_t st,
                      spc_index **out);
// reduce.hip
spc_status one_shell(Arena &ar, hipStream_t st, uint64_t *ws, uint32_t N, uint64_t NNZ,
                     const uint64_t *off, const uint32_t *col, const uint32_t *ord, const uint64_t *tie,
                     const std::vector<uint32_t> &vbase, ShellResult *R);
spc_status twin_reduce(Arena &ar, hipStream_t st, uint64_t *ws, uint32_t N, uint64_t NNZ,
                       const uint64_t *off, uint32_t *col, bool rows_sorted, const uint32_t *ord,
                       const uint64_t *tie, const std::vector<uint32_t> &vbase, ShellResult *R);
// query.hip
spc_status query_impl(const spc_index *ix, uint32_t graph_id, const uint32_t *s, const uint32_t *t,
                      uint64_t nq, void *dist_out, uint64_t *count_out, uint8_t *flags_out,
                      hipStream_t st);
spc_status query_multi_run(const spc_index *ix, const uint32_t *gid, const uint32_t *s,
                           const uint32_t *t, uint64_t nq, void *dist_out, uint64_t *count_out,
                           uint8_t *flags_out, uint32_t *perm, uint32_t *cnt, uint32_t small,
                           uint32_t cfg, hipStream_t st);
spc_status tune_query_buckets_impl(spc_index *ix, const uint32_t *gid, const uint32_t *s,
                                   const uint32_t *t, uint64_t nq, hipStream_t st, uint32_t *small_out);
spc_status query_multi_noalloc_impl(const spc_index *ix, const uint32_t *gid, const uint32_t *s,
                                    const uint32_t *t, uint64_t nq, void *dist_out, uint64_t *count_out,
                                    uint8_t *flags_out, hipStream_t st);
spc_status query_multi_impl(const spc_index *ix, const uint32_t *gid, const uint32_t *s,
                            const uint32_t *t, uint64_t nq, void *dist_out, uint64_t *count_out,
                            uint8_t *flags_out, hipStream_t st);
// order.hip
spc_status hybrid_order_impl(const spc_graph *g, uint32_t delta, uint32_t *order, uint32_t *core_out);
spc_status tune_queries_impl(spc_index *ix, uint32_t graph_id, const uint32_t *s, const uint32_t *t,
                             uint64_t nq, hipStream_t st, uint32_t *cfg_out);
uint32_t query_cfg_count();
spc_status query_cfg_info(uint32_t cfg, uint32_t *stage, uint32_t *tiles);
spc_status export_impl(const spc_index *ix, uint32_t graph_id, uint64_t *off, uint32_t *hub,
                       uint16_t *dist, uint64_t *count, uint32_t *order, int32_t on_device,
                       hipStream_t st);
spc_status export_reduction_impl(const spc_index *ix, uint32_t graph_id, uint32_t *root,
                                 uint32_t *depth, uint32_t *parent, int32_t on_device, hipStream_t st);
}  // namespace spc
