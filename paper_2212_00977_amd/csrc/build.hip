// SPC label index construction on gfx950: vertex ordering, relabelling and
// the round-by-distance PULL propagation of PSPC (Alg. 2, Eq. PSPCdu, Label
// Elimination / Label Merging), then the hub-ordered count array.
//
// Layout in HBM (rank space: vertex id == rank, 0 = most important)
//   graph      goff u64[N+1], gadj u32[2m]
//   labels     lab_off u64[N+1], lab_hd E[entries]: packed (hub, dist), each
//              label sorted by hub; rebuilt each round by merging the round's
//              entries in (double-buffered), so probes always stream sorted
//              labels and the final index needs no sort
//   rounds     one allocation per round: rhub[r] u32[], rcnt[r] u64[]; round
//              r of vertex v is the hub-sorted segment at rstart[r][v],
//              rlen[r][v] of those arrays
//   counts     lab_cnt u64[entries], filled at the end from the rounds' counts
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "spc_internal.h"

namespace spc {

namespace {

// ---------------------------------------------------------------------------
// Preprocessing kernels
// ---------------------------------------------------------------------------
// Copy one graph's CSR into the union, shifting offsets by the graph's edge
// base and neighbour ids by its vertex base; flags out-of-range ids and
// non-monotone offsets.
__global__ void k_union_off(const uint64_t *src, uint64_t *dst, uint32_t n, uint64_t nnz,
                            uint64_t ebase, uint32_t *err) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    uint64_t x = src[i];
    if ((i == 0 && x != 0) || (i == n && x != nnz) || x > nnz) atomicOr(err, 1u);
    if (i < n && src[i + 1] < x) atomicOr(err, 1u);
    dst[i] = x + ebase;
}
__global__ void k_union_col(const uint32_t *src, uint32_t *dst, uint64_t nnz, uint32_t n,
                            uint32_t vbase, uint32_t *err) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nnz) return;
    uint32_t x = src[i];
    if (x >= n) atomicOr(err, 2u);
    dst[i] = x + vbase;
}

__global__ void k_degrees(const uint64_t *off, uint32_t N, uint32_t *deg, uint32_t *maxdeg) {
    uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    uint32_t dv = (uint32_t)(off[v + 1] - off[v]);
    deg[v] = dv;
    atomicMax(maxdeg, dv);
}

// graph id of union vertex v: largest g with vbase[g] <= v
__device__ __forceinline__ uint32_t graph_of(const uint32_t *vbase, uint32_t k, uint32_t v) {
    uint32_t lo = 0, hi = k - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (vbase[mid] <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// key for the degree pass: (graph id, maxdeg - degree), values = vertices in
// their current (stable) order
__global__ void k_degree_keys(const uint32_t *vals, const uint32_t *deg, uint32_t N, uint32_t maxdeg,
                              int degbits, const uint32_t *vbase, uint32_t k, uint64_t *keys) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    uint32_t v = vals[i];
    uint64_t g = (k > 1) ? graph_of(vbase, k, v) : 0;
    keys[i] = (g << degbits) | (uint64_t)(maxdeg - deg[v]);
}
__global__ void k_iota_keys(const uint64_t *tie, uint32_t N, uint64_t *keys, uint32_t *vals) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    keys[i] = tie ? tie[i] : 0;
    vals[i] = i;
}
// explicit per-graph order, shifted into the union; counts hits per vertex
__global__ void k_union_order(const uint32_t *src, uint32_t *dst, uint32_t n, uint32_t vbase,
                              uint32_t *hits, uint32_t *err) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t v = src[i];
    if (v >= n) {
        atomicOr(err, 4u);
        v = 0;
    }
    dst[vbase + i] = v + vbase;
    atomicAdd(&hits[vbase + v], 1u);
}
__global__ void k_check_perm(const uint32_t *hits, uint32_t N, uint32_t *err) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N && hits[i] != 1) atomicOr(err, 4u);
}
__global__ void k_rank_of(const uint32_t *order, uint32_t N, const uint32_t *deg, uint32_t *rank_of,
                          uint32_t *rdeg) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    uint32_t v = order[r];
    rank_of[v] = r;
    rdeg[r] = deg[v];
}
// rank-space adjacency: one wave per rank
__global__ __launch_bounds__(kBlock) void k_relabel(const uint32_t *order, const uint32_t *rank_of,
                                                    const uint64_t *off, const uint32_t *col,
                                                    const uint64_t *roff, uint32_t *radj,
                                                    uint32_t N) {
    uint32_t r = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (r >= N) return;
    uint32_t lane = threadIdx.x & 63;
    uint32_t v = order[r];
    uint64_t s = off[v], len = off[v + 1] - s, o = roff[r];
    for (uint64_t k = lane; k < len; k += 64) radj[o + k] = rank_of[col[s + k]];
}
// keys (row << xbits | neighbour) for sorting each adjacency list
__global__ __launch_bounds__(kBlock) void k_row_keys(const uint64_t *roff, const uint32_t *radj,
                                                     uint32_t N, int xbits, uint64_t *keys) {
    uint32_t r = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (r >= N) return;
    uint32_t lane = threadIdx.x & 63;
    for (uint64_t k = roff[r] + lane; k < roff[r + 1]; k += 64)
        keys[k] = ((uint64_t)r << xbits) | radj[k];
}
__global__ void k_keys_to_adj(const uint64_t *keys, uint64_t nnz, int xbits, uint32_t *radj) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nnz) radj[i] = (uint32_t)(keys[i] & ((1ull << xbits) - 1));
}
// simple (+ symmetric unless `directed`) check on sorted rank-space adjacency
__global__ __launch_bounds__(kBlock) void k_check_adj(const uint64_t *roff, const uint32_t *radj,
                                                      uint32_t N, uint32_t *err, int directed) {
    uint32_t r = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (r >= N) return;
    uint32_t lane = threadIdx.x & 63;
    uint64_t s = roff[r], e = roff[r + 1];
    for (uint64_t k = s + lane; k < e; k += 64) {
        uint32_t x = radj[k];
        if (x == r) atomicOr(err, 8u);                       // self loop
        if (k > s && radj[k - 1] == x) atomicOr(err, 16u);   // duplicate
        if (directed) continue;
        uint64_t xs = roff[x];
        uint32_t xl = (uint32_t)(roff[x + 1] - xs);
        uint32_t p = lower_bound_u32(radj + xs, xl, r);
        if (p >= xl || radj[xs + p] != r) atomicOr(err, 32u); // asymmetric
    }
}

// ---------------------------------------------------------------------------
// Round 0: L_0(v) = {(v, 0, 1)}.
// ---------------------------------------------------------------------------
template <int DB>
__global__ void k_round0(uint32_t N, uint32_t nreal, uint32_t *pool_hub, uint64_t *pool_cnt, uint64_t *rstart,
                         uint32_t *rlen, uint64_t *lab_off, typename Ent<DB>::T *lab_hd) {
    uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v > N) return;
    lab_off[v] = v;
    if (v == N) return;
    const uint32_t h = (nreal && v >= nreal) ? v - nreal : v;  // a row's own vertex
    pool_hub[v] = h;
    pool_cnt[v] = 1;
    rstart[v] = v;
    rlen[v] = 1;
    lab_hd[v] = e_make<DB>(h, 0);
}

// ---------------------------------------------------------------------------
// Expand count: raw[u] = number of round d-1 entries of u's neighbours whose
// hub outranks u (Lemma propagation + rank rule).  The round d-1 segment of a
// neighbour v is hub-sorted, so this is a prefix length; when v outranks u
// every hub of that segment does too.  One wave per u.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_expand_count(uint32_t N, uint32_t nreal, const uint64_t *goff,
                                                         const uint32_t *gadj, const uint64_t *pstart,
                                                         const uint32_t *plen,
                                                         const uint32_t *pool_hub, uint64_t *raw) {
    uint32_t u = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (u >= N) return;
    uint32_t lane = threadIdx.x & 63;
    // rows of a directed build: hubs are real vertices (row - nreal for
    // in-label rows)
    const uint32_t ur = (nreal && u >= nreal) ? u - nreal : u;
    uint64_t s = 0;
    for (uint64_t k = goff[u] + lane; k < goff[u + 1]; k += 64) {
        uint32_t v = gadj[k];
        uint32_t ln = plen[v];
        if (ln == 0) continue;
        const uint32_t vr = (nreal && v >= nreal) ? v - nreal : v;
        s += (vr < ur) ? ln : lower_bound_u32(pool_hub + pstart[v], ln, ur);
    }
    s = wave_sum(s);
    if (lane == 0) raw[u] = s;
}

// ---------------------------------------------------------------------------
// Landmark rows.  The kLand highest-ranked vertices of every graph are
// landmarks (Section "Landmark-Based Filtering": the highest-degree vertices,
// whose entries dominate every round).  Each vertex keeps a dense row with
// its label distance to every landmark (INF = type max when the landmark is
// not one of its hubs), so the part of a 2-hop query that goes through a
// landmark is one coalesced row load and register compares instead of label
// streaming.  Rows hold exactly the label entries with landmark hubs; they
// change the cost of a query, never its answer.
// ---------------------------------------------------------------------------
constexpr int kLand = 256;
template <int DB>
struct Land;
template <>
struct Land<8> {
    using T = uint8_t;
    using W = uint32_t;  // 4 landmarks per lane
};
template <>
struct Land<16> {
    using T = uint16_t;
    using W = uint64_t;
};
// true if some of the 4 packed landmark distances satisfies a + b < d; an
// absent entry is the type max, so its sum is never below d (d <= max-1)
// Is d_x + d_y < d for some landmark of the word (four distances each)?
// SWAR: the even and the odd distances are summed in lanes twice as wide
// (no carry between lanes), and each lane's (d - 1) - sum keeps its guard
// bit exactly when sum < d.  d >= 1.
__device__ __forceinline__ bool land_hit(uint32_t x, uint32_t y, uint32_t d) {
    constexpr uint32_t m = 0x00FF00FFu, g = 0x80008000u;
    const uint32_t dd = ((d - 1) * 0x00010001u) | g;
    const uint32_t te = dd - ((x & m) + (y & m));
    const uint32_t to = dd - (((x >> 8) & m) + ((y >> 8) & m));
    return ((te | to) & g) != 0;
}
__device__ __forceinline__ bool land_hit(uint64_t x, uint64_t y, uint32_t d) {
    constexpr uint64_t m = 0x0000FFFF0000FFFFull, g = 0x8000000080000000ull;
    const uint64_t dd = ((uint64_t)(d - 1) * 0x0000000100000001ull) | g;
    const uint64_t te = dd - ((x & m) + (y & m));
    const uint64_t to = dd - (((x >> 16) & m) + ((y >> 16) & m));
    return ((te | to) & g) != 0;
}

__device__ __forceinline__ uint32_t land_count_le(uint32_t x, uint32_t lim) {
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) c += ((x >> (8 * i)) & 0xFFu) <= lim;
    return c;
}
__device__ __forceinline__ uint32_t land_count_le(uint64_t x, uint32_t lim) {
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) c += (uint32_t)((x >> (16 * i)) & 0xFFFFu) <= lim;
    return c;
}

// Landmark masks: per row and distance k in [1, kMaskK], the 256-bit set of
// landmarks held at distance exactly k (32 bytes), so the landmark test of a
// round d <= kMaskK + 2 reads (d-2) x 32 bytes of a candidate's masks, not
// its row.
constexpr int kMaskK = 6;
constexpr int kMaskWords = kLand / 32;  // u32 words per mask

template <int DB>
__global__ void k_land_init(uint32_t N, uint32_t nreal, const uint32_t *gbase, typename Land<DB>::T *land) {
    using LT = typename Land<DB>::T;
    const uint64_t n = (uint64_t)N * kLand;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t v = (uint32_t)(i / kLand), l = (uint32_t)(i % kLand);
        uint32_t base = gbase ? gbase[v] : 0;
        const uint32_t h = (nreal && v >= nreal) ? v - nreal : v;
        land[i] = (h - base == l) ? (LT)0 : (LT)~(LT)0;
    }
}
__global__ void k_land_widen(const uint8_t *src, uint16_t *dst, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i] == 0xFF ? (uint16_t)0xFFFF : (uint16_t)src[i];
}

// ---------------------------------------------------------------------------
// The fused round kernel.  One workgroup per puller u (largest rank ids
// first: they have the most candidates).
//   1. stage u's landmark row (registers + LDS) and the rest of L_{<d}(u)
//      (hub -> dist, hubs past the landmarks) in an LDS hash table; a part
//      longer than the table allows is staged chunk by chunk instead (the
//      entries with hubs in the chunk's range, which is capped to fit);
//   2. walk the hub range [0, u) in chunks: pull every neighbour's round d-1
//      entries with hub in the chunk, drop hubs u already holds (Label
//      Elimination: they hold a smaller distance) and merge equal hubs in an
//      LDS hash by summing counts (Label Merging, saturating).  A chunk whose
//      distinct hubs overflow the table is retried with half the width;
//   3. prune each merged candidate w with the 2-hop query over entries of
//      distance < d (Eq. PSPCdu), 16 lanes per candidate: first through the
//      landmark rows of u and w; if no landmark proves a shorter path and w
//      is not a landmark itself, through the two labels' other entries of
//      distance <= d-2 (only those can prove anything, since a common hub
//      h != u, w forces d_u, d_w >= 1) with hubs ranked above w, from the
//      previous round's merged labels.  A hub with d_u(h) + d_w(h) < d
//      prunes; equality keeps;
//   4. rank the survivors by hub (counting, LDS);
//   5. append them to u's slot of the temp buffer.
// ---------------------------------------------------------------------------
// LDS budget of the round kernel (about 32 KB with the defaults; the
// 128-VGPR bound keeps four workgroups per CU).  u's L_{<=d-2} part is staged for the probes in the
// candidate table's count array, which is idle between a chunk's merge and
// its sort, so it costs no occupancy.
#ifndef SPC_LBITS
#define SPC_LBITS 11
#endif
constexpr int kLBits = SPC_LBITS;
#ifndef SPC_LBITS_LONG
#define SPC_LBITS_LONG 12
#endif
// the instances of rounds past kMergeRound (long-diameter graphs, small
// candidate sets per puller, labels of about a thousand entries) take a
// table of 2^12 8-bit-label entries or 2^11 16-bit ones (16 KB; three
// workgroups per CU by LDS)
constexpr int kLBitsLong = SPC_LBITS_LONG;
#ifndef SPC_CBITS
#define SPC_CBITS 10
#endif
constexpr int kCBits = SPC_CBITS;  // >= 9: a candidate slot per thread at least
constexpr int kCCap = 1 << kCBits;   // candidate hash slots
constexpr int kULimit = kCCap / 2;   // distinct candidates per chunk
static_assert(kULimit <= 65536 && kCCap * 2 <= 65536, "filtered probes pack (candidate, entry) in 16 + 16 bits");
constexpr uint32_t kNone = 0xFFFFFFFFu;
#ifndef SPC_ROUND_BLOCK
#define SPC_ROUND_BLOCK 256
#endif
constexpr int kRoundBlock = SPC_ROUND_BLOCK;  // threads per puller workgroup
static_assert((1 << (SPC_CBITS - 1)) >= SPC_ROUND_BLOCK, "candidate limit below one per thread");
#ifndef SPC_TAIL_STEPS
#define SPC_TAIL_STEPS 4
#endif
// merge trips over u's unstaged label per tile of w's entries before the
// remaining hubs are binary-searched
constexpr uint32_t kTailSteps = SPC_TAIL_STEPS;
#ifndef SPC_PROBE_GROUP
#define SPC_PROBE_GROUP 16
#endif
#ifndef SPC_PULL_UNROLL
#define SPC_PULL_UNROLL 4
#endif
#ifndef SPC_LAND_UNROLL
#define SPC_LAND_UNROLL 1
#endif
// pulled entries per thread whose loads are in flight together
constexpr int kPullUnroll = SPC_PULL_UNROLL;
// filter lookups per thread in flight together: pairs, and distances per pair
#ifndef SPC_PROBE_UNROLL
#define SPC_PROBE_UNROLL 2
#endif
constexpr int kProbeUnroll = SPC_PROBE_UNROLL;
constexpr int kFiltProbes = 2;
// older label entries per membership-filter word: 2 (32 bits an entry)
// where the memory allows, else 4
constexpr uint32_t kFiltShiftLo = 1, kFiltShiftHi = 2;
#ifndef SPC_FILT_LIST
#define SPC_FILT_LIST 512
#endif
// filter hits listed for the searches after the lookups (more are searched
// at once)
constexpr uint32_t kFiltList = SPC_FILT_LIST;
// candidates per 16-lane group whose landmark slices are in flight together
constexpr int kLandUnroll = SPC_LAND_UNROLL;
// lanes per candidate in the probes past the landmarks (a power of two <= 64)
constexpr uint32_t kProbeGroup = SPC_PROBE_GROUP;
static_assert(kProbeGroup >= 2 && kProbeGroup <= 64 && (kProbeGroup & (kProbeGroup - 1)) == 0,
              "probe group: a power of two from 2 to 64");

struct RoundArgs {
    uint32_t d, u_lo, u_hi;
    // directed builds: rows [0, nreal) are out-labels, rows [nreal, 2 nreal)
    // in-labels of the same vertices (0: undirected, row = vertex)
    uint32_t nreal;
    const uint64_t *goff;
    const uint32_t *gadj;
    const uint64_t *lab_off;         // L_{<=d-1}: staged for u
    const void *lab_hd;
    const uint64_t *prev_off;        // L_{<=d-2}: probed for candidates w
    const void *prev_hd;
    const uint32_t *lc_cur;          // landmark entries of L_{<=d-1}(v) / L_{<=d-2}(v)
    const uint32_t *lc_prev;
    const void *land;                // landmark rows [N][kLand]
    const uint4 *lmask;              // landmark masks [N][kMaskK][kLand / 32], or null
    const uint32_t *gbase;           // first rank of each vertex's graph, or null
    const uint64_t *pstart;          // round d-1: segment start / length per vertex
    const uint32_t *plen;
    const uint32_t *pool_hub;        // round d-1 entries
    const uint64_t *pool_cnt;
    const uint32_t *adj_w;           // per adjacency slot: the neighbour's weight (W only)
    uint32_t *cur, *nxt;             // per adjacency slot: segment positions at lo / hi
    const uint64_t *raw_off;  // exclusive prefix of raw over all vertices
    // survivors of puller u go to the temp buffer at its pull offset
    // raw_off[u] - raw_off[u_lo] (it has at most raw_u of them)
    uint32_t *tmp_hub;
    uint64_t *tmp_cnt;
    uint32_t *surv;
    unsigned long long *ctr;  // raw, merged, kept, tail, staged, row bytes, headers, filter bytes
    // membership filter of L_{<=d-2}'s (row, hub, distance) triples past the
    // landmarks (null: none this round), filt_words 64-bit words, 2^filt_shift
    // older entries a word
    const unsigned long long *filt = nullptr;
    uint64_t filt_words = 0;
    uint32_t filt_shift = kFiltShiftHi;
};

__device__ __forceinline__ uint32_t hash_slot(uint32_t h, int bits) {
    return (h * 0x9E3779B1u) >> (32 - bits);
}

// Membership filter over the (row, hub, distance) triples of the older
// labels past the landmarks: a Bloom filter with one 64-bit word per key, in
// which a key sets (and a lookup tests) up to 4 bits.  A clear bit proves
// the triple absent; a hit is confirmed in the label itself.  Keys are mixed
// with the 64-bit finalizer of MurmurHash3; the low 32 bits pick the word
// among the row's own ones, the top 24 bits the 4 bit positions.  A row owns
// the words its older label's entries span at 2^s entries a word
// (neighbouring rows may share an end word), so the lookups of one candidate
// row fall in a few cache lines rather than all over the filter.
__device__ __forceinline__ uint64_t filt_mix(uint32_t row, uint32_t hub, uint32_t dist) {
    uint64_t x = (((uint64_t)row << 32) | hub) ^ ((uint64_t)dist * 0x9E3779B97F4A7C15ull);
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}
// row words [x, x + y) from the row's older label offsets [o0, o1), within
// the filter's nw >= 1 words whatever the offsets
__device__ __forceinline__ uint2 filt_region(uint64_t o0, uint64_t o1, uint64_t nw, uint32_t s) {
    uint64_t b1 = (o1 + (1ull << s) - 1) >> s;
    if (b1 > nw) b1 = nw;
    if (b1 == 0) b1 = 1;
    uint64_t b0 = o0 >> s;
    if (b0 >= b1) b0 = b1 - 1;
    return make_uint2((uint32_t)b0, (uint32_t)(b1 - b0));
}
__device__ __forceinline__ uint32_t filt_word(uint2 reg, uint64_t x) {
    return reg.x + (uint32_t)(((x & 0xFFFFFFFFull) * reg.y) >> 32);
}
__device__ __forceinline__ unsigned long long filt_bits(uint64_t x) {
    return (1ull << ((x >> 40) & 63)) | (1ull << ((x >> 46) & 63)) | (1ull << ((x >> 52) & 63)) |
           (1ull << (x >> 58));
}

// first position p in [0, n) with hub(a[p]) >= key (packed entries sorted by
// hub): exponential steps from 0, then a binary search
template <int DB>
__device__ __forceinline__ uint64_t gallop_hub(const typename Ent<DB>::T *a, uint64_t n, uint32_t key) {
    uint64_t lo = 0, step = 1, end = n;
    while (lo < n) {
        const uint64_t p = lo + step - 1;
        if (p >= n) break;
        if (e_hub<DB>(a[p]) >= key) {
            end = p;
            break;
        }
        lo = p + 1;
        step <<= 1;
    }
    return lo + lower_bound_hub<DB>(a + lo, end - lo, key);
}

// first position p in [c, n) with a[p] >= key, where every position below c
// holds a smaller value: exponential steps from c, then a binary search
__device__ __forceinline__ uint32_t gallop_u32(const uint32_t *a, uint32_t c, uint32_t n, uint32_t key) {
    uint32_t lo = c, step = 1, end = n;
    while (lo < n) {
        const uint32_t p = lo + step - 1;
        if (p >= n) break;
        if (a[p] >= key) {
            end = p;
            break;
        }
        lo = p + 1;
        step <<= 1;
    }
    return lo + lower_bound_u32(a + lo, end - lo, key);
}

template <int DB, int LB>
struct LabelLookup {
    using E = typename Ent<DB>::T;
    const E *tab;     // LDS table
    const E *tail;    // unstaged entries in HBM, hub-sorted
    uint64_t ntail;
    uint32_t x;       // hubs >= x live in the tail
    __device__ __forceinline__ uint32_t operator()(uint32_t h) const {
        if (h < x) {
            uint32_t s = hash_slot(h, LB);
            while (true) {
                E e = tab[s];
                if (e == (E)~(E)0) return kNone;
                if (e_hub<DB>(e) == h) return e_dist<DB>(e);
                s = (s + 1) & ((1u << LB) - 1);
            }
        }
        uint64_t p = lower_bound_hub<DB>(tail, ntail, h);
        if (p < ntail && e_hub<DB>(tail[p]) == h) return e_dist<DB>(tail[p]);
        return kNone;
    }
};

// TM: w's entries past u's staged label are matched by a merge with u's
// unstaged part (labels of similar length: high-diameter graphs) rather than
// by binary searches
// W: vertex weights (neighbourhood equivalence, rounds >= 2): a pulled
// count is multiplied by the weight of the neighbour it is pulled from.
template <int DB, int RB, bool TM, bool W>
__global__ __launch_bounds__(RB, 4) void k_round(RoundArgs a) {  // at most 128 VGPRs: 4 waves per SIMD
    constexpr int RW = RB / 64;          // waves per workgroup
    constexpr int PER = kULimit / RB;    // candidate slots per thread
    using E = typename Ent<DB>::T;
    using LT = typename Land<DB>::T;
    using LW = typename Land<DB>::W;
    // L(u) hash: 2^LB slots (in the long-diameter instances the same bytes
    // for both entry widths), at most half of them staged
    constexpr int LB = TM ? kLBitsLong - (DB == 16 ? 1 : 0) : kLBits;
    constexpr int kLCap = 1 << LB;
    constexpr int kLStage = kLCap / 2;
    __shared__ E ltab[kLCap];
    __shared__ LW lrow[kLand / 4];
    __shared__ uint32_t ckey[kCCap];
    __shared__ unsigned long long cval[kCCap];
    __shared__ uint8_t cwrap[kCCap];
    __shared__ __align__(16) uint32_t lhub[kULimit];
    __shared__ unsigned long long lcnt[kULimit];
    __shared__ uint8_t lkeep[kULimit];   // 0 pruned, 1 kept, 2 needs the tail check
    // candidates that need the tail check (probe phase)
    __shared__ uint16_t tlist[kULimit];
    __shared__ uint2 freg[kULimit];      // filtered probes: tlist[t]'s filter words
    __shared__ uint64_t nb_start[RB];
    __shared__ uint32_t nb_off[RB];
    __shared__ uint32_t red32[RW];
    __shared__ uint32_t s_nuniq, s_ovf, s_next, s_nver;
    __shared__ unsigned long long s_tail, s_hdr, s_rowb, s_filt;

    const E *hd = static_cast<const E *>(a.lab_hd);
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint32_t grp = lane >> 4, gl = lane & 15;  // 16-lane groups
    const uint32_t u = a.u_hi - 1 - blockIdx.x;
    const uint64_t raw_u = a.raw_off[u + 1] - a.raw_off[u];
    // a row's hubs are real vertices ranked at or above the row's own
    // vertex ur; a candidate hub w is probed against w's in-label for an
    // out-label row, w's out-label for an in-label row, w itself otherwise
    auto real = [&](uint32_t p) -> uint32_t { return (a.nreal && p >= a.nreal) ? p - a.nreal : p; };
    const uint32_t ur = real(u);
    const uint32_t poff = (a.nreal && u < a.nreal) ? a.nreal : 0;
    if (raw_u == 0) {  // uniform over the workgroup
        if (tid == 0) a.surv[u] = 0;
        return;
    }
    const uint32_t d = a.d;
    const E kEmptyE = (E)~(E)0;
    const LT kInfL = (LT)~(LT)0;
    const uint32_t base = a.gbase ? a.gbase[u] : 0;
    const uint32_t land_end = base + kLand;  // hubs below this are landmarks
    const LW *lands = static_cast<const LW *>(a.land);

    // 1. stage u's landmark row and the rest of L_{<d}(u); the landmark
    //    entries of a hub-sorted label are its first lc entries
    if (wv == 0) lrow[lane] = lands[(uint64_t)u * (kLand / 4) + lane];
    const uint64_t l0 = a.lab_off[u];
    const uint64_t nL = a.lab_off[u + 1] - l0;
    const uint64_t s0 = a.lc_cur[u];
    const uint64_t nsp = nL - s0;
    const E *lab = hd + l0 + s0;  // u's label past the landmarks, hub-sorted
    // a label that fits the table is staged once; a longer one chunk by
    // chunk, the chunk's hub range capped so that its slice fits
    const bool big = nsp > (uint64_t)kLStage;
    auto stage = [&](const E *src, uint32_t cnt) {
        for (uint32_t i = tid; i < cnt; i += RB) {
            E e = src[i];
            uint32_t s = hash_slot(e_hub<DB>(e), LB);
            while (atomicCAS(&ltab[s], kEmptyE, e) != kEmptyE) s = (s + 1) & (kLCap - 1);
        }
    };
    for (int i = tid; i < kLCap; i += RB) ltab[i] = kEmptyE;
    if (tid == 0) {
        s_tail = 0;
        s_hdr = 0;
        s_rowb = 0;
        s_filt = 0;
    }
    __syncthreads();
    if (!big) stage(lab, (uint32_t)nsp);
    // u's entries of distance <= d-2 past the landmarks, hub-sorted (from
    // the previous round's merged label), for probes that stream u's side
    const E *pu = nullptr;
    uint64_t npu = 0;
    if (d >= 3) {
        const uint64_t q0 = a.prev_off[u];
        const uint64_t qs = a.lc_prev[u];
        pu = static_cast<const E *>(a.prev_hd) + q0 + qs;
        npu = a.prev_off[u + 1] - q0 - qs;
    }
    // the table, which holds the current chunk's hubs of u's label
    LabelLookup<DB, LB> tabl;
    tabl.tab = ltab;
    tabl.tail = lab + nsp;
    tabl.ntail = 0;
    tabl.x = 0xFFFFFFFFu;
    // u's whole label past the landmarks for the probes: the table when
    // staged once, else HBM
    LabelLookup<DB, LB> look = tabl;
    if (big) {
        look.tail = lab;
        look.ntail = nsp;
        look.x = 0;
    }
    __syncthreads();
    const LT *lrow_t = reinterpret_cast<const LT *>(lrow);
    // is hub w of the current chunk already held by u (at a distance < d)?
    uint64_t tcur = 0, tend = 0;  // u's slice of the chunk in lab (big labels)
    auto held = [&](uint32_t w) -> bool {
        if (w < land_end) return lrow_t[w - base] != kInfL;
        return tabl(w) != kNone;
    };
    // this lane's 16 landmarks of u, and whether any of them is within d-2
    // (a landmark farther from u cannot prove d_u + d_w < d since d_w >= 1)
    LW uw[4];
    bool slice_useful = false;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        uw[q] = lrow[4 * gl + q];
        slice_useful |= d >= 3 && land_count_le(uw[q], d - 2) > 0;
    }

    const uint64_t g0 = a.goff[u];
    const uint32_t deg = (uint32_t)(a.goff[u + 1] - g0);
    const uint64_t tbase = a.raw_off[u] - a.raw_off[a.u_lo];
    uint32_t nout = 0;
    uint64_t st_raw = 0, st_merged = 0, st_kept = 0;
    // Chunks of the hub range [0, u).  Every neighbour keeps a cursor into
    // its round d-1 segment (first entry with hub >= lo), so a chunk costs one
    // galloping search per neighbour; a chunk is sized from its exact pull
    // count and the pulls-per-distinct-candidate ratio seen so far, so that
    // the candidate table rarely overflows.
    constexpr uint32_t kTarget = kULimit * 3 / 4;  // distinct candidates aimed at
    constexpr int kSizePasses = 8;                  // pull counts taken per chunk at most
    const bool one_group = deg <= (uint32_t)RB;   // cursors live in registers
    uint32_t my_v = 0, my_ln = 0, my_c = 0, my_e = 0;
    uint64_t my_ps = 0;
    if (one_group && tid < deg) {
        my_v = a.gadj[g0 + tid];
        my_ln = a.plen[my_v];
        my_ps = my_ln ? a.pstart[my_v] : 0;
    }
    float ratio = 2.0f;      // pulls per distinct candidate
    bool may_widen = true;   // false from an overflow until a chunk completes
    // u's hubs are vertices of its own graph, ids [base, ur): the chunks
    // start at base (a batch's other graphs hold none)
    const uint32_t lo0 = base < ur ? base : ur;
    uint32_t lo = lo0, width = ur - lo0;
    if (raw_u > (uint64_t)(2 * kTarget)) {
        uint64_t parts = (raw_u + 2 * kTarget - 1) / (2 * kTarget);
        width = (uint32_t)((ur - lo0) / parts) > 0 ? (uint32_t)((ur - lo0) / parts) : 1;
    }

    // 2-5, chunk by chunk
    while (lo < ur) {
        // A. size the chunk.  With cursors in registers the exact pull count
        //    of [lo, hi) is cheap: the range is narrowed or widened, up to
        //    kSizePasses - 1 times, until the expected distinct count falls
        //    in the band (the count is exact for each try).  Wider pullers take the
        //    width learned from the previous chunk.  A label staged chunk by
        //    chunk caps the range at the hub of its entry kLStage past the
        //    cursor (which is above lo).
        uint32_t hend = ur;
        if (big && tcur + kLStage < nsp) {
            const uint32_t hc = e_hub<DB>(lab[tcur + kLStage]);
            hend = hc < ur ? hc : ur;
        }
        uint32_t hi = (width >= hend - lo) ? hend : lo + width, tot = 0;
        if (one_group) {
            for (int it = 0;; it++) {
                hi = (width >= hend - lo) ? hend : lo + width;
                uint32_t t = 0;
                if (tid < deg) {
                    // hubs of v's segment are <= v
                    my_e = (real(my_v) >= lo && my_c < my_ln) ? gallop_u32(a.pool_hub + my_ps, my_c, my_ln, hi)
                                                        : my_c;
                    t = my_e - my_c;
                }
                block_excl_scan<uint32_t, RW>(t, red32, tot);
                if (it + 1 == kSizePasses) break;
                const float expect = (float)tot / ratio;
                if (expect > 1.25f * kTarget && hi - lo > 1) {
                    uint32_t w2 = (uint32_t)((float)(hi - lo) * ((float)kTarget / expect));
                    width = w2 ? w2 : 1;
                    continue;
                }
                if (may_widen && expect < 0.75f * kTarget && hi < hend) {
                    float f = expect > 1.0f ? (float)kTarget / expect : 8.0f;
                    f = f > 8.0f ? 8.0f : f;
                    uint64_t w2 = (uint64_t)((double)(hi - lo) * f);
                    width = w2 >= (uint64_t)(hend - lo) ? hend - lo : (uint32_t)w2;
                    continue;
                }
                break;
            }
        }

        // B. pull: Label Elimination, then Label Merging in the table
        for (int i = tid; i < kCCap; i += RB) {
            ckey[i] = kEmpty32;
            cval[i] = 0;
            cwrap[i] = 0;
        }
        // a long label: stage its entries with hubs in [lo, hi), from the
        // cursor (first entry with hub >= lo), RB per trip
        if (big) {
            for (int i = tid; i < kLCap; i += RB) ltab[i] = kEmptyE;
            __syncthreads();
            uint64_t b = tcur;
            while (true) {
                const uint64_t j = b + tid;
                const E e = j < nsp ? lab[j] : (E)0;
                const bool in = j < nsp && e_hub<DB>(e) < hi;  // a prefix of the trip
                if (in) {
                    uint32_t s = hash_slot(e_hub<DB>(e), LB);
                    while (atomicCAS(&ltab[s], kEmptyE, e) != kEmptyE) s = (s + 1) & (kLCap - 1);
                }
                const uint32_t cnt = (uint32_t)__syncthreads_count(in);
                b += cnt;
                if (cnt < (uint32_t)RB) break;
            }
            tend = b;
        }
        if (tid == 0) {
            s_nuniq = 0;
            s_ovf = 0;
        }
        __syncthreads();
        for (uint32_t nb0 = 0; nb0 < deg; nb0 += RB) {
            const uint32_t nb = nb0 + tid;
            uint64_t sb = 0;
            uint32_t len = 0;
            if (nb < deg) {
                uint32_t c = my_c, e = my_e;
                uint64_t ps = my_ps;
                if (!one_group) {
                    const uint32_t v = a.gadj[g0 + nb];
                    const uint32_t ln = a.plen[v];
                    ps = ln ? a.pstart[v] : 0;
                    c = lo > lo0 ? a.cur[g0 + nb] : 0;  // the first chunk starts the cursors
                    e = (real(v) >= lo && c < ln) ? gallop_u32(a.pool_hub + ps, c, ln, hi) : c;
                    a.nxt[g0 + nb] = e;
                }
                sb = ps + c;
                len = e - c;
            }
            uint32_t gt;
            const uint32_t ex = block_excl_scan<uint32_t, RW>(len, red32, gt);
            if (!one_group) tot += gt;
            nb_start[tid] = sb;
            nb_off[tid] = ex;
            __syncthreads();
            uint32_t jl = 0;  // owner of k: last j with nb_off[j] <= k (monotone in k)
            // kPullUnroll pulled entries per thread and trip: their loads are
            // issued together, then each is eliminated or merged
            for (uint32_t k0 = tid; k0 < gt; k0 += kPullUnroll * RB) {
                if (*(volatile uint32_t *)&s_ovf) break;
                uint32_t wq[kPullUnroll];
                uint64_t cq[kPullUnroll];
#pragma unroll
                for (int r = 0; r < kPullUnroll; r++) {
                    const uint32_t k = k0 + r * RB;
                    wq[r] = kEmpty32;  // no hub: past the chunk's pulls
                    cq[r] = 0;
                    if (k < gt) {
                        if (jl + 1 < (uint32_t)RB && nb_off[jl + 1] <= k) {
                            uint32_t lo2 = jl + 1, hi2 = RB - 1;
                            while (lo2 < hi2) {
                                uint32_t mid = (lo2 + hi2 + 1) >> 1;
                                if (nb_off[mid] <= k)
                                    lo2 = mid;
                                else
                                    hi2 = mid - 1;
                            }
                            jl = lo2;
                        }
                        const uint64_t idx = nb_start[jl] + (k - nb_off[jl]);
                        wq[r] = a.pool_hub[idx];
                        cq[r] = a.pool_cnt[idx];
                        if constexpr (W) cq[r] = sat_mul(cq[r], (uint64_t)a.adj_w[g0 + nb0 + jl]);
                    }
                }
#pragma unroll
                for (int r = 0; r < kPullUnroll; r++) {
                    const uint32_t w = wq[r];
                    const uint64_t c = cq[r];
                    if (w == kEmpty32 || held(w)) continue;  // Label Elimination
                    uint32_t s = hash_slot(w, kCBits);
                    bool ok = true;
                    for (uint32_t probes = 0;; probes++) {
                        uint32_t kk = ckey[s];
                        if (kk == w) break;
                        if (kk == kEmpty32) {
                            uint32_t old = atomicCAS(&ckey[s], kEmpty32, w);
                            if (old == kEmpty32) {
                                if (atomicAdd(&s_nuniq, 1u) + 1 > (uint32_t)kULimit) s_ovf = 1;
                                break;
                            }
                            if (old == w) break;
                        }
                        s = (s + 1) & (kCCap - 1);
                        if (probes + 1 >= (uint32_t)kCCap) {
                            s_ovf = 1;
                            ok = false;
                            break;
                        }
                    }
                    if (ok) {  // Label Merging: saturating sum, wrap recorded
                        unsigned long long old = atomicAdd(&cval[s], (unsigned long long)c);
                        if (old + c < old) cwrap[s] = 1;
                    }
                }
            }
            __syncthreads();
        }
        if (s_ovf) {
            // too many distinct hubs after all: at least s_nuniq of them came
            // from at most tot pulls, so the ratio is lowered to match and
            // the range only narrows until a chunk completes (a range of one
            // hub always fits)
            const float r = (float)tot / (float)(s_nuniq > 0 ? s_nuniq : 1);
            ratio = r < ratio ? r : ratio;
            may_widen = false;
            width = (hi - lo) > 1 ? (hi - lo) >> 1 : 1;
            __syncthreads();
            continue;
        }
        // the chunk is complete: advance the cursors
        tcur = tend;
        if (one_group) {
            my_c = my_e;
        } else {
            for (uint32_t nb = tid; nb < deg; nb += RB) a.cur[g0 + nb] = a.nxt[g0 + nb];
        }
        const uint64_t chunk_raw = tot;

        // compact the table into a list (any order: survivors are ranked by
        // hub at the end)
        uint32_t nv = 0;
        for (int j = 0; j < kCCap / RB; j++) nv += ckey[tid * (kCCap / RB) + j] != kEmpty32;
        uint32_t M;
        uint32_t ex = block_excl_scan<uint32_t, RW>(nv, red32, M);
        for (int j = 0; j < kCCap / RB; j++) {
            uint32_t s = tid * (kCCap / RB) + j;
            uint32_t kk = ckey[s];
            if (kk != kEmpty32) {
                lhub[ex] = kk;
                lcnt[ex] = cwrap[s] ? kSat : cval[s];
                ex++;
            }
        }
        __syncthreads();

        // 4. prune probes (nothing can prune before round 3: a common hub
        //    with d_u + d_w < 2 would be u or w itself).
        //  4a. landmark pass, 16 lanes per candidate (4 candidates per wave):
        //      lane gl compares landmarks [16 gl, 16 gl + 16) of the two rows,
        //      reading w's slice only if u has a landmark within d-2 there.
        uint64_t my_tail = 0, my_hdr = 0, my_rowb = 0, my_filt = 0;
        if (d >= 3 && a.lmask && d - 2 <= (uint32_t)kMaskK) {
            // by the landmark masks, one candidate per thread: w is pruned
            // if some landmark l it holds at distance k in [1, d-2] is held
            // by u at distance <= d-1-k, i.e. E_k(w) meets A_{d-1-k}(u)
            // with A_j(u) = {l : d_u(l) <= j}, built here from u's row in
            // nb_off (idle outside the pull)
            uint32_t *amask = nb_off;
            static_assert(kLand == RB && kLand / 64 * 2 == kMaskWords, "one landmark per thread");
            for (uint32_t j = 1; j + 2 <= d; j++) {
                const uint64_t bal = __ballot((uint32_t)lrow_t[tid] <= j);
                if (lane == 0) {
                    amask[(j - 1) * kMaskWords + 2 * wv] = (uint32_t)bal;
                    amask[(j - 1) * kMaskWords + 2 * wv + 1] = (uint32_t)(bal >> 32);
                }
            }
            __syncthreads();
            const uint32_t nk = d - 2;
            for (uint32_t i0 = tid; i0 < M; i0 += kLandUnroll * RB) {
                bool hit[kLandUnroll];
#pragma unroll
                for (int r = 0; r < kLandUnroll; r++) hit[r] = false;
                // two levels per trip: their loads are in flight together
                for (uint32_t k = 1; k <= nk; k += 2) {
                    uint4 ev[kLandUnroll][4];
#pragma unroll
                    for (int r = 0; r < kLandUnroll; r++) {
                        const uint32_t i = i0 + r * RB;
                        if (i < M) {
                            const uint4 *em = a.lmask + ((uint64_t)(lhub[i] + poff) * kMaskK + (k - 1)) * 2;
                            ev[r][0] = em[0];
                            ev[r][1] = em[1];
                            if (k + 1 <= nk) {
                                ev[r][2] = em[2];
                                ev[r][3] = em[3];
                            } else {
                                ev[r][2] = ev[r][3] = make_uint4(0, 0, 0, 0);
                            }
                        } else {
                            ev[r][0] = ev[r][1] = ev[r][2] = ev[r][3] = make_uint4(0, 0, 0, 0);
                        }
                    }
                    const uint32_t *a0 = amask + (d - 2 - k) * kMaskWords;  // A_{d-1-k}
                    const uint32_t *a1 = amask + (k + 1 <= nk ? d - 3 - k : 0) * kMaskWords;  // A_{d-2-k}
#pragma unroll
                    for (int r = 0; r < kLandUnroll; r++) {
                        const uint4 x0 = ev[r][0], x1 = ev[r][1], y0 = ev[r][2], y1 = ev[r][3];
                        uint32_t o = (x0.x & a0[0]) | (x0.y & a0[1]) | (x0.z & a0[2]) | (x0.w & a0[3]) |
                                     (x1.x & a0[4]) | (x1.y & a0[5]) | (x1.z & a0[6]) | (x1.w & a0[7]);
                        o |= (y0.x & a1[0]) | (y0.y & a1[1]) | (y0.z & a1[2]) | (y0.w & a1[3]) |
                             (y1.x & a1[4]) | (y1.y & a1[5]) | (y1.z & a1[6]) | (y1.w & a1[7]);
                        hit[r] |= o != 0;
                    }
                }
#pragma unroll
                for (int r = 0; r < kLandUnroll; r++) {
                    const uint32_t i = i0 + r * RB;
                    if (i < M) {
                        lkeep[i] = hit[r] ? 0 : (lhub[i] - base >= (uint32_t)kLand ? 2 : 1);
                        my_rowb += (uint64_t)nk * kMaskWords * sizeof(uint32_t);
                    }
                }
            }
        } else if (d >= 3) {
            // kLandUnroll candidates per group and trip, their row slices
            // loaded together
            for (uint32_t i0 = wv * 4; i0 < M; i0 += kLandUnroll * (RB / 16)) {
                LW rv[kLandUnroll][4];
                uint32_t wl[kLandUnroll];
                bool rd[kLandUnroll];
#pragma unroll
                for (int r = 0; r < kLandUnroll; r++) {
                    const uint32_t i = i0 + r * (RB / 16) + grp;
                    wl[r] = i < M ? lhub[i] - base : 0;
                    rd[r] = i < M && slice_useful && 16 * gl <= wl[r];  // landmarks above w are not its hubs
                    if (rd[r]) {
                        const LW *rw = lands + (uint64_t)(lhub[i] + poff) * (kLand / 4) + 4 * gl;
#pragma unroll
                        for (int q = 0; q < 4; q++) rv[r][q] = rw[q];
                    }
                }
#pragma unroll
                for (int r = 0; r < kLandUnroll; r++) {
                    const uint32_t i = i0 + r * (RB / 16) + grp;
                    bool hit = false;
                    if (rd[r]) {
#pragma unroll
                        for (int q = 0; q < 4; q++) hit |= land_hit(uw[q], rv[r][q], d);
                    }
                    const bool ghit = ((__ballot(hit) >> (16 * grp)) & 0xFFFFull) != 0;
                    uint32_t loads = rd[r] ? 1 : 0;
#pragma unroll
                    for (int o = 8; o > 0; o >>= 1) loads += __shfl_xor(loads, o, 16);
                    if (i < M && gl == 0) {
                        lkeep[i] = ghit ? 0 : (wl[r] >= (uint32_t)kLand ? 2 : 1);
                        my_rowb += (uint64_t)loads * 16 * sizeof(LT);
                    }
                }
            }
        } else {
            for (uint32_t i = tid; i < M; i += RB) lkeep[i] = 1;
        }
        // u's entries of distance <= d-2 past the landmarks go to the
        // candidate table's count array (idle until the next chunk) when they
        // fit, for the probes below
        E *pl = reinterpret_cast<E *>(cval);
        constexpr uint64_t kPuCap = (uint64_t)kCCap * sizeof(unsigned long long) / sizeof(E);
        const bool pstaged = d >= 3 && npu <= kPuCap;
        if (pstaged)
            for (uint32_t j = tid; j < (uint32_t)npu; j += RB) pl[j] = pu[j];
        __syncthreads();
        //  4b. the other hubs of the surviving non-landmark candidates: their
        //      entries of distance <= d-2 past the landmarks on both sides
        //      (L_{<=d-2} is the previous round's merged label).  Either stream
        //      w's entries and look each hub up in u's table, or stream u's
        //      entries with hub < w (a common hub ranks at or above w) and
        //      binary-search each in w's sorted label, whichever reads fewer
        //      entries.  16 lanes per candidate.
        uint32_t T = 0;
        if (d >= 3) {
            uint32_t f[PER], nf = 0;
#pragma unroll
            for (int q = 0; q < PER; q++) {
                uint32_t i = PER * tid + q;
                f[q] = (i < M && lkeep[i] == 2) ? 1 : 0;
                // a common hub ranks above w: none of u's hubs below w, no probe
                if (f[q] && pstaged && (npu == 0 || e_hub<DB>(pl[0]) >= lhub[i])) {
                    lkeep[i] = 1;
                    f[q] = 0;
                }
                nf += f[q];
            }
            if (tid == 0) s_next = 0;
            uint32_t p = block_excl_scan<uint32_t, RW>(nf, red32, T);
#pragma unroll
            for (int q = 0; q < PER; q++)
                if (f[q]) tlist[p++] = (uint16_t)(PER * tid + q);
            __syncthreads();
        }
        // The candidates' scans differ widely in length, so the 16-lane
        // groups take them from a shared counter: a group that finishes one
        // takes the next, one 16-entry step per trip, and no group waits for
        // a slow one of another wave.
        if (T > 0 && pstaged && a.filt) {
            // Filtered probes.  Every pair (candidate w, entry (h, d_u) of
            // pl[0, cu_w)) is looked up in the membership filter first, as
            // (w, h, d_w) for each d_w < d - d_u (at most kFiltProbes of
            // them; more count as a hit): misses prove that no entry of w
            // past its landmarks gives d_u + d_w < d through h.  The pairs
            // that hit (the proving ones and the filter's rare false
            // positives) are listed, then binary-searched in w's label, one
            // per thread.
            // Pairs are numbered candidate by candidate: pre[t] is the first
            // pair of tlist[t] (the candidate table's key array is idle here),
            // freg[t] its row's filter words.
            uint32_t *pre = ckey;
            uint32_t *vlist = reinterpret_cast<uint32_t *>(nb_start);  // (t << 16) | j
            constexpr uint32_t kVCap = kFiltList < RB * 2 ? kFiltList : RB * 2;  // nb_start's bytes
            uint32_t P = 0;
            {
                uint32_t cq[PER], sum = 0;
                uint64_t o0[PER], o1[PER];
#pragma unroll
                for (int q = 0; q < PER; q++) {
                    const uint32_t t = PER * tid + q;
                    cq[q] = 0;
                    o0[q] = o1[q] = 0;
                    if (t < T) {
                        const uint32_t w = lhub[tlist[t]];
                        o0[q] = a.prev_off[w + poff];
                        o1[q] = a.prev_off[w + poff + 1];
                        cq[q] = (uint32_t)lower_bound_hub<DB>(pl, npu, w);  // >= 1
                    }
                    sum += cq[q];
                }
                uint32_t ex = block_excl_scan<uint32_t, RW>(sum, red32, P);
#pragma unroll
                for (int q = 0; q < PER; q++) {
                    const uint32_t t = PER * tid + q;
                    if (t < T) {
                        pre[t] = ex;
                        ex += cq[q];
                        freg[t] = filt_region(o0[q], o1[q], a.filt_words, a.filt_shift);
                        lkeep[tlist[t]] = 1;  // until a search proves a shorter path
                    }
                }
                if (tid == 0) {
                    pre[T] = P;
                    s_nver = 0;
                }
                __syncthreads();
            }
            // binary search of u's entry pl[j] in w = lhub[tlist[t]]'s label
            auto search = [&](uint32_t t, uint32_t j) {
                const uint32_t i = tlist[t];
                if (!lkeep[i]) return;  // another pair has proved it already
                const uint32_t wr = lhub[i] + poff;
                const uint64_t q0 = a.prev_off[wr];
                const uint64_t np = a.prev_off[wr + 1] - q0 - 1;  // the last entry is (w, 0)
                const uint64_t p0 = a.lc_prev[wr];
                const E *pw = static_cast<const E *>(a.prev_hd) + q0;
                const E e = pl[j];
                const uint32_t h = e_hub<DB>(e);
                const uint64_t nw = np - p0;
                const uint64_t q = p0 + lower_bound_hub<DB>(pw + p0, nw, h);
                if (q < np && e_hub<DB>(pw[q]) == h && e_dist<DB>(e) + e_dist<DB>(pw[q]) < d) lkeep[i] = 0;
                uint32_t steps = 1;
                while ((1ull << steps) <= nw) steps++;
                my_tail += steps;
                my_hdr++;
            };
            uint32_t own = 0;  // owner of pair p: last t with pre[t] <= p (monotone in p)
            for (uint32_t pb = tid; pb < P; pb += kProbeUnroll * RB) {
                uint32_t tq[kProbeUnroll], jq[kProbeUnroll];
                bool vq[kProbeUnroll], hq[kProbeUnroll];
                unsigned long long mq[kProbeUnroll][kFiltProbes], wq[kProbeUnroll][kFiltProbes];
#pragma unroll
                for (int r = 0; r < kProbeUnroll; r++) {
                    const uint32_t p = pb + r * RB;
                    vq[r] = p < P;
                    hq[r] = false;  // a hit without lookups (too many distances)
                    tq[r] = jq[r] = 0;
#pragma unroll
                    for (int k = 0; k < kFiltProbes; k++) {
                        mq[r][k] = 0;  // no lookup
                        wq[r][k] = 0;
                    }
                    if (vq[r]) {
                        if (pre[own + 1] <= p) {
                            uint32_t lo2 = own + 1, hi2 = T - 1;
                            while (lo2 < hi2) {
                                const uint32_t mid = (lo2 + hi2 + 1) >> 1;
                                if (pre[mid] <= p)
                                    lo2 = mid;
                                else
                                    hi2 = mid - 1;
                            }
                            own = lo2;
                        }
                        tq[r] = own;
                        jq[r] = p - pre[own];
                        const E e = pl[jq[r]];
                        const uint32_t wr = lhub[tlist[own]] + poff, h = e_hub<DB>(e);
                        const uint2 reg = freg[own];
                        const uint32_t nd = d - 1 - e_dist<DB>(e);  // d_w in [1, nd]; d_u <= d-2
                        hq[r] = nd > (uint32_t)kFiltProbes;
#pragma unroll
                        for (int k = 0; k < kFiltProbes; k++)
                            if (!hq[r] && (uint32_t)k < nd) {
                                const uint64_t x = filt_mix(wr, h, (uint32_t)k + 1);
                                mq[r][k] = filt_bits(x);
                                wq[r][k] = a.filt[filt_word(reg, x)];
                                my_filt += sizeof(unsigned long long);
                            }
                    }
                }
#pragma unroll
                for (int r = 0; r < kProbeUnroll; r++) {
                    bool hit = hq[r];
#pragma unroll
                    for (int k = 0; k < kFiltProbes; k++)
                        hit |= mq[r][k] != 0 && (wq[r][k] & mq[r][k]) == mq[r][k];
                    if (!vq[r] || !hit) continue;  // no pair, or absent
                    const uint32_t slot = atomicAdd(&s_nver, 1u);
                    if (slot < kVCap)
                        vlist[slot] = (tq[r] << 16) | jq[r];
                    else
                        search(tq[r], jq[r]);  // the list is full
                }
            }
            __syncthreads();
            const uint32_t nver = s_nver < kVCap ? s_nver : kVCap;
            for (uint32_t v = tid; v < nver; v += RB) search(vlist[v] >> 16, vlist[v] & 0xFFFFu);
        } else if (T > 0 && pstaged) {
            // u's side is pl[0, cu), its hubs below w, in LDS.  Groups of PG
            // lanes take one candidate each and either
            //  B. binary-search u's cu hubs in w's entries, PG at a time, or
            //  A. stream w's entries, 4 PG per trip (each PG-lane load
            //     contiguous), looking each hub up in u's table, until a hit
            //     or a hub past u's last one below w,
            // whichever reads fewer entries; the last levels of a binary
            // search stay within one cache line.  The next candidate's label
            // offsets are loaded one trip ahead, with the current entries.
            constexpr uint32_t PG = kProbeGroup;
            constexpr uint64_t kPGMask = PG == 64 ? ~0ull : ((1ull << PG) - 1);
            const uint32_t pgi = lane / PG, pgl = lane % PG;
            bool have = false, nhave = false, useu = false;
            uint32_t i = 0, ni = 0, it = 0, nit = 0, cu = 0, hmax = 0, nlc = 0;
            uint64_t nq0 = 0, nq1 = 0, np = 0, p0 = 0, nw = 0, read = 0, wt = 1;
            const E *pw = nullptr;
            auto grab = [&]() {  // called by whole groups
                uint32_t got = 0;
                if (pgl == 0) got = atomicAdd(&s_next, 1u);
                got = (uint32_t)__shfl((int)got, (int)(pgi * PG), 64);
                nhave = got < T;
                if (nhave) {
                    ni = tlist[got];
                    const uint32_t wr = lhub[ni] + poff;
                    nq0 = a.prev_off[wr];
                    nq1 = a.prev_off[wr + 1];
                    nlc = a.lc_prev[wr];
                }
            };
            // u's distance to hub h <= hmax of w's label (kNone: not held
            // within d-2 past the landmarks)
            auto du_of = [&](uint32_t h) -> uint32_t {
                if (h < look.x) return look(h);
                const uint32_t p = (uint32_t)lower_bound_hub<DB>(pl, cu, h);
                return (p < cu && e_hub<DB>(pl[p]) == h) ? e_dist<DB>(pl[p]) : kNone;
            };
            grab();
            while (true) {
                if (!have && nhave) {  // uniform within the group
                    i = ni;
                    const uint32_t w = lhub[i];
                    pw = static_cast<const E *>(a.prev_hd) + nq0;
                    np = nq1 - nq0 - 1;  // the last entry is (w, 0)
                    p0 = nlc;
                    nw = np - p0;
                    grab();
                    cu = (uint32_t)lower_bound_hub<DB>(pl, npu, w);  // >= 1
                    hmax = e_hub<DB>(pl[cu - 1]);
                    uint32_t steps = 1;
                    while ((1ull << steps) <= nw) steps++;
                    useu = (uint64_t)cu * steps < nw;
                    nit = useu ? (cu + PG - 1) / PG : (uint32_t)((nw + 4 * PG - 1) / (4 * PG));
                    wt = useu ? steps : 1;
                    it = 0;
                    read = 0;
                    have = nit > 0;
                    if (!have && pgl == 0) {  // w holds nothing past its landmarks: kept
                        lkeep[i] = 1;
                        my_hdr++;
                    }
                }
                if (__ballot(have || nhave) == 0) break;
                bool h2 = false, past = false;
                if (have) {
                    if (useu) {
                        const uint32_t j = it * PG + pgl;
                        if (j < cu) {
                            const E e = pl[j];
                            const uint32_t h = e_hub<DB>(e);
                            const uint64_t q = p0 + lower_bound_hub<DB>(pw + p0, nw, h);
                            h2 = q < np && e_hub<DB>(pw[q]) == h && e_dist<DB>(e) + e_dist<DB>(pw[q]) < d;
                        }
                    } else {
                        const uint64_t j0 = (uint64_t)it * (4 * PG) + pgl;
                        E ev[4];
                        bool ok[4];
#pragma unroll
                        for (int k = 0; k < 4; k++) {
                            ok[k] = j0 + PG * k < nw;
                            ev[k] = ok[k] ? pw[p0 + j0 + PG * k] : (E)0;
                        }
#pragma unroll
                        for (int k = 0; k < 4; k++) {
                            if (!ok[k]) continue;
                            const uint32_t h = e_hub<DB>(ev[k]);
                            if (h > hmax) {
                                past = true;  // and every later entry of w
                                continue;
                            }
                            const uint32_t du = du_of(h);
                            h2 |= du != kNone && du + e_dist<DB>(ev[k]) < d;
                        }
                    }
                }
                const bool ghit = ((__ballot(h2) >> (PG * pgi)) & kPGMask) != 0;
                const bool gpast = ((__ballot(past) >> (PG * pgi)) & kPGMask) != 0;
                if (have) {
                    const uint64_t tile = useu ? PG : 4 * PG, lenx = useu ? cu : nw;
                    const uint64_t done = (uint64_t)it * tile;
                    read += (lenx - done < tile ? lenx - done : tile) * wt;
                    if (ghit || gpast || ++it >= nit) {
                        if (pgl == 0) {
                            lkeep[i] = ghit ? 0 : 1;
                            my_tail += read;
                            my_hdr++;
                        }
                        have = false;
                    }
                }
            }
        } else if (T > 0) {
            bool have = false, retired = false;
            uint32_t i = 0, it = 0, nit = 0;
            uint64_t np = 0, p0 = 0, nw = 0, len = 0, read = 0, wt = 1;
            const E *pw = nullptr;
            bool useu = false;
            // w's side: the current tile of w's entries (one per lane), which
            // of them are decided, and a cursor into the part of u's label
            // not staged in LDS
            bool fresh = true, res = true, hit = false;
            E ew = (E)0;
            uint64_t ut = 0, upos = 0;
            uint32_t usteps = 0;
            bool tmerge = false;  // merge with u's unstaged part (labels of similar size)
            while (true) {
                if (!have && !retired) {  // uniform within the group
                    uint32_t got = 0;
                    if (gl == 0) got = atomicAdd(&s_next, 1u);
                    got = (uint32_t)__shfl((int)got, (int)(grp * 16), 64);
                    if (got < T) {
                        i = tlist[got];
                        const uint32_t w = lhub[i];
                        const uint64_t q0 = a.prev_off[w + poff];
                        np = a.prev_off[w + poff + 1] - q0 - 1;  // the last entry is (w, 0)
                        p0 = a.lc_prev[w + poff];
                        pw = static_cast<const E *>(a.prev_hd) + q0;
                        nw = np - p0;
                        const uint64_t cu = lower_bound_hub<DB>(pu, npu, w);
                        uint32_t steps = 1;
                        while ((1ull << steps) <= nw) steps++;
                        useu = cu * steps < nw;
                        len = useu ? cu : nw;
                        wt = useu ? steps : 1;
                        nit = (uint32_t)((len + 15) / 16);
                        it = 0;
                        read = 0;
                        fresh = true;
                        ut = 0;
                        tmerge = look.ntail <= 4 * nw;
                        have = true;
                        if (nit == 0) {  // nothing to scan: kept
                            if (gl == 0) {
                                lkeep[i] = 1;
                                my_hdr++;
                            }
                            have = false;
                        }
                    } else {
                        retired = true;
                    }
                }
                if (__ballot(have || !retired) == 0) break;
                bool h2 = false, step_done = true;
                if (have) {
                    if (useu) {
                        const uint64_t j = (uint64_t)it * 16 + gl;
                        if (j < len) {
                            const E e = pu[j];
                            const uint32_t h = e_hub<DB>(e);
                            const uint64_t q = p0 + lower_bound_hub<DB>(pw + p0, nw, h);
                            h2 = q < np && e_hub<DB>(pw[q]) == h && e_dist<DB>(e) + e_dist<DB>(pw[q]) < d;
                        }
                    } else if (!TM || look.ntail == 0) {
                        // u's label all in LDS, or no merge: u's unstaged part
                        // (if any) is binary-searched by look()
                        const uint64_t j = (uint64_t)it * 16 + gl;
                        if (j < len) {
                            const E e = pw[p0 + j];
                            const uint32_t du = look(e_hub<DB>(e));
                            h2 = du != kNone && du + e_dist<DB>(e) < d;
                        }
                    } else {
                        if (fresh) {  // next 16 entries of w; hubs staged for u are looked up in LDS
                            const uint64_t j = (uint64_t)it * 16 + gl;
                            ew = j < len ? pw[p0 + j] : (E)0;
                            res = j >= len;
                            hit = false;
                            const uint32_t h = e_hub<DB>(ew);
                            if (!res && h < look.x) {
                                const uint32_t du = look(h);
                                hit = du != kNone && du + e_dist<DB>(ew) < d;
                                res = true;
                            }
                            fresh = false;
                            usteps = 0;
                            upos = ut;
                        }
                        // the others in the part of u's label not staged: a
                        // 16-wide merge from the cursor for a few trips (the near
                        // hubs), then parallel binary searches past the cursor;
                        // the cursor ends at the furthest position found, since
                        // the next tile's hubs are larger
                        if (!tmerge && ((__ballot(!res) >> (16 * grp)) & 0xFFFFull)) {
                            // u's unstaged part is much longer than w's entries:
                            // binary searches from the cursor
                            uint64_t q = ut;
                            if (!res) {
                                const uint32_t h = e_hub<DB>(ew);
                                q = ut + lower_bound_hub<DB>(look.tail + ut, look.ntail - ut, h);
                                hit = q < look.ntail && e_hub<DB>(look.tail[q]) == h &&
                                      e_dist<DB>(look.tail[q]) + e_dist<DB>(ew) < d;
                                res = true;
                            }
#pragma unroll
                            for (int o = 8; o > 0; o >>= 1) {
                                const uint64_t y = __shfl_xor(q, o, 16);
                                q = y > q ? y : q;
                            }
                            ut = q;
                        } else if ((__ballot(!res) >> (16 * grp)) & 0xFFFFull) {
                            const bool tv = ut + gl < look.ntail;
                            const E te = tv ? look.tail[ut + gl] : (E)0;
                            const uint32_t th = tv ? e_hub<DB>(te) : 0xFFFFFFFFu;
                            const uint32_t lastu = (uint32_t)__shfl((int)th, 15, 16);
                            const uint32_t h = e_hub<DB>(ew);
                            uint32_t pp = 0;
#pragma unroll
                            for (uint32_t st = 8; st > 0; st >>= 1) {
                                const uint32_t y = (uint32_t)__shfl((int)th, (int)(pp + st - 1), 16);
                                if (y < h) pp += st;
                            }
                            const uint32_t hp = (uint32_t)__shfl((int)th, (int)pp, 16);
                            const E ep = (E)__shfl(te, (int)pp, 16);
                            if (!res && h <= lastu) {
                                hit = hp == h && e_dist<DB>(ep) + e_dist<DB>(ew) < d;
                                upos = ut + pp;
                                res = true;
                            }
                            if (ut < look.ntail) read += (look.ntail - ut < 16) ? look.ntail - ut : 16;
                            const bool more = ((__ballot(!res) >> (16 * grp)) & 0xFFFFull) != 0;
                            if (more && ++usteps < kTailSteps) {
                                ut += 16;  // merge on next trip; this tile waits
                                step_done = false;
                            } else {
                                if (!res) {
                                    const uint64_t b = ut + 16;
                                    const uint64_t q =
                                        b + lower_bound_hub<DB>(look.tail + b, look.ntail - b, h);
                                    hit = q < look.ntail && e_hub<DB>(look.tail[q]) == h &&
                                          e_dist<DB>(look.tail[q]) + e_dist<DB>(ew) < d;
                                    upos = q;
                                    res = true;
                                }
                                uint64_t mx = upos;
#pragma unroll
                                for (int o = 8; o > 0; o >>= 1) {
                                    const uint64_t y = __shfl_xor(mx, o, 16);
                                    mx = y > mx ? y : mx;
                                }
                                ut = mx;
                            }
                        }
                        h2 = hit;
                    }
                }
                const uint64_t m = __ballot(h2 && step_done);
                const uint32_t gm = (uint32_t)((m >> (16 * grp)) & 0xFFFFull);
                if (have && step_done) {
                    bool fin = false, found = false;
                    if (gm) {
                        found = fin = true;
                        read += (uint64_t)__ffs(gm) * wt;
                    } else {
                        const uint64_t k = len - (uint64_t)it * 16;
                        read += (k < 16 ? k : 16) * wt;
                        fin = ++it >= nit;
                        fresh = true;
                    }
                    if (fin) {
                        if (gl == 0) {
                            lkeep[i] = found ? 0 : 1;
                            my_tail += read;
                            my_hdr++;
                        }
                        have = false;
                    }
                }
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            my_tail += __shfl_xor(my_tail, o, 64);
            my_hdr += __shfl_xor(my_hdr, o, 64);
            my_rowb += __shfl_xor(my_rowb, o, 64);
            my_filt += __shfl_xor(my_filt, o, 64);
        }
        if (lane == 0) {
            atomicAdd(&s_tail, (unsigned long long)my_tail);
            atomicAdd(&s_hdr, (unsigned long long)my_hdr);
            atomicAdd(&s_rowb, (unsigned long long)my_rowb);
            atomicAdd(&s_filt, (unsigned long long)my_filt);
        }
        __syncthreads();

        // 5. survivors: compact, sort by hub, write out
        uint32_t kk[PER], hh[PER], nk = 0;
        unsigned long long cc[PER];
#pragma unroll
        for (int q = 0; q < PER; q++) {
            uint32_t i = PER * tid + q;
            kk[q] = (i < M) ? lkeep[i] : 0;
            hh[q] = kk[q] ? lhub[i] : 0;
            cc[q] = kk[q] ? lcnt[i] : 0;
            nk += kk[q];
        }
        uint32_t S;
        uint32_t pos = block_excl_scan<uint32_t, RW>(nk, red32, S);
#pragma unroll
        for (int q = 0; q < PER; q++)
            if (kk[q]) {
                lhub[pos] = hh[q];
                lcnt[pos] = cc[q];
                pos++;
            }
        __syncthreads();
        // place them in hub order: a survivor's rank is the number of
        // survivors with a smaller hub (hubs are distinct), counted over the
        // list read four hubs at a time (the same LDS words in every lane);
        // the list is padded to a multiple of 4 with hubs above all
        if (tid < ((4 - (S & 3)) & 3)) lhub[S + tid] = 0xFFFFFFFFu;
        __syncthreads();
        const uint64_t obase = tbase + nout;
        const uint4 *h4 = reinterpret_cast<const uint4 *>(lhub);
        const uint32_t S4 = (S + 3) >> 2;
        for (uint32_t i = tid; i < S; i += RB) {
            const uint32_t h = lhub[i];
            uint32_t r = 0;
            for (uint32_t j = 0; j < S4; j++) {
                const uint4 v = h4[j];
                r += (v.x < h) + (v.y < h) + (v.z < h) + (v.w < h);
            }
            a.tmp_hub[obase + r] = h;
            a.tmp_cnt[obase + r] = lcnt[i];
        }
        nout += S;
        st_raw += chunk_raw;
        st_merged += M;
        st_kept += S;
        lo = hi;
        if (M) ratio = (float)chunk_raw / (float)M;
        if (!one_group) {  // next width from this chunk's distinct count
            float f = M ? (float)kTarget / (float)M : 4.0f;
            f = f > 4.0f ? 4.0f : (f < 0.5f ? 0.5f : f);
            uint64_t w2 = (uint64_t)((double)width * f);
            width = w2 < 1 ? 1 : (w2 > 0x7FFFFFFFull ? 0x7FFFFFFFu : (uint32_t)w2);
        }
        may_widen = true;
        __syncthreads();
    }
    if (tid == 0) {
        a.surv[u] = nout;
        atomicAdd(&a.ctr[0], (unsigned long long)st_raw);
        atomicAdd(&a.ctr[1], (unsigned long long)st_merged);
        atomicAdd(&a.ctr[2], (unsigned long long)st_kept);
        atomicAdd(&a.ctr[3], s_tail);
        atomicAdd(&a.ctr[4], (unsigned long long)nsp);
        atomicAdd(&a.ctr[5], s_rowb);
        atomicAdd(&a.ctr[6], s_hdr);
        atomicAdd(&a.ctr[7], s_filt);
    }
}

// Move a batch's survivors from the temp buffer (each puller's at its pull
// offset) to the round pool, record the round's segment of every vertex of
// the batch, and write the round's landmark entries into the landmark rows.
// One wave per vertex.
template <int DB>
__global__ __launch_bounds__(kBlock) void k_compact(uint32_t u_lo, uint32_t u_hi, uint32_t d,
                                                    const uint64_t *raw_off, const uint64_t *soff,
                                                    const uint32_t *surv, const uint32_t *tmp_hub,
                                                    const uint64_t *tmp_cnt, uint64_t pool_base,
                                                    uint32_t *pool_hub, uint64_t *pool_cnt,
                                                    uint64_t *rstart, uint32_t *rlen,
                                                    const uint32_t *gbase,
                                                    typename Land<DB>::T *land, uint32_t *lmask) {
    uint32_t u = u_lo + blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (u >= u_hi) return;
    uint32_t lane = threadIdx.x & 63;
    uint32_t s = surv[u];
    uint32_t base = gbase ? gbase[u] : 0;
    uint64_t src = raw_off[u] - raw_off[u_lo];
    uint64_t dst = pool_base + soff[u - u_lo];
    for (uint32_t i = lane; i < s; i += 64) {
        uint32_t h = tmp_hub[src + i];
        pool_hub[dst + i] = h;
        pool_cnt[dst + i] = tmp_cnt[src + i];
        if (h - base < (uint32_t)kLand) {
            const uint32_t l = h - base;
            land[(uint64_t)u * kLand + l] = (typename Land<DB>::T)d;
            if (lmask && d >= 1 && d <= (uint32_t)kMaskK)
                atomicOr(&lmask[((uint64_t)u * kMaskK + (d - 1)) * kMaskWords + (l >> 5)], 1u << (l & 31));
        }
    }
    if (lane == 0) {
        rstart[u] = dst;
        rlen[u] = s;
    }
}

__global__ void k_fill_gbase(uint32_t N, const uint32_t *vbase, uint32_t k, uint32_t *gbase) {
    uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < N) gbase[v] = vbase[graph_of(vbase, k, v)];
}

__global__ void k_new_len(uint32_t N, const uint64_t *lab_off, const uint32_t *rlen, uint64_t *nlen) {
    uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u < N) nlen[u] = (lab_off[u + 1] - lab_off[u]) + rlen[u];
}

// L_{<=d}(u) = merge of L_{<d}(u) and round d (disjoint hubs, both sorted).
// Each element's output position is its own index plus the number of smaller
// hubs in the other list.  Also the number of landmark entries of the merged
// label (its landmark prefix).  One wave per vertex.
// outputs of one merge-path step of k_merge (a multiple of 64)
constexpr uint32_t kMergeW = 256;

template <int DB>
__global__ __launch_bounds__(kBlock) void k_merge(uint32_t N, uint32_t d, const uint64_t *lab_off,
                                                  const typename Ent<DB>::T *lab_hd,
                                                  const uint64_t *rstart, const uint32_t *rlen,
                                                  const uint32_t *pool_hub, const uint64_t *new_off,
                                                  typename Ent<DB>::T *new_hd, const uint32_t *gbase,
                                                  const uint32_t *lc_in, uint32_t *lc_out) {
    using E = typename Ent<DB>::T;
    uint32_t u = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (u >= N) return;
    uint32_t lane = threadIdx.x & 63;
    uint64_t a0 = lab_off[u], na = lab_off[u + 1] - a0;
    uint32_t nb = rlen[u];
    const E *A = lab_hd + a0;
    const uint32_t *B = pool_hub + rstart[u];
    E *out = new_hd + new_off[u];
    if (lane == 0) {
        uint32_t land_end = (gbase ? gbase[u] : 0) + kLand;
        lc_out[u] = lc_in[u] + (nb ? lower_bound_u32(B, nb, land_end) : 0);
    }
    if (nb == 0) {
        for (uint64_t i = lane; i < na; i += 64) out[i] = A[i];
        return;
    }
    // Merge path, kMergeW outputs per step: the next kMergeW entries of each
    // list go to LDS (hubs; past a list's end a hub above every vertex), and
    // an entry's place among the step's outputs is its index in its own
    // window plus the count of smaller hubs in the other window (the hubs of
    // the two lists are distinct).  That place is below kMergeW exactly for
    // the entries that come first in the merge, so every step writes the
    // next kMergeW outputs (fewer at the end) and consumes them from A and B.
    constexpr uint32_t K = kMergeW / 64;
    constexpr uint32_t kPast = 0xFFFFFFFFu;
    __shared__ uint32_t sa[kWaves][kMergeW], sb[kWaves][kMergeW];
    const uint32_t wv = threadIdx.x >> 6;
    // entries of window s smaller than x
    auto below = [](const uint32_t *s, uint32_t x) -> uint32_t {
        uint32_t pos = 0;
#pragma unroll
        for (uint32_t step = kMergeW; step > 0; step >>= 1)
            if (pos + step <= kMergeW && s[pos + step - 1] < x) pos += step;
        return pos;
    };
    const uint64_t nt = na + nb;
    uint64_t ia = 0, ib = 0;
    while (ia + ib < nt) {
        E ea[K];
        uint32_t ha[K], hb[K];
#pragma unroll
        for (uint32_t k = 0; k < K; k++) {
            const uint64_t i = ia + k * 64 + lane;
            ea[k] = i < na ? A[i] : (E)0;
            const uint64_t j = ib + k * 64 + lane;
            hb[k] = j < nb ? B[j] : kPast;
        }
#pragma unroll
        for (uint32_t k = 0; k < K; k++) {
            ha[k] = ia + k * 64 + lane < na ? e_hub<DB>(ea[k]) : kPast;
            sa[wv][k * 64 + lane] = ha[k];
            sb[wv][k * 64 + lane] = hb[k];
        }
        wave_lds_sync();
        E *o = out + ia + ib;
        uint32_t take_a = 0;
#pragma unroll
        for (uint32_t k = 0; k < K; k++) {
            if (ha[k] != kPast) {
                const uint32_t r = k * 64 + lane + below(sb[wv], ha[k]);
                if (r < kMergeW) {
                    o[r] = ea[k];
                    take_a++;
                }
            }
            if (hb[k] != kPast) {
                const uint32_t r = k * 64 + lane + below(sa[wv], hb[k]);
                if (r < kMergeW) o[r] = e_make<DB>(hb[k], d);
            }
        }
        const uint32_t na_step = wave_sum(take_a);
        const uint64_t left = nt - ia - ib;
        const uint32_t made = left < kMergeW ? (uint32_t)left : kMergeW;
        ia += na_step;
        ib += made - na_step;
        wave_lds_sync();  // the windows are rewritten next
    }
}

__global__ void k_lc_init(uint32_t N, uint32_t nreal, const uint32_t *gbase, uint32_t *lc) {
    uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t h = (nreal && v >= nreal) ? v - nreal : v;
    if (v < N) lc[v] = (h - (gbase ? gbase[v] : 0)) < (uint32_t)kLand ? 1u : 0u;
}

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
// The round's membership filter: cleared, then every row's older label
// entries past its landmarks, but its own entry (r, 0), inserted with their
// distances into the row's words (one wave per row).
__global__ void k_filt_clear(unsigned long long *f, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        f[i] = 0;
}
template <int DB>
__global__ __launch_bounds__(kBlock) void k_filt_insert(uint32_t N, const uint64_t *off, const void *hd,
                                                        const uint32_t *lc, unsigned long long *f, uint64_t nw,
                                                        uint32_t shift) {
    using E = typename Ent<DB>::T;
    const uint32_t r = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (r >= N) return;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t o0 = off[r], b = o0 + lc[r], e = off[r + 1];
    if (e <= b + 1) return;
    const uint2 reg = filt_region(o0, e, nw, shift);
    const E *lab = static_cast<const E *>(hd);
    for (uint64_t i = b + lane; i < e - 1; i += 64) {
        const uint64_t x = filt_mix(r, e_hub<DB>(lab[i]), e_dist<DB>(lab[i]));
        atomicOr(&f[filt_word(reg, x)], filt_bits(x));
    }
}

// Widen packed entries from 8-bit to 16-bit distances.

__global__ void k_widen(const uint32_t *src, uint64_t *dst, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t e = src[i];
        dst[i] = e_make<16>(e_hub<8>(e), e_dist<8>(e));
    }
}

// Count of every final entry by searching its hub in its round's segment
// (any distance width).
template <int DB>
__global__ __launch_bounds__(kBlock) void k_finalize(uint32_t N, const uint64_t *lab_off,
                                                     const typename Ent<DB>::T *lab_hd,
                                                     const uint64_t *const *rstart_tab,
                                                     const uint32_t *const *rlen_tab,
                                                     const uint32_t *const *hub_tab,
                                                     const uint64_t *const *cnt_tab, uint64_t *lab_cnt,
                                                     unsigned long long *nsat) {
    uint32_t u = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (u >= N) return;
    uint32_t lane = threadIdx.x & 63;
    uint64_t a0 = lab_off[u], na = lab_off[u + 1] - a0;
    uint32_t sat = 0;
    for (uint64_t i = lane; i < na; i += 64) {
        auto e = lab_hd[a0 + i];
        uint32_t r = e_dist<DB>(e), h = e_hub<DB>(e);
        uint64_t ps = rstart_tab[r][u];
        uint32_t ln = rlen_tab[r][u];
        uint32_t p = lower_bound_u32(hub_tab[r] + ps, ln, h);
        uint64_t c = cnt_tab[r][ps + p];
        lab_cnt[a0 + i] = c;
        sat += (c == kSat);
    }
    sat = wave_sum(sat);
    if (lane == 0 && sat) atomicAdd(nsat, (unsigned long long)sat);
}

// Count of every final entry by rank (8-bit distances): a label and each of
// its round segments are sorted by hub, so the j-th entry of distance r in
// L(u) is the j-th entry of u's round-r segment.  One wave per vertex walks
// L(u) kFinalK chunks of 64 at a time (their loads, then their count
// gathers, in flight together), ranking lanes of equal distance with ballots
// and keeping a running count per distance in LDS.
constexpr uint32_t kFinalK = 4;
__global__ __launch_bounds__(kBlock) void k_finalize_rank(uint32_t N, uint32_t R,
                                                          const uint64_t *lab_off,
                                                          const uint32_t *lab_hd,
                                                          const uint64_t *const *rstart_tab,
                                                          const uint64_t *const *cnt_tab,
                                                          uint64_t *lab_cnt, unsigned long long *nsat) {
    __shared__ uint32_t seen[kWaves][256];
    __shared__ uint64_t seg[kWaves][256];
    __shared__ const uint64_t *ctab[256];
    for (uint32_t r = threadIdx.x; r < 256; r += blockDim.x) ctab[r] = r < R ? cnt_tab[r] : nullptr;
    __syncthreads();
    const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t u = blockIdx.x * kWaves + wv;
    if (u >= N) return;
    for (uint32_t r = lane; r < 256; r += 64) {
        seen[wv][r] = 0;
        seg[wv][r] = r < R ? rstart_tab[r][u] : 0;
    }
    wave_lds_sync();
    const uint64_t a0 = lab_off[u], na = lab_off[u + 1] - a0;
    uint32_t sat = 0;
    for (uint64_t i0 = 0; i0 < na; i0 += 64 * kFinalK) {
        uint32_t r[kFinalK];
        bool valid[kFinalK];
#pragma unroll
        for (uint32_t k = 0; k < kFinalK; k++) {
            const uint64_t i = i0 + k * 64 + lane;
            valid[k] = i < na;
            r[k] = valid[k] ? e_dist<8>(lab_hd[a0 + i]) : 0;
        }
        uint64_t at[kFinalK];
#pragma unroll
        for (uint32_t k = 0; k < kFinalK; k++) {
            uint64_t peers = __ballot(valid[k]);
#pragma unroll
            for (int b = 0; b < 8; b++) {
                const uint64_t bb = __ballot((r[k] >> b) & 1);
                peers &= ((r[k] >> b) & 1) ? bb : ~bb;
            }
            const uint32_t rank = __popcll(peers & lanemask_lt());
            const uint32_t base = seen[wv][r[k]];
            at[k] = seg[wv][r[k]] + base + rank;
            wave_lds_sync();
            if (valid[k] && (peers & lanemask_lt()) == 0) seen[wv][r[k]] = base + (uint32_t)__popcll(peers);
            wave_lds_sync();
        }
        uint64_t c[kFinalK];
#pragma unroll
        for (uint32_t k = 0; k < kFinalK; k++) c[k] = valid[k] ? ctab[r[k]][at[k]] : 0;
#pragma unroll
        for (uint32_t k = 0; k < kFinalK; k++)
            if (valid[k]) {
                lab_cnt[a0 + i0 + k * 64 + lane] = c[k];
                sat += (c[k] == kSat);
            }
    }
    sat = wave_sum(sat);
    if (lane == 0 && sat) atomicAdd(nsat, (unsigned long long)sat);
}

inline uint32_t grid_for(uint64_t items, uint32_t per_block) {
    return (uint32_t)((items + per_block - 1) / per_block);
}
// grid of a grid-stride kernel over `items` (one per thread): a launch's
// work-item count must stay below 2^32
inline uint32_t grid_stride(uint64_t items) {
    uint64_t b = (items + kBlock - 1) / kBlock;
    return (uint32_t)(b < (1u << 20) ? (b ? b : 1) : (1u << 20));
}

inline int bit_width(uint64_t x) {
    int b = 0;
    while (x) {
        b++;
        x >>= 1;
    }
    return b;
}

// ---------------------------------------------------------------------------
// Host-side build state
// ---------------------------------------------------------------------------
constexpr uint64_t kMaxVertices = (1ull << 26) - 1024;
constexpr uint64_t kMaxAdjacency = (1ull << 32) - (1ull << 20);

// rounds that may insert at least this many entries grow in place (mapped
// address ranges); smaller ones are copied when they grow
constexpr uint64_t kVmmMinEntries = 1ull << 24;

struct Build {
    Arena arena;
    hipStream_t st;
    uint32_t N = 0;
    uint64_t NNZ = 0;
    uint32_t k = 1;
    // directed build: N = 2 nreal rows, out-labels then in-labels
    uint32_t nreal = 0;
    std::vector<uint32_t> vbase, gn;
    bool simple = false;  // the input was validated simple and symmetric
    uint32_t prop = 0;    // SPC_PROPAGATE_*
    // PUSH rounds: every puller's merged candidates as the segment of one
    // virtual neighbour (itself)
    uint64_t *vgoff = nullptr, *vpstart = nullptr;
    uint32_t *vgadj = nullptr, *vplen = nullptr;
    ShellResult shell;  // SPC_REDUCE_*: what was cut off, and the core ids
    bool reduced = false;
    uint32_t *hub_w = nullptr;  // neighbourhood equivalence: class size per rank
    uint32_t *adj_w = nullptr;  // and of the neighbour in every adjacency slot
    std::vector<uint32_t> obase, on;  // input vertex ranges when reduced
    // graph
    uint64_t *goff = nullptr;
    uint32_t *gadj = nullptr;
    uint32_t *rank_of = nullptr, *order = nullptr;
    // labels
    uint64_t *lab_off = nullptr, *lab_off2 = nullptr;
    void *lab_hd = nullptr, *lab_hd2 = nullptr;
    uint64_t lab_cap = 0, lab_cap2 = 0, entries = 0, entries_prev = 0;
    int db = 8;
    // rounds: entries (one allocation per round) and per-vertex segments
    std::vector<uint32_t *> rhub;
    std::vector<uint64_t *> rcnt;
    std::vector<uint64_t> rcap, rused;
    std::vector<uint64_t *> rstart;
    std::vector<uint32_t *> rlen;
    bool vmm = false;              // round arrays grow in place (virtual memory API)
    bool filter = true;            // membership filters for the prune probes
    bool filter_dense = true;      // 32 bits per entry where the memory allows
    uint64_t dev_bytes = 0;        // device memory size (bounds reservations)
    std::vector<std::unique_ptr<VArray>> vhub, vcnt;
    uint64_t **rs_tab = nullptr;  // device copies of the per-round pointers
    uint32_t **rl_tab = nullptr;
    uint32_t **hub_tab = nullptr;
    uint64_t **cnt_tab = nullptr;
    size_t tab_cap = 0;
    void *land = nullptr;         // landmark rows [N][kLand]
    uint32_t *lmask = nullptr;    // landmark masks [N][kMaskK][kLand / 32] (null: rows only)
    uint32_t *gbase = nullptr;    // per-rank graph base (batches only)
    uint32_t *lc = nullptr, *lc2 = nullptr;  // landmark prefix lengths of the two label buffers
    // per-round scratch
    uint64_t *raw = nullptr, *raw_off = nullptr, *soff = nullptr, *nlen = nullptr;
    uint32_t *surv = nullptr;
    uint32_t *cur = nullptr, *nxt = nullptr;  // per adjacency slot (round kernel cursors)
    uint32_t *tmp_hub = nullptr;
    uint64_t *tmp_cnt = nullptr;
    uint64_t tmp_cap = 0;
    uint64_t *ws = nullptr;
    unsigned long long *ctr = nullptr;
    uint64_t *h_pin = nullptr;  // pinned host scratch
    std::vector<RoundCounters> stats;
    double ms_round_kernel = 0;
    uint64_t alg_bytes = 0;
    uint64_t launches = 0;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;

    Build(uint64_t budget, hipStream_t s) : arena(budget, s), st(s) {}
    ~Build() {
        (void)hipStreamSynchronize(st);  // before the round arrays are unmapped
    }

    // record round r's segment arrays (host list + device pointer tables)
    spc_status add_round(uint64_t *rs, uint32_t *rl) {
        size_t r = rstart.size();
        if (r >= tab_cap) return SPC_ERR_DIST_RANGE;
        rstart.push_back(rs);
        rlen.push_back(rl);
        rhub.push_back(nullptr);
        rcnt.push_back(nullptr);
        vhub.emplace_back();
        vcnt.emplace_back();
        rcap.push_back(0);
        rused.push_back(0);
        SPC_HIP(hipMemcpyAsync(rs_tab + r, &rstart[r], sizeof(uint64_t *), hipMemcpyHostToDevice, st));
        SPC_HIP(hipMemcpyAsync(rl_tab + r, &rlen[r], sizeof(uint32_t *), hipMemcpyHostToDevice, st));
        SPC_HIP(hipStreamSynchronize(st));  // the host vectors may reallocate
        return SPC_OK;
    }
    // address space for round r's arrays, up to `max_entries` (in-place
    // growth only)
    spc_status reserve_round(size_t r, uint64_t max_entries) {
        if (!vmm || max_entries < kVmmMinEntries) return SPC_OK;  // small rounds copy cheaply
        uint64_t m = std::max<uint64_t>(std::min(max_entries, dev_bytes / sizeof(uint32_t)), 1);
        std::unique_ptr<VArray> h(new (std::nothrow) VArray()), c(new (std::nothrow) VArray());
        if (!h || !c) return SPC_ERR_OUT_OF_MEMORY;
        SPC_TRY(h->reserve(m * sizeof(uint32_t)));
        SPC_TRY(c->reserve(std::min<uint64_t>(m, dev_bytes / sizeof(uint64_t) + 1) * sizeof(uint64_t)));
        vhub[r] = std::move(h);
        vcnt[r] = std::move(c);
        rhub[r] = static_cast<uint32_t *>(vhub[r]->ptr());
        rcnt[r] = static_cast<uint64_t *>(vcnt[r]->ptr());
        rcap[r] = 0;
        SPC_HIP(hipMemcpyAsync(hub_tab + r, &rhub[r], sizeof(uint32_t *), hipMemcpyHostToDevice, st));
        SPC_HIP(hipMemcpyAsync(cnt_tab + r, &rcnt[r], sizeof(uint64_t *), hipMemcpyHostToDevice, st));
        SPC_HIP(hipStreamSynchronize(st));
        return SPC_OK;
    }
    // round r's entries from its mapped ranges into ordinary allocations
    spc_status demote_round(size_t r) {
        uint64_t n = std::max<uint64_t>(rused[r], 1);
        uint32_t *h = nullptr;
        uint64_t *c = nullptr;
        SPC_TRY(arena.alloc(&h, n));
        SPC_TRY(arena.alloc(&c, n));
        if (rused[r]) {
            SPC_HIP(hipMemcpyAsync(h, rhub[r], rused[r] * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
            SPC_HIP(hipMemcpyAsync(c, rcnt[r], rused[r] * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
        }
        SPC_HIP(hipStreamSynchronize(st));
        arena.uncharge(vhub[r]->mapped() + vcnt[r]->mapped());
        vhub[r].reset();
        vcnt[r].reset();
        rhub[r] = h;
        rcnt[r] = c;
        rcap[r] = n;
        SPC_HIP(hipMemcpyAsync(hub_tab + r, &rhub[r], sizeof(uint32_t *), hipMemcpyHostToDevice, st));
        SPC_HIP(hipMemcpyAsync(cnt_tab + r, &rcnt[r], sizeof(uint64_t *), hipMemcpyHostToDevice, st));
        SPC_HIP(hipStreamSynchronize(st));
        return SPC_OK;
    }
    // give back round r's hub array
    void release_round_hub(size_t r) {
        if (vhub[r]) {
            (void)hipStreamSynchronize(st);
            arena.uncharge(vhub[r]->mapped());
            vhub[r].reset();
            rhub[r] = nullptr;
        } else {
            arena.release(rhub[r]);
        }
    }
    // round r's arrays at exactly their used size
    spc_status shrink_round(size_t r) {
        if (vhub[r]) return SPC_OK;  // mapped in bounded pieces already
        uint64_t n = std::max<uint64_t>(rused[r], 1);
        uint32_t *h = nullptr;
        uint64_t *c = nullptr;
        SPC_TRY(arena.alloc(&h, n));
        SPC_TRY(arena.alloc(&c, n));
        if (rused[r]) {
            SPC_HIP(hipMemcpyAsync(h, rhub[r], rused[r] * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
            SPC_HIP(hipMemcpyAsync(c, rcnt[r], rused[r] * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
        }
        arena.release(rhub[r]);
        arena.release(rcnt[r]);
        rhub[r] = h;
        rcnt[r] = c;
        rcap[r] = n;
        SPC_HIP(hipMemcpyAsync(hub_tab + r, &rhub[r], sizeof(uint32_t *), hipMemcpyHostToDevice, st));
        SPC_HIP(hipMemcpyAsync(cnt_tab + r, &rcnt[r], sizeof(uint64_t *), hipMemcpyHostToDevice, st));
        SPC_HIP(hipStreamSynchronize(st));
        return SPC_OK;
    }
    // room for `need` entries in round r's arrays (kept entries are copied)
    spc_status grow_round(size_t r, uint64_t need) {
        if (need <= rcap[r]) return SPC_OK;
        if (vhub[r]) {
            size_t a = 0, b = 0;
            spc_status s = vhub[r]->ensure(need * sizeof(uint32_t), &a);
            SPC_TRY(arena.charge(a));
            if (s == SPC_OK) {
                s = vcnt[r]->ensure(need * sizeof(uint64_t), &b);
                SPC_TRY(arena.charge(b));
            }
            if (s == SPC_OK) {
                rcap[r] = std::min<uint64_t>(vhub[r]->mapped() / sizeof(uint32_t),
                                             vcnt[r]->mapped() / sizeof(uint64_t));
                return SPC_OK;
            }
            if (s != SPC_ERR_DEVICE) return s;
            // the runtime refused a mapping: move the round into ordinary
            // allocations and grow by copying from here on
            SPC_TRY(demote_round(r));
            vmm = false;
        }
        uint64_t nc = need;
        uint64_t c1 = rcap[r], c2 = rcap[r];
        SPC_TRY(grow(&rhub[r], &c1, nc, rused[r]));
        SPC_TRY(grow(&rcnt[r], &c2, nc, rused[r]));
        rcap[r] = std::min(c1, c2);
        SPC_HIP(hipMemcpyAsync(hub_tab + r, &rhub[r], sizeof(uint32_t *), hipMemcpyHostToDevice, st));
        SPC_HIP(hipMemcpyAsync(cnt_tab + r, &rcnt[r], sizeof(uint64_t *), hipMemcpyHostToDevice, st));
        SPC_HIP(hipStreamSynchronize(st));
        return SPC_OK;
    }

    spc_status read_u64(const uint64_t *dev, uint64_t *out, size_t count = 1) {
        SPC_HIP(hipMemcpyAsync(h_pin, dev, count * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
        SPC_HIP(hipStreamSynchronize(st));
        std::memcpy(out, h_pin, count * sizeof(uint64_t));
        return SPC_OK;
    }

    template <typename T>
    spc_status grow(T **p, uint64_t *cap, uint64_t need, uint64_t keep) {
        if (need <= *cap) return SPC_OK;
        uint64_t nc = std::max<uint64_t>(need, *cap + *cap / 2);
        T *q = nullptr;
        spc_status s = arena.alloc(&q, nc);
        if (s != SPC_OK && nc > need) {
            nc = need;
            s = arena.alloc(&q, nc);
        }
        SPC_TRY(s);
        if (keep && *p) SPC_HIP(hipMemcpyAsync(q, *p, keep * sizeof(T), hipMemcpyDeviceToDevice, st));
        if (*p) {
            SPC_HIP(hipStreamSynchronize(st));
            arena.release(*p);
        }
        *p = q;
        *cap = nc;
        return SPC_OK;
    }
};

// out[rank_of[v]] = in[v]
__global__ void k_to_rank(uint32_t N, const uint32_t *rank_of, const uint32_t *in, uint32_t *out) {
    uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < N) out[rank_of[v]] = in[v];
}
// weight of the neighbour in every adjacency slot (rank space)
__global__ void k_adj_weights(const uint32_t *adj, uint64_t nnz, const uint32_t *w, uint32_t *out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += stride) out[i] = w[adj[i]];
}

// simple + symmetric check of a CSR; sorts each row of adj in place
spc_status validate_csr(Build &B, const uint64_t *off, uint32_t *adj, uint32_t N, uint64_t NNZ,
                        uint32_t *err, bool directed = false) {
    if (!NNZ) return SPC_OK;
    int xb = std::max(1, bit_width(N));
    uint64_t *keys = nullptr, *keys2 = nullptr;
    SPC_TRY(B.arena.alloc(&keys, NNZ));
    SPC_TRY(B.arena.alloc(&keys2, NNZ));
    uint64_t *rws = nullptr;
    SPC_TRY(B.arena.alloc(&rws, radix_ws_elems(NNZ)));
    hipLaunchKernelGGL(k_row_keys, dim3(grid_for(N, kWaves)), dim3(kBlock), 0, B.st, off, adj, N, xb,
                       keys);
    SPC_LAUNCHED();
    SPC_TRY(radix_sort_pairs(keys, nullptr, keys2, nullptr, NNZ, 2 * xb, rws, B.st));
    hipLaunchKernelGGL(k_keys_to_adj, dim3(grid_for(NNZ, kBlock)), dim3(kBlock), 0, B.st, keys, NNZ, xb,
                       adj);
    SPC_LAUNCHED();
    SPC_HIP(hipMemsetAsync(err, 0, sizeof(uint32_t), B.st));
    hipLaunchKernelGGL(k_check_adj, dim3(grid_for(N, kWaves)), dim3(kBlock), 0, B.st, off, adj, N, err,
                       directed ? 1 : 0);
    SPC_LAUNCHED();
    uint64_t ev[1];
    SPC_TRY(B.read_u64((const uint64_t *)err, ev));
    B.arena.release(keys);
    B.arena.release(keys2);
    B.arena.release(rws);
    if ((uint32_t)ev[0] != 0) return SPC_ERR_INVALID_ARG;
    return SPC_OK;
}

// union CSR (+ 1-shell reduction) + ordering + relabel (+ validation)
spc_status preprocess(Build &B, const spc_graph *gs, bool use_order, bool use_tie, bool validate,
                      uint32_t reduce) {
    B.simple = validate;  // checked below, or the build fails
    uint32_t N = B.N;
    uint64_t NNZ = B.NNZ;
    uint64_t *off = nullptr;
    uint32_t *col = nullptr, *deg = nullptr, *err = nullptr, *vb_dev = nullptr;
    SPC_TRY(B.arena.alloc(&off, (uint64_t)N + 1));
    SPC_TRY(B.arena.alloc(&col, NNZ));
    SPC_TRY(B.arena.alloc(&deg, (uint64_t)N + 1));
    SPC_TRY(B.arena.alloc(&err, 2));
    SPC_TRY(B.arena.alloc(&vb_dev, (uint64_t)B.k + 1));
    SPC_HIP(hipMemsetAsync(err, 0, 2 * sizeof(uint32_t), B.st));
    SPC_HIP(hipMemcpyAsync(vb_dev, B.vbase.data(), B.k * sizeof(uint32_t), hipMemcpyHostToDevice, B.st));

    // staging for host inputs
    uint64_t max_n1 = 0, max_nnz = 0;
    for (uint32_t g = 0; g < B.k; g++) {
        max_n1 = std::max<uint64_t>(max_n1, (uint64_t)gs[g].n + 1);
        max_nnz = std::max<uint64_t>(max_nnz, gs[g].nnz);
    }
    uint64_t *st_off = nullptr;
    uint32_t *st_col = nullptr;
    uint64_t *st_tie = nullptr;
    uint32_t *st_ord = nullptr;
    bool host_in = !gs[0].on_device;
    if (host_in) {
        SPC_TRY(B.arena.alloc(&st_off, max_n1));
        SPC_TRY(B.arena.alloc(&st_col, std::max<uint64_t>(max_nnz, 1)));
        if (use_order) SPC_TRY(B.arena.alloc(&st_ord, max_n1));
    }
    uint64_t *tie_union = nullptr;
    if (use_tie) SPC_TRY(B.arena.alloc(&tie_union, (uint64_t)N + 1));
    uint32_t *ord_union = nullptr, *hits = nullptr;
    if (use_order) {
        SPC_TRY(B.arena.alloc(&ord_union, (uint64_t)N + 1));
        SPC_TRY(B.arena.alloc(&hits, (uint64_t)N + 1));
        SPC_HIP(hipMemsetAsync(hits, 0, ((uint64_t)N + 1) * sizeof(uint32_t), B.st));
    }

    uint64_t ebase = 0;
    for (uint32_t g = 0; g < B.k; g++) {
        const spc_graph &G = gs[g];
        const uint64_t *src_off = G.row_off;
        const uint32_t *src_col = G.col;
        const uint32_t *src_ord = G.order;
        if (host_in) {
            SPC_HIP(hipMemcpyAsync(st_off, G.row_off, ((uint64_t)G.n + 1) * sizeof(uint64_t),
                                   hipMemcpyHostToDevice, B.st));
            if (G.nnz)
                SPC_HIP(hipMemcpyAsync(st_col, G.col, G.nnz * sizeof(uint32_t), hipMemcpyHostToDevice,
                                       B.st));
            if (use_order && G.n)
                SPC_HIP(hipMemcpyAsync(st_ord, G.order, (uint64_t)G.n * sizeof(uint32_t),
                                       hipMemcpyHostToDevice, B.st));
            src_off = st_off;
            src_col = st_col;
            src_ord = st_ord;
        }
        hipLaunchKernelGGL(k_union_off, dim3(grid_for((uint64_t)G.n + 1, kBlock)), dim3(kBlock), 0,
                           B.st, src_off, off + B.vbase[g], G.n, G.nnz, ebase, err);
        SPC_LAUNCHED();
        if (G.nnz) {
            hipLaunchKernelGGL(k_union_col, dim3(grid_for(G.nnz, kBlock)), dim3(kBlock), 0, B.st,
                               src_col, col + ebase, G.nnz, G.n, B.vbase[g], err);
            SPC_LAUNCHED();
        }
        if (use_order && G.n) {
            hipLaunchKernelGGL(k_union_order, dim3(grid_for(G.n, kBlock)), dim3(kBlock), 0, B.st,
                               src_ord, ord_union, G.n, B.vbase[g], hits, err);
            SPC_LAUNCHED();
        }
        if (use_tie && G.n)
            SPC_HIP(hipMemcpyAsync(tie_union + B.vbase[g], G.tie_key, (uint64_t)G.n * sizeof(uint64_t),
                                   G.on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                   B.st));
        if (host_in) SPC_HIP(hipStreamSynchronize(B.st));  // staging is reused
        ebase += G.nnz;
    }
    if (use_order) {
        hipLaunchKernelGGL(k_check_perm, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, B.st, hits, N,
                           err);
        SPC_LAUNCHED();
    }
    uint64_t e2[1];
    SPC_TRY(B.read_u64((const uint64_t *)err, e2));
    if ((uint32_t)e2[0] != 0) return SPC_ERR_INVALID_ARG;
    B.arena.release(st_off);
    B.arena.release(st_col);
    B.arena.release(st_ord);

    if (reduce) {
        // Sections "Reduction by 1-Shell" and "Reduction by Equivalence
        // Relation": the rest of the build sees the core only.  The input is
        // checked first: both reductions assume a simple symmetric graph.
        const bool sorted = validate && NNZ;  // validation sorts every row
        if (validate) SPC_TRY(validate_csr(B, off, col, N, NNZ, err));
        validate = false;  // the core of a valid graph is valid
        ShellResult &R = B.shell;
        if (reduce & SPC_REDUCE_ONE_SHELL)
            SPC_TRY(one_shell(B.arena, B.st, B.ws, N, NNZ, off, col, ord_union, tie_union, B.vbase, &R));
        else
            SPC_TRY(twin_reduce(B.arena, B.st, B.ws, N, NNZ, off, col, sorted, ord_union, tie_union,
                                B.vbase, &R));
        B.arena.release(off);
        B.arena.release(col);
        B.arena.release(ord_union);
        B.arena.release(tie_union);
        off = R.off;
        col = R.col;
        ord_union = R.ord;
        tie_union = R.tie;
        R.off = nullptr;
        R.col = nullptr;
        R.ord = nullptr;
        R.tie = nullptr;
        B.reduced = true;
        B.obase = B.vbase;
        B.on = B.gn;
        B.vbase = R.cbase;
        for (uint32_t g = 0; g < B.k; g++) B.gn[g] = B.vbase[g + 1] - B.vbase[g];
        B.N = N = R.N;
        B.NNZ = NNZ = R.NNZ;
        SPC_HIP(hipMemcpyAsync(vb_dev, B.vbase.data(), B.k * sizeof(uint32_t), hipMemcpyHostToDevice,
                               B.st));
    }

    // degrees and order
    uint32_t *maxdeg = err + 1;
    hipLaunchKernelGGL(k_degrees, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, B.st, off, N, deg,
                       maxdeg);
    SPC_LAUNCHED();
    SPC_TRY(B.arena.alloc(&B.order, (uint64_t)N + 1));
    SPC_TRY(B.arena.alloc(&B.rank_of, (uint64_t)N + 1));
    if (use_order) {
        SPC_HIP(hipMemcpyAsync(B.order, ord_union, (uint64_t)N * sizeof(uint32_t),
                               hipMemcpyDeviceToDevice, B.st));
    } else {
        uint64_t md[1];
        SPC_TRY(B.read_u64((const uint64_t *)err, md));
        uint32_t maxd = (uint32_t)(md[0] >> 32);
        uint64_t *keys = nullptr, *keys2 = nullptr;
        uint32_t *vals2 = nullptr;
        SPC_TRY(B.arena.alloc(&keys, (uint64_t)N + 1));
        SPC_TRY(B.arena.alloc(&keys2, (uint64_t)N + 1));
        SPC_TRY(B.arena.alloc(&vals2, (uint64_t)N + 1));
        hipLaunchKernelGGL(k_iota_keys, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, B.st,
                           (const uint64_t *)tie_union, N, keys, B.order);
        SPC_LAUNCHED();
        if (use_tie) SPC_TRY(radix_sort_pairs(keys, B.order, keys2, vals2, N, 64, B.ws, B.st));
        int degbits = std::max(1, bit_width(maxd));
        hipLaunchKernelGGL(k_degree_keys, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, B.st, B.order,
                           deg, N, maxd, degbits, vb_dev, B.k, keys);
        SPC_LAUNCHED();
        int gbits = B.k > 1 ? bit_width(B.k - 1) : 0;
        SPC_TRY(radix_sort_pairs(keys, B.order, keys2, vals2, N, degbits + gbits, B.ws, B.st));
        B.arena.release(keys);
        B.arena.release(keys2);
        B.arena.release(vals2);
    }
    B.arena.release(tie_union);
    B.arena.release(ord_union);
    B.arena.release(hits);

    // rank space CSR
    uint32_t *rdeg = nullptr;
    SPC_TRY(B.arena.alloc(&rdeg, (uint64_t)N + 1));
    hipLaunchKernelGGL(k_rank_of, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, B.st, B.order, N, deg,
                       B.rank_of, rdeg);
    SPC_LAUNCHED();
    if (B.shell.weight) {  // class sizes into rank space
        SPC_TRY(B.arena.alloc(&B.hub_w, (uint64_t)N + 1));
        hipLaunchKernelGGL(k_to_rank, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, B.st, N, B.rank_of,
                           B.shell.weight, B.hub_w);
        SPC_LAUNCHED();
        B.arena.release(B.shell.weight);
    }
    SPC_TRY(B.arena.alloc(&B.goff, (uint64_t)N + 1));
    SPC_TRY(B.arena.alloc(&B.gadj, std::max<uint64_t>(NNZ, 1)));
    SPC_TRY(scan_u32(rdeg, B.goff, N, B.ws, B.st));
    hipLaunchKernelGGL(k_relabel, dim3(grid_for(N, kWaves)), dim3(kBlock), 0, B.st, B.order,
                       B.rank_of, off, col, B.goff, B.gadj, N);
    SPC_LAUNCHED();
    B.arena.release(rdeg);
    B.arena.release(off);
    B.arena.release(col);
    B.arena.release(deg);

    if (validate) SPC_TRY(validate_csr(B, B.goff, B.gadj, N, NNZ, err));
    if (B.hub_w) {  // after validation, which reorders rows
        SPC_TRY(B.arena.alloc(&B.adj_w, std::max<uint64_t>(NNZ, 1)));
        if (NNZ) {
            hipLaunchKernelGGL(k_adj_weights, dim3(grid_stride(NNZ)), dim3(kBlock), 0, B.st, B.gadj, NNZ,
                               B.hub_w, B.adj_w);
            SPC_LAUNCHED();
        }
    }
    B.arena.release(err);
    B.arena.release(vb_dev);
    return SPC_OK;
}

// Pulled entries per batch (temp buffer entries): at least kRawBatchMax,
// at most kTempMaxEntries (the small-table test build takes tiny ones, so
// small graphs run many batches per round).
#ifndef SPC_TEMP_LOG2
#define SPC_TEMP_LOG2 27
#endif
#ifndef SPC_TEMP_MAX_LOG2
#define SPC_TEMP_MAX_LOG2 30
#endif
constexpr uint64_t kRawBatchMax = 1ull << SPC_TEMP_LOG2;
constexpr uint64_t kTempMaxEntries = 1ull << SPC_TEMP_MAX_LOG2;
// pullers per round-kernel launch (one workgroup each: the launch's
// work-item count stays below 2^32)
constexpr uint32_t kBatchVerts = 1u << 22;
constexpr uint32_t kMergeRound = 16;

// Round 1 of a simple graph: round 0 holds only self entries, so L_1(u) is
// every neighbour ranked above u with count 1 -- nothing is held, merged or
// pruned.  Each puller's neighbours above it are written as (puller, hub)
// keys into its segment of the round kernel's output layout; a radix sort
// then orders every segment by hub.
__global__ __launch_bounds__(kBlock) void k_round1_keys(uint32_t u_lo, uint32_t u_hi, const uint64_t *goff,
                                                         const uint32_t *gadj, const uint64_t *raw_off,
                                                         uint64_t *keys, uint32_t *surv) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t nw = gridDim.x * kWaves;
    for (uint32_t u = u_lo + blockIdx.x * kWaves + (threadIdx.x >> 6); u < u_hi; u += nw) {
        uint64_t out = raw_off[u] - raw_off[u_lo];
        const uint64_t e = goff[u + 1];
        for (uint64_t k0 = goff[u]; k0 < e; k0 += 64) {
            const uint64_t k = k0 + lane;
            const uint32_t v = k < e ? gadj[k] : 0xFFFFFFFFu;
            const bool keep = v < u;
            const uint64_t m = __ballot(keep);
            if (keep) keys[out + (uint64_t)__popcll(m & lanemask_lt())] = ((uint64_t)(u - u_lo) << 32) | v;
            out += (uint64_t)__popcll(m);
        }
        if (lane == 0) surv[u] = (uint32_t)(raw_off[u + 1] - raw_off[u]);
    }
}
// PUSH propagation (Alg. 1): every pusher v scatters the entries of its
// round d-1 segment whose hub lies below a neighbour u to u, for the pullers
// u of the batch [u_lo, u_hi); one wave per pusher, one lane per neighbour.
// A puller's slots start at its raw offset: it receives exactly the entries
// the pull would read.  Counts are multiplied by the pusher's weight (vw,
// neighbourhood equivalence), which lies inside every path it extends.
__global__ __launch_bounds__(kBlock) void k_push_scatter(uint32_t N, uint32_t u_lo, uint32_t u_hi,
                                                          const uint64_t *goff, const uint32_t *gadj,
                                                          const uint64_t *pstart, const uint32_t *plen,
                                                          const uint32_t *pool_hub, const uint64_t *pool_cnt,
                                                          const uint32_t *vw, const uint64_t *raw_off,
                                                          uint32_t *cursor, uint64_t *keys, uint64_t *cnt) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t nw = gridDim.x * kWaves;
    for (uint32_t v = blockIdx.x * kWaves + (threadIdx.x >> 6); v < N; v += nw) {
        const uint32_t ln = plen[v];
        if (!ln) continue;
        const uint64_t ps = pstart[v];
        const uint64_t f = vw ? vw[v] : 1;
        for (uint64_t k = goff[v] + lane; k < goff[v + 1]; k += 64) {
            const uint32_t u = gadj[k];
            if (u < u_lo || u >= u_hi) continue;
            const uint32_t p = (v < u) ? ln : lower_bound_u32(pool_hub + ps, ln, u);
            if (!p) continue;
            const uint32_t pos = atomicAdd(&cursor[u - u_lo], p);
            // u's slots end at its next raw offset (a symmetric graph fills
            // them exactly; the bound only guards the writes)
            const uint64_t lim = raw_off[u + 1] - raw_off[u_lo];
            const uint32_t q = pos >= lim ? 0u : (uint32_t)std::min<uint64_t>(p, lim - pos);
            for (uint32_t j = 0; j < q; j++) {
                keys[pos + j] = ((uint64_t)(u - u_lo) << 32) | pool_hub[ps + j];
                cnt[pos + j] = sat_mul(pool_cnt[ps + j], f);
            }
        }
    }
}
__global__ void k_push_cursor(uint32_t u_lo, uint32_t n, const uint64_t *raw_off, uint32_t *cursor,
                              uint32_t *idx, uint64_t need) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < need || i < n; i += stride) {
        if (i < n) cursor[i] = (uint32_t)(raw_off[u_lo + i] - raw_off[u_lo]);
        if (i < need) idx[i] = (uint32_t)i;
    }
}
__global__ void k_push_heads(const uint64_t *keys, uint64_t n, uint32_t *head) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}
// Label Merging of the sorted pushes: one entry per (puller, hub), its
// counts summed
__global__ void k_push_unique(const uint64_t *keys, const uint32_t *idx, const uint64_t *cnt,
                              const uint32_t *head, const uint64_t *hpos, uint64_t n, uint32_t *uhub,
                              uint64_t *ucnt) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (!head[i]) continue;
        uint64_t sum = cnt[idx[i]];
        for (uint64_t j = i + 1; j < n && !head[j]; j++) sum = sat_add(sum, cnt[idx[j]]);
        uhub[hpos[i]] = (uint32_t)keys[i];
        ucnt[hpos[i]] = sum;
    }
}
// each puller's merged candidates as the segment of one virtual neighbour
// (itself)
__global__ void k_push_segs(uint32_t u_lo, uint32_t u_hi, const uint64_t *raw_off, const uint64_t *hpos,
                            uint64_t *vpstart, uint32_t *vplen) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t u = u_lo + blockIdx.x * blockDim.x + threadIdx.x; u < u_hi; u += stride) {
        const uint64_t t0 = raw_off[u] - raw_off[u_lo], t1 = raw_off[u + 1] - raw_off[u_lo];
        vpstart[u] = hpos[t0];
        vplen[u] = (uint32_t)(hpos[t1] - hpos[t0]);
    }
}
__global__ void k_iota_adj(uint32_t N, uint64_t *off, uint32_t *adj) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v <= N; v += stride) {
        off[v] = v;
        if (v < N) adj[v] = v;
    }
}

// sorted keys -> hubs and unit counts (the keys live in the count array)
__global__ void k_round1_out(uint64_t n, uint32_t *hub, uint64_t *cnt) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t key = cnt[i];
        hub[i] = (uint32_t)key;
        cnt[i] = 1;
    }
}

// One distance round d >= 1.  Returns the number of entries it inserted.
template <int DB>
spc_status run_round(Build &B, uint32_t d, uint64_t *kept_out, bool *any_cand) {
    using E = typename Ent<DB>::T;
    const uint32_t N = B.N;
    const uint64_t *pstart = B.rstart[d - 1];
    const uint32_t *plen = B.rlen[d - 1];
    using LT = typename Land<DB>::T;
    B.arena.begin_window();
    hipLaunchKernelGGL(k_expand_count, dim3(grid_for(N, kWaves)), dim3(kBlock), 0, B.st, N, B.nreal, B.goff,
                       B.gadj, pstart, plen, B.rhub[d - 1], B.raw);
    SPC_LAUNCHED();
    SPC_TRY(scan_u64(B.raw, B.raw_off, N, B.ws, B.st));
    uint64_t total_raw;
    SPC_TRY(B.read_u64(B.raw_off + N, &total_raw));
    *any_cand = total_raw > 0;
    *kept_out = 0;
    if (total_raw == 0) return SPC_OK;

    uint64_t *rs = nullptr;
    uint32_t *rl = nullptr;
    SPC_TRY(B.arena.alloc(&rs, (uint64_t)N + 1));
    SPC_TRY(B.arena.alloc(&rl, (uint64_t)N + 1));
    SPC_TRY(B.add_round(rs, rl));
    SPC_TRY(B.reserve_round(d, total_raw));  // survivors are a subset of the pulls
    SPC_HIP(hipMemsetAsync(B.ctr, 0, 8 * sizeof(unsigned long long), B.st));

    uint64_t kept = 0, fast_raw = 0;
    double round_ms = 0;
    const bool fast1 = d == 1 && B.simple;
    // PUSH (Alg. 1) every round from 2 on, or where the pushes are fewer than
    // the adjacency slots the pull would walk (SPC_PROPAGATE_AUTO)
    // (validated input only: the pushes fill exactly the pull's slots when
    // the graph is symmetric)
    const bool push = d >= 2 && B.simple &&
                      (B.prop == SPC_PROPAGATE_PUSH || (B.prop == SPC_PROPAGATE_AUTO && total_raw < B.NNZ));
    // Batches of pullers whose pulled entries fit the temp buffer (a
    // puller's survivors are a subset of its pulls, written at its pull
    // offset).  The buffer takes up to a sixth of the memory the build has
    // left (2^27 .. 2^30 entries): the more pullers a launch holds, the
    // better the dispatcher balances their very uneven work.  PUSH rounds
    // keep 2^27 (their scratch per pulled entry is larger).
    uint64_t tmp_want = kRawBatchMax;
    if (!push) {
        const uint64_t cap_bytes = B.arena.budget() ? B.arena.budget() : B.dev_bytes;
        const uint64_t left = cap_bytes > B.arena.used() ? cap_bytes - B.arena.used() : 0;
        tmp_want = std::min<uint64_t>(std::max<uint64_t>(left / 6 / 12, kRawBatchMax), kTempMaxEntries);
    }
    tmp_want = std::min<uint64_t>(tmp_want, std::max<uint64_t>(total_raw, 1024));
    if (tmp_want > B.tmp_cap) {
        B.arena.release(B.tmp_hub);
        B.arena.release(B.tmp_cnt);
        B.tmp_cap = 0;
        SPC_TRY(B.arena.alloc(&B.tmp_hub, tmp_want));
        SPC_TRY(B.arena.alloc(&B.tmp_cnt, tmp_want));
        B.tmp_cap = tmp_want;
    }
    // Membership filter of L_{<=d-2}'s (row, hub, distance) triples for the prune probes
    // (32 or else 16 bits per entry, 1/8 of the memory left at most, row
    // words indexed in 32 bits), where inserting the older labels costs less
    // than a quarter of the round's pulls
    unsigned long long *filt = nullptr;
    uint64_t filt_words = 0;
    uint32_t filt_shift = kFiltShiftHi;
    if (B.filter && d >= 3 && !push && !fast1 && B.entries_prev > 0 && B.entries_prev * 4 <= total_raw) {
        const uint64_t cap_bytes = B.arena.budget() ? B.arena.budget() : B.dev_bytes;
        const uint64_t left = cap_bytes > B.arena.used() ? cap_bytes - B.arena.used() : 0;
        auto words_at = [&](uint32_t sh) { return (B.entries_prev + (1ull << sh) - 1) >> sh; };
        auto fits = [&](uint32_t sh) { return words_at(sh) < (1ull << 32) && words_at(sh) * 8 <= left / 8; };
        filt_shift = B.filter_dense && fits(kFiltShiftLo) ? kFiltShiftLo : kFiltShiftHi;
        const uint64_t words = words_at(filt_shift);
        if (fits(filt_shift) && B.arena.alloc(&filt, words) == SPC_OK) {
            filt_words = words;
            hipLaunchKernelGGL(k_filt_clear, dim3(grid_stride(words)), dim3(kBlock), 0, B.st, filt, words);
            SPC_LAUNCHED();
            hipLaunchKernelGGL(k_filt_insert<DB>, dim3(grid_for(N, kWaves)), dim3(kBlock), 0, B.st, N,
                               B.lab_off2, B.lab_hd2, B.lc2, filt, words, filt_shift);
            SPC_LAUNCHED();
        } else {
            filt = nullptr;
        }
    }
    std::vector<uint32_t> bounds{0};
    std::vector<uint64_t> ro;  // raw_off on the host (several batches)
    if (total_raw <= B.tmp_cap && N <= kBatchVerts) {
        bounds.push_back(N);
    } else {
        ro.resize((size_t)N + 1);
        SPC_HIP(hipMemcpyAsync(ro.data(), B.raw_off, ((size_t)N + 1) * sizeof(uint64_t),
                               hipMemcpyDeviceToHost, B.st));
        SPC_HIP(hipStreamSynchronize(B.st));
        uint32_t b0 = 0;
        while (b0 < N) {
            uint64_t lim = ro[b0] + B.tmp_cap;
            uint32_t b1 = (uint32_t)(std::upper_bound(ro.begin() + b0 + 1, ro.end(), lim) - ro.begin()) - 1;
            if (b1 <= b0) b1 = b0 + 1;  // one puller pulling more than the buffer: a buffer of its own
            if (b1 - b0 > kBatchVerts) b1 = b0 + kBatchVerts;
            bounds.push_back(b1);
            b0 = b1;
        }
    }
    uint64_t raw_lo = 0;  // pull offset of the current batch's first puller

    if (push && !B.vgoff) {
        SPC_TRY(B.arena.alloc(&B.vgoff, (uint64_t)N + 1));
        SPC_TRY(B.arena.alloc(&B.vgadj, (uint64_t)N + 1));
        SPC_TRY(B.arena.alloc(&B.vpstart, (uint64_t)N + 1));
        SPC_TRY(B.arena.alloc(&B.vplen, (uint64_t)N + 1));
        hipLaunchKernelGGL(k_iota_adj, dim3(grid_stride((uint64_t)N + 1)), dim3(kBlock), 0, B.st, N, B.vgoff,
                           B.vgadj);
        SPC_LAUNCHED();
    }
    for (size_t bi = 0; bi + 1 < bounds.size(); bi++) {
        const uint32_t b0 = bounds[bi], b1 = bounds[bi + 1];
        // pulled entries of the batch (raw_off[N] = total_raw)
        const uint64_t need = (ro.empty() ? total_raw : ro[b1]) - raw_lo;
        if (need > B.tmp_cap) {  // a single puller pulling more than the buffer holds
            B.arena.release(B.tmp_hub);
            B.arena.release(B.tmp_cnt);
            B.tmp_cap = 0;
            SPC_TRY(B.arena.alloc(&B.tmp_hub, need));
            SPC_TRY(B.arena.alloc(&B.tmp_cnt, need));
            B.tmp_cap = need;
        }
        // PUSH: scatter, sort by (puller, hub), merge equal hubs
        uint64_t *pkeys = nullptr, *pkeys2 = nullptr, *pcnt = nullptr, *phpos = nullptr, *pws = nullptr,
                 *pucnt = nullptr;
        uint32_t *pidx = nullptr, *pidx2 = nullptr, *phead = nullptr, *pcur = nullptr, *puhub = nullptr;
        if (push) {
            const uint64_t n1 = std::max<uint64_t>(need, 1);
            SPC_TRY(B.arena.alloc(&pkeys, n1));
            SPC_TRY(B.arena.alloc(&pkeys2, n1));
            SPC_TRY(B.arena.alloc(&pcnt, n1));
            SPC_TRY(B.arena.alloc(&pidx, n1));
            SPC_TRY(B.arena.alloc(&pidx2, n1));
            SPC_TRY(B.arena.alloc(&phead, n1));
            SPC_TRY(B.arena.alloc(&phpos, n1 + 1));
            SPC_TRY(B.arena.alloc(&puhub, n1));
            SPC_TRY(B.arena.alloc(&pucnt, n1));
            SPC_TRY(B.arena.alloc(&pcur, (uint64_t)(b1 - b0) + 1));
            SPC_TRY(B.arena.alloc(&pws, std::max(radix_ws_elems(n1), scan_ws_elems(n1 + 1))));
            hipLaunchKernelGGL(k_push_cursor, dim3(grid_stride(std::max<uint64_t>(need, b1 - b0))), dim3(kBlock),
                               0, B.st, b0, b1 - b0, B.raw_off, pcur, pidx, need);
            SPC_LAUNCHED();
            hipLaunchKernelGGL(k_push_scatter, dim3(grid_for(N, kWaves)), dim3(kBlock), 0, B.st, N, b0, b1,
                               B.goff, B.gadj, pstart, plen, B.rhub[d - 1], B.rcnt[d - 1], B.hub_w, B.raw_off,
                               pcur, pkeys, pcnt);
            SPC_LAUNCHED();
            if (need) {
                SPC_TRY(radix_sort_pairs(pkeys, pidx, pkeys2, pidx2, need, 32 + std::max(1, bit_width(b1 - b0)),
                                         pws, B.st));
                hipLaunchKernelGGL(k_push_heads, dim3(grid_stride(need)), dim3(kBlock), 0, B.st, pkeys, need,
                                   phead);
                SPC_LAUNCHED();
                SPC_TRY(scan_u32(phead, phpos, need, pws, B.st));
                hipLaunchKernelGGL(k_push_unique, dim3(grid_stride(need)), dim3(kBlock), 0, B.st, pkeys, pidx,
                                   pcnt, phead, phpos, need, puhub, pucnt);
                SPC_LAUNCHED();
            } else {
                SPC_HIP(hipMemsetAsync(phpos, 0, sizeof(uint64_t), B.st));
            }
            hipLaunchKernelGGL(k_push_segs, dim3(grid_stride(b1 - b0)), dim3(kBlock), 0, B.st, b0, b1, B.raw_off,
                               phpos, B.vpstart, B.vplen);
            SPC_LAUNCHED();
        }
        RoundArgs ra;
        ra.d = d;
        ra.u_lo = b0;
        ra.u_hi = b1;
        ra.nreal = B.nreal;
        ra.goff = B.goff;
        ra.gadj = B.gadj;
        ra.lab_off = B.lab_off;
        ra.lab_hd = B.lab_hd;
        ra.prev_off = B.lab_off2;
        ra.prev_hd = B.lab_hd2;
        ra.lc_cur = B.lc;
        ra.lc_prev = B.lc2;
        ra.land = B.land;
        ra.lmask = reinterpret_cast<const uint4 *>(B.lmask);
        ra.gbase = B.gbase;
        ra.pstart = pstart;
        ra.plen = plen;
        ra.pool_hub = B.rhub[d - 1];
        ra.pool_cnt = B.rcnt[d - 1];
        // vertex weights (neighbourhood equivalence): from round 2 on, a
        // pulled entry (w, d-1) of v extends paths that pass through v
        ra.adj_w = B.adj_w;
        if (push) {  // the pushes, merged, arrive through one virtual neighbour
            ra.goff = B.vgoff;
            ra.gadj = B.vgadj;
            ra.pstart = B.vpstart;
            ra.plen = B.vplen;
            ra.pool_hub = puhub;
            ra.pool_cnt = pucnt;
        }
        ra.raw_off = B.raw_off;
        ra.tmp_hub = B.tmp_hub;
        ra.tmp_cnt = B.tmp_cnt;
        ra.surv = B.surv;
        ra.cur = B.cur;
        ra.nxt = B.nxt;
        ra.ctr = B.ctr;
        ra.filt = filt;
        ra.filt_words = filt_words;
        ra.filt_shift = filt_shift;
        SPC_HIP(hipEventRecord(B.ev_a, B.st));
        // from round 17 on the graph has a long diameter: there, neighbours'
        // labels are nearly the same set, which the tail merge exploits
        const bool weighted = B.adj_w && d >= 2 && !push;  // pushes carry their weights
        const dim3 grid(b1 - b0), blk(kRoundBlock);
        if (fast1) {
            // the keys are built in the count array, sorted there, then
            // split into hubs and unit counts
            uint64_t *keys2 = nullptr, *rws = nullptr;
            SPC_TRY(B.arena.alloc(&keys2, std::max<uint64_t>(need, 1)));
            SPC_TRY(B.arena.alloc(&rws, radix_ws_elems(std::max<uint64_t>(need, 1))));
            hipLaunchKernelGGL(k_round1_keys, dim3(grid_for(b1 - b0, kWaves)), dim3(kBlock), 0, B.st, b0, b1,
                               B.goff, B.gadj, B.raw_off, B.tmp_cnt, B.surv);
            SPC_LAUNCHED();
            if (need) {
                SPC_TRY(radix_sort_pairs(B.tmp_cnt, nullptr, keys2, nullptr, need,
                                         32 + std::max(1, bit_width(b1 - b0)), rws, B.st));
                hipLaunchKernelGGL(k_round1_out, dim3(grid_stride(need)), dim3(kBlock), 0, B.st, need,
                                   B.tmp_hub, B.tmp_cnt);
                SPC_LAUNCHED();
            }
            B.arena.release(keys2);
            B.arena.release(rws);
            fast_raw += need;
        } else if (d > kMergeRound) {
            if (weighted)
                k_round<DB, kRoundBlock, true, true><<<grid, blk, 0, B.st>>>(ra);
            else
                k_round<DB, kRoundBlock, true, false><<<grid, blk, 0, B.st>>>(ra);
        } else {
            if (weighted)
                k_round<DB, kRoundBlock, false, true><<<grid, blk, 0, B.st>>>(ra);
            else
                k_round<DB, kRoundBlock, false, false><<<grid, blk, 0, B.st>>>(ra);
        }
        SPC_LAUNCHED();
        if (!fast1) B.launches++;
        SPC_HIP(hipEventRecord(B.ev_b, B.st));
        if (push) {
            for (uint64_t *q : {pkeys, pkeys2, pcnt, phpos, pws, pucnt}) B.arena.release(q);
            for (uint32_t *q : {pidx, pidx2, phead, pcur, puhub}) B.arena.release(q);
        }
        SPC_TRY(scan_u32(B.surv + b0, B.soff, b1 - b0, B.ws, B.st));
        uint64_t sb;
        SPC_TRY(B.read_u64(B.soff + (b1 - b0), &sb));  // synchronises: both events are done
        float ms = 0;
        SPC_HIP(hipEventElapsedTime(&ms, B.ev_a, B.ev_b));
        if (!fast1) B.ms_round_kernel += ms;  // the fused round kernel only
        round_ms += ms;
        if (B.rcap[d] < B.rused[d] + sb) {
            // copied growth: the first batch sizes the round from its
            // survivor density, later batches grow by half; in-place growth
            // maps what is needed
            uint64_t want = B.rused[d] + sb;
            if (!B.vhub[d]) {
                if (bi == 0 && bounds.size() > 2 && need)
                    want = std::max<uint64_t>(want, (uint64_t)((double)sb * total_raw / need * 1.1));
                else if (bi > 0)
                    want = std::max<uint64_t>(want, B.rcap[d] + B.rcap[d] / 2);
            }
            SPC_TRY(B.grow_round(d, want));
        }
        hipLaunchKernelGGL(k_compact<DB>, dim3(grid_for(b1 - b0, kWaves)), dim3(kBlock), 0, B.st, b0,
                           b1, d, B.raw_off, B.soff, B.surv, B.tmp_hub, B.tmp_cnt, B.rused[d],
                           B.rhub[d], B.rcnt[d], rs, rl, (const uint32_t *)B.gbase,
                           static_cast<LT *>(B.land), B.lmask);
        SPC_LAUNCHED();
        B.rused[d] += sb;
        kept += sb;
        raw_lo += need;
    }
    B.arena.release(filt);
    if (B.rcap[d] > B.rused[d] + B.rused[d] / 8 + (1u << 20)) SPC_TRY(B.shrink_round(d));
    uint64_t c[8];
    SPC_TRY(B.read_u64((const uint64_t *)B.ctr, c, 8));
    RoundCounters rc;
    rc.raw = push ? total_raw : c[0] + fast_raw;  // a push round's kernel reads merged candidates
    rc.merged = c[1] + fast_raw;
    rc.kept = c[2] + fast_raw;
    rc.scanned = c[3];
    rc.staged = c[4];
    rc.row_bytes = c[5];
    rc.headers = c[6];
    rc.filter_bytes = c[7];
    rc.kernel_ms = round_ms;
    rc.mem_peak = B.arena.window_peak();
    B.stats.push_back(rc);
    // algorithmic bytes of the fused kernel: the pulled entries (hub +
    // count), u's staged label entries past the landmarks, the candidates'
    // landmark rows (hubs <= w), the other probe entries read up to the first
    // one proving a shorter path and their label offsets, and the survivors
    // written (hub + count), and the filter words looked up
    uint64_t es = sizeof(E);
    B.alg_bytes += c[0] * 12 + c[4] * es + c[5] + c[3] * es + c[6] * 16 + c[2] * 12 + c[7];
    *kept_out = kept;
    if (kept == 0) return SPC_OK;

    // merge the round into the labels
    hipLaunchKernelGGL(k_new_len, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, B.st, N, B.lab_off, rl,
                       B.nlen);
    SPC_LAUNCHED();
    SPC_TRY(scan_u64(B.nlen, B.lab_off2, N, B.ws, B.st));
    uint64_t new_entries = B.entries + kept;
    if (B.lab_cap2 < new_entries) {
        // the older buffer (distances <= d-2) is dead once the round kernel
        // has run: free it first (a large one straight to the runtime: it is
        // outgrown), then take the merged size, plus an eighth (at most 2^28
        // entries) when the labels grew by less than 1/16 this round (the
        // two buffers alternate, so slowly growing labels reuse them for
        // many rounds; a fast-growing index gets no slack)
        E *p2 = static_cast<E *>(B.lab_hd2);
        if (B.arena.size_of(p2) >= (256ull << 20))
            B.arena.release_to_device(p2);
        else
            B.arena.release(p2);
        B.lab_cap2 = 0;
        const uint64_t slack = std::min<uint64_t>(new_entries / 8, 1ull << 28);
        uint64_t cap = new_entries + (kept < B.entries / 16 ? slack : 0);
        if (B.arena.alloc(&p2, cap) != SPC_OK) {
            cap = new_entries;
            SPC_TRY(B.arena.alloc(&p2, cap));
        }
        B.lab_hd2 = p2;
        B.lab_cap2 = cap;
    }
    hipLaunchKernelGGL(k_merge<DB>, dim3(grid_for(N, kWaves)), dim3(kBlock), 0, B.st, N, d, B.lab_off,
                       static_cast<const E *>(B.lab_hd), rs, rl, B.rhub[d], B.lab_off2,
                       static_cast<E *>(B.lab_hd2), (const uint32_t *)B.gbase,
                       (const uint32_t *)B.lc, B.lc2);
    SPC_LAUNCHED();
    std::swap(B.lab_off, B.lab_off2);
    std::swap(B.lab_hd, B.lab_hd2);
    std::swap(B.lc, B.lc2);
    std::swap(B.lab_cap, B.lab_cap2);
    B.entries_prev = B.entries;
    B.entries = new_entries;
    B.stats.back().mem_peak = B.arena.window_peak();
    return SPC_OK;
}

}  // namespace
}  // namespace spc

namespace spc {
namespace {

enum class LoopEnd { Done, Widen };

// Rounds d, d+1, ... with DB-bit distances until a round inserts nothing, the
// cap is reached, or (auto width) distances outgrow 8 bits.
template <int DB>
spc_status rounds_loop(Build &B, uint32_t &d, uint32_t cap, bool auto_width, bool &truncated,
                       uint32_t &last_round, LoopEnd &end) {
    for (;; d++) {
        if (cap && d > cap) {
            // truncated iff round cap+1 would still pull candidates
            const uint32_t N = B.N;
            hipLaunchKernelGGL(k_expand_count, dim3(grid_for(N, kWaves)), dim3(kBlock), 0, B.st, N,
                               B.nreal, B.goff, B.gadj, B.rstart[d - 1], B.rlen[d - 1], B.rhub[d - 1], B.raw);
            SPC_LAUNCHED();
            SPC_TRY(scan_u64(B.raw, B.raw_off, N, B.ws, B.st));
            uint64_t tr;
            SPC_TRY(B.read_u64(B.raw_off + N, &tr));
            truncated = tr > 0;
            last_round = cap;
            end = LoopEnd::Done;
            return SPC_OK;
        }
        if (d > Ent<DB>::kMaxDist) {
            if (DB == 8 && auto_width) {
                end = LoopEnd::Widen;
                return SPC_OK;
            }
            return SPC_ERR_DIST_RANGE;
        }
        uint64_t kept;
        bool any;
        SPC_TRY(run_round<DB>(B, d, &kept, &any));
        if (kept == 0) {
            if (any) {
                // the round ran its kernels but inserted nothing: record an
                // empty segment table is not needed; nothing reads it
            }
            last_round = d;
            end = LoopEnd::Done;
            return SPC_OK;
        }
    }
}

spc_status widen_buffer(Build &B, void **buf, uint64_t *cap, uint64_t n) {
    uint64_t *w = nullptr;
    uint64_t c = std::max<uint64_t>(n, 1);
    SPC_TRY(B.arena.alloc(&w, c));
    if (n) {
        hipLaunchKernelGGL(k_widen, dim3(grid_stride(n)), dim3(kBlock), 0, B.st,
                           static_cast<const uint32_t *>(*buf), w, n);
        SPC_LAUNCHED();
    }
    SPC_HIP(hipStreamSynchronize(B.st));
    uint32_t *old = static_cast<uint32_t *>(*buf);
    B.arena.release(old);
    *buf = w;
    *cap = c;
    return SPC_OK;
}

// 8-bit -> 16-bit distances: both label buffers and the landmark rows
spc_status widen_labels(Build &B) {
    SPC_TRY(widen_buffer(B, &B.lab_hd, &B.lab_cap, B.entries));
    SPC_TRY(widen_buffer(B, &B.lab_hd2, &B.lab_cap2, B.entries_prev));
    uint64_t nl = (uint64_t)B.N * kLand;
    uint16_t *l16 = nullptr;
    SPC_TRY(B.arena.alloc(&l16, nl));
    hipLaunchKernelGGL(k_land_widen, dim3(grid_stride(nl)), dim3(kBlock), 0, B.st,
                       static_cast<const uint8_t *>(B.land), l16, nl);
    SPC_LAUNCHED();
    SPC_HIP(hipStreamSynchronize(B.st));
    uint8_t *l8 = static_cast<uint8_t *>(B.land);
    B.arena.release(l8);
    B.land = l16;
    B.db = 16;
    return SPC_OK;
}

template <int DB>
spc_status finalize_counts(Build &B, uint64_t **lab_cnt, uint64_t *nsat_out) {
    using E = typename Ent<DB>::T;
    // the older label buffer is not needed any more; with 8-bit distances
    // neither are the rounds' hub arrays (counts are placed by rank)
    {
        E *old = static_cast<E *>(B.lab_hd2);
        B.arena.release(old);
        B.lab_hd2 = nullptr;
        B.lab_cap2 = 0;
    }
    B.arena.release(B.cur);
    B.arena.release(B.nxt);
    const uint32_t R = (uint32_t)B.rstart.size();
    const bool by_rank = DB == 8 && R <= 256;
    if (by_rank)
        for (size_t r = 0; r < B.rhub.size(); r++) B.release_round_hub(r);
    SPC_TRY(B.arena.alloc(lab_cnt, std::max<uint64_t>(B.entries, 1)));
    SPC_HIP(hipMemsetAsync(B.ctr, 0, sizeof(unsigned long long), B.st));
    if (by_rank) {
        hipLaunchKernelGGL(k_finalize_rank, dim3(grid_for(B.N, kWaves)), dim3(kBlock), 0, B.st, B.N, R,
                           B.lab_off, static_cast<const uint32_t *>(B.lab_hd),
                           (const uint64_t *const *)B.rs_tab, (const uint64_t *const *)B.cnt_tab,
                           *lab_cnt, B.ctr);
    } else {
        hipLaunchKernelGGL(k_finalize<DB>, dim3(grid_for(B.N, kWaves)), dim3(kBlock), 0, B.st, B.N,
                           B.lab_off, static_cast<const E *>(B.lab_hd),
                           (const uint64_t *const *)B.rs_tab, (const uint32_t *const *)B.rl_tab,
                           (const uint32_t *const *)B.hub_tab, (const uint64_t *const *)B.cnt_tab,
                           *lab_cnt, B.ctr);
    }
    SPC_LAUNCHED();
    SPC_TRY(B.read_u64((const uint64_t *)B.ctr, nsat_out));
    return SPC_OK;
}

inline float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0;
    return ms;
}

}  // namespace

// ---------------------------------------------------------------------------
// Directed input (Section "2-Hop Labeling for Shortest Path Counting": an
// out-label and an in-label per vertex).  The build labels 2n rows: row r is
// the out-label of rank r, row n + r its in-label.  Row r pulls from the
// out-labels of the heads of r's out-arcs (a path r -> x -> ... -> w), row
// n + r from the in-labels of the tails of r's in-arcs (w -> ... -> y -> r),
// so the rows' adjacency is the rank-space out-arcs for the first half and
// the in-arcs, shifted by n, for the second.  A row's hubs are real vertices
// ranked at or above its own, and a candidate of an out-label row is pruned
// through the candidate's in-label (and vice versa): the round kernel's
// `nreal`.
// ---------------------------------------------------------------------------
__global__ void k_in_degree(const uint32_t *col, uint64_t nnz, uint32_t *indeg) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz;
         i += (uint64_t)gridDim.x * blockDim.x)
        atomicAdd(&indeg[col[i]], 1u);
}
// total degree (out + in), and its maximum
__global__ void k_total_degree(const uint64_t *off, const uint32_t *indeg, uint32_t n, uint32_t *deg,
                               uint32_t *maxdeg) {
    uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const uint32_t dv = (uint32_t)(off[v + 1] - off[v]) + indeg[v];
    deg[v] = dv;
    atomicMax(maxdeg, dv);
}
// row lengths of the pseudo-graph: out-degree of rank r, then in-degree
__global__ void k_dir_rowdeg(const uint32_t *order, const uint64_t *off, const uint32_t *indeg, uint32_t n,
                             uint32_t *pdeg) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint32_t v = order[r];
    pdeg[r] = (uint32_t)(off[v + 1] - off[v]);
    pdeg[n + r] = indeg[v];
}
// in-arc keys (rank of head << xb | rank of tail), one wave per tail
__global__ __launch_bounds__(kBlock) void k_arc_keys(const uint64_t *off, const uint32_t *col,
                                                     const uint32_t *rank_of, uint32_t n, int xb,
                                                     uint64_t *keys) {
    const uint32_t v = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (v >= n) return;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t rv = rank_of[v];
    for (uint64_t k = off[v] + lane; k < off[v + 1]; k += 64)
        keys[k] = ((uint64_t)rank_of[col[k]] << xb) | rv;
}
// sorted in-arc keys -> the in-label rows' neighbours (n + rank of tail)
__global__ void k_dir_in_rows(const uint64_t *keys, uint64_t nnz, int xb, uint32_t n, uint32_t *gadj_in) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz;
         i += (uint64_t)gridDim.x * blockDim.x)
        gadj_in[i] = n + (uint32_t)(keys[i] & ((1ull << xb) - 1));
}

spc_status preprocess_directed(Build &B, const spc_graph &G, bool use_order, bool use_tie, bool validate) {
    B.simple = false;  // no symmetric shortcuts (round 1 sort, PUSH)
    const uint32_t n = B.nreal;
    const uint64_t A = G.nnz;  // arcs
    uint64_t *off = nullptr;
    uint32_t *col = nullptr, *deg = nullptr, *indeg = nullptr, *err = nullptr, *ord = nullptr, *hits = nullptr;
    uint64_t *tie = nullptr;
    SPC_TRY(B.arena.alloc(&off, (uint64_t)n + 1));
    SPC_TRY(B.arena.alloc(&col, std::max<uint64_t>(A, 1)));
    SPC_TRY(B.arena.alloc(&deg, (uint64_t)n + 1));
    SPC_TRY(B.arena.alloc(&indeg, (uint64_t)n + 1));
    SPC_TRY(B.arena.alloc(&err, 2));
    SPC_HIP(hipMemsetAsync(err, 0, 2 * sizeof(uint32_t), B.st));
    SPC_HIP(hipMemsetAsync(indeg, 0, ((uint64_t)n + 1) * sizeof(uint32_t), B.st));
    // inputs on the device (host inputs are staged)
    const uint64_t *src_off = G.row_off;
    const uint32_t *src_col = G.col, *src_ord = G.order;
    const uint64_t *src_tie = G.tie_key;
    uint64_t *st_off = nullptr, *st_tie = nullptr;
    uint32_t *st_col = nullptr, *st_ord = nullptr;
    if (!G.on_device) {
        SPC_TRY(B.arena.alloc(&st_off, (uint64_t)n + 1));
        SPC_TRY(B.arena.alloc(&st_col, std::max<uint64_t>(A, 1)));
        SPC_HIP(hipMemcpyAsync(st_off, G.row_off, ((uint64_t)n + 1) * sizeof(uint64_t), hipMemcpyHostToDevice,
                               B.st));
        if (A) SPC_HIP(hipMemcpyAsync(st_col, G.col, A * sizeof(uint32_t), hipMemcpyHostToDevice, B.st));
        if (use_order) {
            SPC_TRY(B.arena.alloc(&st_ord, (uint64_t)n + 1));
            SPC_HIP(hipMemcpyAsync(st_ord, G.order, (uint64_t)n * sizeof(uint32_t), hipMemcpyHostToDevice, B.st));
        }
        if (use_tie) {
            SPC_TRY(B.arena.alloc(&st_tie, (uint64_t)n + 1));
            SPC_HIP(hipMemcpyAsync(st_tie, G.tie_key, (uint64_t)n * sizeof(uint64_t), hipMemcpyHostToDevice,
                                   B.st));
        }
        src_off = st_off;
        src_col = st_col;
        src_ord = st_ord;
        src_tie = st_tie;
    }
    hipLaunchKernelGGL(k_union_off, dim3(grid_for((uint64_t)n + 1, kBlock)), dim3(kBlock), 0, B.st, src_off, off,
                       n, A, (uint64_t)0, err);
    SPC_LAUNCHED();
    if (A) {
        hipLaunchKernelGGL(k_union_col, dim3(grid_for(A, kBlock)), dim3(kBlock), 0, B.st, src_col, col, A, n, 0u,
                           err);
        SPC_LAUNCHED();
    }
    if (use_order) {
        SPC_TRY(B.arena.alloc(&ord, (uint64_t)n + 1));
        SPC_TRY(B.arena.alloc(&hits, (uint64_t)n + 1));
        SPC_HIP(hipMemsetAsync(hits, 0, ((uint64_t)n + 1) * sizeof(uint32_t), B.st));
        hipLaunchKernelGGL(k_union_order, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, B.st, src_ord, ord, n, 0u,
                           hits, err);
        SPC_LAUNCHED();
        hipLaunchKernelGGL(k_check_perm, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, B.st, hits, n, err);
        SPC_LAUNCHED();
    }
    if (use_tie) {
        SPC_TRY(B.arena.alloc(&tie, (uint64_t)n + 1));
        SPC_HIP(hipMemcpyAsync(tie, src_tie, (uint64_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, B.st));
    }
    uint64_t e2[1];
    SPC_TRY(B.read_u64((const uint64_t *)err, e2));  // also ends the staging copies
    if ((uint32_t)e2[0] != 0) return SPC_ERR_INVALID_ARG;
    B.arena.release(st_off);
    B.arena.release(st_col);
    B.arena.release(st_ord);
    B.arena.release(st_tie);
    if (validate) {  // no self loops, no repeated arcs (sorts each row)
        SPC_TRY(validate_csr(B, off, col, n, A, err, true));
    }
    // total degrees and the order
    if (A) {
        hipLaunchKernelGGL(k_in_degree, dim3(grid_stride(A)), dim3(kBlock), 0, B.st, col, A, indeg);
        SPC_LAUNCHED();
    }
    uint32_t *maxdeg = err + 1;
    SPC_HIP(hipMemsetAsync(maxdeg, 0, sizeof(uint32_t), B.st));
    hipLaunchKernelGGL(k_total_degree, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, B.st, off, indeg, n, deg,
                       maxdeg);
    SPC_LAUNCHED();
    SPC_TRY(B.arena.alloc(&B.order, (uint64_t)n + 1));
    SPC_TRY(B.arena.alloc(&B.rank_of, (uint64_t)n + 1));
    if (use_order) {
        SPC_HIP(hipMemcpyAsync(B.order, ord, (uint64_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, B.st));
    } else {
        uint64_t md[1];
        SPC_TRY(B.read_u64((const uint64_t *)err, md));
        const uint32_t maxd = (uint32_t)(md[0] >> 32);
        uint64_t *keys = nullptr, *keys2 = nullptr;
        uint32_t *vals2 = nullptr;
        SPC_TRY(B.arena.alloc(&keys, (uint64_t)n + 1));
        SPC_TRY(B.arena.alloc(&keys2, (uint64_t)n + 1));
        SPC_TRY(B.arena.alloc(&vals2, (uint64_t)n + 1));
        hipLaunchKernelGGL(k_iota_keys, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, B.st, (const uint64_t *)tie, n,
                           keys, B.order);
        SPC_LAUNCHED();
        if (use_tie) SPC_TRY(radix_sort_pairs(keys, B.order, keys2, vals2, n, 64, B.ws, B.st));
        const int degbits = std::max(1, bit_width(maxd));
        hipLaunchKernelGGL(k_degree_keys, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, B.st, B.order, deg, n, maxd,
                           degbits, (const uint32_t *)nullptr, 1u, keys);
        SPC_LAUNCHED();
        SPC_TRY(radix_sort_pairs(keys, B.order, keys2, vals2, n, degbits, B.ws, B.st));
        B.arena.release(keys);
        B.arena.release(keys2);
        B.arena.release(vals2);
    }
    B.arena.release(ord);
    B.arena.release(hits);
    B.arena.release(tie);
    // the pseudo-graph in rank space
    uint32_t *pdeg = nullptr, *rdeg = nullptr;
    SPC_TRY(B.arena.alloc(&pdeg, 2 * (uint64_t)n + 1));
    SPC_TRY(B.arena.alloc(&rdeg, (uint64_t)n + 1));
    hipLaunchKernelGGL(k_rank_of, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, B.st, B.order, n, deg, B.rank_of,
                       rdeg);
    SPC_LAUNCHED();
    hipLaunchKernelGGL(k_dir_rowdeg, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, B.st, B.order, off, indeg, n,
                       pdeg);
    SPC_LAUNCHED();
    SPC_TRY(B.arena.alloc(&B.goff, 2 * (uint64_t)n + 1));
    SPC_TRY(B.arena.alloc(&B.gadj, std::max<uint64_t>(2 * A, 1)));
    SPC_TRY(scan_u32(pdeg, B.goff, 2 * n, B.ws, B.st));
    // out rows: the heads of each rank's out-arcs, in rank space
    hipLaunchKernelGGL(k_relabel, dim3(grid_for(n, kWaves)), dim3(kBlock), 0, B.st, B.order, B.rank_of, off, col,
                       B.goff, B.gadj, n);
    SPC_LAUNCHED();
    // in rows: arcs sorted by (head rank, tail rank); row n + r gets r's tails
    if (A) {
        const int xb = std::max(1, bit_width(n));
        uint64_t *keys = nullptr, *keys2 = nullptr, *rws = nullptr;
        SPC_TRY(B.arena.alloc(&keys, A));
        SPC_TRY(B.arena.alloc(&keys2, A));
        SPC_TRY(B.arena.alloc(&rws, radix_ws_elems(A)));
        hipLaunchKernelGGL(k_arc_keys, dim3(grid_for(n, kWaves)), dim3(kBlock), 0, B.st, off, col, B.rank_of, n, xb,
                           keys);
        SPC_LAUNCHED();
        SPC_TRY(radix_sort_pairs(keys, nullptr, keys2, nullptr, A, 2 * xb, rws, B.st));
        hipLaunchKernelGGL(k_dir_in_rows, dim3(grid_stride(A)), dim3(kBlock), 0, B.st, keys, A, xb, n, B.gadj + A);
        SPC_LAUNCHED();
        SPC_HIP(hipStreamSynchronize(B.st));
        B.arena.release(keys);
        B.arena.release(keys2);
        B.arena.release(rws);
    }
    for (uint32_t *p : {pdeg, rdeg, col, deg, indeg, err}) B.arena.release(p);
    B.arena.release(off);
    return SPC_OK;
}

// Per graph (vbase, gn, obase, on) on the device, for queries that name
// their graph one by one; owned by the index.
spc_status attach_graph_table(Build &B, spc_index *ix) {
    const size_t k = ix->gn.size();
    std::vector<uint32_t> h(4 * std::max<size_t>(k, 1), 0);
    for (size_t g = 0; g < k; g++) {
        h[4 * g] = ix->vbase[g];
        h[4 * g + 1] = ix->gn[g];
        h[4 * g + 2] = ix->reduced ? ix->obase[g] : ix->vbase[g];
        h[4 * g + 3] = ix->reduced ? ix->on[g] : ix->gn[g];
    }
    uint32_t *d = nullptr;
    SPC_TRY(B.arena.alloc(&d, (uint64_t)h.size()));
    SPC_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(uint32_t), hipMemcpyHostToDevice, B.st));
    SPC_HIP(hipStreamSynchronize(B.st));
    const uint64_t b = B.arena.detach(d);
    ix->blocks.emplace_back(d, (size_t)b);
    ix->index_bytes += b;
    ix->g_tab = d;
    return SPC_OK;
}

spc_status build_impl(const spc_graph *gs, uint32_t k, const spc_build_opts *o, hipStream_t st,
                      spc_index **out) {
    if (!gs || !o || !out || k == 0) return SPC_ERR_INVALID_ARG;
    // one reduction at a time
    if (o->reduce != 0 && o->reduce != SPC_REDUCE_ONE_SHELL && o->reduce != SPC_REDUCE_EQUIVALENCE)
        return SPC_ERR_INVALID_ARG;
    if (o->propagation > SPC_PROPAGATE_AUTO || o->reserved != 0) return SPC_ERR_INVALID_ARG;
    if (o->dist_bits != 0 && o->dist_bits != 8 && o->dist_bits != 16) return SPC_ERR_INVALID_ARG;
    // a directed graph is built alone and unreduced: 2n label rows
    const bool directed = gs[0].directed != 0;
    for (uint32_t g = 0; g < k; g++)
        if ((gs[g].directed != 0) != directed) return SPC_ERR_INVALID_ARG;
    if (directed && k > 1) return SPC_ERR_UNSUPPORTED;
    if (directed && o->reduce != 0) return SPC_ERR_INVALID_ARG;
    uint64_t N64 = 0, NNZ = 0;
    uint32_t n_order = 0, n_tie = 0, n_dev = 0;
    for (uint32_t g = 0; g < k; g++) {
        const spc_graph &G = gs[g];
        if (!G.row_off || (G.nnz && !G.col)) return SPC_ERR_INVALID_ARG;
        if (!directed && (G.nnz & 1)) return SPC_ERR_INVALID_ARG;  // symmetric: every edge twice
        N64 += G.n;
        NNZ += G.nnz;
        n_order += G.order != nullptr;
        n_tie += G.tie_key != nullptr;
        n_dev += G.on_device != 0;
    }
    if ((n_order && n_order != k) || (n_tie && n_tie != k) || (n_dev && n_dev != k))
        return SPC_ERR_INVALID_ARG;
    // one wave per vertex in several kernels, one work-item per adjacency
    // slot in others: a launch's work-item count must stay below 2^32
    const uint64_t rows64 = directed ? 2 * N64 : N64, slots64 = directed ? 2 * NNZ : NNZ;
    if (rows64 > kMaxVertices || slots64 > kMaxAdjacency) return SPC_ERR_UNSUPPORTED;
    int db = (o->dist_bits == 16) ? 16 : 8;
    if (db == 8 && N64 > Ent<8>::kMaxHub - 1) {
        if (o->dist_bits == 8) return SPC_ERR_UNSUPPORTED;
        db = 16;
    }
    const bool auto_width = o->dist_bits == 0;

    int dev = 0;
    SPC_HIP(hipGetDevice(&dev));
    Build B(o->mem_budget, st);
    {
        size_t fr = 0, tot = 0;
        SPC_HIP(hipMemGetInfo(&fr, &tot));
        B.dev_bytes = tot;
        // SPC_VMM=0 in the environment turns in-place growth off
        const char *ev = std::getenv("SPC_VMM");
        B.vmm = vmm_supported() && !(ev && ev[0] == '0');
        // SPC_FILTER=0 turns the prune probes' membership filter off, 16
        // keeps it at 16 bits per entry (the density where memory is short)
        const char *ef = std::getenv("SPC_FILTER");
        B.filter = !(ef && ef[0] == '0');
        B.filter_dense = !(ef && std::strcmp(ef, "16") == 0);
    }
    B.N = (uint32_t)rows64;
    B.NNZ = slots64;
    B.nreal = directed ? (uint32_t)N64 : 0;
    B.prop = directed ? (uint32_t)SPC_PROPAGATE_PULL : o->propagation;
    B.k = k;
    B.db = db;
    {
        uint32_t base = 0;
        for (uint32_t g = 0; g < k; g++) {
            B.vbase.push_back(base);
            B.gn.push_back(gs[g].n);
            base += gs[g].n;
        }
        B.vbase.push_back(base);
    }
    SPC_HIP(hipHostMalloc((void **)&B.h_pin, 64 * sizeof(uint64_t), hipHostMallocDefault));
    SPC_HIP(hipEventCreate(&B.ev_a));
    SPC_HIP(hipEventCreate(&B.ev_b));
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            for (int i = 0; i < 4; i++)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } evg{ev};
    for (int i = 0; i < 4; i++) SPC_HIP(hipEventCreate(&ev[i]));
    if (B.N == 0) {  // nothing to order or label: an empty index
        if (NNZ) return SPC_ERR_INVALID_ARG;
        spc_index *ix = new (std::nothrow) spc_index();
        if (!ix) return SPC_ERR_OUT_OF_MEMORY;
        SPC_TRY(B.arena.alloc(&ix->lab_off, 1));
        SPC_HIP(hipMemsetAsync(ix->lab_off, 0, sizeof(uint64_t), st));
        uint32_t *hd = nullptr;
        SPC_TRY(B.arena.alloc(&hd, 1));
        ix->lab_hd = hd;
        SPC_TRY(B.arena.alloc(&ix->lab_cnt, 1));
        SPC_TRY(B.arena.alloc(&ix->rank_of, 1));
        SPC_TRY(B.arena.alloc(&ix->order, 1));
        SPC_HIP(hipStreamSynchronize(st));
        ix->device = dev;
        ix->dist_bits = (uint32_t)db;
        ix->out_bits = (uint32_t)db;
        ix->vbase.assign(B.vbase.begin(), B.vbase.end());
        ix->gn = B.gn;
        ix->round_stats.push_back(RoundCounters());
        for (void *blk : {(void *)ix->lab_off, (void *)hd, (void *)ix->lab_cnt, (void *)ix->rank_of,
                          (void *)ix->order}) {
            uint64_t b = B.arena.detach(blk);
            ix->blocks.emplace_back(blk, (size_t)b);
            ix->index_bytes += b;
        }
        if (spc_status e = attach_graph_table(B, ix); e != SPC_OK) {
            spc_free(ix);
            return e;
        }
        *out = ix;
        return SPC_OK;
    }
    SPC_TRY(B.arena.alloc(&B.ws, std::max(radix_ws_elems((uint64_t)B.N + 1), scan_ws_elems((uint64_t)B.N + 1))));
    SPC_TRY(B.arena.alloc(&B.ctr, 8));

    SPC_HIP(hipEventRecord(ev[0], st));
    if (directed)
        SPC_TRY(preprocess_directed(B, gs[0], n_order == k, n_tie == k, o->validate != 0));
    else
        SPC_TRY(preprocess(B, gs, n_order == k, n_tie == k, o->validate != 0, o->reduce));
    SPC_HIP(hipEventRecord(ev[1], st));
    // from here on the graph is the core when the 1-shell was cut off
    const uint32_t N = B.N;
    const uint64_t NNZ_in = NNZ;
    NNZ = B.NNZ;

    // round 0
    SPC_TRY(B.arena.alloc(&B.raw, (uint64_t)N + 1));
    SPC_TRY(B.arena.alloc(&B.raw_off, (uint64_t)N + 1));
    SPC_TRY(B.arena.alloc(&B.soff, (uint64_t)N + 1));
    SPC_TRY(B.arena.alloc(&B.nlen, (uint64_t)N + 1));
    SPC_TRY(B.arena.alloc(&B.surv, (uint64_t)N + 1));
    SPC_TRY(B.arena.alloc(&B.cur, std::max<uint64_t>(NNZ, 1)));
    SPC_TRY(B.arena.alloc(&B.nxt, std::max<uint64_t>(NNZ, 1)));
    SPC_TRY(B.arena.alloc(&B.lab_off, (uint64_t)N + 1));
    SPC_TRY(B.arena.alloc(&B.lab_off2, (uint64_t)N + 1));
    {
        B.tab_cap = (size_t)Ent<16>::kMaxDist + 2;
        SPC_TRY(B.arena.alloc(&B.rs_tab, B.tab_cap));
        SPC_TRY(B.arena.alloc(&B.rl_tab, B.tab_cap));
        SPC_TRY(B.arena.alloc(&B.hub_tab, B.tab_cap));
        SPC_TRY(B.arena.alloc(&B.cnt_tab, B.tab_cap));
        uint64_t *rs = nullptr;
        uint32_t *rl = nullptr;
        SPC_TRY(B.arena.alloc(&rs, (uint64_t)N + 1));
        SPC_TRY(B.arena.alloc(&rl, (uint64_t)N + 1));
        SPC_TRY(B.add_round(rs, rl));
        SPC_TRY(B.reserve_round(0, N));
        SPC_TRY(B.grow_round(0, N));
        B.rused[0] = N;
        if (k > 1) {
            uint32_t *vb_dev = nullptr;
            SPC_TRY(B.arena.alloc(&vb_dev, (uint64_t)k + 1));
            SPC_HIP(hipMemcpyAsync(vb_dev, B.vbase.data(), k * sizeof(uint32_t), hipMemcpyHostToDevice,
                                   st));
            SPC_TRY(B.arena.alloc(&B.gbase, (uint64_t)N));
            hipLaunchKernelGGL(k_fill_gbase, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, st, N, vb_dev, k,
                               B.gbase);
            SPC_LAUNCHED();
            SPC_HIP(hipStreamSynchronize(st));
            B.arena.release(vb_dev);
        }
        {
            uint64_t nl = (uint64_t)N * kLand;
            if (db == 8) {
                uint8_t *l8 = nullptr;
                SPC_TRY(B.arena.alloc(&l8, nl));
                B.land = l8;
                hipLaunchKernelGGL(k_land_init<8>, dim3(grid_stride(nl)), dim3(kBlock), 0, st, N,
                                   B.nreal, (const uint32_t *)B.gbase, l8);
            } else {
                uint16_t *l16 = nullptr;
                SPC_TRY(B.arena.alloc(&l16, nl));
                B.land = l16;
                hipLaunchKernelGGL(k_land_init<16>, dim3(grid_stride(nl)), dim3(kBlock), 0, st, N,
                                   B.nreal, (const uint32_t *)B.gbase, l16);
            }
            SPC_LAUNCHED();
        }
        {
            // landmark masks (optional: without them the rows serve)
            const uint64_t nw = (uint64_t)N * kMaskK * kMaskWords;
            if (B.arena.alloc(&B.lmask, nw) == SPC_OK) {
                hipLaunchKernelGGL(k_fill_u32, dim3(grid_stride(nw)), dim3(kBlock), 0, st, B.lmask, nw, 0u);
                SPC_LAUNCHED();
            } else {
                B.lmask = nullptr;
            }
        }
        SPC_TRY(B.arena.alloc(&B.lc, (uint64_t)N + 1));
        SPC_TRY(B.arena.alloc(&B.lc2, (uint64_t)N + 1));
        hipLaunchKernelGGL(k_lc_init, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, st, N, B.nreal,
                           (const uint32_t *)B.gbase, B.lc);
        SPC_LAUNCHED();
        uint64_t lcap = std::max<uint64_t>((uint64_t)N + NNZ / 2, 1024);
        if (db == 8) {
            uint32_t *h = nullptr;
            SPC_TRY(B.arena.alloc(&h, lcap));
            B.lab_hd = h;
            hipLaunchKernelGGL(k_round0<8>, dim3(grid_for((uint64_t)N + 1, kBlock)), dim3(kBlock), 0,
                               st, N, B.nreal, B.rhub[0], B.rcnt[0], rs, rl, B.lab_off, h);
        } else {
            uint64_t *h = nullptr;
            SPC_TRY(B.arena.alloc(&h, lcap));
            B.lab_hd = h;
            hipLaunchKernelGGL(k_round0<16>, dim3(grid_for((uint64_t)N + 1, kBlock)), dim3(kBlock), 0,
                               st, N, B.nreal, B.rhub[0], B.rcnt[0], rs, rl, B.lab_off, h);
        }
        SPC_LAUNCHED();
        B.lab_cap = lcap;
        B.entries = N;
        RoundCounters r0;
        r0.kept = N;
        B.stats.push_back(r0);
    }

    uint32_t d = 1, last_round = 0;
    bool truncated = false;
    if (N > 0) {
        while (true) {
            LoopEnd end;
            if (B.db == 8)
                SPC_TRY(rounds_loop<8>(B, d, o->round_cap, auto_width, truncated, last_round, end));
            else
                SPC_TRY(rounds_loop<16>(B, d, o->round_cap, auto_width, truncated, last_round, end));
            if (end == LoopEnd::Widen) {
                SPC_TRY(widen_labels(B));
                continue;
            }
            break;
        }
    }
    SPC_HIP(hipEventRecord(ev[2], st));
    uint64_t *lab_cnt = nullptr;
    uint64_t nsat = 0;
    if (B.db == 8)
        SPC_TRY(finalize_counts<8>(B, &lab_cnt, &nsat));
    else
        SPC_TRY(finalize_counts<16>(B, &lab_cnt, &nsat));
    SPC_HIP(hipEventRecord(ev[3], st));
    SPC_HIP(hipStreamSynchronize(st));

    uint32_t maxd = 0;
    for (size_t r = 0; r < B.stats.size(); r++)
        if (B.stats[r].kept) maxd = (uint32_t)r;
    // a query distance is at most two label distances plus two fringe
    // depths: the outputs take the narrowest width that holds every one
    uint64_t qmax = 2ull * maxd + (B.reduced ? 2ull * B.shell.max_depth : 0ull);
    if (B.hub_w && qmax < 2) qmax = 2;  // two twins with common neighbours
    if (qmax > Ent<16>::kMaxDist) return SPC_ERR_DIST_RANGE;
    const uint32_t out_bits = (B.db == 16 || qmax > Ent<8>::kMaxDist) ? 16u : 8u;

    spc_index *ix = new (std::nothrow) spc_index();
    if (!ix) return SPC_ERR_OUT_OF_MEMORY;
    ix->device = dev;
    ix->n = directed ? B.nreal : N;
    ix->m = directed ? NNZ_in : NNZ_in / 2;  // arcs of a directed graph
    ix->nreal = B.nreal;
    ix->dist_bits = (uint32_t)B.db;
    ix->out_bits = out_bits;
    ix->rounds = last_round;
    ix->round_cap = o->round_cap;
    ix->truncated = truncated;
    ix->entries = B.entries;
    ix->saturated = nsat;
    ix->max_dist = maxd;
    ix->vbase.assign(B.vbase.begin(), B.vbase.end());
    ix->gn = B.gn;
    ix->round_stats = B.stats;
    ix->peak_build_bytes = B.arena.peak();
    ix->ms_order = elapsed(ev[0], ev[1]);
    ix->ms_rounds = elapsed(ev[1], ev[2]);
    ix->ms_finalize = elapsed(ev[2], ev[3]);
    ix->ms_total = elapsed(ev[0], ev[3]);
    ix->ms_round_kernel = B.ms_round_kernel;
    ix->alg_bytes_round_kernel = B.alg_bytes;
    ix->round_kernel_launches = B.launches;
    ix->lab_off = B.lab_off;
    ix->lab_hd = B.lab_hd;
    ix->lab_cnt = lab_cnt;
    ix->rank_of = B.rank_of;
    ix->order = B.order;
    for (void *blk : {(void *)B.lab_off, B.lab_hd, (void *)lab_cnt, (void *)B.rank_of, (void *)B.order}) {
        uint64_t b = B.arena.detach(blk);
        ix->blocks.emplace_back(blk, (size_t)b);
        ix->index_bytes += b;
    }
    if (B.reduced) {
        ShellResult &R = B.shell;
        ix->reduced = true;
        ix->obase = B.obase;
        ix->on = B.on;
        ix->red_root = R.root;
        ix->red_depth = R.depth;
        ix->red_parent = R.parent;
        ix->core_vid = R.core_vid;
        ix->fringe = R.fringe;
        ix->fringe_depth = R.max_depth;
        ix->twins = R.twins;
        ix->red_same = R.same;
        ix->hub_w = B.hub_w;
        for (void *blk : {(void *)R.root, (void *)R.depth, (void *)R.parent, (void *)R.core_vid,
                          (void *)R.same, (void *)B.hub_w}) {
            if (!blk) continue;
            uint64_t b = B.arena.detach(blk);
            ix->blocks.emplace_back(blk, (size_t)b);
            ix->index_bytes += b;
        }
    }
    if (spc_status e = attach_graph_table(B, ix); e != SPC_OK) {
        spc_free(ix);
        return e;
    }
    *out = ix;
    return SPC_OK;
}

}  // namespace spc
