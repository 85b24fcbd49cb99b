// SPC queries over the finished index (Eq. con:spc1 and con:spc2) and label
// export, gfx950.
//
// A query (s, t) joins the hub-sorted labels L(s) and L(t): the common hubs
// with the least d_s + d_t form H, and the answer is the saturating sum of
// count_s * count_t over H.  One wave per query: L(s) is staged in LDS a
// slice at a time and the part of L(t) in the slice's hub range is streamed
// past it, several tiles per round of loads, each entry binary-searched in
// LDS.  The loads of a round are independent, so a query waits for a few
// memory round trips per slice rather than one per tile.
//
// On an index with the 1-shell cut off, s and t are first mapped to their
// roots: equal roots leave the tree path as the only shortest path; other
// roots are joined as above and the two depths added.  On an index reduced
// by neighbourhood equivalence they are mapped to their classes'
// representatives: two members of one class are answered from the class
// alone, others by the join of the representatives, where a common hub
// inside the path counts once per member of its class.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <mutex>

#include <type_traits>

#include "spc_internal.h"

// Scratch of spc_query_batch_multi_noalloc: the bucket permutation of at
// most kNoAllocQueries queries, then the two bucket counters.  One copy per
// GPU, resident while the library is loaded.  Host code reaches it only
// through the address hipGetSymbolAddress returns for the device.
constexpr uint64_t kNoAllocQueries = 1ull << 22;
static __device__ __align__(256) uint32_t scratch[kNoAllocQueries + 64];

namespace spc {

namespace {

// queries bucketed per pass (perm entries of spc_query_batch_multi's scratch)
constexpr uint64_t kMultiChunk = 1ull << 24;

struct QueryArgs {
    const uint64_t *lab_off;
    const void *lab_hd;
    const uint64_t *lab_cnt;
    const uint32_t *rank_of;
    const uint32_t *s, *t;
    uint64_t nq;
    uint32_t vbase, gn;     // graph view
    uint32_t cap;           // round cap of a truncated index, 0 otherwise
    // 1-shell (null when not reduced): per input vertex, core id of the
    // root, depth, parent; the graph's input vertex range
    const uint32_t *red_root, *red_depth, *red_parent;
    uint32_t obase, on;
    // neighbourhood equivalence (null otherwise): class size per hub (rank
    // space); per input vertex the answer for two members of its class
    const uint32_t *hub_w, *red_same;
    void *dist_out;
    uint64_t *count_out;
    uint8_t *flags_out;
    // queries that name their graph (null: every query is on the graph
    // view above): graph id per query, and per graph (vbase, gn, obase, on)
    const uint32_t *gid;
    const uint32_t *g_tab;
    uint32_t ngraphs;
    // bucketed launches: this launch answers queries perm[i] (back: perm[nq
    // - 1 - i]) for i < *cnt; perm null: queries 0 .. nq-1
    const uint32_t *perm;
    const uint32_t *cnt;
    bool back;
    // directed index: t's row is its in-label, t_row past its out-label
    uint32_t t_row;
};

// neighbouring workgroups of a query launch kept on one XCD (k_query)
constexpr uint32_t kXcdRun = 16;

// kQStage: L(s) entries staged per query; kQTiles: L(t) tiles of G entries
// requested together; G: lanes per query (64: one query per wave, fewer:
// several queries per wave for short labels).  The triple is a launch
// configuration (see kQueryCfg).  DB: label distance bits; OB: output
// distance bits; RED: the index was built with a reduction (the plain
// instances carry none of its code).
template <int DB, int OB, bool RED, uint32_t kQStage, int kQTiles, int G>
__global__ __launch_bounds__(kBlock) void k_query(QueryArgs a) {
    using E = typename Ent<DB>::T;
    using DT = typename std::conditional<OB == 8, uint8_t, uint16_t>::type;
    static_assert(G == 64 || G == 32 || G == 16, "lanes per query");
    constexpr bool kWave = G == 64;  // one query per wave: uniform values in scalar registers
    __shared__ E stage[kBlock / G][kQStage];
    // Workgroups go to the 8 XCDs in turn; within every 8 kXcdRun
    // consecutive blocks, XCD x takes the kXcdRun neighbouring ones from
    // x kXcdRun, so that the neighbouring queries of an ordered batch (which
    // share their staged label) meet in one L2 while the XCDs still share
    // the batch evenly (a block past the last whole span keeps its index).
    constexpr uint32_t span = 8 * kXcdRun;
    const uint32_t b0 = blockIdx.x / span * span;
    const uint32_t bk = b0 + span <= gridDim.x
                            ? b0 + (blockIdx.x % 8) * kXcdRun + ((blockIdx.x / 8) % kXcdRun)
                            : blockIdx.x;
    const uint64_t q = ((uint64_t)bk * kBlock + threadIdx.x) / G;
    const uint64_t nq = a.cnt ? (uint64_t)*a.cnt : a.nq;
    if (q >= nq) return;
    const uint32_t lane = threadIdx.x & (G - 1);
    // this query's lanes within the wave
    const uint64_t gmask = kWave ? ~0ull : (((1ull << G) - 1) << ((threadIdx.x & 63) & ~(uint32_t)(G - 1)));
    E *st = stage[threadIdx.x / G];
    const E *hd = static_cast<const E *>(a.lab_hd);
    auto uni = [](uint32_t x) -> uint32_t { return kWave ? __builtin_amdgcn_readfirstlane(x) : x; };
    const uint64_t qi = a.perm ? a.perm[a.back ? a.nq - 1 - q : q] : q;
    uint32_t vbase = a.vbase, gn = a.gn, obase = a.obase, on = a.on;
    bool bad = false;
    if (a.gid) {
        const uint32_t g = uni(a.gid[qi]);
        if (g < a.ngraphs) {
            vbase = uni(a.g_tab[4 * g]);
            gn = uni(a.g_tab[4 * g + 1]);
            obase = uni(a.g_tab[4 * g + 2]);
            on = uni(a.g_tab[4 * g + 3]);
        } else {
            bad = true;
        }
    }
    const uint32_t s = uni(a.s[qi]), t = uni(a.t[qi]);
    const DT kInf = (DT)~(DT)0;
    const uint32_t lim = RED ? on : gn;
    if (bad || s >= lim || t >= lim) {
        if (lane == 0) {
            static_cast<DT *>(a.dist_out)[qi] = kInf;
            a.count_out[qi] = 0;
            if (a.flags_out) a.flags_out[qi] = SPC_FLAG_INVALID;
        }
        return;
    }
    uint32_t rs, rt, extra = 0;
    if constexpr (RED) {
        const uint32_t gs = obase + s, gt = obase + t;
        const uint32_t cs = a.red_root[gs], ct = a.red_root[gt];
        if (cs == ct && a.red_same) {
            // one class: the same vertex (0, 1); adjacent twins (1, 1);
            // others share all k neighbours: (2, k), unreachable when k = 0
            if (lane == 0) {
                const uint32_t k = a.red_same[gs];
                DT dd = 0;
                uint64_t cc = 1;
                uint8_t fl = 0;
                if (s != t) {
                    if (k == 0xFFFFFFFFu) {
                        dd = 1;
                    } else if (k == 0) {
                        dd = kInf;
                        cc = 0;
                        fl = SPC_FLAG_UNREACHABLE;
                    } else {
                        dd = 2;
                        cc = k;
                    }
                }
                static_cast<DT *>(a.dist_out)[qi] = dd;
                a.count_out[qi] = cc;
                if (a.flags_out) a.flags_out[qi] = fl;
            }
            return;
        }
        if (cs == ct) {
            // one tree: climb to the lowest common ancestor (every step
            // lowers the depth by one, so the walk ends by depth 0)
            if (lane == 0) {
                uint32_t x = gs, y = gt, dx = a.red_depth[gs], dy = a.red_depth[gt];
                const uint32_t tot = dx + dy;
                for (; dx > dy; dx--) x = a.red_parent[x];
                for (; dy > dx; dy--) y = a.red_parent[y];
                for (; x != y && dx > 0; dx--) {
                    x = a.red_parent[x];
                    y = a.red_parent[y];
                }
                static_cast<DT *>(a.dist_out)[qi] = (DT)(tot - 2 * dx);
                a.count_out[qi] = 1;
                if (a.flags_out) a.flags_out[qi] = 0;
            }
            return;
        }
        extra = uni(a.red_depth[gs] + a.red_depth[gt]);
        rs = uni(a.rank_of[cs]);
        rt = uni(a.rank_of[ct]);
    } else {
        rs = uni(a.rank_of[vbase + s]);
        rt = uni(a.rank_of[vbase + t]) + a.t_row;
    }
    uint64_t as = a.lab_off[rs], na = a.lab_off[rs + 1] - as;
    uint64_t bs = a.lab_off[rt], nb = a.lab_off[rt + 1] - bs;
    // an undirected query is symmetric: the longer label is the staged one
    // (the binary searches in the stage are per streamed entry)
    if (a.t_row == 0 && na < nb) {
        const uint64_t x = as, y = na;
        as = bs;
        na = nb;
        bs = x;
        nb = y;
    }
    uint32_t best = 0xFFFFFFFFu;
    uint64_t sum = 0;
    uint64_t ia = 0, ib = 0;
    // L(s) is taken kQStage entries at a time into LDS (one round of
    // independent loads); the entries of L(t) whose hubs fall in the staged
    // hub range are streamed kQTiles tiles at a time and each is binary-
    // searched in the staged part.  Hub ranges of consecutive stages abut,
    // so every common hub is met exactly once.
    E eb[kQTiles];
    auto load_tiles = [&]() {
#pragma unroll
        for (int j = 0; j < kQTiles; j++) {
            const uint64_t i = ib + (uint64_t)j * G + lane;
            eb[j] = i < nb ? hd[bs + i] : (E)~(E)0;
        }
    };
    while (ia < na && ib < nb) {
        const uint32_t cnt = (uint32_t)((na - ia) < kQStage ? (na - ia) : kQStage);
        // the slice of L(s) and the first tiles of L(t) are requested
        // together (the tiles do not depend on the slice)
        E sv[kQStage / G];
#pragma unroll
        for (uint32_t j = 0; j < kQStage / G; j++) {
            const uint32_t k = j * G + lane;
            sv[j] = k < cnt ? hd[as + ia + k] : (E)0;
        }
        E nxt = (E)~(E)0;
        if (lane == 0 && ia + cnt < na) nxt = hd[as + ia + cnt];
        load_tiles();
#pragma unroll
        for (uint32_t j = 0; j < kQStage / G; j++) {
            const uint32_t k = j * G + lane;
            if (k < cnt) st[k] = sv[j];
        }
        wave_lds_sync();
        // staged hubs are [first, hub_hi): up to the next stage's first hub
        const uint32_t hub_hi = (ia + cnt < na) ? e_hub<DB>((E)__shfl(nxt, 0, G))
                                                : e_hub<DB>(st[cnt - 1]) + 1;
        bool more = true, first = true;
        while (more && ib < nb) {
            if (!first) load_tiles();
            first = false;
            uint32_t pos[kQTiles];
            bool in[kQTiles];
            uint32_t n_in = 0;
#pragma unroll
            for (int j = 0; j < kQTiles; j++) {
                const uint64_t i = ib + (uint64_t)j * G + lane;
                in[j] = i < nb && e_hub<DB>(eb[j]) < hub_hi;
                n_in += (uint32_t)__popcll(__ballot(in[j]) & gmask);
                pos[j] = 0;
            }
            // lower bound of each streamed hub among the staged hubs; the
            // searches of a lane's tiles interleave
            for (uint32_t step = kQStage / 2; step > 0; step >>= 1) {
#pragma unroll
                for (int j = 0; j < kQTiles; j++) {
                    const uint32_t c = pos[j] + step;
                    if (in[j] && c <= cnt && e_hub<DB>(st[c - 1]) < e_hub<DB>(eb[j])) pos[j] = c;
                }
            }
            uint32_t dd[kQTiles];
            uint32_t gmin = best;
#pragma unroll
            for (int j = 0; j < kQTiles; j++) {
                dd[j] = 0xFFFFFFFFu;
                if (in[j] && pos[j] < cnt && e_hub<DB>(st[pos[j]]) == e_hub<DB>(eb[j]))
                    dd[j] = e_dist<DB>(st[pos[j]]) + e_dist<DB>(eb[j]);
                gmin = dd[j] < gmin ? dd[j] : gmin;
            }
            // counts of this lane's matches at its least distance, loaded
            // together
            if (gmin != 0xFFFFFFFFu && gmin <= best) {
                uint64_t cs[kQTiles], ct[kQTiles];
#pragma unroll
                for (int j = 0; j < kQTiles; j++) {
                    cs[j] = 0;
                    ct[j] = 0;
                    if (dd[j] == gmin) {
                        cs[j] = a.lab_cnt[as + ia + pos[j]];
                        ct[j] = a.lab_cnt[bs + ib + (uint64_t)j * G + lane];
                        // a hub other than s and t lies inside the path
                        if (RED && a.hub_w) {
                            const uint32_t h = e_hub<DB>(eb[j]);
                            if (h != rs && h != rt) ct[j] = sat_mul(ct[j], a.hub_w[h]);
                        }
                    }
                }
                if (gmin < best) {
                    sum = 0;
                    best = gmin;
                }
#pragma unroll
                for (int j = 0; j < kQTiles; j++)
                    if (dd[j] == gmin) sum = sat_add(sum, sat_mul(cs[j], ct[j]));
            }
            // L(t) is sorted: the in-range entries are a prefix
            ib += n_in;
            more = n_in == (uint32_t)(kQTiles * G);
        }
        ia += cnt;
        wave_lds_sync();  // the stage is rewritten next
    }
    // reduction over the query's lanes: least distance, then the saturating
    // sum at it
    uint32_t mn = best;
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) mn = min(mn, (uint32_t)__shfl_xor(mn, o, G));
    uint64_t part = (best == mn) ? sum : 0;
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) part = sat_add(part, __shfl_xor(part, o, G));
    if (lane == 0) {
        uint8_t fl = 0;
        DT dout;
        uint64_t cout;
        if (mn == 0xFFFFFFFFu) {
            dout = kInf;
            cout = 0;
            fl |= SPC_FLAG_UNREACHABLE;
            if (a.cap) fl |= SPC_FLAG_HORIZON;
        } else {
            dout = (DT)(mn + extra);
            cout = part;
            if (part == kSat) fl |= SPC_FLAG_SATURATED;
            if (a.cap && mn > a.cap) fl |= SPC_FLAG_HORIZON;
        }
        static_cast<DT *>(a.dist_out)[qi] = dout;
        a.count_out[qi] = cout;
        if (a.flags_out) a.flags_out[qi] = fl;
    }
}

// Locality order of a large batch: the queries grouped by the label row the
// query kernel stages (the longer label of an undirected query, L(s) of a
// directed one), so that the queries sharing it run side by side and find it
// in cache.  A counting sort: row[q] and per-row counts, their exclusive
// scan, then each query at its row's next slot (the order within a row is
// arbitrary: answers are written by query index).  Invalid queries go to
// row 0.  Single-graph launches (no gid).
__global__ void k_qrow(QueryArgs a, uint32_t *row, uint32_t *cnt) {
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < a.nq;
         q += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t s = a.s[q], t = a.t[q];
        const uint32_t lim = a.red_root ? a.on : a.gn;
        uint32_t r = 0;
        if (s < lim && t < lim) {
            uint32_t rs, rt;
            if (a.red_root) {
                rs = a.rank_of[a.red_root[a.obase + s]];
                rt = a.rank_of[a.red_root[a.obase + t]];
            } else {
                rs = a.rank_of[a.vbase + s];
                rt = a.rank_of[a.vbase + t] + a.t_row;
            }
            const uint64_t na = a.lab_off[rs + 1] - a.lab_off[rs];
            const uint64_t nb = a.lab_off[rt + 1] - a.lab_off[rt];
            r = (a.t_row == 0 && na < nb) ? rt : rs;
        }
        row[q] = r;
        atomicAdd(&cnt[r], 1u);
    }
}
__global__ void k_qplace(const uint32_t *row, uint64_t nq, uint64_t *next, uint32_t *perm) {
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq;
         q += (uint64_t)gridDim.x * blockDim.x)
        perm[atomicAdd((unsigned long long *)&next[row[q]], 1ull)] = (uint32_t)q;
}
__global__ void k_qfill0(uint32_t *p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Bucketing of a query batch by its work, |L(s)| + |L(t)|: queries at most
// `small` go to the front of perm (answered G < 64 lanes each), the others
// to the back (a wave each).  cnt[0] counts the front, cnt[1] the back;
// both start at zero.  The order within a bucket is arbitrary (answers are
// written by query index).
__global__ void k_qbucket(QueryArgs a, uint32_t small, uint32_t *perm, uint32_t *cnt) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.nq) return;
    uint32_t vbase = a.vbase, gn = a.gn, obase = a.obase, on = a.on;
    bool big = false;
    if (a.gid) {
        const uint32_t g = a.gid[q];
        if (g < a.ngraphs) {
            vbase = a.g_tab[4 * g];
            gn = a.g_tab[4 * g + 1];
            obase = a.g_tab[4 * g + 2];
            on = a.g_tab[4 * g + 3];
        } else {
            gn = on = 0;  // invalid: answered at once by either kernel
        }
    }
    const uint32_t s = a.s[q], t = a.t[q];
    const uint32_t lim = a.red_root ? on : gn;
    if (s < lim && t < lim) {
        uint32_t rs, rt;
        if (a.red_root) {
            rs = a.rank_of[a.red_root[obase + s]];
            rt = a.rank_of[a.red_root[obase + t]];
        } else {
            rs = a.rank_of[vbase + s];
            rt = a.rank_of[vbase + t] + a.t_row;
        }
        const uint64_t w = (a.lab_off[rs + 1] - a.lab_off[rs]) + (a.lab_off[rt + 1] - a.lab_off[rt]);
        big = w > small;
    }
    if (big)
        perm[a.nq - 1 - atomicAdd(&cnt[1], 1u)] = (uint32_t)q;
    else
        perm[atomicAdd(&cnt[0], 1u)] = (uint32_t)q;
}

__global__ void k_qzero(uint32_t *cnt, uint32_t n) {
    if (threadIdx.x < n) cnt[threadIdx.x] = 0;
}

// Export kernels: labels of one graph, rank space of that graph.
__global__ void k_export_off(const uint64_t *lab_off, uint32_t vbase, uint32_t n, uint64_t *off) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) off[i] = lab_off[vbase + i] - lab_off[vbase];
}
template <int DB>
__global__ void k_export_ent(const typename Ent<DB>::T *hd, const uint64_t *cnt, uint64_t e0,
                             uint64_t ne, uint32_t vbase, uint32_t *hub, uint16_t *dist,
                             uint64_t *count) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    auto e = hd[e0 + i];
    if (hub) hub[i] = e_hub<DB>(e) - vbase;
    if (dist) dist[i] = (uint16_t)e_dist<DB>(e);
    if (count) count[i] = cnt[e0 + i];
}
// rank -> vertex id of the graph; through core -> input ids when reduced
__global__ void k_export_order(const uint32_t *order, uint32_t vbase, uint32_t n,
                               const uint32_t *core_vid, uint32_t obase, uint32_t *out) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = core_vid ? core_vid[order[vbase + i]] - obase : order[vbase + i] - vbase;
}
// the 1-shell of one graph in its input ids (identity when not reduced)
__global__ void k_export_shell(const uint32_t *root, const uint32_t *depth, const uint32_t *parent,
                               const uint32_t *core_vid, uint32_t obase, uint32_t n, uint32_t *root_out,
                               uint32_t *depth_out, uint32_t *parent_out) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t v = obase + i;
    if (root_out) root_out[i] = root ? core_vid[root[v]] - obase : i;
    if (depth_out) depth_out[i] = depth ? depth[v] : 0;
    if (parent_out) parent_out[i] = parent ? parent[v] - obase : i;
}

inline uint32_t grid1(uint64_t items) { return (uint32_t)((items + kBlock - 1) / kBlock); }

// Query launch configurations (staged L(s) entries, L(t) tiles per round of
// loads); spc_tune_queries picks one per index by timing them all.
struct QueryCfg {
    uint32_t stage, tiles;
};
constexpr QueryCfg kQueryCfg[] = {{512, 2}, {512, 1}, {512, 4}, {256, 1}, {256, 2},
                                  {1024, 1}, {1024, 2}, {2048, 1}};
constexpr uint32_t kQueryCfgs = sizeof(kQueryCfg) / sizeof(kQueryCfg[0]);

template <int DB, int OB, bool RED>
void launch_cfg(uint32_t cfg, dim3 g, hipStream_t st, const QueryArgs &c) {
    switch (cfg) {
        case 1: hipLaunchKernelGGL((k_query<DB, OB, RED, 512, 1, 64>), g, dim3(kBlock), 0, st, c); break;
        case 2: hipLaunchKernelGGL((k_query<DB, OB, RED, 512, 4, 64>), g, dim3(kBlock), 0, st, c); break;
        case 3: hipLaunchKernelGGL((k_query<DB, OB, RED, 256, 1, 64>), g, dim3(kBlock), 0, st, c); break;
        case 4: hipLaunchKernelGGL((k_query<DB, OB, RED, 256, 2, 64>), g, dim3(kBlock), 0, st, c); break;
        case 5: hipLaunchKernelGGL((k_query<DB, OB, RED, 1024, 1, 64>), g, dim3(kBlock), 0, st, c); break;
        case 6: hipLaunchKernelGGL((k_query<DB, OB, RED, 1024, 2, 64>), g, dim3(kBlock), 0, st, c); break;
        case 7: hipLaunchKernelGGL((k_query<DB, OB, RED, 2048, 1, 64>), g, dim3(kBlock), 0, st, c); break;
        default: hipLaunchKernelGGL((k_query<DB, OB, RED, 512, 2, 64>), g, dim3(kBlock), 0, st, c); break;
    }
}
// short labels: 16 lanes per query (16 queries per workgroup), L(s) staged
// 128 entries at a time, L(t) streamed two 16-entry tiles per round
constexpr int kSmallG = 16;
template <int DB, int OB, bool RED>
void launch_small(dim3 g, hipStream_t st, const QueryArgs &c) {
    hipLaunchKernelGGL((k_query<DB, OB, RED, 128, 2, kSmallG>), g, dim3(kBlock), 0, st, c);
}
template <int DB, int OB>
void launch_red(uint32_t cfg, bool small, dim3 g, hipStream_t st, const QueryArgs &c) {
    if (small) {
        if (c.red_root)
            launch_small<DB, OB, true>(g, st, c);
        else
            launch_small<DB, OB, false>(g, st, c);
    } else if (c.red_root) {
        launch_cfg<DB, OB, true>(cfg, g, st, c);
    } else {
        launch_cfg<DB, OB, false>(cfg, g, st, c);
    }
}

// 16-bit labels always come with 16-bit outputs.  Work-items of a launch:
// nq * (lanes per query), kept below 2^32 by the callers' chunks.
spc_status launch_query(uint32_t dist_bits, uint32_t out_bits, uint32_t cfg, const QueryArgs &c,
                        hipStream_t st, bool small = false) {
    const uint64_t per_block = small ? kBlock / kSmallG : kWaves;
    const dim3 g((uint32_t)((c.nq + per_block - 1) / per_block));
    if (dist_bits == 16)
        launch_red<16, 16>(cfg, small, g, st, c);
    else if (out_bits == 16)
        launch_red<8, 16>(cfg, small, g, st, c);
    else
        launch_red<8, 8>(cfg, small, g, st, c);
    SPC_LAUNCHED();
    return SPC_OK;
}

// The index's arrays in the arguments of a query launch.
QueryArgs index_args(const spc_index *ix) {
    QueryArgs a = {};
    a.lab_off = ix->lab_off;
    a.lab_hd = ix->lab_hd;
    a.lab_cnt = ix->lab_cnt;
    a.rank_of = ix->rank_of;
    a.cap = ix->truncated ? ix->round_cap : 0;
    a.red_root = ix->reduced ? ix->red_root : nullptr;
    a.red_depth = ix->red_depth;
    a.red_parent = ix->red_parent;
    a.hub_w = ix->hub_w;
    a.red_same = ix->red_same;
    a.t_row = ix->nreal;
    return a;
}

}  // namespace

namespace {

__global__ void k_same(const uint8_t *a, const uint8_t *b, uint64_t n, unsigned int *diff) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        if (a[i] != b[i]) atomicOr(diff, 1u);
}

spc_status query_run(const spc_index *ix, uint32_t graph_id, const uint32_t *s, const uint32_t *t,
                     uint64_t nq, void *dist_out, uint64_t *count_out, uint8_t *flags_out,
                     uint32_t cfg, hipStream_t st);

// batches of at least this many queries are answered in locality order
// (k_qrow) unless SPC_QUERY_ORDER=0 in the environment
constexpr uint64_t kOrderMin = 1ull << 20;

bool order_enabled() {
    const char *eo = std::getenv("SPC_QUERY_ORDER");
    return !(eo && eo[0] == '0');
}

// A batch answered in locality order with configuration cfg.
spc_status query_ordered(const spc_index *ix, uint32_t graph_id, const uint32_t *s, const uint32_t *t,
                         uint64_t nq, void *dist_out, uint64_t *count_out, uint8_t *flags_out,
                         uint32_t cfg, hipStream_t st) {
    if (nq == 0) return SPC_OK;
    if (graph_id >= ix->gn.size()) return SPC_ERR_INVALID_ARG;
    if (!s || !t || !dist_out || !count_out) return SPC_ERR_INVALID_ARG;
    QueryArgs a = index_args(ix);
    a.vbase = ix->vbase[graph_id];
    a.gn = ix->gn[graph_id];
    a.obase = ix->reduced ? ix->obase[graph_id] : 0;
    a.on = ix->reduced ? ix->on[graph_id] : 0;
    // scratch in stream order, freed after the launches that read it:
    // row and perm per query, counts and offsets per label row, scan space
    const uint64_t rows = (uint64_t)ix->n + ix->nreal;
    const uint64_t np = std::min<uint64_t>(nq, kMultiChunk);
    const uint64_t wse = scan_ws_elems(rows + 1);
    const uint64_t bytes = (2 * np + rows + 64) * sizeof(uint32_t) + (rows + 1 + wse + 8) * sizeof(uint64_t);
    void *buf = nullptr;
    if (hipMallocAsync(&buf, bytes, st) != hipSuccess) return SPC_ERR_OUT_OF_MEMORY;
    uint64_t *next = static_cast<uint64_t *>(buf);
    uint64_t *ws = next + rows + 1;
    uint32_t *cnt = reinterpret_cast<uint32_t *>(ws + wse + 8);
    uint32_t *row = cnt + rows;
    uint32_t *perm = row + np;
    const size_t dsz = ix->out_bits == 8 ? 1 : 2;
    spc_status r = SPC_OK;
    for (uint64_t q0 = 0; q0 < nq && r == SPC_OK; q0 += kMultiChunk) {
        const uint64_t nc = std::min<uint64_t>(kMultiChunk, nq - q0);
        QueryArgs c = a;
        c.s = s + q0;
        c.t = t + q0;
        c.nq = nc;
        c.dist_out = static_cast<char *>(dist_out) + q0 * dsz;
        c.count_out = count_out + q0;
        c.flags_out = flags_out ? flags_out + q0 : nullptr;
        const uint32_t gq = std::min<uint32_t>(grid1(nc), 8192);
        hipLaunchKernelGGL(k_qfill0, dim3(std::min<uint32_t>(grid1(rows), 4096)), dim3(kBlock), 0, st, cnt,
                           rows);
        hipLaunchKernelGGL(k_qrow, dim3(gq), dim3(kBlock), 0, st, c, row, cnt);
        if (hipGetLastError() != hipSuccess) {
            r = SPC_ERR_DEVICE;
            break;
        }
        r = scan_u32(cnt, next, rows, ws, st);
        if (r != SPC_OK) break;
        hipLaunchKernelGGL(k_qplace, dim3(gq), dim3(kBlock), 0, st, row, nc, next, perm);
        if (hipGetLastError() != hipSuccess) {
            r = SPC_ERR_DEVICE;
            break;
        }
        c.perm = perm;
        r = launch_query(ix->dist_bits, ix->out_bits, cfg, c, st);
    }
    if (hipFreeAsync(buf, st) != hipSuccess && r == SPC_OK) r = SPC_ERR_DEVICE;
    return r;
}

}  // namespace

spc_status query_impl(const spc_index *ix, uint32_t graph_id, const uint32_t *s, const uint32_t *t,
                      uint64_t nq, void *dist_out, uint64_t *count_out, uint8_t *flags_out,
                      hipStream_t st) {
    if (!ix) return SPC_ERR_INVALID_ARG;
    if (nq < kOrderMin || !order_enabled())
        return query_run(ix, graph_id, s, t, nq, dist_out, count_out, flags_out, ix->query_cfg, st);
    return query_ordered(ix, graph_id, s, t, nq, dist_out, count_out, flags_out, ix->query_cfg, st);
}

spc_status query_multi_impl(const spc_index *ix, const uint32_t *gid, const uint32_t *s,
                            const uint32_t *t, uint64_t nq, void *dist_out, uint64_t *count_out,
                            uint8_t *flags_out, hipStream_t st) {
    if (!ix) return SPC_ERR_INVALID_ARG;
    if (nq == 0) return SPC_OK;
    if (!s || !t || !dist_out || !count_out) return SPC_ERR_INVALID_ARG;
    if (ix->query_small == 0)
        return query_multi_run(ix, gid, s, t, nq, dist_out, count_out, flags_out, nullptr, nullptr, 0,
                               ix->query_cfg, st);
    // scratch in stream order: freed after the launches that read it
    const uint64_t np = std::min<uint64_t>(nq, kMultiChunk);
    void *buf = nullptr;
    if (hipMallocAsync(&buf, (np + 64) * sizeof(uint32_t), st) != hipSuccess) return SPC_ERR_OUT_OF_MEMORY;
    uint32_t *perm = static_cast<uint32_t *>(buf);
    spc_status r = query_multi_run(ix, gid, s, t, nq, dist_out, count_out, flags_out, perm, perm + np,
                                   ix->query_small, ix->query_cfg, st);
    if (hipFreeAsync(buf, st) != hipSuccess && r == SPC_OK) r = SPC_ERR_DEVICE;
    return r;
}

// Bucket thresholds the tuner times (0: no bucketing).
constexpr uint32_t kSmallChoices[] = {0, 64, 128, 256, 512, 1024, 2048};

spc_status tune_query_buckets_impl(spc_index *ix, const uint32_t *gid, const uint32_t *s,
                                   const uint32_t *t, uint64_t nq, hipStream_t st, uint32_t *small_out) {
    if (!ix || !s || !t || nq == 0 || ix->gn.empty()) return SPC_ERR_INVALID_ARG;
    const size_t dsz = ix->out_bits == 8 ? 1 : 2;
    const uint64_t per = (nq * (dsz + 8 + 1) + 255) & ~uint64_t(255);
    const uint64_t np = std::min<uint64_t>(nq, kMultiChunk);
    Arena tmp(0, st);
    uint8_t *buf = nullptr;
    unsigned int *diff = nullptr;
    uint32_t *perm = nullptr;
    SPC_TRY(tmp.alloc(&buf, 2 * per + 16));
    SPC_TRY(tmp.alloc(&diff, 1));
    SPC_TRY(tmp.alloc(&perm, np + 64));
    auto outs = [&](int side, void **d, uint64_t **c, uint8_t **f) {
        uint8_t *b = buf + side * per;
        *c = reinterpret_cast<uint64_t *>(b);
        *d = b + nq * 8;
        *f = b + nq * (8 + dsz);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SPC_HIP(hipEventCreate(&e0));
    SPC_HIP(hipEventCreate(&e1));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } guard{e0, e1};
    float best_ms = 0;
    uint32_t best = ix->query_small;
    bool first = true;
    for (uint32_t small : kSmallChoices) {
        void *d;
        uint64_t *c;
        uint8_t *f;
        outs(first ? 0 : 1, &d, &c, &f);
        float ms = 0;
        for (int rep = 0; rep < 2; rep++) {  // the first run warms caches
            SPC_HIP(hipEventRecord(e0, st));
            SPC_TRY(query_multi_run(ix, gid, s, t, nq, d, c, f, perm, perm + np, small, ix->query_cfg, st));
            SPC_HIP(hipEventRecord(e1, st));
            SPC_HIP(hipEventSynchronize(e1));
            SPC_HIP(hipEventElapsedTime(&ms, e0, e1));
        }
        if (!first) {  // every threshold must give the same answers
            SPC_HIP(hipMemsetAsync(diff, 0, sizeof(unsigned int), st));
            const uint64_t used = nq * (dsz + 8 + 1);
            hipLaunchKernelGGL(k_same, dim3(grid1(used) < 4096 ? grid1(used) : 4096), dim3(kBlock), 0, st,
                               buf, buf + per, used, diff);
            SPC_LAUNCHED();
            unsigned int h = 0;
            SPC_HIP(hipMemcpyAsync(&h, diff, sizeof(h), hipMemcpyDeviceToHost, st));
            SPC_HIP(hipStreamSynchronize(st));
            if (h) return SPC_ERR_DEVICE;
        }
        if (first || ms < best_ms) {
            best_ms = ms;
            best = small;
        }
        first = false;
    }
    ix->query_small = best;
    if (small_out) *small_out = best;
    return SPC_OK;
}

uint32_t query_cfg_count() { return kQueryCfgs; }

spc_status query_cfg_info(uint32_t cfg, uint32_t *stage, uint32_t *tiles) {
    if (cfg >= kQueryCfgs) return SPC_ERR_INVALID_ARG;
    if (stage) *stage = kQueryCfg[cfg].stage;
    if (tiles) *tiles = kQueryCfg[cfg].tiles;
    return SPC_OK;
}

spc_status tune_queries_impl(spc_index *ix, uint32_t graph_id, const uint32_t *s, const uint32_t *t,
                             uint64_t nq, hipStream_t st, uint32_t *cfg_out) {
    if (!ix || graph_id >= ix->gn.size() || !s || !t || nq == 0) return SPC_ERR_INVALID_ARG;
    const size_t dsz = ix->out_bits == 8 ? 1 : 2;
    // one output set per side of the comparison, in one block:
    // dist | count | flags, reference then candidate
    const uint64_t per = (nq * (dsz + 8 + 1) + 255) & ~uint64_t(255);
    Arena tmp(0, st);
    uint8_t *buf = nullptr;
    unsigned int *diff = nullptr;
    SPC_TRY(tmp.alloc(&buf, 2 * per + 16));
    SPC_TRY(tmp.alloc(&diff, 1));
    auto outs = [&](int side, void **d, uint64_t **c, uint8_t **f) {
        uint8_t *b = buf + side * per;
        *c = reinterpret_cast<uint64_t *>(b);  // counts first: 8-byte aligned
        *d = b + nq * 8;
        *f = b + nq * (8 + dsz);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SPC_HIP(hipEventCreate(&e0));
    SPC_HIP(hipEventCreate(&e1));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } guard{e0, e1};
    float best_ms = 0;
    uint32_t best = ix->query_cfg;
    for (uint32_t cfg = 0; cfg < kQueryCfgs; cfg++) {
        void *d;
        uint64_t *c;
        uint8_t *f;
        outs(cfg == 0 ? 0 : 1, &d, &c, &f);
        float ms = 0;
        for (int rep = 0; rep < 2; rep++) {  // the first run warms caches
            SPC_HIP(hipEventRecord(e0, st));
            // the path large batches take
            if (order_enabled())
                SPC_TRY(query_ordered(ix, graph_id, s, t, nq, d, c, f, cfg, st));
            else
                SPC_TRY(query_run(ix, graph_id, s, t, nq, d, c, f, cfg, st));
            SPC_HIP(hipEventRecord(e1, st));
            SPC_HIP(hipEventSynchronize(e1));
            SPC_HIP(hipEventElapsedTime(&ms, e0, e1));
        }
        if (cfg > 0) {  // every configuration must give the same answers
            SPC_HIP(hipMemsetAsync(diff, 0, sizeof(unsigned int), st));
            const uint64_t used = nq * (dsz + 8 + 1);  // the padding is not compared
            hipLaunchKernelGGL(k_same, dim3(grid1(used) < 4096 ? grid1(used) : 4096), dim3(kBlock), 0, st,
                               buf, buf + per, used, diff);
            SPC_LAUNCHED();
            unsigned int h = 0;
            SPC_HIP(hipMemcpyAsync(&h, diff, sizeof(h), hipMemcpyDeviceToHost, st));
            SPC_HIP(hipStreamSynchronize(st));
            if (h) return SPC_ERR_DEVICE;
        }
        if (cfg == 0 || ms < best_ms) {
            best_ms = ms;
            best = cfg;
        }
    }
    ix->query_cfg = best;
    if (cfg_out) *cfg_out = best;
    return SPC_OK;
}

namespace {

spc_status query_run(const spc_index *ix, uint32_t graph_id, const uint32_t *s, const uint32_t *t,
                     uint64_t nq, void *dist_out, uint64_t *count_out, uint8_t *flags_out,
                     uint32_t cfg, hipStream_t st) {
    if (graph_id >= ix->gn.size()) return SPC_ERR_INVALID_ARG;
    if (nq == 0) return SPC_OK;
    if (!s || !t || !dist_out || !count_out) return SPC_ERR_INVALID_ARG;
    QueryArgs a = index_args(ix);
    a.s = s;
    a.t = t;
    a.nq = nq;
    a.vbase = ix->vbase[graph_id];
    a.gn = ix->gn[graph_id];
    a.obase = ix->reduced ? ix->obase[graph_id] : 0;
    a.on = ix->reduced ? ix->on[graph_id] : 0;
    a.dist_out = dist_out;
    a.count_out = count_out;
    a.flags_out = flags_out;
    // one wave per query: launches of at most 2^24 queries keep the
    // work-item count of each below 2^32
    constexpr uint64_t kChunk = 1ull << 24;
    const size_t dsz = ix->out_bits == 8 ? 1 : 2;
    for (uint64_t q0 = 0; q0 < nq; q0 += kChunk) {
        const uint64_t nc = std::min(kChunk, nq - q0);
        QueryArgs c = a;
        c.s = s + q0;
        c.t = t + q0;
        c.nq = nc;
        c.dist_out = static_cast<char *>(dist_out) + q0 * dsz;
        c.count_out = count_out + q0;
        c.flags_out = flags_out ? flags_out + q0 : nullptr;
        SPC_TRY(launch_query(ix->dist_bits, ix->out_bits, cfg, c, st));
    }
    return SPC_OK;
}

}  // namespace

// Queries that name their graph (gid null: graph 0), bucketed by the work
// |L(s)| + |L(t)|: up to `small` entries 16 lanes per query, the rest a wave
// each with the index's configuration (small = 0: no bucketing).  perm
// holds min(nq, kMultiChunk) entries and cnt two; both are scratch written
// before they are read, on `st`, so calls sharing them must not overlap.
spc_status query_multi_run(const spc_index *ix, const uint32_t *gid, const uint32_t *s,
                           const uint32_t *t, uint64_t nq, void *dist_out, uint64_t *count_out,
                           uint8_t *flags_out, uint32_t *perm, uint32_t *cnt, uint32_t small,
                           uint32_t cfg, hipStream_t st) {
    if (!ix) return SPC_ERR_INVALID_ARG;
    if (nq == 0) return SPC_OK;
    if (!s || !t || !dist_out || !count_out) return SPC_ERR_INVALID_ARG;
    if (cfg >= kQueryCfgs) return SPC_ERR_INVALID_ARG;
    QueryArgs a = index_args(ix);
    a.gid = gid;
    a.g_tab = ix->g_tab;
    a.ngraphs = (uint32_t)ix->gn.size();
    if (!gid) {  // every query on graph 0
        if (ix->gn.empty()) return SPC_ERR_INVALID_ARG;
        a.vbase = ix->vbase[0];
        a.gn = ix->gn[0];
        a.obase = ix->reduced ? ix->obase[0] : 0;
        a.on = ix->reduced ? ix->on[0] : 0;
    }
    const size_t dsz = ix->out_bits == 8 ? 1 : 2;
    for (uint64_t q0 = 0; q0 < nq; q0 += kMultiChunk) {
        const uint64_t nc = std::min<uint64_t>(kMultiChunk, nq - q0);
        QueryArgs c = a;
        c.s = s + q0;
        c.t = t + q0;
        c.gid = gid ? gid + q0 : nullptr;
        c.nq = nc;
        c.dist_out = static_cast<char *>(dist_out) + q0 * dsz;
        c.count_out = count_out + q0;
        c.flags_out = flags_out ? flags_out + q0 : nullptr;
        if (small == 0) {
            SPC_TRY(launch_query(ix->dist_bits, ix->out_bits, cfg, c, st));
            continue;
        }
        hipLaunchKernelGGL(k_qzero, dim3(1), dim3(64), 0, st, cnt, 2u);
        SPC_LAUNCHED();
        hipLaunchKernelGGL(k_qbucket, dim3(grid1(nc)), dim3(kBlock), 0, st, c, small, perm, cnt);
        SPC_LAUNCHED();
        QueryArgs cs = c, cl = c;
        cs.perm = perm;
        cs.cnt = cnt;
        cs.back = false;
        cl.perm = perm;
        cl.cnt = cnt + 1;
        cl.back = true;
        SPC_TRY(launch_query(ix->dist_bits, ix->out_bits, cfg, cs, st, true));
        SPC_TRY(launch_query(ix->dist_bits, ix->out_bits, cfg, cl, st, false));
    }
    return SPC_OK;
}


spc_status export_impl(const spc_index *ix, uint32_t graph_id, uint64_t *off, uint32_t *hub,
                       uint16_t *dist, uint64_t *count, uint32_t *order, int32_t on_device,
                       hipStream_t st) {
    if (!ix || graph_id >= ix->gn.size()) return SPC_ERR_INVALID_ARG;
    // label rows (twice the vertices of a directed graph); the order has
    // one entry per vertex
    const uint32_t vb = ix->vbase[graph_id], nv = ix->gn[graph_id];
    const uint32_t n = ix->nreal ? 2 * nv : nv;
    uint64_t e0 = 0, e1 = 0;
    SPC_HIP(hipMemcpy(&e0, ix->lab_off + vb, sizeof(uint64_t), hipMemcpyDeviceToHost));
    SPC_HIP(hipMemcpy(&e1, ix->lab_off + vb + n, sizeof(uint64_t), hipMemcpyDeviceToHost));
    const uint64_t ne = e1 - e0;
    // device staging when the destination is host memory
    uint64_t *d_off = off;
    uint32_t *d_hub = hub, *d_ord = order;
    uint16_t *d_dist = dist;
    uint64_t *d_cnt = count;
    Arena tmp(0, st);
    if (!on_device) {
        if (off) SPC_TRY(tmp.alloc(&d_off, (uint64_t)n + 1));
        if (hub) SPC_TRY(tmp.alloc(&d_hub, ne));
        if (dist) SPC_TRY(tmp.alloc(&d_dist, ne));
        if (count) SPC_TRY(tmp.alloc(&d_cnt, ne));
        if (order) SPC_TRY(tmp.alloc(&d_ord, (uint64_t)nv));
    }
    if (off) {
        hipLaunchKernelGGL(k_export_off, dim3(grid1((uint64_t)n + 1)), dim3(kBlock), 0, st,
                           ix->lab_off, vb, n, d_off);
        SPC_LAUNCHED();
    }
    // entries in launches of at most 2^30 (one work-item each)
    constexpr uint64_t kChunk = 1ull << 30;
    for (uint64_t i0 = 0; (hub || dist || count) && i0 < ne; i0 += kChunk) {
        const uint64_t nc = std::min(kChunk, ne - i0);
        uint32_t *h = hub ? d_hub + i0 : nullptr;
        uint16_t *dd = dist ? d_dist + i0 : nullptr;
        uint64_t *cc = count ? d_cnt + i0 : nullptr;
        if (ix->dist_bits == 8)
            hipLaunchKernelGGL(k_export_ent<8>, dim3(grid1(nc)), dim3(kBlock), 0, st,
                               static_cast<const uint32_t *>(ix->lab_hd), ix->lab_cnt, e0 + i0, nc,
                               vb, h, dd, cc);
        else
            hipLaunchKernelGGL(k_export_ent<16>, dim3(grid1(nc)), dim3(kBlock), 0, st,
                               static_cast<const uint64_t *>(ix->lab_hd), ix->lab_cnt, e0 + i0, nc,
                               vb, h, dd, cc);
        SPC_LAUNCHED();
    }
    if (order && nv) {
        hipLaunchKernelGGL(k_export_order, dim3(grid1(nv)), dim3(kBlock), 0, st, ix->order, vb, nv,
                           ix->reduced ? ix->core_vid : nullptr, ix->reduced ? ix->obase[graph_id] : 0,
                           d_ord);
        SPC_LAUNCHED();
    }
    if (!on_device) {
        if (off) SPC_HIP(hipMemcpyAsync(off, d_off, ((uint64_t)n + 1) * 8, hipMemcpyDeviceToHost, st));
        if (hub && ne) SPC_HIP(hipMemcpyAsync(hub, d_hub, ne * 4, hipMemcpyDeviceToHost, st));
        if (dist && ne) SPC_HIP(hipMemcpyAsync(dist, d_dist, ne * 2, hipMemcpyDeviceToHost, st));
        if (count && ne) SPC_HIP(hipMemcpyAsync(count, d_cnt, ne * 8, hipMemcpyDeviceToHost, st));
        if (order && nv) SPC_HIP(hipMemcpyAsync(order, d_ord, (uint64_t)nv * 4, hipMemcpyDeviceToHost, st));
    }
    SPC_HIP(hipStreamSynchronize(st));
    return SPC_OK;
}

spc_status export_reduction_impl(const spc_index *ix, uint32_t graph_id, uint32_t *root,
                                 uint32_t *depth, uint32_t *parent, int32_t on_device, hipStream_t st) {
    if (!ix || graph_id >= ix->gn.size()) return SPC_ERR_INVALID_ARG;
    const uint32_t n = ix->reduced ? ix->on[graph_id] : ix->gn[graph_id];
    const uint32_t ob = ix->reduced ? ix->obase[graph_id] : ix->vbase[graph_id];
    if (n == 0) return SPC_OK;
    uint32_t *d[3] = {root, depth, parent};
    Arena tmp(0, st);
    if (!on_device)
        for (auto &p : d)
            if (p) SPC_TRY(tmp.alloc(&p, n));
    hipLaunchKernelGGL(k_export_shell, dim3(grid1(n)), dim3(kBlock), 0, st,
                       ix->reduced ? ix->red_root : nullptr, ix->reduced ? ix->red_depth : nullptr,
                       ix->reduced ? ix->red_parent : nullptr, ix->core_vid, ob, n, d[0], d[1], d[2]);
    SPC_LAUNCHED();
    if (!on_device) {
        uint32_t *h[3] = {root, depth, parent};
        for (int i = 0; i < 3; i++)
            if (h[i]) SPC_HIP(hipMemcpyAsync(h[i], d[i], (uint64_t)n * 4, hipMemcpyDeviceToHost, st));
    }
    SPC_HIP(hipStreamSynchronize(st));
    return SPC_OK;
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch[kMaxDevices];  // device address of `scratch`, per device

// The device address of `scratch` on device `dev`, looked up once per
// device with that device current.
spc_status scratch_on(int dev, uint32_t **out) {
    if (dev < 0 || dev >= kMaxDevices) return SPC_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        int cur = 0;
        SPC_HIP(hipGetDevice(&cur));
        if (cur != dev) SPC_HIP(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) SPC_HIP(hipSetDevice(cur));
        if (e != hipSuccess || !p) return SPC_ERR_DEVICE;
        g_scratch[dev] = static_cast<uint32_t *>(p);
    }
    *out = g_scratch[dev];
    return SPC_OK;
}
}  // namespace

spc_status query_multi_noalloc_impl(const spc_index *ix, const uint32_t *gid, const uint32_t *s,
                                    const uint32_t *t, uint64_t nq, void *dist_out, uint64_t *count_out,
                                    uint8_t *flags_out, hipStream_t st) {
    if (!ix) return SPC_ERR_INVALID_ARG;
    if (nq == 0) return SPC_OK;
    if (!s || !t || !dist_out || !count_out) return SPC_ERR_INVALID_ARG;
    if (nq > kNoAllocQueries) return SPC_ERR_UNSUPPORTED;
    uint32_t *p = nullptr;
    SPC_TRY(scratch_on(ix->device, &p));
    // perm = p[0 .. nq), counters at p[kNoAllocQueries]: cleared by a kernel
    // at the start of the call (query_multi_run)
    return query_multi_run(ix, gid, s, t, nq, dist_out, count_out, flags_out, p, p + kNoAllocQueries,
                           ix->query_small, ix->query_cfg, st);
}

}  // namespace spc
