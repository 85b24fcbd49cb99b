// 1-shell reduction (Section "Reduction by 1-Shell"), gfx950.
//
// The fringe -- every vertex outside the 2-core -- is stripped on the device
// by synchronous leaf removal: in round r every vertex with exactly one
// remaining neighbour (a leaf) is removed, and that neighbour becomes its
// parent.  A vertex whose remaining degree drops to one joins the next
// round's leaves.  Two leaves joined to each other are the last edge of a
// tree component: the smaller id stays, so a tree component keeps its
// centre (the smaller of two centres), and a tree hanging off the 2-core
// keeps its core end.  Roots and depths then follow the parents, rounds in
// reverse.  The core is relabelled in id order into its own CSR, and the
// caller's order and tie keys are restricted to it.  The neighbourhood-
// equivalence reduction (further below) keeps one vertex per class of
// twins the same way.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "spc_internal.h"

namespace spc {

namespace {

inline uint32_t waves_grid(uint64_t waves) {
    uint64_t b = (waves + kWaves - 1) / kWaves;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(b, 1u << 16));
}
inline uint32_t items_grid(uint64_t n) {
    uint64_t b = (n + kBlock - 1) / kBlock;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(b, 1u << 16));
}

// append the lanes with `pred` to q (one atomic per wave)
__device__ __forceinline__ void wave_push(bool pred, uint32_t val, uint32_t *q, uint32_t *cnt) {
    const uint64_t m = __ballot(pred);
    if (!m) return;
    const uint32_t leader = (uint32_t)__ffsll((long long)m) - 1;
    uint32_t base = 0;
    if ((threadIdx.x & 63) == leader) base = atomicAdd(cnt, (uint32_t)__popcll(m));
    base = __shfl(base, leader, 64);
    if (pred) q[base + (uint32_t)__popcll(m & lanemask_lt())] = val;
}

__global__ __launch_bounds__(kBlock) void k_shell_init(const uint64_t *off, uint32_t N, uint32_t *deg,
                                                        uint32_t *alive, uint32_t *inq, uint32_t *parent,
                                                        uint32_t *root, uint32_t *depth, uint32_t *fr,
                                                        uint32_t *fr_cnt) {
    const uint32_t stride = gridDim.x * blockDim.x;
    // whole waves iterate together (wave_push is wave-collective)
    const uint32_t span = (N + 63) & ~63u;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < span; v += stride) {
        bool leaf = false;
        if (v < N) {
            const uint32_t d = (uint32_t)(off[v + 1] - off[v]);
            deg[v] = d;
            alive[v] = 1;
            parent[v] = v;
            root[v] = v;
            depth[v] = 0;
            leaf = d == 1;
            inq[v] = leaf ? 1u : 0u;
        }
        wave_push(leaf, v, fr, fr_cnt);
    }
}

// One removal round r over the leaves fr[0, nfr): one wave per leaf finds
// its one remaining neighbour p.  The leaf stays when it has none (a tree
// component's centre) or when p is a leaf of this round too and has the
// larger id; otherwise it is removed with parent p, and p joins round r+1
// when this removal leaves it one neighbour.  Only leaves of this round are
// removed and each reads the flags of its own neighbours, so the one race
// (two leaves joined to each other) is settled by the id rule whichever
// flag value the smaller leaf sees.
__global__ __launch_bounds__(kBlock) void k_shell_round(uint32_t r, const uint32_t *fr, uint32_t nfr,
                                                         const uint64_t *off, const uint32_t *col,
                                                         uint32_t *alive, uint32_t *inq, uint32_t *deg,
                                                         uint32_t *parent, uint32_t *rem,
                                                         uint32_t *rem_cnt, uint32_t *nxt,
                                                         uint32_t *nxt_cnt) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t nw = gridDim.x * kWaves;
    volatile uint32_t *valive = alive;
    volatile uint32_t *vinq = inq;
    for (uint32_t i = blockIdx.x * kWaves + (threadIdx.x >> 6); i < nfr; i += nw) {
        const uint32_t v = fr[i];
        const uint64_t e = off[v + 1];
        uint32_t p = kEmpty32;
        for (uint64_t k0 = off[v]; k0 < e && p == kEmpty32; k0 += 64) {
            const uint64_t k = k0 + lane;
            const uint32_t w = k < e ? col[k] : kEmpty32;
            const bool a = w != kEmpty32 && w != v && valive[w] != 0;
            const uint64_t m = __ballot(a);
            if (m) p = __shfl(w, (int)__ffsll((long long)m) - 1, 64);
        }
        if (lane == 0 && p != kEmpty32 && !(vinq[p] == r && v < p)) {
            valive[v] = 0;
            parent[v] = p;
            rem[atomicAdd(rem_cnt, 1u)] = v;
            if (atomicSub(&deg[p], 1u) == 2u) {
                vinq[p] = r + 1;
                nxt[atomicAdd(nxt_cnt, 1u)] = p;
            }
        }
    }
}

// roots and depths of the vertices removed in one round (later rounds and
// the core are final already)
__global__ void k_shell_resolve(const uint32_t *rem, uint32_t cnt, const uint32_t *parent,
                                uint32_t *root, uint32_t *depth, uint32_t *maxd) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride) {
        const uint32_t v = rem[i], p = parent[v];
        root[v] = root[p];
        const uint32_t d = depth[p] + 1;
        depth[v] = d;
        atomicMax(maxd, d);
    }
}

// core ids: cpos = exclusive scan of alive; roots as core ids; the core's
// tie keys.  A root outside the core only comes from an asymmetric input.
__global__ void k_shell_ids(uint32_t N, const uint32_t *alive, const uint64_t *cpos, uint32_t *root,
                            uint32_t *core_vid, const uint64_t *tie, uint64_t *ctie, const uint32_t *pay,
                            uint32_t *cpay, uint32_t *err) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride) {
        const uint32_t r = root[v];
        if (!alive[r]) atomicOr(err, 1u);
        root[v] = alive[r] ? (uint32_t)cpos[r] : 0u;
        if (alive[v]) {
            const uint32_t c = (uint32_t)cpos[v];
            core_vid[c] = v;
            if (tie) ctie[c] = tie[v];
            if (pay) cpay[c] = pay[v];
        }
    }
}

// core degree of every core vertex (neighbours in the core), one wave each
__global__ __launch_bounds__(kBlock) void k_shell_cdeg(uint32_t N, const uint64_t *off,
                                                        const uint32_t *col, const uint32_t *alive,
                                                        const uint64_t *cpos, uint32_t *cdeg) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t nw = gridDim.x * kWaves;
    for (uint32_t v = blockIdx.x * kWaves + (threadIdx.x >> 6); v < N; v += nw) {
        if (!alive[v]) continue;
        uint32_t c = 0;
        for (uint64_t k = off[v] + lane; k < off[v + 1]; k += 64) c += alive[col[k]] ? 1u : 0u;
        c = wave_sum(c);
        if (lane == 0) cdeg[cpos[v]] = c;
    }
}

// core adjacency in core ids, input order kept within each row
__global__ __launch_bounds__(kBlock) void k_shell_fill(uint32_t N, const uint64_t *off,
                                                        const uint32_t *col, const uint32_t *alive,
                                                        const uint64_t *cpos, const uint64_t *coff,
                                                        uint32_t *ccol) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t nw = gridDim.x * kWaves;
    for (uint32_t v = blockIdx.x * kWaves + (threadIdx.x >> 6); v < N; v += nw) {
        if (!alive[v]) continue;
        uint64_t out = coff[cpos[v]];
        const uint64_t e = off[v + 1];
        for (uint64_t k0 = off[v]; k0 < e; k0 += 64) {
            const uint64_t k = k0 + lane;
            const uint32_t w = k < e ? col[k] : 0;
            const bool keep = k < e && alive[w] != 0;
            const uint64_t m = __ballot(keep);
            if (keep) ccol[out + (uint64_t)__popcll(m & lanemask_lt())] = (uint32_t)cpos[w];
            out += (uint64_t)__popcll(m);
        }
    }
}

// the caller's order restricted to the core: flag, then scatter
__global__ void k_shell_ord_flag(uint32_t N, const uint32_t *ord, const uint32_t *alive, uint32_t *flag) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < N; r += stride)
        flag[r] = alive[ord[r]];
}
__global__ void k_shell_ord_put(uint32_t N, const uint32_t *ord, const uint32_t *flag,
                                const uint64_t *pos, const uint64_t *cpos, uint32_t *cord) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < N; r += stride)
        if (flag[r]) cord[pos[r]] = (uint32_t)cpos[ord[r]];
}

__global__ void k_gather_u64(const uint64_t *src, const uint32_t *idx, uint32_t n, uint64_t *dst) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

// Neighbourhood equivalence (Section "Reduction by Equivalence Relation"):
// u ~ v when nbr(u) minus {v} equals nbr(v) minus {u}.  Candidates are
// grouped by a hash of the open neighbourhood (non-adjacent twins share it)
// and then, among vertices left alone, of the closed one (adjacent twins
// share nbr + self); every member is checked against its group's first
// vertex with the definition itself, so a hash collision only loses a merge.

// one 64-bit mix per vertex id (the splitmix64 finaliser)
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// row sort keys (row << xb | column), one wave per row
__global__ __launch_bounds__(kBlock) void k_tw_rowkeys(const uint64_t *off, const uint32_t *col, uint32_t N,
                                                        int xb, uint64_t *keys) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t nw = gridDim.x * kWaves;
    for (uint32_t v = blockIdx.x * kWaves + (threadIdx.x >> 6); v < N; v += nw)
        for (uint64_t k = off[v] + lane; k < off[v + 1]; k += 64) keys[k] = ((uint64_t)v << xb) | col[k];
}
__global__ void k_tw_keys2col(const uint64_t *keys, uint64_t nnz, int xb, uint32_t *col) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += stride)
        col[i] = (uint32_t)(keys[i] & ((1ull << xb) - 1));
}

// graph of union vertex v: largest g with vbase[g] <= v (vbase[0] = 0)
__device__ __forceinline__ uint32_t graph_index(const uint32_t *vbase, uint32_t k, uint32_t v) {
    uint32_t lo = 0, hi = k - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (vbase[mid] <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// hash keys of the open (closed = false) or closed neighbourhood of the
// listed vertices, salted by the graph (isolated vertices of different
// graphs of a batch are not twins); ids listed in vals
__global__ __launch_bounds__(kBlock) void k_tw_hash(const uint64_t *off, const uint32_t *col,
                                                     const uint32_t *list, uint32_t cnt, bool closed,
                                                     const uint32_t *vbase, uint32_t k,
                                                     uint64_t *keys, uint32_t *vals) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t nw = gridDim.x * kWaves;
    for (uint32_t i = blockIdx.x * kWaves + (threadIdx.x >> 6); i < cnt; i += nw) {
        const uint32_t v = list ? list[i] : i;
        uint64_t h = 0;
        for (uint64_t e = off[v] + lane; e < off[v + 1]; e += 64) h += mix64(col[e]);
        h = wave_sum(h);
        if (lane == 0) {
            h += mix64(~(uint64_t)graph_index(vbase, k, v));
            keys[i] = closed ? h + mix64(v) : h;
            vals[i] = v;
        }
    }
}

// segment heads of sorted keys
__global__ void k_tw_heads(const uint64_t *keys, uint32_t cnt, uint32_t *head) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride)
        head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}
// first position of every segment
__global__ void k_tw_starts(const uint32_t *head, const uint64_t *hpos, uint32_t cnt, uint32_t *start) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride)
        if (head[i]) start[hpos[i]] = i;
}

// is x in the sorted row a[0, len)?  position or len
__device__ __forceinline__ uint64_t find_sorted(const uint32_t *a, uint64_t len, uint32_t x) {
    uint64_t lo = 0, hi = len;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (a[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < len && a[lo] == x) ? lo : len;
}

// the definition, member m against leader L (sorted rows): nbr(m) minus
// {L} and nbr(L) minus {m} hold the same ids (and both lie in one graph).
// One wave per sorted position; a match records L as m's class, and marks
// the class as adjacent twins when m and L are neighbours.
__global__ __launch_bounds__(kBlock) void k_tw_verify(const uint64_t *off, const uint32_t *col,
                                                       const uint32_t *vals, const uint32_t *head,
                                                       const uint64_t *hpos, const uint32_t *start,
                                                       uint32_t cnt, const uint32_t *vbase, uint32_t k,
                                                       uint32_t *cls, uint32_t *kind) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t nw = gridDim.x * kWaves;
    for (uint32_t i = blockIdx.x * kWaves + (threadIdx.x >> 6); i < cnt; i += nw) {
        if (head[i]) continue;
        const uint32_t m = vals[i], L = vals[start[hpos[i] - 1]];
        if (graph_index(vbase, k, m) != graph_index(vbase, k, L)) continue;
        const uint32_t *rm = col + off[m], *rl = col + off[L];
        const uint64_t lm = off[m + 1] - off[m], ll = off[L + 1] - off[L];
        const uint64_t pm = find_sorted(rm, lm, L), pl = find_sorted(rl, ll, m);
        const uint64_t nm = lm - (pm < lm), nl = ll - (pl < ll);
        bool same = nm == nl;
        for (uint64_t k0 = 0; same && k0 < nm; k0 += 64) {
            const uint64_t k = k0 + lane;
            bool ok = true;
            if (k < nm) ok = rm[k + (k >= pm)] == rl[k + (k >= pl)];
            same = __ballot(!ok) == 0;
        }
        if (same && lane == 0) {
            cls[m] = L;
            if (pm < lm) kind[L] = 1;
        }
    }
}

__global__ void k_tw_init(uint32_t N, uint32_t *cls, uint32_t *kind, uint32_t *size) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride) {
        cls[v] = v;
        kind[v] = 0;
        size[v] = 0;
    }
}
__global__ void k_tw_count(uint32_t N, const uint32_t *cls, uint32_t *size) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride) atomicAdd(&size[cls[v]], 1u);
}
// vertices still alone after the open-neighbourhood pass
__global__ void k_tw_alone(uint32_t N, const uint32_t *cls, const uint32_t *size, uint32_t *flag) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride)
        flag[v] = (cls[v] == v && size[v] == 1) ? 1u : 0u;
}
__global__ void k_tw_list(uint32_t N, const uint32_t *flag, const uint64_t *pos, uint32_t *list) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride)
        if (flag[v]) list[pos[v]] = v;
}
// final per-vertex arrays: representative flag, root = representative,
// depth 0, parent = itself; same-class answer (~0: adjacent twins, else the
// degree); class size of representatives
__global__ void k_tw_finish(uint32_t N, const uint64_t *off, const uint32_t *cls, const uint32_t *kind,
                            const uint32_t *size, uint32_t *alive, uint32_t *root, uint32_t *depth,
                            uint32_t *parent, uint32_t *same, uint32_t *weight) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride) {
        const uint32_t c = cls[v];
        alive[v] = c == v ? 1u : 0u;
        root[v] = c;
        depth[v] = 0;
        parent[v] = v;
        same[v] = kind[c] ? 0xFFFFFFFFu : (uint32_t)(off[v + 1] - off[v]);
        weight[v] = c == v ? size[v] : 0u;
    }
}

}  // namespace

namespace {

// The core (alive vertices) in input id order: core ids, its CSR, the given
// order and tie keys restricted to it, roots as core ids, and the payload
// of core vertices.  deg is scratch of N+1 entries; ctr of 4.
spc_status induce_core(Arena &ar, hipStream_t st, uint64_t *ws, uint32_t N, uint64_t NNZ,
                       const uint64_t *off, const uint32_t *col, const uint32_t *ord, const uint64_t *tie,
                       const std::vector<uint32_t> &vbase, const uint32_t *alive, uint32_t removed,
                       uint32_t *deg, uint32_t *ctr, const uint32_t *pay, uint32_t **cpay,
                       ShellResult *R) {
    uint64_t *cpos = nullptr;
    SPC_TRY(ar.alloc(&cpos, (uint64_t)N + 1));
    SPC_TRY(scan_u32(alive, cpos, N, ws, st));
    const uint32_t Nc = N - removed;
    SPC_TRY(ar.alloc(&R->core_vid, (uint64_t)Nc + 1));
    if (tie) SPC_TRY(ar.alloc(&R->tie, (uint64_t)Nc + 1));
    if (pay) SPC_TRY(ar.alloc(cpay, (uint64_t)Nc + 1));
    SPC_HIP(hipMemsetAsync(ctr, 0, sizeof(uint32_t), st));  // error flag
    hipLaunchKernelGGL(k_shell_ids, dim3(items_grid(N)), dim3(kBlock), 0, st, N, alive, cpos, R->root,
                       R->core_vid, tie, R->tie, pay, pay ? *cpay : nullptr, ctr);
    SPC_LAUNCHED();
    uint32_t *cdeg = deg;
    hipLaunchKernelGGL(k_shell_cdeg, dim3(waves_grid(N)), dim3(kBlock), 0, st, N, off, col, alive, cpos,
                       cdeg);
    SPC_LAUNCHED();
    SPC_TRY(ar.alloc(&R->off, (uint64_t)Nc + 1));
    SPC_TRY(scan_u32(cdeg, R->off, Nc, ws, st));
    uint64_t nnzc = 0;
    SPC_HIP(hipMemcpyAsync(&nnzc, R->off + Nc, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    SPC_HIP(hipStreamSynchronize(st));
    if (nnzc > NNZ) return SPC_ERR_DEVICE;
    SPC_TRY(ar.alloc(&R->col, std::max<uint64_t>(nnzc, 1)));
    hipLaunchKernelGGL(k_shell_fill, dim3(waves_grid(N)), dim3(kBlock), 0, st, N, off, col, alive, cpos,
                       R->off, R->col);
    SPC_LAUNCHED();
    if (ord) {
        uint32_t *flag = deg;  // core degrees are in R->off now
        uint64_t *pos = nullptr;
        SPC_TRY(ar.alloc(&pos, (uint64_t)N + 1));
        hipLaunchKernelGGL(k_shell_ord_flag, dim3(items_grid(N)), dim3(kBlock), 0, st, N, ord, alive, flag);
        SPC_LAUNCHED();
        SPC_TRY(scan_u32(flag, pos, N, ws, st));
        SPC_TRY(ar.alloc(&R->ord, (uint64_t)Nc + 1));
        hipLaunchKernelGGL(k_shell_ord_put, dim3(items_grid(N)), dim3(kBlock), 0, st, N, ord, flag, pos,
                           cpos, R->ord);
        SPC_LAUNCHED();
        ar.release(pos);
    }
    // each graph's vertices stay contiguous: core range starts at cpos[vbase]
    const uint32_t k1 = (uint32_t)vbase.size();
    uint32_t *vb = nullptr;
    uint64_t *cb = nullptr;
    SPC_TRY(ar.alloc(&vb, k1));
    SPC_TRY(ar.alloc(&cb, k1));
    SPC_HIP(hipMemcpyAsync(vb, vbase.data(), k1 * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_gather_u64, dim3((k1 + kBlock - 1) / kBlock), dim3(kBlock), 0, st, cpos, vb, k1, cb);
    SPC_LAUNCHED();
    std::vector<uint64_t> hb(k1);
    uint32_t h[4] = {0, 0, 0, 0};
    SPC_HIP(hipMemcpyAsync(hb.data(), cb, k1 * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    SPC_HIP(hipMemcpyAsync(h, ctr, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    SPC_HIP(hipStreamSynchronize(st));
    if (h[0]) return SPC_ERR_INVALID_ARG;
    R->cbase.assign(hb.begin(), hb.end());
    R->N = Nc;
    R->NNZ = nnzc;
    ar.release(vb);
    ar.release(cb);
    ar.release(cpos);
    return SPC_OK;
}

}  // namespace

spc_status one_shell(Arena &ar, hipStream_t st, uint64_t *ws, uint32_t N, uint64_t NNZ,
                     const uint64_t *off, const uint32_t *col, const uint32_t *ord, const uint64_t *tie,
                     const std::vector<uint32_t> &vbase, ShellResult *R) {
    uint32_t *deg = nullptr, *alive = nullptr, *inq = nullptr, *qa = nullptr, *qb = nullptr,
             *ctr = nullptr;
    SPC_TRY(ar.alloc(&deg, (uint64_t)N + 1));
    SPC_TRY(ar.alloc(&alive, (uint64_t)N + 1));
    SPC_TRY(ar.alloc(&inq, (uint64_t)N + 1));
    SPC_TRY(ar.alloc(&qa, (uint64_t)N + 1));
    SPC_TRY(ar.alloc(&qb, (uint64_t)N + 1));
    SPC_TRY(ar.alloc(&ctr, 4));  // frontier count, next count, removed count, max depth
    SPC_TRY(ar.alloc(&R->parent, (uint64_t)N + 1));
    SPC_TRY(ar.alloc(&R->root, (uint64_t)N + 1));
    SPC_TRY(ar.alloc(&R->depth, (uint64_t)N + 1));
    uint32_t *rem = nullptr;
    SPC_TRY(ar.alloc(&rem, (uint64_t)N + 1));
    SPC_HIP(hipMemsetAsync(ctr, 0, 4 * sizeof(uint32_t), st));
    hipLaunchKernelGGL(k_shell_init, dim3(items_grid(N)), dim3(kBlock), 0, st, off, N, deg, alive, inq,
                       R->parent, R->root, R->depth, qa, ctr);
    SPC_LAUNCHED();
    uint32_t h[4] = {0, 0, 0, 0};
    SPC_HIP(hipMemcpyAsync(h, ctr, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    SPC_HIP(hipStreamSynchronize(st));
    // removal offsets per round: rem[roff[i], roff[i+1]) left in round i+1;
    // every vertex is a leaf in at most one round, so at most N rounds run
    std::vector<uint32_t> roff{0};
    uint32_t nfr = h[0];
    for (uint32_t r = 1; nfr > 0; r++) {
        SPC_HIP(hipMemsetAsync(ctr + 1, 0, sizeof(uint32_t), st));
        hipLaunchKernelGGL(k_shell_round, dim3(waves_grid(nfr)), dim3(kBlock), 0, st, r, qa, nfr, off,
                           col, alive, inq, deg, R->parent, rem, ctr + 2, qb, ctr + 1);
        SPC_LAUNCHED();
        SPC_HIP(hipMemcpyAsync(h, ctr, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        SPC_HIP(hipStreamSynchronize(st));
        roff.push_back(h[2]);
        nfr = h[1];
        std::swap(qa, qb);
    }
    const uint32_t removed = roff.back();
    for (size_t i = roff.size() - 1; i-- > 0;) {
        const uint32_t c = roff[i + 1] - roff[i];
        if (!c) continue;
        hipLaunchKernelGGL(k_shell_resolve, dim3(items_grid(c)), dim3(kBlock), 0, st, rem + roff[i], c,
                           R->parent, R->root, R->depth, ctr + 3);
        SPC_LAUNCHED();
    }
    SPC_HIP(hipMemcpyAsync(h, ctr, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    SPC_HIP(hipStreamSynchronize(st));
    R->max_depth = h[3];
    R->fringe = removed;
    ar.release(rem);
    ar.release(qa);
    ar.release(qb);
    ar.release(inq);
    SPC_TRY(induce_core(ar, st, ws, N, NNZ, off, col, ord, tie, vbase, alive, removed, deg, ctr, nullptr,
                        nullptr, R));
    ar.release(deg);
    ar.release(alive);
    ar.release(ctr);
    return SPC_OK;
}

spc_status twin_reduce(Arena &ar, hipStream_t st, uint64_t *ws, uint32_t N, uint64_t NNZ,
                       const uint64_t *off, uint32_t *col, bool rows_sorted, const uint32_t *ord,
                       const uint64_t *tie, const std::vector<uint32_t> &vbase, ShellResult *R) {
    if (!rows_sorted && NNZ) {  // the definition check walks sorted rows
        int xb = 1;
        while (xb < 32 && (1ull << xb) < (uint64_t)N) xb++;
        uint64_t *keys = nullptr, *keys2 = nullptr, *rws = nullptr;
        SPC_TRY(ar.alloc(&keys, NNZ));
        SPC_TRY(ar.alloc(&keys2, NNZ));
        SPC_TRY(ar.alloc(&rws, radix_ws_elems(NNZ)));
        hipLaunchKernelGGL(k_tw_rowkeys, dim3(waves_grid(N)), dim3(kBlock), 0, st, off, col, N, xb, keys);
        SPC_LAUNCHED();
        SPC_TRY(radix_sort_pairs(keys, nullptr, keys2, nullptr, NNZ, 2 * xb, rws, st));
        hipLaunchKernelGGL(k_tw_keys2col, dim3(items_grid(NNZ)), dim3(kBlock), 0, st, keys, NNZ, xb, col);
        SPC_LAUNCHED();
        ar.release(keys);
        ar.release(keys2);
        ar.release(rws);
    }
    uint32_t *cls = nullptr, *kind = nullptr, *size = nullptr, *vals = nullptr, *vals2 = nullptr,
             *head = nullptr, *start = nullptr, *list = nullptr, *ctr = nullptr;
    uint64_t *keys = nullptr, *keys2 = nullptr, *hpos = nullptr;
    const uint64_t n1 = (uint64_t)N + 1;
    SPC_TRY(ar.alloc(&cls, n1));
    SPC_TRY(ar.alloc(&kind, n1));
    SPC_TRY(ar.alloc(&size, n1));
    SPC_TRY(ar.alloc(&vals, n1));
    SPC_TRY(ar.alloc(&vals2, n1));
    SPC_TRY(ar.alloc(&head, n1));
    SPC_TRY(ar.alloc(&start, n1));
    SPC_TRY(ar.alloc(&list, n1));
    SPC_TRY(ar.alloc(&ctr, 4));
    SPC_TRY(ar.alloc(&keys, n1));
    SPC_TRY(ar.alloc(&keys2, n1));
    SPC_TRY(ar.alloc(&hpos, n1));
    uint64_t *rws = nullptr;
    SPC_TRY(ar.alloc(&rws, radix_ws_elems(n1)));
    const uint32_t k = (uint32_t)vbase.size() - 1;  // graphs; vbase ends with N
    uint32_t *vb = nullptr;
    SPC_TRY(ar.alloc(&vb, (uint64_t)k + 1));
    SPC_HIP(hipMemcpyAsync(vb, vbase.data(), ((uint64_t)k + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_tw_init, dim3(items_grid(N)), dim3(kBlock), 0, st, N, cls, kind, size);
    SPC_LAUNCHED();
    // pass 1: open neighbourhoods of every vertex; pass 2: closed
    // neighbourhoods of the vertices pass 1 left alone
    for (int pass = 0; pass < 2; pass++) {
        const bool closed = pass == 1;
        uint32_t cnt = N;
        const uint32_t *lst = nullptr;
        if (closed) {
            hipLaunchKernelGGL(k_tw_count, dim3(items_grid(N)), dim3(kBlock), 0, st, N, cls, size);
            SPC_LAUNCHED();
            hipLaunchKernelGGL(k_tw_alone, dim3(items_grid(N)), dim3(kBlock), 0, st, N, cls, size, head);
            SPC_LAUNCHED();
            SPC_TRY(scan_u32(head, hpos, N, ws, st));
            uint64_t c64 = 0;
            SPC_HIP(hipMemcpyAsync(&c64, hpos + N, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
            SPC_HIP(hipStreamSynchronize(st));
            cnt = (uint32_t)c64;
            hipLaunchKernelGGL(k_tw_list, dim3(items_grid(N)), dim3(kBlock), 0, st, N, head, hpos, list);
            SPC_LAUNCHED();
            lst = list;
        }
        if (cnt < 2) continue;
        hipLaunchKernelGGL(k_tw_hash, dim3(waves_grid(cnt)), dim3(kBlock), 0, st, off, col, lst, cnt, closed,
                           vb, k, keys, vals);
        SPC_LAUNCHED();
        SPC_TRY(radix_sort_pairs(keys, vals, keys2, vals2, cnt, 64, rws, st));
        hipLaunchKernelGGL(k_tw_heads, dim3(items_grid(cnt)), dim3(kBlock), 0, st, keys, cnt, head);
        SPC_LAUNCHED();
        SPC_TRY(scan_u32(head, hpos, cnt, ws, st));
        hipLaunchKernelGGL(k_tw_starts, dim3(items_grid(cnt)), dim3(kBlock), 0, st, head, hpos, cnt, start);
        SPC_LAUNCHED();
        hipLaunchKernelGGL(k_tw_verify, dim3(waves_grid(cnt)), dim3(kBlock), 0, st, off, col, vals, head,
                           hpos, start, cnt, vb, k, cls, kind);
        SPC_LAUNCHED();
    }
    SPC_HIP(hipMemsetAsync(size, 0, n1 * sizeof(uint32_t), st));
    hipLaunchKernelGGL(k_tw_count, dim3(items_grid(N)), dim3(kBlock), 0, st, N, cls, size);
    SPC_LAUNCHED();
    uint32_t *alive = head, *weight = start;  // reuse
    SPC_TRY(ar.alloc(&R->root, n1));
    SPC_TRY(ar.alloc(&R->depth, n1));
    SPC_TRY(ar.alloc(&R->parent, n1));
    SPC_TRY(ar.alloc(&R->same, n1));
    hipLaunchKernelGGL(k_tw_finish, dim3(items_grid(N)), dim3(kBlock), 0, st, N, off, cls, kind, size, alive,
                       R->root, R->depth, R->parent, R->same, weight);
    SPC_LAUNCHED();
    uint64_t *apos = hpos;
    SPC_TRY(scan_u32(alive, apos, N, ws, st));
    uint64_t reps = 0;
    SPC_HIP(hipMemcpyAsync(&reps, apos + N, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    SPC_HIP(hipStreamSynchronize(st));
    const uint32_t removed = N - (uint32_t)reps;
    R->twins = removed;
    ar.release(rws);
    ar.release(keys);
    ar.release(keys2);
    ar.release(vals);
    ar.release(vals2);
    SPC_TRY(induce_core(ar, st, ws, N, NNZ, off, col, ord, tie, vbase, alive, removed, size, ctr, weight,
                        &R->weight, R));
    ar.release(cls);
    ar.release(kind);
    ar.release(size);
    ar.release(head);
    ar.release(start);
    ar.release(list);
    ar.release(hpos);
    ar.release(ctr);
    ar.release(vb);
    return SPC_OK;
}

}  // namespace spc
