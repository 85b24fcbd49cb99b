// Hybrid vertex order ("Vertex Ordering Strategies": road-network order by
// tree decomposition for the fringe, degree order for the core).  Host code:
// the elimination is a sequential greedy process; its output is the explicit
// order a build takes.
//
// Fringe: repeatedly remove a vertex of least current degree (ties: smaller
// id) while that degree is at most delta, and connect its remaining
// neighbours pairwise (fill-in), so later degrees are those of the
// elimination graph.  Core: the vertices left, ranked first by their degree
// in the input graph (descending, ties by id).  The fringe follows in
// reverse order of removal (the last removed ranks highest among them).
#include <algorithm>
#include <cstdint>
#include <functional>
#include <queue>
#include <utility>
#include <vector>

#include "spc_internal.h"

namespace spc {

spc_status hybrid_order_impl(const spc_graph *g, uint32_t delta, uint32_t *order, uint32_t *core_out) {
    if (!g || !order || !g->row_off || (g->nnz && !g->col) || g->on_device) return SPC_ERR_INVALID_ARG;
    const uint32_t n = g->n;
    if (g->row_off[0] != 0 || g->row_off[n] != g->nnz) return SPC_ERR_INVALID_ARG;
    std::vector<std::vector<uint32_t>> adj(n);
    for (uint32_t v = 0; v < n; v++) {
        const uint64_t b = g->row_off[v], e = g->row_off[v + 1];
        if (e < b || e > g->nnz) return SPC_ERR_INVALID_ARG;
        auto &a = adj[v];
        a.reserve(e - b);
        for (uint64_t i = b; i < e; i++) {
            const uint32_t w = g->col[i];
            if (w >= n) return SPC_ERR_INVALID_ARG;
            if (w != v) a.push_back(w);
        }
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
    }
    std::vector<uint32_t> deg0(n);
    for (uint32_t v = 0; v < n; v++) deg0[v] = (uint32_t)adj[v].size();
    std::vector<uint8_t> removed(n, 0);
    using Item = std::pair<uint32_t, uint32_t>;  // (current degree, vertex)
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
    for (uint32_t v = 0; v < n; v++)
        if (adj[v].size() <= delta) heap.push({(uint32_t)adj[v].size(), v});
    std::vector<uint32_t> elim;
    elim.reserve(n);
    std::vector<uint32_t> merged;
    while (!heap.empty()) {
        const Item top = heap.top();
        heap.pop();
        const uint32_t v = top.second;
        if (removed[v] || top.first != adj[v].size()) continue;  // stale
        if (top.first > delta) break;
        removed[v] = 1;
        elim.push_back(v);
        const std::vector<uint32_t> nb = std::move(adj[v]);
        adj[v].clear();
        // each remaining neighbour loses v and gains the others (fill-in):
        // one sorted union per neighbour rather than one insertion per edge
        for (uint32_t a : nb) {
            const auto &x = adj[a];
            merged.clear();
            merged.reserve(x.size() + nb.size());
            size_t i = 0, j = 0;
            while (i < x.size() || j < nb.size()) {
                uint32_t c;
                if (j >= nb.size() || (i < x.size() && x[i] < nb[j])) {
                    c = x[i++];
                } else if (i >= x.size() || nb[j] < x[i]) {
                    c = nb[j++];
                } else {
                    c = x[i++];
                    j++;
                }
                if (c != a && c != v) merged.push_back(c);
            }
            adj[a].swap(merged);
        }
        for (uint32_t a : nb)
            if (adj[a].size() <= delta) heap.push({(uint32_t)adj[a].size(), a});
    }
    std::vector<uint32_t> core;
    for (uint32_t v = 0; v < n; v++)
        if (!removed[v]) core.push_back(v);
    std::stable_sort(core.begin(), core.end(),
                     [&](uint32_t a, uint32_t b) { return deg0[a] > deg0[b]; });
    uint32_t r = 0;
    for (uint32_t v : core) order[r++] = v;
    for (size_t i = elim.size(); i-- > 0;) order[r++] = elim[i];
    if (core_out) *core_out = (uint32_t)core.size();
    return SPC_OK;
}

}  // namespace spc
