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
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <mutex>
#include <queue>
#include <thread>
#include <utility>
#include <vector>

#include "spc_internal.h"

namespace spc {

namespace {

// adj[a] <- (adj[a] union nb) minus {a, v}: one sorted merge, written from
// the back into the row's own buffer (it only grows), then moved to the front
void merge_row(std::vector<uint32_t> &x, const std::vector<uint32_t> &nb, uint32_t a, uint32_t v,
               std::vector<uint32_t> &) {
    const size_t nx = x.size(), nn = nb.size();
    x.resize(nx + nn);
    size_t i = nx, j = nn, w = nx + nn;  // merge from the largest ids down
    uint32_t last = 0xFFFFFFFFu;        // no id equals it (ids < n < 2^32 - 1)
    while (i > 0 || j > 0) {
        uint32_t c;
        if (j == 0 || (i > 0 && x[i - 1] > nb[j - 1])) {
            c = x[--i];
        } else if (i == 0 || nb[j - 1] > x[i - 1]) {
            c = nb[--j];
        } else {
            c = x[--i];
            --j;
        }
        if (c != a && c != v && c != last) {
            x[--w] = c;
            last = c;
        }
    }
    const size_t len = nx + nn - w;
    if (w) std::copy(x.begin() + w, x.end(), x.begin());
    x.resize(len);
}

// Host threads that share the neighbour merges of one elimination (each
// neighbour's row is written by one thread only; the eliminated vertex's
// row is read-only meanwhile), started once per order computation.
class MergePool {
  public:
    explicit MergePool(unsigned n) {
        for (unsigned t = 1; t < n; t++) th_.emplace_back([this, t, n] { run(t, n); });
        nth_ = n;
    }
    ~MergePool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            gen_++;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    unsigned threads() const { return nth_; }
    // merge nb into the rows of all of nb's vertices, spread over the threads
    void merge_all(std::vector<std::vector<uint32_t>> &adj, const std::vector<uint32_t> &nb, uint32_t v) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            adj_ = &adj;
            nb_ = &nb;
            v_ = v;
            pending_ = nth_ - 1;
            gen_++;
        }
        cv_.notify_all();
        work(0, nth_);
        std::unique_lock<std::mutex> lk(mu_);
        done_.wait(lk, [this] { return pending_ == 0; });
    }

  private:
    void work(unsigned t, unsigned n) {
        std::vector<uint32_t> &merged = scratch_[t];
        const std::vector<uint32_t> &nb = *nb_;
        for (size_t k = t; k < nb.size(); k += n) merge_row((*adj_)[nb[k]], nb, nb[k], v_, merged);
    }
    void run(unsigned t, unsigned n) {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return gen_ != seen; });
                seen = gen_;
                if (stop_) return;
            }
            work(t, n);
            {
                std::lock_guard<std::mutex> lk(mu_);
                if (--pending_ == 0) done_.notify_one();
            }
        }
    }
    std::vector<std::thread> th_;
    unsigned nth_ = 1;
    std::mutex mu_;
    std::condition_variable cv_, done_;
    uint64_t gen_ = 0;
    unsigned pending_ = 0;
    bool stop_ = false;
    std::vector<std::vector<uint32_t>> *adj_ = nullptr;
    const std::vector<uint32_t> *nb_ = nullptr;
    uint32_t v_ = 0;
    std::vector<uint32_t> scratch_[64];
};

// eliminations whose neighbourhood is at least this large share the merges
constexpr size_t kParallelNeighbours = 48;

}  // namespace

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
    const unsigned hw = std::thread::hardware_concurrency();
    MergePool pool(std::min(16u, std::max(1u, hw)));
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
        // one sorted union per neighbour rather than one insertion per edge;
        // the merges of a large neighbourhood are independent and shared by
        // the pool's threads
        if (nb.size() >= kParallelNeighbours && pool.threads() > 1)
            pool.merge_all(adj, nb, v);
        else
            for (uint32_t a : nb) merge_row(adj[a], nb, a, v, merged);
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
