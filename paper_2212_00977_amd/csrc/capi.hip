// C ABI entry points (declared in include/spc.h).  Each call validates its
// host-side arguments, then runs the library's kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <unistd.h>

#include <atomic>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "spc_internal.h"

namespace {
// The cache keeps at most g_cache_limit bytes of freed memory after a build
// or a free (0: a quarter of the current device's memory, enough for the
// next build of a similar graph); the rest goes back to the runtime for
// other allocators.
std::atomic<uint64_t> g_cache_limit{0};
void trim_cache() {
    const uint64_t lim = g_cache_limit.load();
    if (lim == UINT64_MAX) return;
    if (lim) {
        spc::cache_trim(lim);
        return;
    }
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess)
        spc::cache_trim(tot / 4);
    else
        (void)hipGetLastError();
}

// On-disk tuning cache (spc_build_opts.tune_cache): lines "<key> <cfg>
// <small>", key in 16 hex digits.
uint64_t tune_key(const spc_index *ix) {
    char dev[320] = {0};
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ix->device) == hipSuccess)
        std::snprintf(dev, sizeof(dev), "%s/%s", prop.name, prop.gcnArchName);
    else
        (void)hipGetLastError();
    const uint64_t vals[] = {ix->n, ix->m, ix->entries, ix->rounds, ix->max_dist, ix->gn.size(),
                             ix->nreal ? 1u : 0u, ix->out_bits};
    uint64_t h = 1469598103934665603ull;  // FNV-1a, 64 bit
    auto mix = [&](const void *p, size_t n) {
        for (size_t i = 0; i < n; i++) {
            h ^= static_cast<const unsigned char *>(p)[i];
            h *= 1099511628211ull;
        }
    };
    mix(vals, sizeof(vals));
    mix(dev, std::strlen(dev));
    // the configuration table: a cached number means the same launch shape
    for (uint32_t c = 0; c < spc::query_cfg_count(); c++) {
        uint32_t st[2] = {0, 0};
        (void)spc::query_cfg_info(c, &st[0], &st[1]);
        mix(st, sizeof(st));
    }
    return h;
}

std::vector<std::string> read_lines(const std::string &path) {
    std::vector<std::string> out;
    std::ifstream f(path);
    std::string line;
    while (f && std::getline(f, line))
        if (!line.empty()) out.push_back(line);
    return out;
}

void load_tune_cache(spc_index *ix, const char *path) {
    ix->tune_cache = path;
    ix->tune_key = tune_key(ix);
    char key[17];
    std::snprintf(key, sizeof(key), "%016llx", (unsigned long long)ix->tune_key);
    for (const std::string &line : read_lines(path)) {
        std::istringstream is(line);
        std::string k;
        uint32_t cfg = 0, small = 0;
        if (!(is >> k >> cfg >> small) || k != key) continue;
        if (cfg < spc::query_cfg_count()) {
            ix->query_cfg = cfg;
            ix->query_small = small;
            ix->tune_cached = true;
        }
    }
}

void store_tune_cache(const spc_index *ix) {
    if (ix->tune_cache.empty()) return;
    char key[17];
    std::snprintf(key, sizeof(key), "%016llx", (unsigned long long)ix->tune_key);
    std::vector<std::string> lines;
    for (const std::string &line : read_lines(ix->tune_cache))
        if (line.compare(0, 16, key) != 0) lines.push_back(line);
    char mine[64];
    std::snprintf(mine, sizeof(mine), "%s %u %u", key, ix->query_cfg, ix->query_small);
    lines.push_back(mine);
    const std::string tmp = ix->tune_cache + ".tmp." + std::to_string((unsigned long)getpid());
    {
        std::ofstream f(tmp, std::ios::trunc);
        for (const std::string &l : lines) f << l << '\n';
        if (!f) {
            std::remove(tmp.c_str());
            return;
        }
    }
    if (std::rename(tmp.c_str(), ix->tune_cache.c_str()) != 0) std::remove(tmp.c_str());
}
}  // namespace

extern "C" {

const char *spc_status_string(spc_status s) {
    switch (s) {
        case SPC_OK: return "ok";
        case SPC_ERR_INVALID_ARG: return "invalid argument";
        case SPC_ERR_OUT_OF_MEMORY: return "out of device memory";
        case SPC_ERR_DEVICE: return "device error";
        case SPC_ERR_DIST_RANGE: return "distance exceeds the label width";
        case SPC_ERR_UNSUPPORTED: return "unsupported size";
    }
    return "unknown status";
}

spc_status spc_build_index(const spc_graph *g, const spc_build_opts *opts, void *stream,
                           spc_index **out) {
    if (!g || !opts || !out) return SPC_ERR_INVALID_ARG;
    spc_status s = spc::build_impl(g, 1, opts, static_cast<hipStream_t>(stream), out);
    if (s == SPC_OK && opts->tune_cache) load_tune_cache(*out, opts->tune_cache);
    trim_cache();
    return s;
}

spc_status spc_build_index_batch(const spc_graph *gs, uint32_t k, const spc_build_opts *opts,
                                 void *stream, spc_index **out) {
    if (!gs || k == 0 || !opts || !out) return SPC_ERR_INVALID_ARG;
    spc_status s = spc::build_impl(gs, k, opts, static_cast<hipStream_t>(stream), out);
    if (s == SPC_OK && opts->tune_cache) load_tune_cache(*out, opts->tune_cache);
    trim_cache();
    return s;
}

spc_status spc_query_batch(const spc_index *ix, uint32_t graph_id, const uint32_t *s,
                           const uint32_t *t, uint64_t nq, void *dist_out, uint64_t *count_out,
                           uint8_t *flags_out, void *stream) {
    return spc::query_impl(ix, graph_id, s, t, nq, dist_out, count_out, flags_out,
                           static_cast<hipStream_t>(stream));
}

spc_status spc_query_batch_multi(const spc_index *ix, const uint32_t *graph_ids, const uint32_t *s,
                                 const uint32_t *t, uint64_t nq, void *dist_out, uint64_t *count_out,
                                 uint8_t *flags_out, void *stream) {
    return spc::query_multi_impl(ix, graph_ids, s, t, nq, dist_out, count_out, flags_out,
                                 static_cast<hipStream_t>(stream));
}

spc_status spc_query_batch_multi_noalloc(const spc_index *ix, const uint32_t *graph_ids,
                                         const uint32_t *s, const uint32_t *t, uint64_t nq,
                                         void *dist_out, uint64_t *count_out, uint8_t *flags_out,
                                         void *stream) {
    return spc::query_multi_noalloc_impl(ix, graph_ids, s, t, nq, dist_out, count_out, flags_out,
                                         static_cast<hipStream_t>(stream));
}

spc_status spc_tune_query_buckets(spc_index *ix, const uint32_t *graph_ids, const uint32_t *s,
                                  const uint32_t *t, uint64_t nq, void *stream, uint32_t *small_out) {
    spc_status r = spc::tune_query_buckets_impl(ix, graph_ids, s, t, nq, static_cast<hipStream_t>(stream),
                                                small_out);
    if (r == SPC_OK) store_tune_cache(ix);
    return r;
}

spc_status spc_set_query_buckets(spc_index *ix, uint32_t small) {
    if (!ix) return SPC_ERR_INVALID_ARG;
    ix->query_small = small;
    return SPC_OK;
}

void spc_free(spc_index *ix) {
    if (!ix) return;
    int cur = 0;
    bool switched = hipGetDevice(&cur) == hipSuccess && cur != ix->device &&
                    hipSetDevice(ix->device) == hipSuccess;
    (void)hipDeviceSynchronize();  // queries may still read the index
    for (auto &b : ix->blocks) spc::cache_free(b.first, b.second);
    trim_cache();
    if (switched) (void)hipSetDevice(cur);
    delete ix;
}

void spc_release_cached_memory(void) { spc::cache_flush(); }

void spc_set_cache_limit(uint64_t bytes) { g_cache_limit.store(bytes ? bytes : 1); }

spc_status spc_index_stats(const spc_index *ix, spc_stats *out) {
    if (!ix || !out) return SPC_ERR_INVALID_ARG;
    std::memset(out, 0, sizeof(*out));
    out->n = ix->n;
    out->num_graphs = (uint32_t)ix->gn.size();
    out->m = ix->m;
    out->entries = ix->entries;
    out->rounds = ix->rounds;
    out->max_dist = ix->max_dist;
    out->dist_bits = ix->out_bits;
    out->label_bits = ix->dist_bits;
    out->fringe_vertices = ix->fringe;
    out->fringe_depth = ix->fringe_depth;
    out->twin_vertices = (uint32_t)ix->twins;
    out->truncated = ix->truncated ? 1u : 0u;
    out->saturated_entries = ix->saturated;
    out->index_bytes = ix->index_bytes;
    out->peak_build_bytes = ix->peak_build_bytes;
    out->ms_order = ix->ms_order;
    out->ms_rounds = ix->ms_rounds;
    out->ms_finalize = ix->ms_finalize;
    out->ms_total = ix->ms_total;
    out->ms_round_kernel = ix->ms_round_kernel;
    out->alg_bytes_round_kernel = ix->alg_bytes_round_kernel;
    out->round_kernel_launches = ix->round_kernel_launches;
    out->directed = ix->nreal ? 1u : 0u;
    out->query_config = ix->query_cfg;
    out->query_small = ix->query_small;
    out->tune_cached = ix->tune_cached ? 1u : 0u;
    return SPC_OK;
}

uint32_t spc_query_config_count(void) { return spc::query_cfg_count(); }

spc_status spc_query_config_info(uint32_t cfg, uint32_t *stage, uint32_t *tiles) {
    return spc::query_cfg_info(cfg, stage, tiles);
}

spc_status spc_tune_queries(spc_index *ix, uint32_t graph_id, const uint32_t *s, const uint32_t *t,
                            uint64_t nq, void *stream, uint32_t *cfg_out) {
    spc_status r = spc::tune_queries_impl(ix, graph_id, s, t, nq, static_cast<hipStream_t>(stream), cfg_out);
    if (r == SPC_OK) store_tune_cache(ix);
    return r;
}

spc_status spc_hybrid_order(const spc_graph *g, uint32_t delta, uint32_t *order_out,
                            uint32_t *core_out) {
    return spc::hybrid_order_impl(g, delta, order_out, core_out);
}

spc_status spc_set_query_config(spc_index *ix, uint32_t cfg) {
    if (!ix || cfg >= spc::query_cfg_count()) return SPC_ERR_INVALID_ARG;
    ix->query_cfg = cfg;
    return SPC_OK;
}

spc_status spc_round_stats(const spc_index *ix, uint32_t max_rounds, uint64_t *raw, uint64_t *merged,
                           uint64_t *kept, uint64_t *scanned) {
    if (!ix) return SPC_ERR_INVALID_ARG;
    for (uint32_t r = 0; r < max_rounds; r++) {
        spc::RoundCounters c;
        if (r < ix->round_stats.size()) c = ix->round_stats[r];
        if (raw) raw[r] = c.raw;
        if (merged) merged[r] = c.merged;
        if (kept) kept[r] = c.kept;
        if (scanned) scanned[r] = c.scanned;
    }
    return SPC_OK;
}

spc_status spc_round_profile(const spc_index *ix, uint32_t max_rounds, double *kernel_ms,
                             uint64_t *staged, uint64_t *row_bytes, uint64_t *headers,
                             uint64_t *mem_peak, uint64_t *filter_bytes) {
    if (!ix) return SPC_ERR_INVALID_ARG;
    for (uint32_t r = 0; r < max_rounds; r++) {
        spc::RoundCounters c;
        if (r < ix->round_stats.size()) c = ix->round_stats[r];
        if (kernel_ms) kernel_ms[r] = c.kernel_ms;
        if (staged) staged[r] = c.staged;
        if (row_bytes) row_bytes[r] = c.row_bytes;
        if (headers) headers[r] = c.headers;
        if (mem_peak) mem_peak[r] = c.mem_peak;
        if (filter_bytes) filter_bytes[r] = c.filter_bytes;
    }
    return SPC_OK;
}

spc_status spc_graph_entries(const spc_index *ix, uint32_t graph_id, uint32_t *n_out,
                             uint64_t *entries_out) {
    if (!ix || graph_id >= ix->gn.size()) return SPC_ERR_INVALID_ARG;
    // label rows: the graph's vertices, twice for a directed graph
    uint32_t vb = ix->vbase[graph_id], n = ix->gn[graph_id] * (ix->nreal ? 2u : 1u);
    uint64_t e[2] = {0, 0};
    if (hipMemcpy(&e[0], ix->lab_off + vb, 8, hipMemcpyDeviceToHost) != hipSuccess) return SPC_ERR_DEVICE;
    if (hipMemcpy(&e[1], ix->lab_off + vb + n, 8, hipMemcpyDeviceToHost) != hipSuccess)
        return SPC_ERR_DEVICE;
    if (n_out) *n_out = n;
    if (entries_out) *entries_out = e[1] - e[0];
    return SPC_OK;
}

spc_status spc_export_labels(const spc_index *ix, uint32_t graph_id, uint64_t *off, uint32_t *hub,
                             uint16_t *dist, uint64_t *count, uint32_t *order, int32_t on_device,
                             void *stream) {
    return spc::export_impl(ix, graph_id, off, hub, dist, count, order, on_device,
                            static_cast<hipStream_t>(stream));
}

spc_status spc_export_reduction(const spc_index *ix, uint32_t graph_id, uint32_t *root,
                                uint32_t *depth, uint32_t *parent, int32_t on_device, void *stream) {
    return spc::export_reduction_impl(ix, graph_id, root, depth, parent, on_device,
                                      static_cast<hipStream_t>(stream));
}

}  // extern "C"
