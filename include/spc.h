/*
 * spc.h -- C ABI of the MI355X (gfx950) shortest-path-counting label library.
 *
 * The library builds the 2-hop SPC label index of PSPC (Peng, Yu, Wang,
 * "PSPC: Efficient Parallel Shortest Path Counting on Large-Scale Graphs")
 * round by round over the distance d = 0, 1, 2, ... with the PULL
 * propagation (Alg. 2, label propagation function Eq. PSPCdu, Label
 * Elimination / Label Merging), and answers SPC queries with the label merge
 * of Eq. (con:spc1)-(con:spc2).  Every step runs in the library's own HIP
 * kernels on the GPU; no entry point falls back to the CPU.
 *
 * Index semantics (Section "The Construction of an ESPC Index"): with the
 * vertices ranked by a total order (rank 0 = most important), L(v) holds
 * (w, sd(v,w), tau(v,w)) for every w ranked at or above v with tau >= 1, where
 * tau counts the shortest v-w paths whose vertices other than w all rank
 * below w.  Both canonical and non-canonical hubs are kept; this is exactly
 * the set that makes the query return (sd(s,t), number of shortest paths).
 *
 * Integer semantics: distances are uint8 or uint16 (dist_bits); counts are
 * uint64 and saturate: every stored or returned count is
 * min(true count, 2^64-1), and 2^64-1 itself is reported as saturated.
 *
 * Conventions for every entry point
 *   - Status codes only; nothing throws across the ABI.  On error, *out
 *     arguments are left untouched and no memory is leaked.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Build and stats calls synchronise that stream before returning; query
 *     calls are asynchronous on it.
 *   - Device pointers are plain device addresses (e.g. a torch tensor's
 *     data_ptr()); the caller owns them.  The index owns all device memory it
 *     allocates until spc_free.
 *   - Thread safety: concurrent spc_query_batch calls on one index, from any
 *     streams, are safe (the index is read-only once built).
 */
#ifndef SPC_H
#define SPC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spc_index spc_index;

typedef enum {
    SPC_OK = 0,
    SPC_ERR_INVALID_ARG = 1,   /* NULL pointer, bad size, id >= n, not a simple symmetric CSR */
    SPC_ERR_OUT_OF_MEMORY = 2, /* device allocation failed or mem_budget exceeded */
    SPC_ERR_DEVICE = 3,        /* a HIP runtime call failed */
    SPC_ERR_DIST_RANGE = 4,    /* a distance does not fit the requested dist_bits */
    SPC_ERR_UNSUPPORTED = 5    /* graph larger than the packed label layout allows */
} spc_status;

/* Per-query flag bits written by spc_query_batch. */
#define SPC_FLAG_SATURATED 0x1u  /* count is 2^64-1: true count >= 2^64-1 */
#define SPC_FLAG_UNREACHABLE 0x2u /* no common hub: dist = INF (type max), count 0 */
#define SPC_FLAG_HORIZON 0x4u    /* truncated index: answer not proven exact (dist > round cap or none found) */
#define SPC_FLAG_INVALID 0x8u    /* s or t >= n: dist = INF, count 0 */

/* Propagation paradigm (spc_build_opts.propagation). */
#define SPC_PROPAGATE_PULL 0u
#define SPC_PROPAGATE_PUSH 1u
#define SPC_PROPAGATE_AUTO 2u

/* Index reductions (spc_build_opts.reduce). */
#define SPC_REDUCE_ONE_SHELL 0x1u   /* Section "Reduction by 1-Shell": label only the core */
#define SPC_REDUCE_EQUIVALENCE 0x2u /* Section "Reduction by Equivalence Relation" */

/* An undirected, unweighted graph (Preliminaries: G = (V, E)) as a symmetric
 * CSR: the neighbours of v are col[row_off[v] .. row_off[v+1]).  Every edge
 * appears in both directions; no self loops, no duplicate entries.
 * nnz = row_off[n] = 2m.  All pointers are device pointers when on_device is
 * nonzero, host pointers otherwise; they are only read during the call. */
typedef struct {
    uint32_t n;
    uint64_t nnz;
    const uint64_t *row_off; /* [n+1] */
    const uint32_t *col;     /* [nnz] */
    /* Optional explicit total order, order[r] = vertex of rank r (a
     * permutation of 0..n-1).  NULL: degree-based order (Section "Vertex
     * Ordering Strategies": higher degree ranks higher), ties by tie_key
     * ascending when tie_key is given, then by vertex id. */
    const uint32_t *order;
    const uint64_t *tie_key; /* [n] or NULL */
    int32_t on_device;
    /* Nonzero: a directed graph (Section "2-Hop Labeling for Shortest Path
     * Counting").  row_off/col then hold each arc a -> b once, in row a
     * (nnz = arcs); no self loops or repeated arcs (checked when
     * opts.validate is set).  The index holds an out-label and an in-label
     * per vertex: L_out(v) = {(w, sd(v,w), c)} and L_in(v) = {(w, sd(w,v), c)}
     * for hubs w ranked at or above v that reach v (or are reached) along a
     * shortest path on which every other vertex ranks below w, c counting
     * those paths; spc_query_batch answers SPC(s, t) for paths from s to t
     * by Eq. (con:spc1)-(con:spc2) over L_out(s) and L_in(t).  Without an
     * explicit order, vertices rank by total degree (out + in) descending,
     * ties by tie_key, then id (the paper fixes no directed order).  One
     * graph per build (spc_build_index_batch: SPC_ERR_UNSUPPORTED), no
     * reduction (SPC_ERR_INVALID_ARG), and every round pulls whatever
     * propagation asks.  Exports (spc_graph_entries, spc_export_labels) cover
     * 2n label rows: rank r's out-label, then at n + r its in-label; the
     * order export has n entries. */
    int32_t directed;
} spc_graph;

typedef struct {
    uint32_t dist_bits;  /* 0 = 8-bit labels, widened to 16 bits when a round passes 254;
                            8 = fail with SPC_ERR_DIST_RANGE past 254; 16 = 16-bit labels */
    uint32_t round_cap;  /* 0 = build to completion; D > 0 = build the distance-partial
                            set L_{<=D} (Def. DPLS) and mark the index truncated if
                            round D+1 would have had candidates */
    uint64_t mem_budget; /* device bytes the build may hold at once; 0 = unlimited */
    uint32_t validate;   /* nonzero: check that the CSR is simple and symmetric */
    /* 0, or SPC_REDUCE_ONE_SHELL (Section "Reduction by 1-Shell"): the
     * fringe -- every vertex outside the 2-core, i.e. the trees hanging off
     * the rest of the graph by one edge, and whole tree components but one
     * vertex each -- is cut off and only the remaining core is labelled
     * (ordered by its own degrees when no order is given, else by the given
     * order restricted to it).  Each fringe vertex v keeps root(v) (the core
     * vertex its tree hangs from; the centre of a tree component, the smaller
     * id of two centres), its depth (distance to root(v)) and its parent (next
     * vertex towards root(v)); queries answer from these and the core labels
     * (spc_query_batch).
     * SPC_REDUCE_EQUIVALENCE (Section "Reduction by Equivalence Relation"):
     * u and v are twins when nbr(u) minus {v} equals nbr(v) minus {u}; each
     * class of twins keeps its smallest id as representative, weighted by the
     * class size, and only the subgraph induced by the representatives is
     * labelled (its own degree order, or the given order restricted).  Label
     * counts then weight every path by the product of the class sizes of its
     * inner vertices, and spc_export_reduction reports root(v) = v's
     * representative, depth 0.  One reduction per build: any other value of
     * reduce is SPC_ERR_INVALID_ARG. */
    uint32_t reduce;
    /* SPC_PROPAGATE_PULL (0, Alg. 2), SPC_PROPAGATE_PUSH (Alg. 1: from round 2
     * on, every vertex scatters its newest entries to its neighbours, the
     * pushes are sorted and equal hubs merged before elimination and
     * pruning), or SPC_PROPAGATE_AUTO (push in a round whose pushes are
     * fewer than the adjacency slots, else pull).  The index is the same
     * either way.  Pushing needs a validated graph (validate nonzero);
     * without validation every round pulls.  Other values:
     * SPC_ERR_INVALID_ARG. */
    uint32_t propagation;
    uint32_t reserved;   /* must be 0 */
    /* Path of an on-disk tuning cache, or NULL.  The file holds text lines
     * "<key> <cfg> <small>": key = 16 hex digits naming an index (a hash of
     * its vertex, edge, entry and round counts, largest distance, graph
     * count, direction, output width, the device's name and the table of
     * launch configurations), cfg its query
     * launch configuration (spc_tune_queries), small its bucket threshold
     * (spc_tune_query_buckets).  A build that finds its key takes both;
     * the tuners, on an index built with a cache path, write their results
     * back (the file is rewritten whole through a temporary file renamed
     * over it).  A missing or unreadable file leaves the defaults; a failed
     * write is ignored.  spc_stats.tune_cached tells whether the build found
     * its key. */
    const char *tune_cache;
} spc_build_opts;

typedef struct {
    uint32_t n;               /* vertices (all graphs of a batch) */
    uint32_t num_graphs;      /* 1, or k for spc_build_index_batch */
    uint64_t m;               /* undirected edges */
    uint64_t entries;         /* label entries, self entries included */
    uint32_t rounds;          /* last round run: first empty round, or the cap */
    uint32_t max_dist;        /* largest label distance */
    uint32_t dist_bits;       /* 8 or 16: width of query dist outputs (8 when every query
                                 distance fits in 0..254: twice the largest label distance,
                                 plus twice the largest fringe depth, at most 254) */
    uint32_t truncated;       /* 1 if round_cap stopped the build early */
    uint64_t saturated_entries; /* entries whose count is 2^64-1 */
    uint64_t index_bytes;     /* device bytes held by the finished index */
    uint64_t peak_build_bytes;/* largest device footprint during the build */
    double ms_order;          /* vertex ordering + relabel + validation */
    double ms_rounds;         /* distance rounds (expand, aggregate, prune, insert) */
    double ms_finalize;       /* hub-ordered count array */
    double ms_total;          /* whole build on the device */
    double ms_round_kernel;   /* time inside the fused round kernel only */
    uint64_t alg_bytes_round_kernel; /* algorithmic bytes of the fused round kernel */
    uint64_t round_kernel_launches;  /* dispatches of the fused round kernel */
    uint32_t query_config;           /* query launch configuration in use */
    uint32_t label_bits;             /* 8 or 16: width of stored label distances */
    uint64_t fringe_vertices;        /* vertices cut off by SPC_REDUCE_ONE_SHELL (0 otherwise) */
    uint32_t fringe_depth;           /* largest fringe depth */
    uint32_t twin_vertices;          /* vertices merged into a representative by
                                        SPC_REDUCE_EQUIVALENCE (0 otherwise) */
    uint32_t directed;               /* 1 for an index of a directed graph (entries
                                        count both label sets) */
    uint32_t query_small;            /* bucket threshold of spc_query_batch_multi */
    uint32_t tune_cached;            /* 1 if the build took cfg and small from its
                                        tuning cache (spc_build_opts.tune_cache) */
} spc_stats;

/* Build the index of one graph (Alg. 2 rounds until a round adds no entry).
 * g, opts and out must be non-NULL.  Returns SPC_ERR_INVALID_ARG for a
 * malformed graph (ids >= n, self loops, asymmetric or duplicate entries when
 * validate is set, order not a permutation), SPC_ERR_UNSUPPORTED when
 * n >= 2^24 - 1 with dist_bits = 8, n > 2^26 - 1024 (all graphs of a batch
 * together) or nnz > 2^32 - 2^20, SPC_ERR_DIST_RANGE as documented above or
 * when a query distance could exceed 65534 (twice the largest label distance
 * plus twice the largest fringe depth). */
spc_status spc_build_index(const spc_graph *g, const spc_build_opts *opts, void *stream,
                           spc_index **out);

/* Build one index over k independent graphs at once (their disjoint union,
 * each graph ranked by its own order).  Labels never cross graphs, so every
 * graph's labels equal those of a solo build.  gs[k]; queries name a graph. */
spc_status spc_build_index_batch(const spc_graph *gs, uint32_t k, const spc_build_opts *opts,
                                 void *stream, spc_index **out);

/* SPC queries (Eq. con:spc1 and con:spc2) on graph `graph_id` of the index
 * (0 for single-graph indexes).  s, t: device uint32[nq] with vertex ids of
 * that graph.  Outputs (device, caller-owned, nq each): dist_out is uint8 when
 * spc_stats.dist_bits is 8 and uint16 otherwise, INF = the type's maximum;
 * count_out uint64; flags_out uint8 (SPC_FLAG_*, may be NULL).  s = t gives
 * (0, 1).  Asynchronous on `stream`; nq == 0 is a no-op.
 * With SPC_REDUCE_ONE_SHELL ("Query Evaluation in Parallel" of that section):
 * when root(s) = root(t) the only shortest path is the tree path, count 1,
 * distance depth(s) + depth(t) - 2 depth(lowest common ancestor); otherwise
 * the core labels of root(s) and root(t) are joined and depth(s) + depth(t)
 * is added to the distance (the count is unchanged: every s-t path runs
 * through root(s) and root(t), each reached by one path).
 * With SPC_REDUCE_EQUIVALENCE: s = t gives (0, 1); two members of one class
 * are adjacent, (1, 1), or share all their k neighbours, (2, k) (k = 0:
 * unreachable); otherwise the labels of the two representatives are joined,
 * each common hub other than the representatives counting once per member
 * of its class (a shortest path meets a class at most once, and any member
 * can take the place of the one it meets).
 * Queries are independent ("Query Evaluation in Parallel"): a batch of at
 * least 2^20 is answered grouped by the label the kernel stages (the longer
 * of L(s), L(t) when undirected, L_out(s) when directed), so the queries that
 * share it run side by side and read it from cache; answers are the same and
 * are written by query index.  That grouping takes 8 bytes per query (at most
 * 2^24 at a time) and 16 per label row of scratch from the device's
 * stream-ordered allocator on `stream` (SPC_ERR_OUT_OF_MEMORY if it has
 * none); SPC_QUERY_ORDER=0 in the environment turns it off. */
spc_status spc_query_batch(const spc_index *ix, uint32_t graph_id, const uint32_t *s,
                           const uint32_t *t, uint64_t nq, void *dist_out, uint64_t *count_out,
                           uint8_t *flags_out, void *stream);

/* SPC queries over several graphs of an index in one call ("Query
 * Evaluation in Parallel": queries are independent, so they can be grouped
 * freely).  Query i asks SPC(s[i], t[i]) on graph graph_ids[i] (device
 * uint32[nq]; NULL: every query on graph 0); answers, flags and output
 * widths as spc_query_batch (an id past the index's graphs, or a vertex id
 * past its graph, gives SPC_FLAG_INVALID).  The queries are first grouped by
 * their work, |L(s)| + |L(t)|: short ones are answered by 16 lanes each
 * (four per wave), the others by a wave each with the index's query
 * configuration, so graphs with short labels do not leave most of a wave
 * idle.  Scratch: 4 bytes per query (at most 2^24 at a time) taken from the
 * device's stream-ordered allocator on `stream` and given back on it.
 * Asynchronous on `stream`; nq == 0 is a no-op; SPC_ERR_INVALID_ARG for a
 * NULL index or a NULL s, t, dist_out or count_out with nq > 0. */
spc_status spc_query_batch_multi(const spc_index *ix, const uint32_t *graph_ids, const uint32_t *s,
                                 const uint32_t *t, uint64_t nq, void *dist_out, uint64_t *count_out,
                                 uint8_t *flags_out, void *stream);

/* spc_query_batch_multi for callers that cannot allocate device memory
 * while they run: work captured into a HIP graph, tight serving loops, and
 * runtimes that forbid allocation inside a request.  Same arguments and
 * answers; no hipMalloc, no stream-ordered allocation, no allocating library
 * call: the bucketing scratch (4 bytes per query and two counters) is a
 * fixed device array of the library, 16 MiB + 256 B on every GPU the library
 * runs on, held until the process ends.  Limit: nq <= 2^22 queries per call
 * (SPC_ERR_UNSUPPORTED beyond, before any launch).  Every call on one GPU
 * uses that GPU's single array, whose counters a kernel clears at the start
 * of each call: calls that overlap on one GPU (several streams, several host
 * threads) race and must be serialised by the caller, e.g. on one stream.
 * The first call on a device looks the array's address up with the index's
 * device current (SPC_ERR_DEVICE if the runtime refuses). */
spc_status spc_query_batch_multi_noalloc(const spc_index *ix, const uint32_t *graph_ids,
                                         const uint32_t *s, const uint32_t *t, uint64_t nq,
                                         void *dist_out, uint64_t *count_out, uint8_t *flags_out,
                                         void *stream);

/* Bucketing of spc_query_batch_multi: queries with |L(s)| + |L(t)| at most
 * `small` take the 16-lanes-per-query path; 0 turns bucketing off (every
 * query a wave).  A new index starts at 256.  The tuner times the
 * thresholds 0, 64, 128, ..., 2048 on the sample queries (device pointers;
 * graph_ids may be NULL), twice each with events on `stream`, checks that
 * every threshold's answers equal those of 0 (SPC_ERR_DEVICE if not), keeps
 * the fastest and returns it in *small_out (may be NULL).  The tuner
 * allocates scratch, synchronises `stream`, and must not run concurrently
 * with queries on the same index; so must not spc_set_query_buckets.
 * SPC_ERR_INVALID_ARG for a NULL index (or NULL samples, nq == 0). */
spc_status spc_tune_query_buckets(spc_index *ix, const uint32_t *graph_ids, const uint32_t *s,
                                  const uint32_t *t, uint64_t nq, void *stream, uint32_t *small_out);
spc_status spc_set_query_buckets(spc_index *ix, uint32_t small);

/* Release the index (waits for the device to finish work that may still
 * read it).  Its device blocks go to the library's per-device block cache,
 * where later builds reuse them.  spc_free(NULL) is a no-op. */
void spc_free(spc_index *ix);

/* Return every cached device block to the HIP runtime (all devices).  The
 * cache is also flushed automatically when an allocation would fail, and
 * trimmed after every build and free to the limit spc_set_cache_limit sets
 * (default: a quarter of the device's memory). */
void spc_release_cached_memory(void);

/* Most device memory, in bytes, that the cache keeps per device after a
 * build or a free (UINT64_MAX: all of it, until spc_release_cached_memory).
 * Memory the runtime takes back is cleared by the driver before it is
 * handed out again (seconds per 100 GB), so a process that builds large
 * indexes one after another keeps it.  Applies to later builds and frees
 * of every device; there is no error. */
void spc_set_cache_limit(uint64_t bytes);

/* Summary numbers of a finished build (host struct). */
spc_status spc_index_stats(const spc_index *ix, spc_stats *out);

/* Per-round counters, rounds 0 .. min(rounds, max_rounds-1), into host arrays
 * of max_rounds entries (any may be NULL): raw = candidates pulled that pass
 * the rank rule (Lemma prune1), merged = distinct candidate hubs left after
 * Label Elimination and Label Merging, kept = entries inserted (these three
 * are properties of the index and the order alone); scanned = label entries
 * the prune probes read beyond the landmark rows, up to and including the
 * first one proving a shorter distance (a cost counter of this
 * implementation). */
spc_status spc_round_stats(const spc_index *ix, uint32_t max_rounds, uint64_t *raw,
                           uint64_t *merged, uint64_t *kept, uint64_t *scanned);

/* Per-round cost profile of the build, same indexing as spc_round_stats:
 * time inside the fused round kernel (ms), label entries of the pullers
 * staged on chip, landmark-row bytes read by prune probes, round segment
 * headers read by prune probes, the device bytes the build held at the
 * round's high-water mark, and the bytes of membership-filter words the
 * prune probes looked up (0 in a round built without the filter: the filter
 * of the older labels' (vertex, hub, distance) triples is an implementation
 * device that skips most label searches; it changes no result).  Host
 * arrays; any may be NULL. */
spc_status spc_round_profile(const spc_index *ix, uint32_t max_rounds, double *kernel_ms,
                             uint64_t *staged, uint64_t *row_bytes, uint64_t *headers,
                             uint64_t *mem_peak, uint64_t *filter_bytes);

/* Number of labelled vertices (the core under SPC_REDUCE_ONE_SHELL, else
 * every vertex) and label entries of graph `graph_id` (host out). */
spc_status spc_graph_entries(const spc_index *ix, uint32_t graph_id, uint32_t *n_out,
                             uint64_t *entries_out);

/* Export the labels of graph `graph_id` in RANK space (vertex id = rank in
 * that graph, hubs likewise), each label sorted by hub: off[n+1], hub, dist,
 * count[entries], order[n] (rank -> vertex id), n = the labelled vertices of
 * spc_graph_entries (for a reduced index, the core; order then gives the
 * input graph's vertex ids).  Pointers are device pointers when on_device is
 * nonzero, host pointers otherwise; any may be NULL to skip it.
 * Synchronises `stream`. */
spc_status spc_export_labels(const spc_index *ix, uint32_t graph_id, uint64_t *off,
                             uint32_t *hub, uint16_t *dist, uint64_t *count, uint32_t *order,
                             int32_t on_device, void *stream);

/* The 1-shell of graph `graph_id` (Section "Reduction by 1-Shell"), per
 * vertex of the input graph: root[v] (shr(v): the core vertex v's tree hangs
 * from, v itself in the core), depth[v] (distance to root[v]), parent[v]
 * (the neighbour of v on the path to root[v], v itself in the core).  Under
 * SPC_REDUCE_EQUIVALENCE root[v] is v's representative, depth 0, parent v;
 * an index built without a reduction reports every vertex as its own root.
 * Arrays of the graph's input size n; device pointers when on_device is
 * nonzero, host pointers otherwise; any may be NULL.  Synchronises `stream`. */
spc_status spc_export_reduction(const spc_index *ix, uint32_t graph_id, uint32_t *root,
                                uint32_t *depth, uint32_t *parent, int32_t on_device,
                                void *stream);

/* Query launch configurations.  The query kernel stages slices of L(s) in
 * LDS and streams L(t) past them; a configuration fixes the slice length
 * (stage, entries) and the L(t) tiles of 64 requested per round of loads
 * (tiles).  spc_query_config_count() configurations exist, numbered from 0
 * (the default of a new index).  spc_query_config_info returns
 * SPC_ERR_INVALID_ARG for a number out of range; either output may be NULL. */
uint32_t spc_query_config_count(void);
spc_status spc_query_config_info(uint32_t cfg, uint32_t *stage, uint32_t *tiles);

/* Autotuner ("Query Evaluation in Parallel": queries are independent, so
 * any launch shape gives the same answers): run the nq sample queries s, t
 * (device pointers, ids of graph graph_id) once per configuration, twice
 * each, timed with events on `stream`, grouped by staged label as large
 * batches of spc_query_batch are (unless SPC_QUERY_ORDER=0), so a sample of
 * the size of the batches to come tunes for them best; check that every configuration's
 * answers equal configuration 0's (SPC_ERR_DEVICE if not); keep the fastest
 * as the index's configuration and return its number in *cfg_out (may be
 * NULL).  Allocates scratch device memory for the outputs, synchronises
 * `stream`, and must not run concurrently with queries on the same index. */
spc_status spc_tune_queries(spc_index *ix, uint32_t graph_id, const uint32_t *s, const uint32_t *t,
                            uint64_t nq, void *stream, uint32_t *cfg_out);

/* Set the index's query configuration (e.g. one tuned on another index of
 * the same workload).  SPC_ERR_INVALID_ARG for ix NULL or cfg out of range;
 * must not run concurrently with queries on the same index. */
spc_status spc_set_query_config(spc_index *ix, uint32_t cfg);

/* Hybrid vertex order ("Vertex Ordering Strategies": tree-decomposition
 * order for the fringe, degree order for the core), for spc_graph.order.
 * Fringe: vertices are removed one at a time, always one of least current
 * degree (ties: smaller id), while that degree is at most delta; the
 * remaining neighbours of a removed vertex are connected pairwise, so later
 * degrees are those of this elimination graph.  Core: the vertices left,
 * ranked first by input degree (descending, ties by id); then the fringe in
 * reverse order of removal.  delta = 0xFFFFFFFF gives the pure
 * tree-decomposition order.  g is a HOST CSR (on_device = 0; self loops and
 * repeated entries ignored); order_out[n] receives rank -> vertex;
 * *core_out (may be NULL) the core size.  Runs on the host.
 * SPC_ERR_INVALID_ARG for NULL pointers, a device graph or ids >= n. */
spc_status spc_hybrid_order(const spc_graph *g, uint32_t delta, uint32_t *order_out,
                            uint32_t *core_out);

/* Static string for a status code. */
const char *spc_status_string(spc_status s);

#ifdef __cplusplus
}
#endif

#endif /* SPC_H */
