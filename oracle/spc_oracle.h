/*
 * CPU oracle for the shortest-path-counting (SPC) 2-hop label index.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this library.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * Conventions
 *   - Graphs are simple, undirected, unweighted, given as a symmetric CSR
 *     (off[n+1], adj[off[n]]).  Most functions take the graph in RANK space:
 *     vertex id == rank, 0 is the most important vertex.
 *   - A label entry is (hub, dist, count).  Counts saturate at 2^64-1: every
 *     stored count is min(true count, 2^64-1).
 *   - Distances are uint32; ORACLE_INF (0xFFFFFFFF) marks "unreachable".
 *   - depth_cap == 0 means no cap; otherwise only entries with dist <= cap
 *     are built (the distance-partial set L_{<=cap}).
 */
#ifndef SPC_ORACLE_H
#define SPC_ORACLE_H
#include <stdint.h>

#define ORACLE_INF 0xFFFFFFFFu
#define ORACLE_SAT 0xFFFFFFFFFFFFFFFFull

typedef struct oracle_index oracle_index;

/* Degree-descending order; ties by tie_key ascending (if non-NULL), then by id.
 * order[r] = vertex of rank r. */
void oracle_degree_order(uint32_t n, const uint64_t *off, const uint64_t *tie_key,
                         uint32_t *order);

/* CSR in rank space: vertex r is order[r]; adjacency lists sorted ascending. */
void oracle_relabel(uint32_t n, const uint64_t *off, const uint32_t *adj,
                    const uint32_t *order, uint64_t *roff, uint32_t *radj);

/* Breadth-first search with shortest-path counting (saturating).
 * restricted != 0: besides src only vertices with id > src may be entered.
 * dist[] gets ORACLE_INF for unreached vertices, sigma[] gets 0 there. */
void oracle_bfs_count(uint32_t n, const uint64_t *off, const uint32_t *adj,
                      uint32_t src, int restricted, uint32_t depth_cap,
                      uint32_t *dist, uint64_t *sigma);

/* Entries whose hub is w, straight from the trough-path definition.
 * Writes (vertex, dist, count) triples in increasing vertex id; returns the
 * count.  Output arrays need room for n entries. */
uint64_t oracle_hub_column(uint32_t n, const uint64_t *off, const uint32_t *adj,
                           uint32_t w, uint32_t depth_cap,
                           uint32_t *out_v, uint32_t *out_d, uint64_t *out_c);

/* Full index builders (rank-space graph).  All three must agree exactly. */
oracle_index *oracle_build_definition(uint32_t n, const uint64_t *off,
                                      const uint32_t *adj, uint32_t depth_cap);
oracle_index *oracle_build_pruned(uint32_t n, const uint64_t *off,
                                  const uint32_t *adj, uint32_t depth_cap,
                                  uint32_t max_hubs, double time_limit_s);
oracle_index *oracle_build_pull(uint32_t n, const uint64_t *off, const uint32_t *adj,
                                uint32_t depth_cap);
/* oracle_build_pull with the pullers of each round spread over nthreads
 * threads (0 or 1: the calling thread).  Same index and counters. */
/* Nonzero: the PULL builders print progress lines on stderr (one per round,
 * and one every 2^16 pullers within a round). */
void oracle_set_progress(int on);
oracle_index *oracle_build_pull_threads(uint32_t n, const uint64_t *off, const uint32_t *adj,
                                        uint32_t depth_cap, uint32_t nthreads);
/* The definition builder with vertex weights weight[rank]: an entry's count
 * sums, over its trough shortest paths, the product of the weights of the
 * path's inner vertices (all weights 1: the plain index). */
oracle_index *oracle_build_definition_weighted(uint32_t n, const uint64_t *off, const uint32_t *adj,
                                               const uint64_t *weight, uint32_t depth_cap);

/* Directed labels from the definition (rank-space digraph: out-arcs off/adj,
 * in-arcs ioff/iadj, no self loops or repeated arcs).  The index has 2n rows:
 * row v < n is L_out(v) = {(w, sd(v,w), c)}, row n + v is L_in(v) =
 * {(w, sd(w,v), c)}, for hubs w ranked at or above v with a trough path. */
oracle_index *oracle_build_directed_definition(uint32_t n, const uint64_t *off, const uint32_t *adj,
                                               const uint64_t *ioff, const uint32_t *iadj);

uint64_t oracle_index_entries(const oracle_index *ix);
/* Last round run by a round-by-distance build: the first empty round
 * (largest distance + 1) or the depth cap. */
uint32_t oracle_index_rounds(const oracle_index *ix);
uint32_t oracle_index_hubs_done(const oracle_index *ix);
/* Export: off[n+1], hub/dist/count[entries]; per vertex sorted by hub. */
void oracle_index_export(const oracle_index *ix, uint64_t *off, uint32_t *hub,
                         uint32_t *dist, uint64_t *count);
/* Per-round counters of the PULL builder, rounds 0..rounds inclusive:
 * raw  = candidates pulled that pass the rank rule,
 * merged = distinct candidate hubs not already held at a smaller distance,
 * kept = entries inserted, scanned = probe entries scanned in hub order. */
void oracle_index_round_stats(const oracle_index *ix, uint64_t *raw, uint64_t *merged,
                              uint64_t *kept, uint64_t *scanned);
/* Byte-model inputs of a PULL build, rounds 0..rounds: active = pullers with
 * at least one candidate passing the rank rule, active_adj = their adjacency
 * slots, staged = label entries (distance < d) of the pullers with at least
 * one merged candidate.  Zeros for other builders. */
void oracle_index_model_stats(const oracle_index *ix, uint64_t *active, uint64_t *active_adj,
                              uint64_t *staged);
void oracle_index_free(oracle_index *ix);

/* SPC query over an index (rank ids): minimum of d_s+d_t over common hubs and
 * the saturating sum of count products at that minimum.  No common hub gives
 * (ORACLE_INF, 0). */
void oracle_query(const oracle_index *ix, uint32_t s, uint32_t t, uint32_t *dist,
                  uint64_t *count);
void oracle_query_batch(const oracle_index *ix, uint64_t q, const uint32_t *s,
                        const uint32_t *t, uint32_t *dist, uint64_t *count);

/* Same query over exported label arrays (any source of labels). */
void oracle_query_arrays(const uint64_t *off, const uint32_t *hub, const uint32_t *dist,
                         const uint64_t *count, uint64_t q, const uint32_t *s,
                         const uint32_t *t, uint32_t *out_d, uint64_t *out_c);

/* oracle_query_arrays with the queries split over nthreads threads. */
void oracle_query_arrays_threads(const uint64_t *off, const uint32_t *hub, const uint32_t *dist,
                                 const uint64_t *count, uint64_t q, const uint32_t *s,
                                 const uint32_t *t, uint32_t *out_d, uint64_t *out_c,
                                 uint32_t nthreads);

/* Hubs of L(s) and their distances from the definition (no counts), by one
 * BFS from s (rank-space graph); increasing hub order; returns how many.
 * out_hub, out_dist need room for n entries. */
uint64_t oracle_label_hubs(uint32_t n, const uint64_t *off, const uint32_t *adj, uint32_t s,
                           uint32_t *out_hub, uint32_t *out_dist);

#endif
