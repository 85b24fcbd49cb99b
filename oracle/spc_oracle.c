/*
 * CPU oracle for the SPC 2-hop label index of PSPC (Peng, Yu, Wang).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path.  Plain, slow,
 * sequential C99, written to be checked against the paper by eye.
 *
 * What is computed (Section "The Construction of an ESPC Index"): for a
 * total order on V, the entry (w, sd(v,w), tau(v,w)) is in L(v) iff w ranks
 * at or above v and tau(v,w) >= 1, where tau(v,w) is the number of shortest
 * v-w paths on which every vertex other than w ranks strictly below w (the
 * trough shortest paths).  Such a label set is an exact shortest path
 * covering, so the query of Eq. (con:spc1)-(con:spc2) returns the distance
 * and the number of shortest paths for every pair.
 *
 * Three builders produce this same set:
 *   oracle_build_definition  the definition itself: per hub w, one BFS over
 *                            the whole graph (true distances) and one BFS
 *                            over {w} and the vertices ranked below w
 *                            (trough distances and trough path counts);
 *   oracle_build_pruned      hub-by-hub pruned BFS in rank order, pruning a
 *                            vertex when a 2-hop query over the labels of
 *                            earlier hubs is already shorter (the sequential
 *                            construction the paper starts from);
 *   oracle_build_pull        the paper's round-by-distance PULL propagation
 *                            (Alg. 2 with the label propagation function,
 *                            Eq. PSPCdu, and the Label Elimination / Label
 *                            Merging rules), one round per distance.
 *
 * Counts saturate at 2^64-1.  Saturating addition and multiplication of
 * non-negative integers give min(true value, 2^64-1) whatever the order of
 * evaluation, so all builders and the GPU path must agree bit for bit.
 */
#include "spc_oracle.h"

#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

static uint64_t sat_add(uint64_t a, uint64_t b) { return (a > ORACLE_SAT - b) ? ORACLE_SAT : a + b; }
static uint64_t sat_mul(uint64_t a, uint64_t b)
{
    if (a == 0 || b == 0) return 0;
    return (a > ORACLE_SAT / b) ? ORACLE_SAT : a * b;
}

static void *xmalloc(size_t sz)
{
    void *p = malloc(sz ? sz : 1);
    if (!p) abort();
    return p;
}
static void *xcalloc(size_t k, size_t sz)
{
    void *p = calloc(k ? k : 1, sz ? sz : 1);
    if (!p) abort();
    return p;
}

/* ------------------------------------------------------------------------ */
/* Vertex order (Section "Vertex Ordering Strategies", degree-based scheme:  */
/* high degree = high rank).                                                  */
/* ------------------------------------------------------------------------ */
static const uint64_t *g_ord_off;
static const uint64_t *g_ord_tie;

static int cmp_order(const void *pa, const void *pb)
{
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    uint64_t da = g_ord_off[a + 1] - g_ord_off[a];
    uint64_t db = g_ord_off[b + 1] - g_ord_off[b];
    if (da != db) return da > db ? -1 : 1;
    if (g_ord_tie) {
        uint64_t ta = g_ord_tie[a], tb = g_ord_tie[b];
        if (ta != tb) return ta < tb ? -1 : 1;
    }
    return a < b ? -1 : (a > b ? 1 : 0);
}

void oracle_degree_order(uint32_t n, const uint64_t *off, const uint64_t *tie_key,
                         uint32_t *order)
{
    for (uint32_t i = 0; i < n; i++) order[i] = i;
    g_ord_off = off;
    g_ord_tie = tie_key;
    qsort(order, n, sizeof(uint32_t), cmp_order);
    g_ord_off = NULL;
    g_ord_tie = NULL;
}

static int cmp_u32(const void *pa, const void *pb)
{
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    return a < b ? -1 : (a > b ? 1 : 0);
}

void oracle_relabel(uint32_t n, const uint64_t *off, const uint32_t *adj,
                    const uint32_t *order, uint64_t *roff, uint32_t *radj)
{
    uint32_t *rank = xmalloc(sizeof(uint32_t) * (size_t)n);
    for (uint32_t r = 0; r < n; r++) rank[order[r]] = r;
    roff[0] = 0;
    for (uint32_t r = 0; r < n; r++) {
        uint32_t v = order[r];
        uint64_t deg = off[v + 1] - off[v];
        for (uint64_t k = 0; k < deg; k++) radj[roff[r] + k] = rank[adj[off[v] + k]];
        qsort(radj + roff[r], deg, sizeof(uint32_t), cmp_u32);
        roff[r + 1] = roff[r] + deg;
    }
    free(rank);
}

/* ------------------------------------------------------------------------ */
/* BFS with path counting.                                                    */
/* ------------------------------------------------------------------------ */
void oracle_bfs_count(uint32_t n, const uint64_t *off, const uint32_t *adj,
                      uint32_t src, int restricted, uint32_t depth_cap,
                      uint32_t *dist, uint64_t *sigma)
{
    uint32_t *queue = xmalloc(sizeof(uint32_t) * (size_t)n);
    for (uint32_t i = 0; i < n; i++) {
        dist[i] = ORACLE_INF;
        sigma[i] = 0;
    }
    uint64_t head = 0, tail = 0;
    dist[src] = 0;
    sigma[src] = 1;
    queue[tail++] = src;
    while (head < tail) {
        uint32_t v = queue[head++];
        if (depth_cap && dist[v] >= depth_cap) continue; /* do not go past the cap */
        for (uint64_t k = off[v]; k < off[v + 1]; k++) {
            uint32_t x = adj[k];
            if (restricted && x <= src) continue; /* only vertices ranked below src */
            if (dist[x] == ORACLE_INF) {
                dist[x] = dist[v] + 1;
                sigma[x] = sigma[v];
                queue[tail++] = x;
            } else if (dist[x] == dist[v] + 1) {
                sigma[x] = sat_add(sigma[x], sigma[v]);
            }
        }
    }
    free(queue);
}

/* ------------------------------------------------------------------------ */
/* The definition, one hub at a time.                                         */
/* tau(v,w) counts shortest v-w paths whose vertices other than w all rank   */
/* below w.  Such a path lies in the subgraph induced by {w} and the          */
/* vertices ranked below w, so a BFS there counts them whenever its distance */
/* equals the true distance; otherwise tau(v,w) = 0 and there is no entry.    */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t *d_full, *d_res;
    uint64_t *s_full, *s_res;
} hub_scratch;

static void hub_scratch_init(hub_scratch *h, uint32_t n)
{
    h->d_full = xmalloc(sizeof(uint32_t) * (size_t)n);
    h->d_res = xmalloc(sizeof(uint32_t) * (size_t)n);
    h->s_full = xmalloc(sizeof(uint64_t) * (size_t)n);
    h->s_res = xmalloc(sizeof(uint64_t) * (size_t)n);
}
static void hub_scratch_free(hub_scratch *h)
{
    free(h->d_full);
    free(h->d_res);
    free(h->s_full);
    free(h->s_res);
}

static uint64_t hub_column(uint32_t n, const uint64_t *off, const uint32_t *adj, uint32_t w,
                           uint32_t depth_cap, hub_scratch *h, uint32_t *out_v,
                           uint32_t *out_d, uint64_t *out_c)
{
    oracle_bfs_count(n, off, adj, w, 0, depth_cap, h->d_full, h->s_full);
    oracle_bfs_count(n, off, adj, w, 1, depth_cap, h->d_res, h->s_res);
    uint64_t k = 0;
    for (uint32_t v = w; v < n; v++) {
        if (h->d_res[v] == ORACLE_INF) continue;
        if (h->d_res[v] != h->d_full[v]) continue; /* no trough shortest path */
        out_v[k] = v;
        out_d[k] = h->d_res[v];
        out_c[k] = h->s_res[v];
        k++;
    }
    return k;
}

uint64_t oracle_hub_column(uint32_t n, const uint64_t *off, const uint32_t *adj, uint32_t w,
                           uint32_t depth_cap, uint32_t *out_v, uint32_t *out_d,
                           uint64_t *out_c)
{
    hub_scratch h;
    hub_scratch_init(&h, n);
    uint64_t k = hub_column(n, off, adj, w, depth_cap, &h, out_v, out_d, out_c);
    hub_scratch_free(&h);
    return k;
}

/* ------------------------------------------------------------------------ */
/* Index container: one growable label per vertex, plus per-round counters. */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t *hub, *dist;
    uint64_t *cnt;
    uint64_t len, cap;
} olabel;

struct oracle_index {
    uint32_t n;
    olabel *lab;
    uint32_t rounds;
    uint32_t hubs_done;
    uint64_t *st_raw, *st_merged, *st_kept, *st_scanned;
    uint64_t *st_active, *st_active_adj, *st_staged;
    uint32_t st_cap, st_model_cap;
};

static oracle_index *index_new(uint32_t n)
{
    oracle_index *ix = xcalloc(1, sizeof(oracle_index));
    ix->n = n;
    ix->lab = xcalloc(n ? n : 1, sizeof(olabel));
    return ix;
}

static void label_push(olabel *l, uint32_t hub, uint32_t dist, uint64_t cnt)
{
    if (l->len == l->cap) {
        uint64_t nc = l->cap ? 2 * l->cap : 4;
        l->hub = realloc(l->hub, sizeof(uint32_t) * nc);
        l->dist = realloc(l->dist, sizeof(uint32_t) * nc);
        l->cnt = realloc(l->cnt, sizeof(uint64_t) * nc);
        if (!l->hub || !l->dist || !l->cnt) abort();
        l->cap = nc;
    }
    l->hub[l->len] = hub;
    l->dist[l->len] = dist;
    l->cnt[l->len] = cnt;
    l->len++;
}

/* Merge k new entries (hub-sorted, all of distance d, hubs not in the label)
 * into a hub-sorted label, keeping it hub-sorted. */
static void label_merge_sorted(olabel *l, const uint32_t *hub, const uint64_t *cnt, uint64_t k,
                               uint32_t d)
{
    if (k == 0) return;
    uint64_t old = l->len;
    for (uint64_t i = 0; i < k; i++) label_push(l, 0, 0, 0); /* room for k more */
    /* from the back: the larger of the two tails goes last */
    uint64_t a = old, b = k, o = old + k;
    while (b > 0) {
        if (a > 0 && l->hub[a - 1] > hub[b - 1]) {
            a--;
            o--;
            l->hub[o] = l->hub[a];
            l->dist[o] = l->dist[a];
            l->cnt[o] = l->cnt[a];
        } else {
            b--;
            o--;
            l->hub[o] = hub[b];
            l->dist[o] = d;
            l->cnt[o] = cnt[b];
        }
    }
}

static void stats_round(oracle_index *ix, uint32_t d, uint64_t raw, uint64_t merged,
                        uint64_t kept, uint64_t scanned)
{
    if (d >= ix->st_cap) {
        uint32_t nc = ix->st_cap ? 2 * ix->st_cap : 16;
        while (nc <= d) nc *= 2;
        ix->st_raw = realloc(ix->st_raw, sizeof(uint64_t) * nc);
        ix->st_merged = realloc(ix->st_merged, sizeof(uint64_t) * nc);
        ix->st_kept = realloc(ix->st_kept, sizeof(uint64_t) * nc);
        ix->st_scanned = realloc(ix->st_scanned, sizeof(uint64_t) * nc);
        for (uint32_t i = ix->st_cap; i < nc; i++)
            ix->st_raw[i] = ix->st_merged[i] = ix->st_kept[i] = ix->st_scanned[i] = 0;
        ix->st_cap = nc;
    }
    ix->st_raw[d] = raw;
    ix->st_merged[d] = merged;
    ix->st_kept[d] = kept;
    ix->st_scanned[d] = scanned;
}

/* Byte-model inputs of round d (PULL builds; rounds_stats must have run for
 * d first): pullers with at least one candidate passing the rank rule, their
 * adjacency slots, and the label entries (all of distance < d) of the
 * pullers with at least one merged candidate. */
static void stats_model(oracle_index *ix, uint32_t d, uint64_t active, uint64_t active_adj,
                        uint64_t staged)
{
    if (!ix->st_active) {
        ix->st_active = xcalloc(ix->st_cap, sizeof(uint64_t));
        ix->st_active_adj = xcalloc(ix->st_cap, sizeof(uint64_t));
        ix->st_staged = xcalloc(ix->st_cap, sizeof(uint64_t));
        ix->st_model_cap = ix->st_cap;
    }
    if (ix->st_model_cap < ix->st_cap) {
        ix->st_active = realloc(ix->st_active, sizeof(uint64_t) * ix->st_cap);
        ix->st_active_adj = realloc(ix->st_active_adj, sizeof(uint64_t) * ix->st_cap);
        ix->st_staged = realloc(ix->st_staged, sizeof(uint64_t) * ix->st_cap);
        if (!ix->st_active || !ix->st_active_adj || !ix->st_staged) abort();
        for (uint32_t i = ix->st_model_cap; i < ix->st_cap; i++)
            ix->st_active[i] = ix->st_active_adj[i] = ix->st_staged[i] = 0;
        ix->st_model_cap = ix->st_cap;
    }
    ix->st_active[d] = active;
    ix->st_active_adj[d] = active_adj;
    ix->st_staged[d] = staged;
}

static uint32_t max_label_dist(const oracle_index *ix)
{
    uint32_t mx = 0;
    for (uint32_t v = 0; v < ix->n; v++)
        for (uint64_t i = 0; i < ix->lab[v].len; i++)
            if (ix->lab[v].dist[i] > mx) mx = ix->lab[v].dist[i];
    return mx;
}

/* The round in which a round-by-distance build stops: the first round with
 * no entry (one past the largest distance), or the depth cap. */
static uint32_t last_round(const oracle_index *ix, uint32_t depth_cap)
{
    if (ix->n == 0) return 0;
    uint32_t r = max_label_dist(ix) + 1;
    return (depth_cap && r > depth_cap) ? depth_cap : r;
}

/* Sort every label by hub (insertion order may be by round). */
static void sort_labels_by_hub(oracle_index *ix)
{
    for (uint32_t v = 0; v < ix->n; v++) {
        olabel *l = &ix->lab[v];
        for (uint64_t i = 1; i < l->len; i++) { /* insertion sort: plain and stable */
            uint32_t h = l->hub[i], d = l->dist[i];
            uint64_t c = l->cnt[i];
            uint64_t j = i;
            while (j > 0 && l->hub[j - 1] > h) {
                l->hub[j] = l->hub[j - 1];
                l->dist[j] = l->dist[j - 1];
                l->cnt[j] = l->cnt[j - 1];
                j--;
            }
            l->hub[j] = h;
            l->dist[j] = d;
            l->cnt[j] = c;
        }
    }
}

oracle_index *oracle_build_definition(uint32_t n, const uint64_t *off, const uint32_t *adj,
                                      uint32_t depth_cap)
{
    oracle_index *ix = index_new(n);
    hub_scratch h;
    hub_scratch_init(&h, n);
    uint32_t *cv = xmalloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    uint32_t *cd = xmalloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    uint64_t *cc = xmalloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
    for (uint32_t w = 0; w < n; w++) { /* hubs in rank order: labels come out hub-sorted */
        uint64_t k = hub_column(n, off, adj, w, depth_cap, &h, cv, cd, cc);
        for (uint64_t i = 0; i < k; i++) label_push(&ix->lab[cv[i]], w, cd[i], cc[i]);
    }
    free(cv);
    free(cd);
    free(cc);
    hub_scratch_free(&h);
    ix->hubs_done = n;
    ix->rounds = last_round(ix, depth_cap);
    return ix;
}

/* ------------------------------------------------------------------------ */
/* The definition with vertex weights (Section "Reduction by Equivalence    */
/* Relation": one vertex stands for a class of twins and carries its size): */
/* a trough path counts the product of the weights of its inner vertices.   */
/* ------------------------------------------------------------------------ */
oracle_index *oracle_build_definition_weighted(uint32_t n, const uint64_t *off, const uint32_t *adj,
                                               const uint64_t *weight, uint32_t depth_cap)
{
    oracle_index *ix = index_new(n);
    uint32_t *dfull = xmalloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    uint64_t *sfull = xmalloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
    uint32_t *dist = xmalloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    uint64_t *sig = xmalloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
    uint32_t *queue = xmalloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    for (uint32_t w = 0; w < n; w++) {
        oracle_bfs_count(n, off, adj, w, 0, depth_cap, dfull, sfull);
        for (uint32_t i = 0; i < n; i++) {
            dist[i] = ORACLE_INF;
            sig[i] = 0;
        }
        uint64_t head = 0, tail = 0;
        dist[w] = 0;
        sig[w] = 1;
        queue[tail++] = w;
        while (head < tail) {
            uint32_t v = queue[head++];
            if (depth_cap && dist[v] >= depth_cap) continue;
            uint64_t f = v == w ? 1 : weight[v]; /* v is inside every path it extends */
            for (uint64_t k = off[v]; k < off[v + 1]; k++) {
                uint32_t x = adj[k];
                if (x <= w) continue; /* only vertices ranked below w */
                if (dist[x] == ORACLE_INF) {
                    dist[x] = dist[v] + 1;
                    queue[tail++] = x;
                }
                if (dist[x] == dist[v] + 1) sig[x] = sat_add(sig[x], sat_mul(sig[v], f));
            }
        }
        for (uint32_t v = w; v < n; v++)
            if (dist[v] != ORACLE_INF && dist[v] == dfull[v]) label_push(&ix->lab[v], w, dist[v], sig[v]);
    }
    free(dfull);
    free(sfull);
    free(dist);
    free(sig);
    free(queue);
    ix->hubs_done = n;
    ix->rounds = last_round(ix, depth_cap);
    return ix;
}

/* ------------------------------------------------------------------------ */
/* Directed labels (Section "2-Hop Labeling for Shortest Path Counting": an */
/* out-label and an in-label per vertex), from the definition.  Rank-space   */
/* digraph given by its out-arcs (off, adj) and in-arcs (ioff, iadj).  The   */
/* index has 2n rows: row v < n is L_out(v), row n + v is L_in(v).  For a    */
/* hub w and v ranked at or below w: (w, sd(v,w), c) is in L_out(v) when a   */
/* shortest v-to-w path has every vertex but w ranked below w (c counts     */
/* those paths); (w, sd(w,v), c) is in L_in(v) likewise for w-to-v paths.   */
/* Per hub, the v-to-w paths are a BFS from w over the reversed arcs (the    */
/* in-arcs), the w-to-v paths a BFS over the out-arcs; each once over the   */
/* whole digraph (true distances) and once over {w} and the vertices ranked */
/* below w (trough distances and counts).                                   */
/* ------------------------------------------------------------------------ */
static void bfs_count_arcs(uint32_t n, const uint64_t *off, const uint32_t *adj, uint32_t src,
                           int restricted, uint32_t *dist, uint64_t *sigma, uint32_t *queue)
{
    for (uint32_t i = 0; i < n; i++) {
        dist[i] = ORACLE_INF;
        sigma[i] = 0;
    }
    uint64_t head = 0, tail = 0;
    dist[src] = 0;
    sigma[src] = 1;
    queue[tail++] = src;
    while (head < tail) {
        uint32_t v = queue[head++];
        for (uint64_t k = off[v]; k < off[v + 1]; k++) {
            uint32_t x = adj[k];
            if (restricted && x <= src) continue;
            if (dist[x] == ORACLE_INF) {
                dist[x] = dist[v] + 1;
                queue[tail++] = x;
            }
            if (dist[x] == dist[v] + 1) sigma[x] = sat_add(sigma[x], sigma[v]);
        }
    }
}

oracle_index *oracle_build_directed_definition(uint32_t n, const uint64_t *off, const uint32_t *adj,
                                               const uint64_t *ioff, const uint32_t *iadj)
{
    oracle_index *ix = index_new(2 * n);
    uint32_t *df = xmalloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    uint32_t *dr = xmalloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    uint64_t *sf = xmalloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
    uint64_t *sr = xmalloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
    uint32_t *queue = xmalloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    for (uint32_t w = 0; w < n; w++) { /* hubs in rank order: labels come out hub-sorted */
        for (int side = 0; side < 2; side++) {
            /* side 0: L_out (paths v -> w: BFS from w over in-arcs);
             * side 1: L_in (paths w -> v: BFS from w over out-arcs) */
            const uint64_t *o = side ? off : ioff;
            const uint32_t *a = side ? adj : iadj;
            bfs_count_arcs(n, o, a, w, 0, df, sf, queue);
            bfs_count_arcs(n, o, a, w, 1, dr, sr, queue);
            for (uint32_t v = w; v < n; v++)
                if (dr[v] != ORACLE_INF && dr[v] == df[v])
                    label_push(&ix->lab[(size_t)side * n + v], w, dr[v], sr[v]);
        }
    }
    free(df);
    free(dr);
    free(sf);
    free(sr);
    free(queue);
    ix->hubs_done = n;
    ix->rounds = last_round(ix, 0);
    return ix;
}

/* ------------------------------------------------------------------------ */
/* Sequential pruned BFS, hubs in rank order.  While hub r is processed,     */
/* the labels hold only hubs ranked above r, so a vertex v met at depth D is */
/* skipped when a common hub of L(v) and L(r) already gives a distance < D.  */
/* Otherwise (r, D, count) joins L(v), where count sums the counts of the    */
/* unskipped predecessors one level up; equality with a higher hub's         */
/* distance does not skip (that is a non-canonical entry).                   */
/* ------------------------------------------------------------------------ */
static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

oracle_index *oracle_build_pruned(uint32_t n, const uint64_t *off, const uint32_t *adj,
                                  uint32_t depth_cap, uint32_t max_hubs, double time_limit_s)
{
    oracle_index *ix = index_new(n);
    uint32_t *dist = xmalloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    uint64_t *cnt = xmalloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
    uint32_t *tdist = xmalloc(sizeof(uint32_t) * (size_t)(n ? n : 1)); /* d_r(h) by hub */
    uint32_t *queue = xmalloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    for (uint32_t i = 0; i < n; i++) {
        dist[i] = ORACLE_INF;
        tdist[i] = ORACLE_INF;
        cnt[i] = 0;
    }
    uint32_t limit = (max_hubs && max_hubs < n) ? max_hubs : n;
    double t0 = now_s();
    uint32_t r;
    for (r = 0; r < limit; r++) {
        if (time_limit_s > 0 && now_s() - t0 > time_limit_s) break;
        olabel *lr = &ix->lab[r];
        for (uint64_t i = 0; i < lr->len; i++) tdist[lr->hub[i]] = lr->dist[i];
        uint64_t head = 0, tail = 0;
        dist[r] = 0;
        cnt[r] = 1;
        queue[tail++] = r;
        while (head < tail) {
            uint32_t v = queue[head++];
            uint32_t D = dist[v];
            olabel *lv = &ix->lab[v];
            uint32_t q = ORACLE_INF;
            for (uint64_t i = 0; i < lv->len; i++) {
                uint32_t th = tdist[lv->hub[i]];
                if (th != ORACLE_INF && th + lv->dist[i] < q) q = th + lv->dist[i];
            }
            if (q < D) continue; /* pruned: neither labelled nor expanded */
            label_push(lv, r, D, cnt[v]);
            if (depth_cap && D >= depth_cap) continue;
            for (uint64_t k = off[v]; k < off[v + 1]; k++) {
                uint32_t x = adj[k];
                if (x <= r) continue;
                if (dist[x] == ORACLE_INF) {
                    dist[x] = D + 1;
                    cnt[x] = cnt[v];
                    queue[tail++] = x;
                } else if (dist[x] == D + 1) {
                    cnt[x] = sat_add(cnt[x], cnt[v]);
                }
            }
        }
        for (uint64_t i = 0; i < tail; i++) {
            dist[queue[i]] = ORACLE_INF;
            cnt[queue[i]] = 0;
        }
        for (uint64_t i = 0; i < lr->len; i++) tdist[lr->hub[i]] = ORACLE_INF;
    }
    ix->hubs_done = r;
    free(dist);
    free(cnt);
    free(tdist);
    free(queue);
    ix->rounds = last_round(ix, depth_cap);
    return ix;
}

/* ------------------------------------------------------------------------ */
/* PULL propagation by distance rounds (Alg. 2, Eq. PSPCdu).                 */
/* Round 0 puts (v,0,1) in every label.  Round d: every u gathers the hubs   */
/* of the round d-1 entries of its neighbours; a hub that does not outrank u */
/* is dropped (rank rule); a hub u already holds at a smaller distance is     */
/* dropped (Label Elimination); candidates with the same hub are merged by   */
/* summing counts (Label Merging); a merged candidate w is pruned when a     */
/* 2-hop query over the entries of distance < d gives a distance < d (it is  */
/* kept on equality).  The survivors form round d.  Only entries of distance */
/* < d can give a distance < d, so the query reads no entry of round d and   */
/* the rounds have no intra-round dependency.  The build stops after the     */
/* first round with no survivor (or at the depth cap).                       */
/*                                                                           */
/* Within a round the pullers are independent (the paper's parallel         */
/* construction runs them on threads), so the same per-puller step can run  */
/* on several threads: each takes blocks of pullers from a shared counter,  */
/* and the survivors are put in puller order before round d is inserted.    */
/* The result does not depend on the thread count.                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t *acc;     /* merged count per hub */
    uint8_t *seen;     /* hub collected for this u */
    uint32_t *touched; /* hubs collected for this u */
    uint32_t *udist;   /* d_u(h) over u's entries (all of distance < d) */
} pull_scratch;

typedef struct { /* survivors of the pullers one thread handled, in its order */
    uint32_t *hub;
    uint64_t *cnt;
    uint64_t len, cap;
} pull_out;

typedef struct {
    uint64_t raw, merged, kept, scanned;
    uint64_t active, active_adj, staged; /* inputs of the byte model, see below */
} pull_counts;

static void pull_scratch_init(pull_scratch *sc, uint32_t n)
{
    sc->acc = xcalloc(n, sizeof(uint64_t));
    sc->seen = xcalloc(n, 1);
    sc->touched = xmalloc(sizeof(uint32_t) * (size_t)n);
    sc->udist = xmalloc(sizeof(uint32_t) * (size_t)n);
    for (uint32_t i = 0; i < n; i++) sc->udist[i] = ORACLE_INF;
}

static void pull_scratch_free(pull_scratch *sc)
{
    free(sc->acc);
    free(sc->seen);
    free(sc->touched);
    free(sc->udist);
}

static void pull_out_push(pull_out *o, uint32_t hub, uint64_t cnt)
{
    if (o->len == o->cap) {
        o->cap = o->cap ? 2 * o->cap : 1024;
        o->hub = realloc(o->hub, sizeof(uint32_t) * o->cap);
        o->cnt = realloc(o->cnt, sizeof(uint64_t) * o->cap);
        if (!o->hub || !o->cnt) abort();
    }
    o->hub[o->len] = hub;
    o->cnt[o->len] = cnt;
    o->len++;
}

/* Round d for one puller u: appends u's survivors (hub order) to `out`.
 * Reads the labels (entries of distance < d) and the round d-1 entries
 * prev_*; writes nothing shared. */
static void pull_vertex(const oracle_index *ix, const uint64_t *off, const uint32_t *adj,
                        const uint64_t *prev_off, const uint32_t *prev_hub,
                        const uint64_t *prev_cnt, uint32_t u, uint32_t d, pull_scratch *sc,
                        pull_out *out, pull_counts *ct)
{
    const olabel *lu = &ix->lab[u];
    uint64_t raw = 0;
    /* all entries of u so far have distance < d */
    for (uint64_t i = 0; i < lu->len; i++) sc->udist[lu->hub[i]] = lu->dist[i];
    uint32_t ntouch = 0;
    for (uint64_t k = off[u]; k < off[u + 1]; k++) {
        uint32_t v = adj[k];
        for (uint64_t i = prev_off[v]; i < prev_off[v + 1]; i++) {
            uint32_t w = prev_hub[i];
            if (w >= u) continue; /* rank rule: w must outrank u */
            raw++;
            if (sc->udist[w] != ORACLE_INF) continue; /* Label Elimination */
            if (!sc->seen[w]) {
                sc->seen[w] = 1;
                sc->touched[ntouch++] = w;
            }
            sc->acc[w] = sat_add(sc->acc[w], prev_cnt[i]); /* Label Merging */
        }
    }
    ct->raw += raw;
    if (raw) {
        ct->active++;
        ct->active_adj += off[u + 1] - off[u];
    }
    ct->merged += ntouch;
    if (ntouch) ct->staged += lu->len;
    qsort(sc->touched, ntouch, sizeof(uint32_t), cmp_u32);
    for (uint32_t j = 0; j < ntouch; j++) {
        uint32_t w = sc->touched[j];
        /* Query(w, u, entries of distance < d): a scan of L(w) in hub order
         * (labels are kept hub-sorted) that stops at the first hub proving a
         * shorter distance.  The counter `scanned` is the number of entries
         * it reads, that hub included (all of L(w) when none proves one). */
        const olabel *lw = &ix->lab[w];
        int pruned = 0;
        for (uint64_t i = 0; i < lw->len; i++) {
            uint32_t du = sc->udist[lw->hub[i]];
            if (lw->dist[i] >= d) continue; /* entries of round >= d are not read */
            if (du != ORACLE_INF && du + lw->dist[i] < d) {
                pruned = 1;
                ct->scanned += i + 1;
                break;
            }
        }
        if (!pruned) {
            ct->scanned += lw->len;
            pull_out_push(out, w, sc->acc[w]);
            ct->kept++;
        }
        sc->acc[w] = 0;
        sc->seen[w] = 0;
    }
    for (uint64_t i = 0; i < lu->len; i++) sc->udist[lu->hub[i]] = ORACLE_INF;
}

#define PULL_BLOCK 64u

typedef struct pull_round pull_round;
typedef struct {
    pull_round *r;
    pull_scratch sc;
    pull_out out;
    pull_counts ct;
    uint32_t id;
} pull_worker;

struct pull_round { /* shared by the workers of one round */
    oracle_index *ix;
    const uint64_t *off;
    const uint32_t *adj;
    const uint64_t *prev_off;
    const uint32_t *prev_hub;
    const uint64_t *prev_cnt;
    uint32_t n, d;
    uint32_t next;     /* next block of pullers (atomic) */
    uint32_t *owner;   /* per u: worker that pulled it */
    uint64_t *ustart;  /* per u: first survivor in that worker's buffer */
    uint64_t *ulen;    /* per u: survivors */
    uint64_t *cur_off; /* phase 2: round d in puller order */
    uint32_t *cur_hub;
    uint64_t *cur_cnt;
    pull_worker *w;
    int phase;         /* 1: pull; 2: gather + insert */
};

static int g_progress;

static void *pull_worker_run(void *arg)
{
    pull_worker *me = arg;
    pull_round *r = me->r;
    for (;;) {
        uint32_t b = __atomic_fetch_add(&r->next, PULL_BLOCK, __ATOMIC_RELAXED);
        if (b >= r->n) break;
        if (g_progress && r->phase == 1 && (b & ((1u << 16) - 1)) == 0) {
            fprintf(stderr, "oracle pull: round %u, puller %u of %u\n", r->d, b, r->n);
            fflush(stderr);
        }
        uint32_t e = (r->n - b < PULL_BLOCK) ? r->n : b + PULL_BLOCK;
        for (uint32_t u = b; u < e; u++) {
            if (r->phase == 1) {
                r->owner[u] = me->id;
                r->ustart[u] = me->out.len;
                pull_vertex(r->ix, r->off, r->adj, r->prev_off, r->prev_hub, r->prev_cnt, u, r->d,
                            &me->sc, &me->out, &me->ct);
                r->ulen[u] = me->out.len - r->ustart[u];
            } else { /* copy u's survivors into puller order and insert round d */
                const pull_out *src = &r->w[r->owner[u]].out;
                for (uint64_t i = 0; i < r->ulen[u]; i++) {
                    uint64_t k = r->cur_off[u] + i;
                    r->cur_hub[k] = src->hub[r->ustart[u] + i];
                    r->cur_cnt[k] = src->cnt[r->ustart[u] + i];
                }
                label_merge_sorted(&r->ix->lab[u], r->cur_hub + r->cur_off[u], r->cur_cnt + r->cur_off[u],
                                   r->ulen[u], r->d);
            }
        }
    }
    return NULL;
}

/* Runs the current phase on nthreads workers (inline when there is one). */
static void pull_phase(pull_round *r, uint32_t nthreads, int phase)
{
    r->phase = phase;
    r->next = 0;
    if (nthreads <= 1) {
        pull_worker_run(&r->w[0]);
        return;
    }
    pthread_t *th = xmalloc(sizeof(pthread_t) * nthreads);
    for (uint32_t i = 0; i < nthreads; i++)
        if (pthread_create(&th[i], NULL, pull_worker_run, &r->w[i]) != 0) abort();
    for (uint32_t i = 0; i < nthreads; i++) pthread_join(th[i], NULL);
    free(th);
}

/* nonzero: progress lines on stderr (per round, and every 2^16 pullers) */
void oracle_set_progress(int on) { g_progress = on; }

oracle_index *oracle_build_pull_threads(uint32_t n, const uint64_t *off, const uint32_t *adj,
                                        uint32_t depth_cap, uint32_t nthreads)
{
    oracle_index *ix = index_new(n);
    if (n == 0) return ix;
    if (nthreads == 0) nthreads = 1;
    /* previous-round entries of each vertex: prev_hub/prev_cnt at prev_off */
    uint64_t *prev_off = xcalloc((size_t)n + 1, sizeof(uint64_t));
    uint32_t *prev_hub = xmalloc(sizeof(uint32_t) * (size_t)n);
    uint64_t *prev_cnt = xmalloc(sizeof(uint64_t) * (size_t)n);
    for (uint32_t v = 0; v < n; v++) {
        label_push(&ix->lab[v], v, 0, 1);
        prev_off[v] = v;
        prev_hub[v] = v;
        prev_cnt[v] = 1;
    }
    prev_off[n] = n;
    stats_round(ix, 0, 0, 0, n, 0);

    pull_round r;
    memset(&r, 0, sizeof(r));
    r.ix = ix;
    r.off = off;
    r.adj = adj;
    r.n = n;
    r.owner = xmalloc(sizeof(uint32_t) * (size_t)n);
    r.ustart = xmalloc(sizeof(uint64_t) * (size_t)n);
    r.ulen = xmalloc(sizeof(uint64_t) * (size_t)n);
    r.w = xcalloc(nthreads, sizeof(pull_worker));
    for (uint32_t i = 0; i < nthreads; i++) {
        r.w[i].r = &r;
        r.w[i].id = i;
        pull_scratch_init(&r.w[i].sc, n);
    }

    uint32_t d = 1, last = 0;
    for (;; d++) {
        if (depth_cap && d > depth_cap) {
            last = d - 1;
            break;
        }
        r.d = d;
        r.prev_off = prev_off;
        r.prev_hub = prev_hub;
        r.prev_cnt = prev_cnt;
        for (uint32_t i = 0; i < nthreads; i++) {
            r.w[i].out.len = 0;
            memset(&r.w[i].ct, 0, sizeof(pull_counts));
        }
        pull_phase(&r, nthreads, 1);
        pull_counts ct;
        memset(&ct, 0, sizeof(ct));
        for (uint32_t i = 0; i < nthreads; i++) {
            ct.raw += r.w[i].ct.raw;
            ct.merged += r.w[i].ct.merged;
            ct.kept += r.w[i].ct.kept;
            ct.scanned += r.w[i].ct.scanned;
            ct.active += r.w[i].ct.active;
            ct.active_adj += r.w[i].ct.active_adj;
            ct.staged += r.w[i].ct.staged;
        }
        /* round d in puller order, then inserted after every u was pulled */
        uint64_t *cur_off = xmalloc(sizeof(uint64_t) * ((size_t)n + 1));
        cur_off[0] = 0;
        for (uint32_t u = 0; u < n; u++) cur_off[u + 1] = cur_off[u] + r.ulen[u];
        uint64_t cur_len = cur_off[n];
        r.cur_off = cur_off;
        r.cur_hub = xmalloc(sizeof(uint32_t) * (size_t)(cur_len ? cur_len : 1));
        r.cur_cnt = xmalloc(sizeof(uint64_t) * (size_t)(cur_len ? cur_len : 1));
        pull_phase(&r, nthreads, 2);
        stats_round(ix, d, ct.raw, ct.merged, ct.kept, ct.scanned);
        stats_model(ix, d, ct.active, ct.active_adj, ct.staged);
        if (g_progress) {
            fprintf(stderr, "oracle pull: round %u raw %llu merged %llu kept %llu\n", d,
                    (unsigned long long)ct.raw, (unsigned long long)ct.merged,
                    (unsigned long long)ct.kept);
            fflush(stderr);
        }
        free(prev_off);
        free(prev_hub);
        free(prev_cnt);
        prev_off = cur_off;
        prev_hub = r.cur_hub;
        prev_cnt = r.cur_cnt;
        if (cur_len == 0) {
            last = d;
            break;
        }
    }
    ix->rounds = last; /* last round run: the first empty one, or the cap */
    free(prev_off);
    free(prev_hub);
    free(prev_cnt);
    for (uint32_t i = 0; i < nthreads; i++) {
        pull_scratch_free(&r.w[i].sc);
        free(r.w[i].out.hub);
        free(r.w[i].out.cnt);
    }
    free(r.w);
    free(r.owner);
    free(r.ustart);
    free(r.ulen);
    sort_labels_by_hub(ix);
    ix->hubs_done = n;
    return ix;
}

oracle_index *oracle_build_pull(uint32_t n, const uint64_t *off, const uint32_t *adj,
                                uint32_t depth_cap)
{
    return oracle_build_pull_threads(n, off, adj, depth_cap, 1);
}

/* ------------------------------------------------------------------------ */
uint64_t oracle_index_entries(const oracle_index *ix)
{
    uint64_t e = 0;
    for (uint32_t v = 0; v < ix->n; v++) e += ix->lab[v].len;
    return e;
}
uint32_t oracle_index_rounds(const oracle_index *ix) { return ix->rounds; }
uint32_t oracle_index_hubs_done(const oracle_index *ix) { return ix->hubs_done; }

void oracle_index_export(const oracle_index *ix, uint64_t *off, uint32_t *hub, uint32_t *dist,
                         uint64_t *count)
{
    uint64_t e = 0;
    off[0] = 0;
    for (uint32_t v = 0; v < ix->n; v++) {
        const olabel *l = &ix->lab[v];
        for (uint64_t i = 0; i < l->len; i++) {
            hub[e] = l->hub[i];
            dist[e] = l->dist[i];
            count[e] = l->cnt[i];
            e++;
        }
        off[v + 1] = e;
    }
}

void oracle_index_round_stats(const oracle_index *ix, uint64_t *raw, uint64_t *merged,
                              uint64_t *kept, uint64_t *scanned)
{
    for (uint32_t d = 0; d <= ix->rounds; d++) {
        int have = d < ix->st_cap;
        raw[d] = have ? ix->st_raw[d] : 0;
        merged[d] = have ? ix->st_merged[d] : 0;
        kept[d] = have ? ix->st_kept[d] : 0;
        scanned[d] = have ? ix->st_scanned[d] : 0;
    }
}

void oracle_index_model_stats(const oracle_index *ix, uint64_t *active, uint64_t *active_adj,
                              uint64_t *staged)
{
    for (uint32_t d = 0; d <= ix->rounds; d++) {
        int have = ix->st_active && d < ix->st_model_cap;
        active[d] = have ? ix->st_active[d] : 0;
        active_adj[d] = have ? ix->st_active_adj[d] : 0;
        staged[d] = have ? ix->st_staged[d] : 0;
    }
}

void oracle_index_free(oracle_index *ix)
{
    if (!ix) return;
    for (uint32_t v = 0; v < ix->n; v++) {
        free(ix->lab[v].hub);
        free(ix->lab[v].dist);
        free(ix->lab[v].cnt);
    }
    free(ix->lab);
    free(ix->st_raw);
    free(ix->st_merged);
    free(ix->st_kept);
    free(ix->st_scanned);
    free(ix->st_active);
    free(ix->st_active_adj);
    free(ix->st_staged);
    free(ix);
}

/* ------------------------------------------------------------------------ */
/* Query, Eq. (con:spc1) and (con:spc2): H is the set of common hubs with    */
/* the least d_s(h)+d_t(h); the answer sums count_s(h)*count_t(h) over H.     */
/* Both labels are sorted by hub, so a two-pointer merge finds common hubs.  */
/* ------------------------------------------------------------------------ */
static void merge_query(const uint32_t *hs, const uint32_t *ds, const uint64_t *cs, uint64_t ns,
                        const uint32_t *ht, const uint32_t *dt, const uint64_t *ct, uint64_t nt,
                        uint32_t *out_d, uint64_t *out_c)
{
    uint32_t best = ORACLE_INF;
    uint64_t sum = 0;
    uint64_t i = 0, j = 0;
    while (i < ns && j < nt) {
        if (hs[i] < ht[j]) {
            i++;
        } else if (hs[i] > ht[j]) {
            j++;
        } else {
            uint32_t dd = ds[i] + dt[j];
            uint64_t pc = sat_mul(cs[i], ct[j]);
            if (dd < best) {
                best = dd;
                sum = pc;
            } else if (dd == best) {
                sum = sat_add(sum, pc);
            }
            i++;
            j++;
        }
    }
    *out_d = best;
    *out_c = best == ORACLE_INF ? 0 : sum;
}

void oracle_query(const oracle_index *ix, uint32_t s, uint32_t t, uint32_t *dist,
                  uint64_t *count)
{
    const olabel *a = &ix->lab[s], *b = &ix->lab[t];
    merge_query(a->hub, a->dist, a->cnt, a->len, b->hub, b->dist, b->cnt, b->len, dist, count);
}

void oracle_query_batch(const oracle_index *ix, uint64_t q, const uint32_t *s, const uint32_t *t,
                        uint32_t *dist, uint64_t *count)
{
    for (uint64_t i = 0; i < q; i++) oracle_query(ix, s[i], t[i], &dist[i], &count[i]);
}

void oracle_query_arrays(const uint64_t *off, const uint32_t *hub, const uint32_t *dist,
                         const uint64_t *count, uint64_t q, const uint32_t *s, const uint32_t *t,
                         uint32_t *out_d, uint64_t *out_c)
{
    for (uint64_t i = 0; i < q; i++) {
        uint64_t a0 = off[s[i]], a1 = off[s[i] + 1];
        uint64_t b0 = off[t[i]], b1 = off[t[i] + 1];
        merge_query(hub + a0, dist + a0, count + a0, a1 - a0, hub + b0, dist + b0, count + b0,
                    b1 - b0, &out_d[i], &out_c[i]);
    }
}

typedef struct {
    const uint64_t *off;
    const uint32_t *hub, *dist;
    const uint64_t *count;
    const uint32_t *s, *t;
    uint32_t *out_d;
    uint64_t *out_c;
    uint64_t q0, q1;
} query_part;

static void *query_part_run(void *arg)
{
    query_part *p = arg;
    oracle_query_arrays(p->off, p->hub, p->dist, p->count, p->q1 - p->q0, p->s + p->q0,
                        p->t + p->q0, p->out_d + p->q0, p->out_c + p->q0);
    return NULL;
}

void oracle_query_arrays_threads(const uint64_t *off, const uint32_t *hub, const uint32_t *dist,
                                 const uint64_t *count, uint64_t q, const uint32_t *s,
                                 const uint32_t *t, uint32_t *out_d, uint64_t *out_c,
                                 uint32_t nthreads)
{
    if (nthreads <= 1 || q < 2) {
        oracle_query_arrays(off, hub, dist, count, q, s, t, out_d, out_c);
        return;
    }
    pthread_t *th = xmalloc(sizeof(pthread_t) * nthreads);
    query_part *pt = xmalloc(sizeof(query_part) * nthreads);
    for (uint32_t i = 0; i < nthreads; i++) {
        query_part p = {off, hub, dist, count, s, t, out_d, out_c, q * i / nthreads,
                        q * (i + 1) / nthreads};
        pt[i] = p;
        if (pthread_create(&th[i], NULL, query_part_run, &pt[i]) != 0) abort();
    }
    for (uint32_t i = 0; i < nthreads; i++) pthread_join(th[i], NULL);
    free(th);
    free(pt);
}

/* ------------------------------------------------------------------------ */
/* The hubs of one label, from the definition, without their counts: w is a */
/* hub of L(s) iff w = s or some shortest s-w path has every vertex other   */
/* than w ranked strictly below w (larger rank-space id).  One BFS from s   */
/* gives, for every x, top(x) = the largest over the shortest s-x paths of  */
/* the smallest id among the path's vertices other than x (top(s) = none);  */
/* then w is a hub iff w = s or w < top(w).  Writes the hubs in increasing   */
/* order with their distances; returns how many.  Arrays: room for n.       */
/* ------------------------------------------------------------------------ */
uint64_t oracle_label_hubs(uint32_t n, const uint64_t *off, const uint32_t *adj, uint32_t s,
                           uint32_t *out_hub, uint32_t *out_dist)
{
    if (s >= n) return 0;
    uint32_t *dist = xmalloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *top = xmalloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *queue = xmalloc(sizeof(uint32_t) * (size_t)n);
    for (uint32_t i = 0; i < n; i++) dist[i] = ORACLE_INF;
    uint64_t head = 0, tail = 0;
    dist[s] = 0;
    top[s] = ORACLE_INF; /* the path s has no vertex other than s */
    queue[tail++] = s;
    while (head < tail) { /* level order: top(v) is final when v is popped */
        uint32_t v = queue[head++];
        uint32_t via = top[v] < v ? top[v] : v; /* smallest id on the path to v, v included */
        for (uint64_t k = off[v]; k < off[v + 1]; k++) {
            uint32_t x = adj[k];
            if (dist[x] == ORACLE_INF) {
                dist[x] = dist[v] + 1;
                top[x] = via;
                queue[tail++] = x;
            } else if (dist[x] == dist[v] + 1 && via > top[x]) {
                top[x] = via;
            }
        }
    }
    uint64_t k = 0;
    for (uint32_t w = 0; w <= s; w++) {
        if (dist[w] == ORACLE_INF) continue;
        if (w == s || w < top[w]) {
            out_hub[k] = w;
            out_dist[k] = dist[w];
            k++;
        }
    }
    free(dist);
    free(top);
    free(queue);
    return k;
}
