"""Pins of the CPU oracle against facts fixed outside it.

* the paper's worked example (Fig. 2 order, Table 2 labels, Example 1);
* the trough-path definition applied to explicitly enumerated shortest
  paths (brute force, tiny graphs);
* closed forms for path counts (grids, cycles, complete bipartite graphs,
  hypercubes, trees, complete graphs) and saturation checked with Python
  big integers;
* structural invariants and the order independence of (distance, count).
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example_table2.txt")
SAT = oracle.SAT
BUILDERS = ("definition", "pruned", "pull")


def read_table2():
    rows = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v, rest = line.split(":")
        ents = []
        for tok in rest.split():
            h, d, c = tok.split(",")
            ents.append((int(h[1:]) - 1, int(d), int(c)))
        rows[int(v[1:]) - 1] = ents
    return rows


def labels_original_ids(L):
    """{vertex: [(hub, dist, count)]} in original ids, entries by hub rank."""
    out = {}
    for r in range(L.n):
        v = int(L.order[r])
        out[v] = [(int(L.order[L.hub[i]]), int(L.dist[i]), int(L.count[i]))
                  for i in range(int(L.off[r]), int(L.off[r + 1]))]
    return out


@pytest.mark.parametrize("method", BUILDERS)
def test_worked_example_table2(method):
    g = inputs.worked_example()
    L = oracle.build_graph(g, method=method)
    assert L.entries == 35
    assert labels_original_ids(L) == read_table2()
    assert L.rounds == 4


def test_worked_example_edges_are_distance1_entries():
    t2 = read_table2()
    e = {(min(v, h), max(v, h)) for v, ents in t2.items() for h, d, c in ents if d == 1}
    assert e == {tuple(sorted(x)) for x in inputs.worked_example().edges().tolist()}
    assert len(e) == 13


@pytest.mark.parametrize("method", BUILDERS)
def test_worked_example_queries(method):
    g = inputs.worked_example()
    L = oracle.build_graph(g, method=method)
    # Example 1 (arithmetic read from Table 2): SPC(v10, v7) = 4 paths of length 3.
    d, c = L.query([9], [6])
    assert (int(d[0]), int(c[0])) == (3, 4)
    d, c = L.query([8], [3])   # SPC(v9, v4): needs the non-canonical (v4,3,1) in L(v9)
    assert (int(d[0]), int(c[0])) == (3, 3)
    nb = brute.adjacency(10, g.edges())
    s, t = np.meshgrid(np.arange(10), np.arange(10), indexing="ij")
    d, c = L.query(s.ravel(), t.ravel())
    for i, (a, b) in enumerate(zip(s.ravel(), t.ravel())):
        assert (int(d[i]), int(c[i])) == brute.spc_brute(nb, int(a), int(b))


def test_canonical_only_would_be_wrong():
    """Dropping the non-canonical entries breaks SPC(v9, v4) (3 -> 2 paths)."""
    t2 = read_table2()
    nb = brute.adjacency(10, inputs.worked_example().edges())
    assert brute.spc_brute(nb, 8, 3) == (3, 3)
    l9 = [e for e in t2[8] if e[0] != 3]  # remove (v4,3,1)
    common = {h: (d, c) for h, d, c in t2[3]}
    best = min(d + common[h][0] for h, d, c in l9 if h in common)
    cnt = sum(c * common[h][1] for h, d, c in l9 if h in common and d + common[h][0] == best)
    assert (best, cnt) == (3, 2)


def _tiny_graphs(count, nmax, seed0):
    rng = np.random.default_rng(seed0)
    for i in range(count):
        n = int(rng.integers(1, nmax + 1))
        p = float(rng.choice([0.15, 0.3, 0.5, 0.8]))
        yield inputs.random_tiny(n, p, seed=seed0 * 1000 + i)


@pytest.mark.parametrize("method", BUILDERS)
def test_labels_equal_bruteforce_definition(method):
    for g in _tiny_graphs(60, 8, 7):
        nb = brute.adjacency(g.n, g.edges())
        order = oracle.degree_order(g.off)
        rank = np.empty(g.n, dtype=np.int64)
        rank[order] = np.arange(g.n)
        want = brute.labels_by_definition(nb, rank.tolist())
        L = oracle.build(g.off, g.adj, order=order, method=method)
        got = {v: {} for v in range(g.n)}
        for v, ents in labels_original_ids(L).items():
            for h, d, c in ents:
                got[v][h] = (d, c)
        assert got == want, g.name


def test_labels_random_orders_bruteforce():
    rng = np.random.default_rng(11)
    for g in _tiny_graphs(25, 7, 13):
        order = rng.permutation(g.n).astype(np.uint32)
        rank = np.empty(g.n, dtype=np.int64)
        rank[order] = np.arange(g.n)
        nb = brute.adjacency(g.n, g.edges())
        want = brute.labels_by_definition(nb, rank.tolist())
        for method in BUILDERS:
            L = oracle.build(g.off, g.adj, order=order, method=method)
            got = {v: {h: (d, c) for h, d, c in ents}
                   for v, ents in labels_original_ids(L).items()}
            assert got == want


def test_bfs_count_bruteforce():
    for g in _tiny_graphs(40, 9, 3):
        nb = brute.adjacency(g.n, g.edges())
        for s in range(g.n):
            d, c = oracle.bfs_count(g.off, g.adj, s)
            for t in range(g.n):
                bd, bc = brute.spc_brute(nb, s, t)
                if bd is None:
                    assert d[t] == oracle.INF and c[t] == 0
                else:
                    assert (int(d[t]), int(c[t])) == (bd, bc)


@pytest.mark.parametrize("method", BUILDERS)
def test_espc_all_pairs(method):
    """Exact shortest path covering: the query gives (sd, sigma) for every pair."""
    for g in _tiny_graphs(30, 40, 5):
        L = oracle.build_graph(g, method=method)
        nb = brute.adjacency(g.n, g.edges())
        s, t = np.meshgrid(np.arange(g.n), np.arange(g.n), indexing="ij")
        d, c = L.query(s.ravel(), t.ravel())
        k = 0
        for a in range(g.n):
            bd, bc = brute.sigma_bfs_bigint(nb, a)
            for b in range(g.n):
                if bd[b] is None:
                    assert d[k] == oracle.INF and c[k] == 0
                else:
                    assert int(d[k]) == bd[b] and int(c[k]) == min(bc[b], SAT)
                k += 1


def _grid(k, m=None):
    m = k if m is None else m
    e = []
    for i in range(k):
        for j in range(m):
            v = i * m + j
            if j + 1 < m:
                e.append((v, v + 1))
            if i + 1 < k:
                e.append((v, v + m))
    return inputs.from_edges(k * m, np.array(e))


def test_closed_form_grid_binomial():
    g = _grid(9, 7)
    d, c = oracle.bfs_count(g.off, g.adj, 0)
    for i in range(9):
        for j in range(7):
            assert int(d[i * 7 + j]) == i + j
            assert int(c[i * 7 + j]) == math.comb(i + j, i)
    L = oracle.build_graph(g, method="pull")
    s = np.zeros(63, dtype=np.uint32)
    dd, cc = L.query(s, np.arange(63))
    assert [int(x) for x in cc] == [math.comb(i + j, i) for i in range(9) for j in range(7)]


def test_saturation_bigint():
    """36x36 grid: corner-to-corner C(70,35) > 2^64-1 saturates; smaller
    counts stay exact.  Checked against Python big integers."""
    k = 36
    g = _grid(k)
    nb = brute.adjacency(g.n, g.edges())
    bd, bc = brute.sigma_bfs_bigint(nb, 0)
    d, c = oracle.bfs_count(g.off, g.adj, 0)
    assert [int(x) for x in c] == [min(x, SAT) for x in bc]
    assert int(c[-1]) == SAT and math.comb(70, 35) > SAT
    assert math.comb(66, 33) < SAT
    for method in ("pruned", "pull"):
        L = oracle.build_graph(g, method=method)
        dq, cq = L.query(np.zeros(g.n, dtype=np.uint32), np.arange(g.n))
        assert [int(x) for x in cq] == [min(x, SAT) for x in bc]
        assert [int(x) for x in dq] == bd
        # the label counts themselves saturate on this graph
        assert int((L.count == np.uint64(SAT)).sum()) > 0
    # an order where label counts saturate: compare two builders entry by entry
    A = oracle.build_graph(g, method="pruned")
    B = oracle.build_graph(g, method="pull")
    for f in ("off", "hub", "dist", "count"):
        assert np.array_equal(getattr(A, f), getattr(B, f))


def test_closed_forms_small_families():
    # even cycle: 2 shortest paths between antipodes
    for n in (6, 8, 10):
        g = inputs.from_edges(n, np.array([(i, (i + 1) % n) for i in range(n)]))
        L = oracle.build_graph(g, method="pull")
        d, c = L.query(np.arange(n), (np.arange(n) + n // 2) % n)
        assert set(d.tolist()) == {n // 2} and set(c.tolist()) == {2}
    # complete bipartite K_{a,b}: same-side pairs at distance 2 via every vertex of the other side
    a, b = 4, 6
    g = inputs.from_edges(a + b, np.array([(i, a + j) for i in range(a) for j in range(b)]))
    L = oracle.build_graph(g, method="pull")
    d, c = L.query([0, a], [1, a + 1])
    assert d.tolist() == [2, 2] and c.tolist() == [b, a]
    # hypercube Q_h: sigma = (Hamming distance)!
    h = 6
    e = [(x, x ^ (1 << i)) for x in range(1 << h) for i in range(h) if x < x ^ (1 << i)]
    g = inputs.from_edges(1 << h, np.array(e))
    L = oracle.build_graph(g, method="pull")
    t = np.arange(1 << h)
    d, c = L.query(np.zeros_like(t), t)
    hw = [bin(x).count("1") for x in t]
    assert d.tolist() == hw and c.tolist() == [math.factorial(x) for x in hw]
    # complete graph and a random tree: one shortest path per pair
    g = inputs.from_edges(7, np.array(list(itertools.combinations(range(7), 2))))
    L = oracle.build_graph(g, method="pruned")
    s, t = np.meshgrid(np.arange(7), np.arange(7), indexing="ij")
    d, c = L.query(s.ravel(), t.ravel())
    assert set(c.tolist()) == {1} and set(d.tolist()) == {0, 1}
    rng = np.random.default_rng(2)
    par = [int(rng.integers(0, i)) for i in range(1, 50)]
    g = inputs.from_edges(50, np.array([(i + 1, p) for i, p in enumerate(par)]))
    L = oracle.build_graph(g, method="pull")
    s, t = np.meshgrid(np.arange(50), np.arange(50), indexing="ij")
    d, c = L.query(s.ravel(), t.ravel())
    assert set(c.tolist()) == {1}


def test_builders_agree_medium():
    graphs = [inputs.erdos_renyi(300, 900, seed=4), inputs.rmat(9, 8, seed=6),
              inputs.grid_lcc(20, 0.05, seed=3)]
    for g in graphs:
        A = oracle.build_graph(g, method="definition")
        for method in ("pruned", "pull"):
            B = oracle.build_graph(g, method=method)
            for f in ("off", "hub", "dist", "count"):
                assert np.array_equal(getattr(A, f), getattr(B, f)), (g.name, method, f)
            assert A.rounds == B.rounds


def test_invariants_and_stats():
    g = inputs.erdos_renyi(400, 1600, seed=9)
    L = oracle.build_graph(g, method="pull")
    n = g.n
    rows = np.repeat(np.arange(n), np.diff(L.off).astype(np.int64))
    # hubs strictly increasing within a label and never ranked below the owner
    assert np.all(L.hub <= rows)
    same = rows[1:] == rows[:-1]
    assert np.all(L.hub[1:][same] > L.hub[:-1][same])
    # self entry (v,0,1) is the last entry of every label
    last = L.off[1:].astype(np.int64) - 1
    assert np.all(L.hub[last] == np.arange(n)) and np.all(L.dist[last] == 0)
    assert np.all(L.count[last] == 1)
    # one distance-1 entry per edge
    assert int((L.dist == 1).sum()) == g.m
    # kept per round = histogram of distances
    hist = np.bincount(L.dist.astype(np.int64), minlength=L.rounds + 1)
    assert L.stats["kept"].tolist() == hist[:L.rounds + 1].tolist()
    assert int(L.stats["kept"][L.rounds]) == 0
    # raw / merged recounted from the final labels (Lemma of propagation + rank rule)
    roff, radj = oracle.relabel(g.off, g.adj, L.order)
    lab = [dict() for _ in range(n)]
    for r in range(n):
        for i in range(int(L.off[r]), int(L.off[r + 1])):
            lab[r][int(L.hub[i])] = int(L.dist[i])
    for d in range(1, L.rounds + 1):
        raw = merged = 0
        for u in range(n):
            cands = set()
            for k in range(int(roff[u]), int(roff[u + 1])):
                v = int(radj[k])
                ws = [w for w, dv in lab[v].items() if dv == d - 1 and w < u]
                raw += len(ws)
                cands.update(w for w in ws if not (w in lab[u] and lab[u][w] < d))
            merged += len(cands)
        assert raw == int(L.stats["raw"][d]) and merged == int(L.stats["merged"][d]), d


def test_scanned_counter_in_hub_order():
    """Probe entries read in hub order, recounted from the final labels."""
    g = inputs.erdos_renyi(150, 500, seed=21)
    L = oracle.build_graph(g, method="pull")
    n = g.n
    roff, radj = oracle.relabel(g.off, g.adj, L.order)
    lab = [[(int(L.hub[i]), int(L.dist[i])) for i in range(int(L.off[r]), int(L.off[r + 1]))]
           for r in range(n)]
    for d in range(1, L.rounds + 1):
        scanned = 0
        for u in range(n):
            du = {h: x for h, x in lab[u] if x < d}
            cands = set()
            for k in range(int(roff[u]), int(roff[u + 1])):
                v = int(radj[k])
                cands.update(w for w, x in lab[v] if x == d - 1 and w < u and w not in du)
            for w in cands:
                lw = [(h, x) for h, x in lab[w] if x < d]   # hub-sorted already
                k = len(lw)
                for i, (h, x) in enumerate(lw):
                    if h in du and du[h] + x < d:
                        k = i + 1
                        break
                scanned += k
        assert scanned == int(L.stats["scanned"][d]), d


def test_depth_cap_is_distance_partial_set():
    g = inputs.grid_lcc(16, 0.05, seed=3)
    full = oracle.build_graph(g, method="pruned")
    for cap in (1, 3, 7):
        keep = full.dist <= cap
        rows = np.repeat(np.arange(g.n), np.diff(full.off).astype(np.int64))
        want_off = np.zeros(g.n + 1, dtype=np.uint64)
        np.cumsum(np.bincount(rows[keep], minlength=g.n), out=want_off[1:])
        for method in BUILDERS:
            L = oracle.build_graph(g, method=method, depth_cap=cap)
            assert np.array_equal(L.off, want_off), (method, cap)
            assert np.array_equal(L.hub, full.hub[keep])
            assert np.array_equal(L.count, full.count[keep])
            assert L.rounds == cap


def test_answers_independent_of_order():
    g = inputs.rmat(8, 8, seed=12)
    A = oracle.build_graph(g, method="pull")
    rng = np.random.default_rng(1)
    B = oracle.build(g.off, g.adj, order=rng.permutation(g.n).astype(np.uint32), method="pull")
    s, t = inputs.queries(g.n, 3000, seed=7)
    da, ca = A.query(s, t)
    db, cb = B.query(s, t)
    assert np.array_equal(da, db) and np.array_equal(ca, cb)


def test_degree_order_rules():
    g = inputs.erdos_renyi(500, 1500, seed=2)
    order = oracle.degree_order(g.off)
    deg = g.degrees()[order]
    assert np.all(deg[:-1] >= deg[1:])
    ties = deg[:-1] == deg[1:]
    assert np.all(order[:-1][ties] < order[1:][ties])
    tk = np.random.default_rng(0).integers(0, 1 << 62, size=g.n).astype(np.uint64)
    order = oracle.degree_order(g.off, tk)
    deg = g.degrees()[order]
    ties = deg[:-1] == deg[1:]
    assert np.all(tk[order][:-1][ties] <= tk[order][1:][ties])


def test_hub_column_matches_full_index():
    g = inputs.chung_lu(2048, seed=2)
    L = oracle.build_graph(g, method="pruned")
    roff, radj = oracle.relabel(g.off, g.adj, L.order)
    rows = np.repeat(np.arange(g.n), np.diff(L.off).astype(np.int64))
    for w in (0, 1, 5, 100, 1000, 2047):
        v, d, c = oracle.hub_column(roff, radj, w)
        sel = L.hub == w
        assert np.array_equal(v, rows[sel].astype(np.uint32))
        assert np.array_equal(d, L.dist[sel]) and np.array_equal(c, L.count[sel])
