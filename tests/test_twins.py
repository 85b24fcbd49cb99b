"""Pins of the oracle's neighbourhood-equivalence reduction (Section
"Reduction by Equivalence Relation"): the classes against the relation's
literal pairwise definition and closed forms; the weighted label
definition against the plain index when every weight is 1; and the query
rule against explicit path enumeration and big-integer BFS counting on the
input graph for every pair of small graphs full of twins."""
import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests import brute


def csr(n, edges):
    return inputs.from_edges(n, np.array(edges, dtype=np.int64).reshape(-1, 2), name="t")


def literal_classes(g):
    nb = [set(int(w) for w in g.adj[g.off[v]:g.off[v + 1]]) for v in range(g.n)]
    rep = np.arange(g.n)
    for v in range(g.n):
        for u in range(v):
            if nb[u] - {v} == nb[v] - {u}:
                rep[v] = rep[u]
                break
    return rep


def twin_graphs():
    out = []
    for seed in range(5):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(12, 30))
        g = inputs.erdos_renyi(n, int(rng.integers(n // 2, 2 * n)), seed=seed)
        e = [tuple(x) for x in g.edges().tolist()]
        # plant twins: copies of random vertices, adjacent or not to their original
        m = n
        for _ in range(int(rng.integers(3, 8))):
            v = int(rng.integers(0, n))
            nbrs = [b for a, b in e if a == v] + [a for a, b in e if b == v]
            e += [(m, x) for x in nbrs]
            if rng.random() < 0.5:
                e.append((v, m))
            m += 1
        out.append(csr(m, sorted(set(tuple(sorted(x)) for x in e))))
    out.append(inputs.rmat(6, 3, seed=4))
    return out


def test_closed_forms():
    k5 = csr(5, [(a, b) for a in range(5) for b in range(a + 1, 5)])
    assert list(oracle.twin_classes(k5.off, k5.adj)) == [0] * 5
    k23 = csr(5, [(a, b) for a in (0, 1) for b in (2, 3, 4)])
    assert list(oracle.twin_classes(k23.off, k23.adj)) == [0, 0, 2, 2, 2]
    star = csr(6, [(0, i) for i in range(1, 6)])
    assert list(oracle.twin_classes(star.off, star.adj)) == [0, 1, 1, 1, 1, 1]
    c4 = csr(4, [(0, 1), (1, 2), (2, 3), (3, 0)])
    assert list(oracle.twin_classes(c4.off, c4.adj)) == [0, 1, 0, 1]
    p4 = csr(4, [(0, 1), (1, 2), (2, 3)])
    assert list(oracle.twin_classes(p4.off, p4.adj)) == [0, 1, 2, 3]
    iso = csr(4, [(1, 2)])
    assert list(oracle.twin_classes(iso.off, iso.adj)) == [0, 1, 1, 0]


@pytest.mark.parametrize("gi", range(6))
def test_classes_equal_pairwise_definition(gi):
    g = twin_graphs()[gi]
    assert np.array_equal(oracle.twin_classes(g.off, g.adj), literal_classes(g))


@pytest.mark.parametrize("gi", range(6))
def test_unit_weights_give_the_plain_index(gi):
    g = twin_graphs()[gi]
    ref = oracle.build(g.off, g.adj)
    lab = oracle.weighted_labels(g.off, g.adj, np.ones(g.n, dtype=np.uint64))
    for k in ("off", "hub", "dist", "count", "order"):
        assert np.array_equal(getattr(lab, k), getattr(ref, k)), k


def test_weighted_labels_count_inner_vertex_weights():
    # path 0-1-2 with weights 1, 5, 1 ranked 0, 2, 1: L(1) holds (0,1,1); L(2)
    # holds hub 0 at distance 2 through vertex 1 (weight 5)
    g = csr(3, [(0, 1), (1, 2)])
    lab = oracle.weighted_labels(g.off, g.adj, np.array([1, 5, 1], dtype=np.uint64),
                                 order=np.array([0, 2, 1], dtype=np.uint32))
    ent = {(int(lab.order[r]), int(lab.order[h])): (int(d), int(c)) for r in range(3)
           for h, d, c in zip(lab.hub[lab.off[r]:lab.off[r + 1]], lab.dist[lab.off[r]:lab.off[r + 1]],
                              lab.count[lab.off[r]:lab.off[r + 1]])}
    assert ent[(2, 0)] == (2, 5) and ent[(1, 0)] == (1, 1) and ent[(1, 2)] == (1, 1)


@pytest.mark.parametrize("gi", range(6))
def test_twin_query_equals_path_enumeration(gi):
    g = twin_graphs()[gi]
    red = oracle.build_twin_reduced(g.off, g.adj)
    assert red.ids.shape[0] < g.n
    nb = [sorted(set(int(w) for w in g.adj[g.off[v]:g.off[v + 1]])) for v in range(g.n)]
    s, t = (x.ravel().astype(np.uint32) for x in np.meshgrid(np.arange(g.n), np.arange(g.n)))
    d, c = red.query(s, t)
    for i in range(s.shape[0]):
        bd, bc = brute.spc_brute(nb, int(s[i]), int(t[i]))
        if bd is None:
            assert d[i] == oracle.INF and c[i] == 0
        else:
            assert (int(d[i]), int(c[i])) == (bd, bc), (gi, int(s[i]), int(t[i]))


def test_twin_query_on_larger_graphs_equals_bfs_counting():
    for g in (inputs.rmat(9, 4, seed=3), inputs.chung_lu(1 << 9, seed=4),
              csr(40, [(a, b) for a in range(8) for b in range(8, 40)])):
        red = oracle.build_twin_reduced(g.off, g.adj)
        assert red.ids.shape[0] < g.n
        nb = [sorted(set(int(w) for w in g.adj[g.off[v]:g.off[v + 1]])) for v in range(g.n)]
        for src in range(0, g.n, 29):
            bd, bc = brute.sigma_bfs_bigint(nb, src)
            d, c = red.query(np.full(g.n, src, dtype=np.uint32), np.arange(g.n, dtype=np.uint32))
            for v in range(g.n):
                if bd[v] is None:
                    assert d[v] == oracle.INF and c[v] == 0
                else:
                    assert int(d[v]) == bd[v] and int(c[v]) == min(bc[v], brute.SAT), (src, v)


@pytest.mark.parametrize("gi", range(6))
def test_c_weighted_builder_equals_python_definition(gi):
    g = twin_graphs()[gi]
    rng = np.random.default_rng(gi)
    w = rng.integers(1, 9, g.n).astype(np.uint64)
    for cap in (0, 2):
        a = oracle.weighted_labels(g.off, g.adj, w, depth_cap=cap)
        b = oracle.build_weighted(g.off, g.adj, w, depth_cap=cap)
        for k in ("off", "hub", "dist", "count", "order"):
            assert np.array_equal(getattr(a, k), getattr(b, k)), (k, cap)


def test_c_weighted_builder_saturates_like_the_definition():
    # a 12x12 grid with every weight 7: corner-to-corner counts pass 2^64
    k = 12
    e = [(i * k + j, i * k + j + 1) for i in range(k) for j in range(k - 1)]
    e += [(i * k + j, (i + 1) * k + j) for i in range(k - 1) for j in range(k)]
    g = csr(k * k, e)
    w = np.full(g.n, 7, dtype=np.uint64)
    a = oracle.weighted_labels(g.off, g.adj, w)
    b = oracle.build_weighted(g.off, g.adj, w)
    assert np.array_equal(a.count, b.count) and int((b.count == np.uint64(oracle.SAT)).sum()) > 0
