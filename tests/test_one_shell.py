"""Pins of the oracle's 1-shell reduction (Section "Reduction by 1-Shell"):
closed forms on paths, stars, cycles with pendant trees and forests; the
structural facts the section states (the fringe is a forest whose trees
each hang from the core by one edge; the core is the 2-core); and the query
rule checked against explicit shortest-path enumeration and big-integer BFS
counting on every pair of small graphs."""
import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests import brute


def csr(n, edges):
    return inputs.from_edges(n, np.array(edges, dtype=np.int64).reshape(-1, 2), name="t")


def test_path_is_rooted_at_its_centre():
    for n in (1, 2, 3, 4, 7, 10):
        g = csr(n, [(i, i + 1) for i in range(n - 1)])
        sh = oracle.one_shell(g.off, g.adj)
        c = (n - 1) // 2  # the centre; of two centres the smaller id
        assert list(np.nonzero(sh.core)[0]) == [c]
        assert list(sh.root) == [c] * n
        assert list(sh.depth) == [abs(v - c) for v in range(n)]
        assert list(sh.parent) == [v + 1 if v < c else (v - 1 if v > c else v) for v in range(n)]


def test_star_and_isolated_vertices():
    k = 6
    g = csr(k + 3, [(0, i) for i in range(1, k + 1)])  # vertices k+1, k+2 isolated
    sh = oracle.one_shell(g.off, g.adj)
    assert list(np.nonzero(sh.core)[0]) == [0, k + 1, k + 2]
    assert list(sh.root) == [0] * (k + 1) + [k + 1, k + 2]
    assert list(sh.depth) == [0] + [1] * k + [0, 0]


def test_cycle_with_pendant_trees():
    # 5-cycle 0..4; a path 5-6-7 hangs from 0; a star 8(9, 10) hangs from 2
    e = [(i, (i + 1) % 5) for i in range(5)] + [(0, 5), (5, 6), (6, 7), (2, 8), (8, 9), (8, 10)]
    g = csr(11, e)
    sh = oracle.one_shell(g.off, g.adj)
    assert list(np.nonzero(sh.core)[0]) == [0, 1, 2, 3, 4]
    assert list(sh.root) == [0, 1, 2, 3, 4, 0, 0, 0, 2, 2, 2]
    assert list(sh.depth) == [0, 0, 0, 0, 0, 1, 2, 3, 1, 2, 2]
    assert list(sh.parent) == [0, 1, 2, 3, 4, 0, 5, 6, 2, 8, 8]


def test_two_cycles_joined_by_a_path_stay_in_the_core():
    # the path between two cycles lies on the 2-core: nothing is cut
    e = [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (4, 5), (5, 6), (6, 7), (7, 5)]
    g = csr(8, e)
    sh = oracle.one_shell(g.off, g.adj)
    assert sh.core.all() and (sh.depth == 0).all()


def random_graphs():
    out = []
    for seed in range(6):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(20, 45))
        m = int(rng.integers(n // 2, n + n // 2))
        out.append(inputs.erdos_renyi(n, m, seed=seed))
    # a random forest plus a few cycles
    rng = np.random.default_rng(7)
    n = 40
    e = [(v, int(rng.integers(0, v))) for v in range(1, n) if rng.random() < 0.9]
    e += [(0, 5), (5, 9), (3, 17)]
    out.append(csr(n, sorted(set(tuple(sorted(x)) for x in e if x[0] != x[1]))))
    return out


@pytest.mark.parametrize("gi", range(7))
def test_shell_structure(gi):
    g = random_graphs()[gi]
    sh = oracle.one_shell(g.off, g.adj)
    nb = [set(int(w) for w in g.adj[g.off[v]:g.off[v + 1]]) for v in range(g.n)]
    core = sh.core
    for v in range(g.n):
        if core[v]:
            assert sh.root[v] == v and sh.depth[v] == 0 and sh.parent[v] == v
            # 2-core: two core neighbours, unless v is a root kept for a tree component
            k = sum(1 for w in nb[v] if core[w])
            comp_has_cycle = k >= 2
            assert comp_has_cycle or all(not core[w] for w in nb[v])
        else:
            p = int(sh.parent[v])
            assert p in nb[v] and sh.depth[p] + 1 == sh.depth[v] and sh.root[p] == sh.root[v]
    # the fringe is a forest: edges among fringe vertices = vertices - trees
    fr = [v for v in range(g.n) if not core[v]]
    fe = sum(1 for v in fr for w in nb[v] if not core[w] and w > v)
    seen, trees = set(), 0
    for v in fr:
        if v in seen:
            continue
        trees += 1
        st = [v]
        seen.add(v)
        while st:
            x = st.pop()
            for w in nb[x]:
                if not core[w] and w not in seen:
                    seen.add(w)
                    st.append(w)
    assert fe == len(fr) - trees
    # each fringe vertex has at most one core neighbour, and only depth-1
    # vertices have one (one joining edge per tree)
    for v in fr:
        k = sum(1 for w in nb[v] if core[w])
        assert k == (1 if sh.depth[v] == 1 else 0)
    # the core is the 2-core: deleting degree < 2 vertices from the core
    # (with the kept tree-component roots set aside) removes nothing
    cyc = [v for v in range(g.n) if core[v] and any(core[w] for w in nb[v])]
    assert all(sum(1 for w in nb[v] if core[w]) >= 2 for v in cyc)


@pytest.mark.parametrize("gi", range(7))
def test_reduced_query_equals_path_enumeration(gi):
    g = random_graphs()[gi]
    red = oracle.build_reduced(g.off, g.adj)
    nb = [sorted(set(int(w) for w in g.adj[g.off[v]:g.off[v + 1]])) for v in range(g.n)]
    s, t = (x.ravel().astype(np.uint32) for x in np.meshgrid(np.arange(g.n), np.arange(g.n)))
    d, c = red.query(s, t)
    for i in range(s.shape[0]):
        bd, bc = brute.spc_brute(nb, int(s[i]), int(t[i]))
        if bd is None:
            assert d[i] == oracle.INF and c[i] == 0
        else:
            assert (int(d[i]), int(c[i])) == (bd, bc), (int(s[i]), int(t[i]))


def test_reduced_query_on_larger_graphs_equals_bfs_counting():
    for g in (inputs.erdos_renyi(400, 500, seed=3), inputs.chung_lu(1 << 9, seed=4)):
        red = oracle.build_reduced(g.off, g.adj)
        assert (~red.shell.core).sum() > 0
        nb = [sorted(set(int(w) for w in g.adj[g.off[v]:g.off[v + 1]])) for v in range(g.n)]
        for src in range(0, g.n, 37):
            bd, bc = brute.sigma_bfs_bigint(nb, src)
            t = np.arange(g.n, dtype=np.uint32)
            d, c = red.query(np.full(g.n, src, dtype=np.uint32), t)
            for v in range(g.n):
                if bd[v] is None:
                    assert d[v] == oracle.INF and c[v] == 0
                else:
                    assert int(d[v]) == bd[v] and int(c[v]) == min(bc[v], brute.SAT)


def test_core_subgraph_restricts_order_and_tie_keys():
    e = [(i, (i + 1) % 5) for i in range(5)] + [(0, 5), (5, 6), (2, 7)]
    g = csr(8, e)
    sh = oracle.one_shell(g.off, g.adj)
    order = np.array([6, 2, 7, 0, 5, 4, 1, 3], dtype=np.uint32)
    tie = np.arange(8, dtype=np.uint64)[::-1].copy()
    coff, cadj, ids, cid, cord, ctie = oracle.core_subgraph(g.off, g.adj, sh.core, order, tie)
    assert list(ids) == [0, 1, 2, 3, 4]
    assert list(cord) == [2, 0, 4, 1, 3]
    assert list(ctie) == [7, 6, 5, 4, 3]
    assert int(coff[-1]) == 10  # the 5-cycle, both directions
