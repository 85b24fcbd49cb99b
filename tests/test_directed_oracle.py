"""Pins of the oracle's directed labels (in- and out-labels, Section "2-Hop
Labeling for Shortest Path Counting"): every pair of random digraphs
answered as directed BFS counting with big integers does, closed forms on
directed paths, cycles and layered graphs, and the symmetric case equal to
the undirected index."""
from collections import deque

import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs


def digraph_bfs(n, arcs, s):
    fwd = [set() for _ in range(n)]
    for a, b in arcs:
        if a != b:
            fwd[int(a)].add(int(b))
    d, c = [None] * n, [0] * n
    d[s], c[s] = 0, 1
    q = deque([s])
    while q:
        u = q.popleft()
        for x in sorted(fwd[u]):
            if d[x] is None:
                d[x] = d[u] + 1
                c[x] = c[u]
                q.append(x)
            elif d[x] == d[u] + 1:
                c[x] += c[u]
    return d, c


@pytest.mark.parametrize("seed", range(8))
def test_random_digraphs_match_bfs_counting(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 40))
    m = int(rng.integers(n, 4 * n))
    arcs = [(int(a), int(b)) for a, b in rng.integers(0, n, (m, 2)) if a != b]
    order = rng.permutation(n) if seed % 2 else None
    lab = oracle.directed_labels(n, arcs, order=order)
    for s in range(n):
        bd, bc = digraph_bfs(n, arcs, s)
        d, c = lab.query(np.full(n, s), np.arange(n))
        for t in range(n):
            if bd[t] is None:
                assert d[t] == oracle.INF and c[t] == 0, (seed, s, t)
            else:
                assert (int(d[t]), int(c[t])) == (bd[t], min(bc[t], oracle.SAT)), (seed, s, t)


def test_closed_forms():
    n = 7
    path = oracle.directed_labels(n, [(i, i + 1) for i in range(n - 1)])
    s, t = (x.ravel() for x in np.meshgrid(np.arange(n), np.arange(n), indexing="ij"))
    d, c = path.query(s, t)
    for a, b, dd, cc in zip(s, t, d, c):
        assert (int(dd), int(cc)) == ((int(b - a), 1) if b >= a else (oracle.INF, 0))
    cyc = oracle.directed_labels(n, [(i, (i + 1) % n) for i in range(n)])
    d, c = cyc.query(s, t)
    assert all(int(dd) == (int(b) - int(a)) % n and int(cc) == 1 for a, b, dd, cc in zip(s, t, d, c))
    # layers 0 -> {1..4} -> {5..7} -> 8: 4 * 3 shortest paths from 0 to 8
    arcs = [(0, i) for i in range(1, 5)] + [(i, j) for i in range(1, 5) for j in range(5, 8)] + \
           [(j, 8) for j in range(5, 8)]
    lay = oracle.directed_labels(9, arcs)
    d, c = lay.query(np.array([0, 8, 1]), np.array([8, 0, 7]))
    assert [int(x) for x in d] == [3, oracle.INF, 1] and [int(x) for x in c] == [12, 0, 1]


def test_symmetric_digraph_is_the_undirected_index():
    for g in (inputs.worked_example(), inputs.erdos_renyi(60, 120, seed=3)):
        arcs = [(int(a), int(b)) for a, b in g.edges()] + [(int(b), int(a)) for a, b in g.edges()]
        order = g.order if g.order is not None else oracle.degree_order(g.off)
        lab = oracle.directed_labels(g.n, arcs, order=order)
        ref = oracle.build(g.off, g.adj, order=order)
        rank = ref.rank_of()
        for v in range(g.n):
            r = int(rank[v])
            want = {int(ref.order[h]): (int(dd), int(cc)) for h, dd, cc in
                    zip(ref.hub[ref.off[r]:ref.off[r + 1]], ref.dist[ref.off[r]:ref.off[r + 1]],
                        ref.count[ref.off[r]:ref.off[r + 1]])}
            assert lab.out[v] == want and lab.inn[v] == want, v


def _arcs_csr(n, arcs):
    arcs = sorted(set((int(a), int(b)) for a, b in arcs if a != b))
    off = np.zeros(n + 1, dtype=np.uint64)
    for a, _ in arcs:
        off[a + 1] += 1
    off = np.cumsum(off).astype(np.uint64)
    adj = np.array([b for _, b in arcs], dtype=np.uint32)
    return off, adj


@pytest.mark.parametrize("seed", range(6))
def test_c_directed_definition_equals_python(seed):
    """The C builder (rows: L_out then L_in, rank space) holds exactly the
    Python definition's entries."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(5, 45))
    m = int(rng.integers(n, 5 * n))
    arcs = [(int(a), int(b)) for a, b in rng.integers(0, n, (m, 2)) if a != b]
    off, adj = _arcs_csr(n, arcs)
    order = oracle.directed_order(n, off, adj)
    py = oracle.directed_labels(n, arcs, order=order)
    C = oracle.build_directed(n, off, adj, order=order)
    for r in range(n):
        v = int(order[r])
        for side, lab in ((0, py.out), (1, py.inn)):
            row = side * n + r
            got = {int(order[C.hub[i]]): (int(C.dist[i]), int(C.count[i]))
                   for i in range(int(C.off[row]), int(C.off[row + 1]))}
            assert got == lab[v], (seed, side, v)


def test_c_directed_symmetric_is_undirected_index():
    g = inputs.erdos_renyi(120, 360, seed=5)
    off, adj = g.off, g.adj   # both directions of every edge
    order = oracle.degree_order(g.off)
    U = oracle.build_graph(g, method="definition")
    D = oracle.build_directed(g.n, off, adj, order=order)
    n = g.n
    for side in (0, 1):
        a, b = int(D.off[side * n]), int(D.off[side * n + n])
        assert np.array_equal(D.off[side * n: side * n + n + 1] - D.off[side * n], U.off)
        assert np.array_equal(D.hub[a:b], U.hub) and np.array_equal(D.dist[a:b], U.dist)
        assert np.array_equal(D.count[a:b], U.count)
