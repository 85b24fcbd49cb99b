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
