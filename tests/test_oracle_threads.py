"""Pins of the oracle's threaded PULL build, its byte-model counters, the
single-label hub set and the threaded merge-join query.

* the threaded PULL (pullers of a round spread over host threads, the
  paper's parallel construction) gives the sequential PULL's index and every
  counter, and both equal the trough-path definition;
* the byte-model inputs (active pullers, their adjacency slots, staged label
  entries) are recounted here from the final labels in plain Python;
* the hub set of one label from a single BFS equals the hubs of the full
  index (Table 2 for the worked example, the definition elsewhere);
* the threaded query answers as the single-threaded one.
"""
import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests.test_oracle_pins import labels_original_ids, read_table2

FIELDS = ("off", "hub", "dist", "count")


def _graphs():
    return [inputs.worked_example(), inputs.erdos_renyi(300, 1200, seed=5),
            inputs.rmat(10, 8, seed=8), inputs.grid_lcc(24, 0.05, seed=3),
            inputs.chung_lu(1024, seed=2), inputs.random_tiny(40, 0.08, seed=3)]


@pytest.mark.parametrize("threads", [2, 3, 8])
def test_threaded_pull_equals_sequential_and_definition(threads):
    for g in _graphs():
        A = oracle.build_graph(g, method="definition")
        S = oracle.build_graph(g, method="pull")
        T = oracle.build_graph(g, method="pull", threads=threads)
        for f in FIELDS:
            assert np.array_equal(getattr(A, f), getattr(T, f)), (g.name, f)
            assert np.array_equal(getattr(S, f), getattr(T, f)), (g.name, f)
        assert S.rounds == T.rounds == A.rounds
        for k in S.stats:
            assert np.array_equal(S.stats[k], T.stats[k]), (g.name, k)


def test_threaded_pull_with_depth_cap():
    g = inputs.grid_lcc(20, 0.05, seed=3)
    for cap in (1, 4, 9):
        A = oracle.build_graph(g, method="definition", depth_cap=cap)
        T = oracle.build_graph(g, method="pull", depth_cap=cap, threads=4)
        for f in FIELDS:
            assert np.array_equal(getattr(A, f), getattr(T, f)), (cap, f)
        assert T.rounds == cap


def test_model_counters_recounted_from_labels():
    """active = pullers with a candidate passing the rank rule, active_adj =
    their adjacency slots, staged = entries of distance < d of pullers with a
    merged candidate; all from the final labels and the graph alone."""
    for g in (inputs.erdos_renyi(200, 700, seed=11), inputs.grid_lcc(14, 0.05, seed=3),
              inputs.worked_example()):
        L = oracle.build_graph(g, method="pull", threads=3)
        n = g.n
        roff, radj = oracle.relabel(g.off, g.adj, L.order)
        lab = [{int(L.hub[i]): int(L.dist[i]) for i in range(int(L.off[r]), int(L.off[r + 1]))}
               for r in range(n)]
        assert int(L.stats["active"][0]) == 0 and int(L.stats["staged"][0]) == 0
        for d in range(1, L.rounds + 1):
            active = active_adj = staged = 0
            for u in range(n):
                nbrs = [int(radj[k]) for k in range(int(roff[u]), int(roff[u + 1]))]
                raw = [w for v in nbrs for w, dv in lab[v].items() if dv == d - 1 and w < u]
                held = {w for w, x in lab[u].items() if x < d}
                if raw:
                    active += 1
                    active_adj += len(nbrs)
                if any(w not in held for w in raw):
                    staged += len(held)
            assert active == int(L.stats["active"][d]), (g.name, d)
            assert active_adj == int(L.stats["active_adj"][d]), (g.name, d)
            assert staged == int(L.stats["staged"][d]), (g.name, d)


def test_label_hubs_worked_example_table2():
    g = inputs.worked_example()
    want = read_table2()
    L = oracle.build_graph(g, method="pull")
    roff, radj = oracle.relabel(g.off, g.adj, L.order)
    rank = L.rank_of()
    for v, ents in want.items():
        h, d = oracle.label_hubs(roff, radj, int(rank[v]))
        got = sorted((int(L.order[x]), int(y)) for x, y in zip(h, d))
        assert got == sorted((w, dd) for w, dd, _ in ents), v
    # and the full index's labels in original ids agree with the golden table
    ids = labels_original_ids(L)
    for v, ents in want.items():
        assert sorted(ids[v]) == sorted(ents)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_label_hubs_equal_full_index(seed):
    rng = np.random.default_rng(seed)
    for g in (inputs.erdos_renyi(150, 400, seed=seed), inputs.rmat(8, 8, seed=seed),
              inputs.grid_lcc(12, 0.05, seed=seed), inputs.random_tiny(30, 0.1, seed=seed)):
        for order in (None, rng.permutation(g.n).astype(np.uint32)):
            A = oracle.build(g.off, g.adj, order=order, tie_key=g.tie_key, method="definition")
            roff, radj = oracle.relabel(g.off, g.adj, A.order)
            for s in range(g.n):
                h, d = oracle.label_hubs(roff, radj, s)
                a, b = int(A.off[s]), int(A.off[s + 1])
                assert np.array_equal(h, A.hub[a:b]), (g.name, s)
                assert np.array_equal(d, A.dist[a:b]), (g.name, s)


def test_threaded_query_equals_single():
    g = inputs.rmat(11, 8, seed=4)
    L = oracle.build_graph(g, method="pull", threads=4)
    s, t = inputs.queries(g.n, 50_000, seed=9)
    rk = L.rank_of()
    rs, rt = rk[s], rk[t]
    d1, c1 = oracle.query_arrays(L.off, L.hub, L.dist, L.count, rs, rt)
    for th in (2, 7):
        d2, c2 = oracle.query_arrays(L.off, L.hub, L.dist, L.count, rs, rt, threads=th)
        assert np.array_equal(d1, d2) and np.array_equal(c1, c2)
    # and against BFS counting from a few sources
    for src in (0, 5, 77):
        bd, bc = oracle.bfs_count(g.off, g.adj, src)
        tt = np.arange(g.n, dtype=np.uint32)
        qd, qc = L.query(np.full(g.n, src, dtype=np.uint32), tt)
        assert np.array_equal(qd, bd) and np.array_equal(qc, bc)
