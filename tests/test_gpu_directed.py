"""Directed labels on the GPU (Section "2-Hop Labeling for Shortest Path
Counting": an out-label and an in-label per vertex, the query over L_out(s)
and L_in(t)).  Labels entry for entry against the oracle's directed
definition (2n rows), answers against directed BFS path counting, a
symmetric digraph equal to the undirected index, closed forms, and the
refused inputs."""
import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests.gpu_util import all_pairs, assert_labels_equal, gpu_query

pytestmark = pytest.mark.gpu


def _build(g, order=None, **kw):
    from paper_2212_00977_amd import spc

    return spc.build_index(g.off, g.adj, order=order, directed=True, **kw)


def _check(g, order=None, pairs=None, **kw):
    ix = _build(g, order=order, **kw)
    ref = oracle.build_directed(g.n, g.off, g.adj, order=order)
    assert_labels_equal(ix.export(), ref, g.name)
    st = ix.stats()
    assert st["directed"] == 1 and st["entries"] == ref.entries and st["m"] == g.m
    s, t = all_pairs(g.n) if pairs is None else pairs
    d, c, f = gpu_query(ix, s, t)
    # every answer against the oracle's labels (rows: out-label of s, in-label of t)
    rk = np.zeros(g.n, dtype=np.uint32)
    rk[ref.order] = np.arange(g.n, dtype=np.uint32)
    rd, rc = oracle.query_arrays(ref.off, ref.hub, ref.dist, ref.count, rk[s], g.n + rk[t])
    assert np.array_equal(d, rd) and np.array_equal(c, rc), g.name
    # and those of some sources against BFS path counting along the arcs
    for src in np.unique(s)[:60]:
        sel = s == src
        bd, bc = oracle.bfs_count(g.off, g.adj, int(src))
        assert np.array_equal(d[sel], bd[t[sel]]) and np.array_equal(c[sel], bc[t[sel]]), (g.name, src)
    return ix


@pytest.mark.parametrize("seed", range(10))
def test_random_digraphs_all_pairs(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 70))
    g = inputs.random_digraph(n, int(rng.integers(n, 5 * n)), seed=seed)
    print(f"[case] directed {g.name}", flush=True)
    order = rng.permutation(n).astype(np.uint32) if seed % 3 == 0 else None
    _check(g, order=order).free()


def test_directed_rmat_and_er():
    for g in (inputs.rmat_digraph(11, 8, seed=4), inputs.random_digraph(2000, 9000, seed=2),
              inputs.rmat_digraph(12, 16, seed=5)):
        print(f"[case] directed {g.name} n={g.n} arcs={g.m}", flush=True)
        s, t = inputs.queries(g.n, 30000, seed=3)
        _check(g, pairs=(s, t)).free()


def test_directed_closed_forms_and_widening():
    # directed path: (b - a, 1) forward, unreachable backward; 300 vertices
    # pass 254 rounds: 16-bit labels
    n = 300
    g = inputs.digraph_from_arcs(n, [(i, i + 1) for i in range(n - 1)], name="dpath300")
    print("[case] directed path 300", flush=True)
    ix = _build(g)
    assert ix.stats()["label_bits"] == 16
    s, t = all_pairs(n)
    d, c, f = gpu_query(ix, s, t)
    fwd = t >= s
    assert np.array_equal(d[fwd], (t - s)[fwd]) and np.all(c[fwd] == 1)
    assert np.all(d[~fwd] == oracle.INF) and np.all(c[~fwd] == 0)
    ix.free()
    # directed cycle: one path each way round
    g = inputs.digraph_from_arcs(9, [(i, (i + 1) % 9) for i in range(9)], name="dcycle9")
    ix = _build(g)
    s, t = all_pairs(9)
    d, c, f = gpu_query(ix, s, t)
    assert np.array_equal(d, (t.astype(np.int64) - s) % 9) and np.all(c == 1)
    ix.free()


def test_symmetric_digraph_is_undirected_index():
    from paper_2212_00977_amd import spc

    g = inputs.erdos_renyi(400, 1500, seed=7)
    print("[case] symmetric digraph vs undirected index", flush=True)
    dg = inputs.Graph(g.n, g.off, g.adj, name="sym", directed=True)
    ix = _build(dg)
    und = spc.build_graph(g).export()
    ex = ix.export()
    n = g.n
    off = ex["off"].astype(np.int64)
    assert np.array_equal(ex["order"], und["order"])
    for side in (0, 1):
        a, b = off[side * n], off[side * n + n]
        assert np.array_equal(off[side * n: side * n + n + 1] - a, und["off"].astype(np.int64))
        assert np.array_equal(ex["hub"][a:b], und["hub"]) and np.array_equal(ex["count"][a:b], und["count"])
    ix.free()


def test_directed_multi_query_and_refusals():
    from paper_2212_00977_amd import spc

    g = inputs.rmat_digraph(10, 8, seed=9)
    ix = _build(g)
    ref = oracle.build_directed(g.n, g.off, g.adj)
    s, t = inputs.queries(g.n, 20000, seed=4)
    rk = np.zeros(g.n, dtype=np.uint32)
    rk[ref.order] = np.arange(g.n, dtype=np.uint32)
    rd, rc = oracle.query_arrays(ref.off, ref.hub, ref.dist, ref.count, rk[s], g.n + rk[t])
    import torch
    from tests.gpu_util import dist_as_u32
    for th in (0, 256, 1 << 30):
        ix.set_query_buckets(th)
        d, c, f = ix.query_multi(None, s, t)
        torch.cuda.synchronize()
        assert np.array_equal(dist_as_u32(spc.as_dist(d), ix.dist_bits), rd)
        assert np.array_equal(spc.as_u64(c), rc)
    ix.free()
    # self loop, repeated arc: refused when validating
    bad = inputs.Graph(3, np.array([0, 1, 2, 2], dtype=np.uint64), np.array([0, 2], dtype=np.uint32),
                       directed=True)
    with pytest.raises(spc.SpcError):
        _build(bad)
    dup = inputs.Graph(3, np.array([0, 2, 2, 2], dtype=np.uint64), np.array([1, 1], dtype=np.uint32),
                       directed=True)
    with pytest.raises(spc.SpcError):
        _build(dup)
    with pytest.raises(spc.SpcError):
        _build(g, opts=spc.BuildOptions(one_shell=True))
