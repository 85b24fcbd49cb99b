"""Queries over many graphs in one call (spc_query_batch_multi): bucketed
by label length, answered 16 lanes per short query and a wave per long one.
Every answer equals the per-graph call's and the oracle's, for every bucket
threshold, with invalid graph and vertex ids mixed in, on reduced indexes,
16-bit labels and a single graph."""
import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests.gpu_util import dist_as_u32

pytestmark = pytest.mark.gpu

THRESHOLDS = (0, 64, 256, 1024, 1 << 30)


def _multi(ix, gid, s, t):
    import torch
    from paper_2212_00977_amd import spc

    d, c, f = ix.query_multi(gid, s, t)
    torch.cuda.synchronize()
    return dist_as_u32(spc.as_dist(d), ix.dist_bits), spc.as_u64(c), f.cpu().numpy()


def _mixed_queries(graphs, per, seed):
    rng = np.random.default_rng(seed)
    gid = rng.integers(0, len(graphs), size=per * len(graphs)).astype(np.uint32)
    n = np.array([g.n for g in graphs], dtype=np.int64)[gid]
    s = (rng.random(gid.shape[0]) * n).astype(np.uint32)
    t = (rng.random(gid.shape[0]) * n).astype(np.uint32)
    return gid, s, t


def test_multi_batch_every_threshold():
    from paper_2212_00977_amd import spc

    graphs = inputs.rmat_batch(40, seed=4, scale_lo=6, scale_hi=12)
    print(f"[case] multi-graph queries over {len(graphs)} graphs", flush=True)
    ix = spc.build_index_batch(graphs)
    refs = [oracle.build_graph(g) for g in graphs]
    gid, s, t = _mixed_queries(graphs, 500, seed=1)
    # invalid graph ids and vertex ids
    gid[:5] = len(graphs) + np.arange(5, dtype=np.uint32)
    s[5:10] = 1 << 30
    want_d = np.zeros(gid.shape[0], dtype=np.uint32)
    want_c = np.zeros(gid.shape[0], dtype=np.uint64)
    for gi, ref in enumerate(refs):
        sel = np.nonzero((gid == gi) & (s < graphs[gi].n))[0]
        want_d[sel], want_c[sel] = ref.query(s[sel], t[sel])
    bad = np.zeros(gid.shape[0], dtype=bool)
    bad[:10] = True
    for th in THRESHOLDS:
        ix.set_query_buckets(th)
        d, c, f = _multi(ix, gid, s, t)
        assert np.all(f[bad] == spc.FLAG_INVALID), th
        assert np.array_equal(d[~bad], want_d[~bad]), th
        assert np.array_equal(c[~bad], want_c[~bad]), th
    # the per-graph call agrees bit for bit, flags included
    ix.set_query_buckets(256)
    d, c, f = _multi(ix, gid, s, t)
    for gi in range(len(graphs)):
        sel = np.nonzero(gid == gi)[0]
        import torch
        dd, cc, ff = ix.query(s[sel], t[sel], graph_id=gi)
        torch.cuda.synchronize()
        assert np.array_equal(dist_as_u32(spc.as_dist(dd), ix.dist_bits), d[sel])
        assert np.array_equal(spc.as_u64(cc), c[sel]) and np.array_equal(ff.cpu().numpy(), f[sel])
    th = ix.tune_query_buckets(gid, s, t)
    assert th in (0, 64, 128, 256, 512, 1024, 2048)
    d2, c2, f2 = _multi(ix, gid, s, t)
    assert np.array_equal(d2, d) and np.array_equal(c2, c) and np.array_equal(f2, f)
    ix.free()


@pytest.mark.parametrize("kind", ["one_shell", "equivalence"])
def test_multi_reduced_batch(kind):
    from paper_2212_00977_amd import spc

    graphs = inputs.rmat_batch(12, seed=9, scale_lo=6, scale_hi=10)
    print(f"[case] multi-graph queries, {kind} batch", flush=True)
    ix = spc.build_index_batch(graphs, opts=spc.BuildOptions(**{kind: True}))
    gid, s, t = _mixed_queries(graphs, 800, seed=2)
    for th in THRESHOLDS:
        ix.set_query_buckets(th)
        d, c, f = _multi(ix, gid, s, t)
        for gi, g in enumerate(graphs):
            sel = np.nonzero(gid == gi)[0]
            bd = np.zeros(sel.shape[0], dtype=np.uint32)
            bc = np.zeros(sel.shape[0], dtype=np.uint64)
            for j, q in enumerate(sel):
                dd, cc = oracle.bfs_count(g.off, g.adj, int(s[q]))
                bd[j], bc[j] = dd[t[q]], cc[t[q]]
            assert np.array_equal(d[sel], bd) and np.array_equal(c[sel], bc), (kind, th, gi)
    ix.free()


def test_multi_single_graph_16bit_and_none_ids():
    from paper_2212_00977_amd import spc

    g = inputs.from_edges(300, np.stack([np.arange(299), np.arange(1, 300)], axis=1), name="path300")
    print("[case] multi-graph queries, 16-bit path graph", flush=True)
    ix = spc.build_graph(g)
    assert ix.dist_bits == 16
    ref = oracle.build_graph(g)
    s, t = inputs.queries(g.n, 20000, seed=3)
    rd, rc = ref.query(s, t)
    for th in THRESHOLDS:
        ix.set_query_buckets(th)
        d, c, f = _multi(ix, None, s, t)
        assert np.array_equal(d, rd) and np.array_equal(c, rc), th
        d, c, f = _multi(ix, np.zeros(s.shape[0], dtype=np.uint32), s, t)
        assert np.array_equal(d, rd) and np.array_equal(c, rc), th
    ix.free()


def test_multi_empty_and_bad_args():
    import torch
    from paper_2212_00977_amd import native, spc

    g = inputs.erdos_renyi(100, 300, seed=1)
    ix = spc.build_graph(g)
    d, c, f = ix.query_multi(None, np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    torch.cuda.synchronize()
    assert d.numel() == 0
    L = native.load()
    assert L.spc_query_batch_multi(None, None, None, None, 1, None, None, None, None) == 1
    with pytest.raises(ValueError):
        ix.query(np.zeros(4, np.uint32), np.zeros(4, np.uint32),
                 out=(torch.empty(4, dtype=torch.int16, device="cuda"),
                      torch.empty(4, dtype=torch.int64, device="cuda"), None))
    ix.free()
