"""Parity at the benchmark's full size (Chung-Lu n = 2^20, mean degree 10,
seed 2), in the configuration bench.py times.

The whole index is too large for the oracle to rebuild, so outputs the
oracle computes one by one are checked:
  * hub columns: every entry with hub w, for sampled hubs w (top-ranked,
    middle and low ranks), from the trough-path definition;
  * query answers for all targets of sampled sources, against BFS path
    counting;
  * properties that hold at any size: one distance-1 entry per edge, the
    self entry closing every label, hubs strictly increasing and never
    below the owner, per-round insert counts equal to the distance
    histogram.
"""
import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests.gpu_util import gpu_query

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def built():
    import torch

    from paper_2212_00977_amd import spc

    print("[case] chung-lu n=2^20 seed 2: generate", flush=True)
    g = inputs.workload("chunglu")
    print(f"[case] build n={g.n} m={g.m}", flush=True)
    ix = spc.build_graph(g)
    torch.cuda.synchronize()
    return g, ix


def test_fullsize_invariants(built):
    import torch

    g, ix = built
    st = ix.stats()
    ex = ix.export_device()
    off, hub, dist = ex["off"], ex["hub"].long(), ex["dist"].long()
    n = g.n
    deg = off[1:] - off[:-1]
    rows = torch.repeat_interleave(torch.arange(n, device=off.device), deg)
    assert int((dist == 1).sum()) == g.m
    last = off[1:] - 1
    assert torch.equal(hub[last], torch.arange(n, device=off.device))
    assert int(dist[last].abs().sum()) == 0
    assert bool((hub <= rows).all())
    same = rows[1:] == rows[:-1]
    assert bool((hub[1:][same] > hub[:-1][same]).all())
    hist = torch.bincount(dist, minlength=st["rounds"] + 1).cpu().numpy()
    kept = ix.round_stats()["kept"]
    assert hist[: st["rounds"] + 1].tolist() == kept.tolist()
    assert st["entries"] == int(off[-1])
    assert np.array_equal(ex["order"].cpu().numpy().astype(np.uint32),
                          oracle.degree_order(g.off))


def test_fullsize_hub_columns(built):
    import torch

    g, ix = built
    ex = ix.export_device()
    roff, radj = oracle.relabel(g.off, g.adj, oracle.degree_order(g.off))
    off, hub = ex["off"], ex["hub"]
    rng = np.random.default_rng(7)
    hubs = [0, 1, 2, 3, 10, 100, 1000] + sorted(rng.integers(1000, g.n, size=8).tolist())
    for w in hubs:
        print(f"[case] hub column {w}", flush=True)
        v, d, c = oracle.hub_column(roff, radj, int(w))
        idx = torch.nonzero(hub == int(w)).flatten()
        rows = torch.searchsorted(off[1:], idx, right=True)
        assert np.array_equal(rows.cpu().numpy().astype(np.uint32), v), w
        assert np.array_equal(ex["dist"][idx].cpu().numpy().astype(np.uint32), d), w
        assert np.array_equal(ex["count"][idx].cpu().numpy().view(np.uint64), c), w


def test_fullsize_queries_vs_bfs(built):
    g, ix = built
    rng = np.random.default_rng(11)
    for src in rng.integers(0, g.n, size=6).tolist():
        print(f"[case] bfs source {src}", flush=True)
        t = np.arange(g.n, dtype=np.uint32)
        s = np.full(g.n, src, dtype=np.uint32)
        d, c, f = gpu_query(ix, s, t)
        bd, bc = oracle.bfs_count(g.off, g.adj, src)
        assert np.array_equal(d, bd) and np.array_equal(c, bc), src
