"""Parity at the workloads' own sizes, in the configurations the benchmark
runs (the index is the same under any schedule: the theorem that the PULL
rounds give the sequential construction's labels, and the paper's
experiment finding PSPC and PSPC+ indexes identical).

* Batched: the 512 R-MAT graphs (scales 10..16, edge factor 8, seed 4) in one
  batched build.  Every graph: invariants, its degree order, answers from two
  BFS sources (1,000 targets each); graphs of scale <= 12: full labels
  against the oracle's PULL build; larger graphs: three hub columns from the
  trough-path definition.  The union's per-round inserts equal the summed
  distance histograms.
* High diameter, complete: the 256 x 256 grid (5% of edges deleted, seed 3,
  largest component) under the tree-decomposition order, 397 rounds with
  16-bit labels: full labels against the oracle's threaded PULL build.
* Power law, served-graph family: R-MAT scale 16, edge factor 16, seed 5
  (same generator as the served index at scale 21): full labels.
"""
import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests.gpu_util import (assert_labels_equal, check_hub_column_device,
                            check_invariants_device, check_source_answers, gpu_query)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch512():
    import torch

    from paper_2212_00977_amd import spc

    print("[case] rmat_batch(512, seed=4): generate", flush=True)
    graphs = inputs.rmat_batch(512, seed=4)
    print(f"[case] batched build of 512 graphs, n={sum(g.n for g in graphs)}", flush=True)
    ix = spc.build_index_batch(graphs)
    torch.cuda.synchronize()
    yield graphs, ix
    ix.free()


def test_batch512_every_graph(batch512):
    graphs, ix = batch512
    threads = oracle.host_threads()
    st = ix.stats()
    assert st["num_graphs"] == 512
    hist_sum = np.zeros(st["rounds"] + 2, dtype=np.int64)
    entries = 0
    rng = np.random.default_rng(44)
    full = cols = 0
    for gi, g in enumerate(graphs):
        if gi % 64 == 0:
            print(f"[case] batch graph {gi} ({g.name})", flush=True)
        ex = ix.export_device(gi)
        n, e = ix.graph_entries(gi)
        assert n == g.n
        entries += e
        h = check_invariants_device(ex, g.m, g.n)
        hist_sum[: h.shape[0]] += h
        order = ex["order"].cpu().numpy().astype(np.uint32)
        assert np.array_equal(order, oracle.degree_order(g.off)), g.name
        scale = int(g.n).bit_length() - 1
        if scale <= 12:
            ref = oracle.build_graph(g, method="pull", threads=threads)
            assert_labels_equal(ix.export(gi), ref, g.name)
            full += 1
        else:
            roff, radj = oracle.relabel(g.off, g.adj, order)
            for w in (0, int(rng.integers(1, 64)), int(rng.integers(64, g.n))):
                check_hub_column_device(ex, roff, radj, w)
            cols += 1
        for src in rng.integers(0, g.n, size=2).tolist():
            check_source_answers(ix, g, int(src), rng.integers(0, g.n, size=1000), graph_id=gi)
        del ex
    assert st["entries"] == entries
    kept = ix.round_stats()["kept"]
    assert hist_sum[: kept.shape[0]].tolist() == kept.astype(np.int64).tolist()
    assert int(hist_sum[kept.shape[0]:].sum()) == 0
    print(f"[case] batch: {full} graphs in full, {cols} by hub columns", flush=True)


def test_grid256_td_complete_full_labels():
    from paper_2212_00977_amd import spc

    print("[case] grid 256x256 LCC seed 3, tree-decomposition order", flush=True)
    g = inputs.grid_lcc(256, 0.05, seed=3)
    order, _ = spc.hybrid_order(g.off, g.adj, 0xFFFFFFFF)
    assert np.array_equal(order, oracle.hybrid_order(g.off, g.adj, 0xFFFFFFFF)[0])
    ix = spc.build_index(g.off, g.adj, order=order)
    st = ix.stats()
    assert st["truncated"] == 0 and st["label_bits"] == 16
    print(f"[case] oracle PULL build ({st['entries']} entries, {st['rounds']} rounds)", flush=True)
    ref = oracle.build(g.off, g.adj, order=order, method="pull", threads=oracle.host_threads())
    assert st["rounds"] == ref.rounds
    assert_labels_equal(ix.export(), ref, "grid256 td")
    kept = ix.round_stats()["kept"]
    assert kept.tolist() == ref.stats["kept"].tolist()
    s, t = inputs.queries(g.n, 200_000, seed=5)
    d, c, f = gpu_query(ix, s, t)
    rd, rc = ref.query(s, t)
    assert np.array_equal(d, rd) and np.array_equal(c, rc)
    ix.free()


def test_rmat16_ef16_full_labels():
    from paper_2212_00977_amd import spc

    print("[case] R-MAT scale 16 ef 16 seed 5", flush=True)
    g = inputs.rmat(16, 16, seed=5)
    ix = spc.build_graph(g)
    st = ix.stats()
    print(f"[case] oracle PULL build ({st['entries']} entries)", flush=True)
    ref = oracle.build_graph(g, method="pull", threads=oracle.host_threads())
    assert_labels_equal(ix.export(), ref, "rmat16 ef16")
    rs = ix.round_stats()
    for k in ("raw", "merged", "kept"):
        assert rs[k].tolist() == ref.stats[k].tolist(), k
    s, t = inputs.queries(g.n, 500_000, seed=6)
    d, c, f = gpu_query(ix, s, t)
    rd, rc = ref.query(s, t)
    assert np.array_equal(d, rd) and np.array_equal(c, rc)
    ix.free()
