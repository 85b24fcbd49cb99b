"""Batched build: one index over many independent R-MAT graphs of uneven
sizes equals the solo index of every graph (labels entry for entry, against
the oracle), and per-graph queries address the right graph."""
import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests.gpu_util import assert_labels_equal, gpu_query

pytestmark = pytest.mark.gpu


def test_rmat_batch_labels_and_queries():
    from paper_2212_00977_amd import spc

    graphs = inputs.rmat_batch(48, seed=4, scale_lo=6, scale_hi=12)
    print(f"[case] batch of {len(graphs)} R-MAT graphs, n={sum(g.n for g in graphs)}", flush=True)
    ix = spc.build_index_batch(graphs)
    st = ix.stats()
    assert st["num_graphs"] == len(graphs)
    total = 0
    for gi, g in enumerate(graphs):
        ref = oracle.build_graph(g)
        assert_labels_equal(ix.export(gi), ref, g.name)
        total += ref.entries
        s, t = inputs.queries(g.n, 1000, seed=100 + gi)
        d, c, f = gpu_query(ix, s, t, graph_id=gi)
        rd, rc = ref.query(s, t)
        assert np.array_equal(d, rd) and np.array_equal(c, rc), g.name
    assert st["entries"] == total
    # per-round counters of the union are the sums over the graphs
    rs = ix.round_stats()
    kept = np.zeros_like(rs["kept"])
    for g in graphs:
        p = oracle.build_graph(g, method="pull").stats["kept"]
        kept[: p.shape[0]] += p
    assert rs["kept"].tolist() == kept.tolist()


def test_batch_mixed_sizes_with_empty_graphs():
    from paper_2212_00977_amd import spc

    graphs = [inputs.from_edges(0, np.zeros((0, 2)), name="empty"),
              inputs.rmat(9, 8, seed=1),
              inputs.from_edges(1, np.zeros((0, 2)), name="single"),
              inputs.erdos_renyi(300, 700, seed=2)]
    print("[case] batch with empty graphs", flush=True)
    ix = spc.build_index_batch(graphs)
    for gi, g in enumerate(graphs):
        if g.n == 0:
            continue
        assert_labels_equal(ix.export(gi), oracle.build_graph(g), g.name)
    d, c, f = gpu_query(ix, np.array([0]), np.array([0]), graph_id=0)
    assert int(f[0]) == 8  # no vertex in the empty graph
    with pytest.raises(spc.SpcError):
        gpu_query(ix, np.array([0]), np.array([0]), graph_id=len(graphs))
