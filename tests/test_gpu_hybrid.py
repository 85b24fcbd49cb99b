"""Builds under the hybrid and tree-decomposition vertex orders (the
library's spc_hybrid_order): labels equal the oracle's for the same explicit
order, answers equal BFS path counts (answers do not depend on the order),
and on a grid the tree-decomposition order gives a much smaller index than
the degree order."""
import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests.gpu_util import assert_labels_equal, gpu_query

pytestmark = pytest.mark.gpu

PURE = 0xFFFFFFFF

CASES = [
    ("grid32_pure", lambda: inputs.grid_lcc(32, 0.05, seed=3), PURE),
    ("grid32_d5", lambda: inputs.grid_lcc(32, 0.05, seed=3), 5),
    ("grid48_d16", lambda: inputs.grid_lcc(48, 0.05, seed=3), 16),
    ("er2000_d5", lambda: inputs.erdos_renyi(2000, 8000, seed=1), 5),
    ("rmat11_d5", lambda: inputs.rmat(11, 8, seed=4), 5),
    ("chunglu12_pure", lambda: inputs.chung_lu(1 << 12, seed=2), PURE),
]


@pytest.mark.parametrize("name,make,delta", CASES, ids=[c[0] for c in CASES])
def test_hybrid_order_build_matches_oracle(name, make, delta):
    from paper_2212_00977_amd import spc

    g = make()
    order, core = spc.hybrid_order(g.off, g.adj, delta)
    print(f"[case] {name}: n={g.n} core={core}", flush=True)
    ix = spc.build_index(g.off, g.adj, order=order)
    ref = oracle.build(g.off, g.adj, order=order)
    assert_labels_equal(ix.export(), ref, name)
    s, t = inputs.queries(g.n, 5000, seed=12)
    d, c, f = gpu_query(ix, s, t)
    rd, rc = oracle.build_graph(g).query(s, t)  # degree order: same answers
    assert np.array_equal(d, rd) and np.array_equal(c, rc), name


def test_tree_decomposition_order_shrinks_grid_index():
    from paper_2212_00977_amd import spc

    g = inputs.grid_lcc(64, 0.05, seed=3)
    order, _ = spc.hybrid_order(g.off, g.adj, PURE)
    td = spc.build_index(g.off, g.adj, order=order).stats()["entries"]
    deg = spc.build_graph(g).stats()["entries"]
    print(f"[case] grid64 entries: degree order {deg}, tree-decomposition order {td}", flush=True)
    assert td * 3 < deg
