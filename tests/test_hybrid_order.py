"""Hybrid vertex order ("Vertex Ordering Strategies": tree-decomposition
order for the fringe, degree order for the core).

The oracle's order is pinned by closed forms and by the degree order it
reduces to; the library's host implementation (spc_hybrid_order) must give
the oracle's order exactly.  CPU only."""
import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs

PURE = 0xFFFFFFFF  # no degree bound: the pure tree-decomposition order


def _edges(n, pairs, name=""):
    return inputs.from_edges(n, np.asarray(pairs, dtype=np.int64).reshape(-1, 2), name=name)


def test_path_pure_order_closed_form():
    # ends have degree 1; ties go to the smaller id, so 0, 1, ..., n-1 are
    # removed in turn and the order is their reverse
    n = 12
    g = _edges(n, [(i, i + 1) for i in range(n - 1)])
    order, core = oracle.hybrid_order(g.off, g.adj, PURE)
    assert core == 0 and order.tolist() == list(range(n - 1, -1, -1))


def test_cycle_pure_order_closed_form():
    # every vertex has degree 2; removing i links i+1 to n-1, keeping all
    # degrees at 2 until the last two
    n = 9
    g = _edges(n, [(i, (i + 1) % n) for i in range(n)])
    order, core = oracle.hybrid_order(g.off, g.adj, PURE)
    assert core == 0 and order.tolist() == list(range(n - 1, -1, -1))


def test_star_pure_order_closed_form():
    # centre 0, leaves 1..k: leaves 1..k-1 go first (degree 1, by id); then
    # the centre and leaf k both have degree 1 and the centre's id is smaller
    k = 7
    g = _edges(k + 1, [(0, i) for i in range(1, k + 1)])
    order, core = oracle.hybrid_order(g.off, g.adj, PURE)
    assert core == 0 and order.tolist() == [k, 0] + list(range(k - 1, 0, -1))


def test_fill_in_changes_the_order():
    # 4-cycle 0-2-1-3-0, all degree 2.  Removing 0 links 2 and 3, so 1, 2, 3
    # keep degree 2 and 1 (smallest id) goes next, then 2, then 3: order
    # 3, 2, 1, 0.  Without the fill-in edge, 2 and 3 would drop to degree 1
    # and 2 would go before 1.
    g = _edges(4, [(1, 3), (1, 2), (0, 3), (0, 2)])
    order, core = oracle.hybrid_order(g.off, g.adj, PURE)
    assert core == 0 and order.tolist() == [3, 2, 1, 0]


def test_complete_graph_core_or_fringe():
    n = 6
    g = _edges(n, [(a, b) for a in range(n) for b in range(a + 1, n)])
    order, core = oracle.hybrid_order(g.off, g.adj, n - 2)  # all degrees n-1 > delta: all core
    assert core == n and order.tolist() == list(range(n))
    order, core = oracle.hybrid_order(g.off, g.adj, n - 1)  # all removable, no fill-in
    assert core == 0 and order.tolist() == list(range(n - 1, -1, -1))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_delta_zero_is_degree_order(seed):
    # no vertex of degree 0 -> nothing is removed: the degree order (ties by
    # id), computed by an independent routine
    g = inputs.erdos_renyi(300, 1500, seed=seed)
    assert int(np.diff(g.off).min()) > 0
    order, core = oracle.hybrid_order(g.off, g.adj, 0)
    assert core == g.n
    assert np.array_equal(order, oracle.degree_order(g.off))


def test_core_fringe_properties():
    g = inputs.grid_lcc(20, 0.05, seed=3)
    for delta in (2, 3, 5, 8):
        order, core = oracle.hybrid_order(g.off, g.adj, delta)
        assert sorted(order.tolist()) == list(range(g.n))
        deg = np.diff(g.off.astype(np.int64))
        cdeg = deg[order[:core]]
        assert np.all(cdeg[:-1] >= cdeg[1:])  # core by input degree, descending


GRAPHS = [
    ("grid24", lambda: inputs.grid_lcc(24, 0.05, seed=3)),
    ("er400", lambda: inputs.erdos_renyi(400, 1600, seed=5)),
    ("rmat10", lambda: inputs.rmat(10, 8, seed=4)),
    ("chunglu11", lambda: inputs.chung_lu(1 << 11, seed=2)),
    ("path50", lambda: _edges(50, [(i, i + 1) for i in range(49)])),
    ("empty", lambda: _edges(3, np.zeros((0, 2)))),
]


@pytest.mark.parametrize("name,make", GRAPHS, ids=[g[0] for g in GRAPHS])
@pytest.mark.parametrize("delta", [0, 2, 5, PURE])
def test_library_order_equals_oracle(name, make, delta):
    from paper_2212_00977_amd import spc

    g = make()
    got, gcore = spc.hybrid_order(g.off, g.adj, delta)
    ref, rcore = oracle.hybrid_order(g.off, g.adj, delta)
    assert gcore == rcore and np.array_equal(got, ref), (name, delta)


def test_library_rejects_bad_input():
    from paper_2212_00977_amd import spc

    g = _edges(4, [(0, 1), (1, 2)])
    bad = g.adj.copy()
    bad[0] = 9  # id >= n
    with pytest.raises(spc.SpcError):
        spc.hybrid_order(g.off, bad, 5)
