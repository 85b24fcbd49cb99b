"""Builds with the neighbourhood-equivalence reduction (Section "Reduction
by Equivalence Relation", SPC_REDUCE_EQUIVALENCE): the device's classes
equal the oracle's; the labels of the representatives (weighted counts)
equal the oracle's weighted definition entry for entry; every answer equals
the oracle's reduced index and the oracle's unreduced index (itself pinned
to path enumeration); batches (isolated vertices stay in their own graph),
explicit orders, tie keys and truncated builds."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests.gpu_util import all_pairs, assert_labels_equal, gpu_query
from tests.test_twins import twin_graphs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spc():
    import torch

    assert torch.cuda.is_available()
    from paper_2212_00977_amd import spc as mod

    return mod


def _say(msg):
    print(f"[case] {msg}", flush=True)


def csr(n, edges, name):
    return inputs.from_edges(n, np.array(edges, dtype=np.int64).reshape(-1, 2), name=name)


CASES = [
    ("worked_example", inputs.worked_example),
    ("planted0", lambda: twin_graphs()[0]),
    ("planted3", lambda: twin_graphs()[3]),
    ("rmat6", lambda: twin_graphs()[5]),
    ("rmat11", lambda: inputs.rmat(11, 8, seed=4)),
    ("rmat12_ef4", lambda: inputs.rmat(12, 4, seed=5)),
    ("chunglu12", lambda: inputs.chung_lu(1 << 12, seed=2)),
    ("er2000_sparse", lambda: inputs.erdos_renyi(2000, 2400, seed=1)),
    ("grid40", lambda: inputs.grid_lcc(40, 0.05, seed=3)),
    ("k7", lambda: csr(7, [(a, b) for a in range(7) for b in range(a + 1, 7)], "k7")),
    ("k_3_40", lambda: csr(43, [(a, b) for a in range(3) for b in range(3, 43)], "k_3_40")),
    ("star50", lambda: csr(51, [(0, i) for i in range(1, 51)], "star50")),
    ("isolated5", lambda: inputs.from_edges(5, np.zeros((0, 2)), name="isolated5")),
    ("single", lambda: inputs.from_edges(1, np.zeros((0, 2)), name="single")),
]


def check_twins(g, queries=20000, order=None, tie_key=None, cap=0):
    from paper_2212_00977_amd import spc as S

    order = g.order if order is None else order
    tie_key = g.tie_key if tie_key is None else tie_key
    ix = S.build_index(g.off, g.adj, order=order, tie_key=tie_key,
                       opts=S.BuildOptions(equivalence=True, round_cap=cap))
    red = oracle.build_twin_reduced(g.off, g.adj, order=order, tie_key=tie_key, depth_cap=cap)
    ex = ix.export_reduction()
    assert np.array_equal(ex["root"], red.rep), f"{g.name}: classes differ"
    assert not ex["depth"].any() and np.array_equal(ex["parent"], np.arange(g.n))
    st = ix.stats()
    assert st["twin_vertices"] == g.n - red.ids.shape[0] and st["n"] == red.ids.shape[0]
    ref = dataclasses.replace(red.labels, order=red.ids[red.labels.order])
    assert_labels_equal(ix.export(), ref, g.name)
    if g.n:
        if g.n * g.n <= 4 * queries:
            s, t = all_pairs(g.n)
        else:
            s, t = inputs.queries(g.n, queries, seed=5)
        d, c, f = gpu_query(ix, s, t)
        rd, rc = red.query(s, t)
        assert np.array_equal(d, rd), g.name
        assert np.array_equal(c, rc), g.name
        if not cap:
            full = oracle.build(g.off, g.adj, order=order, tie_key=tie_key)
            fd, fc = full.query(s, t)
            assert np.array_equal(d, fd) and np.array_equal(c, fc), g.name
            assert not (f & 0x4).any()
    return ix, red


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_twin_build_matches_oracle(spc, name, make):
    g = make()
    _say(f"{name} n={g.n} m={g.m}")
    ix, red = check_twins(g)
    _say(f"{name}: {g.n - red.ids.shape[0]} twins merged, {ix.stats()['entries']} entries")


def test_twin_with_explicit_order_and_tie_keys(spc):
    g = inputs.rmat(11, 8, seed=7)
    rng = np.random.default_rng(3)
    check_twins(g, order=rng.permutation(g.n).astype(np.uint32))
    check_twins(g, tie_key=rng.integers(0, 1 << 40, g.n).astype(np.uint64))


def test_twin_truncated(spc):
    for g in (inputs.rmat(11, 8, seed=4), inputs.erdos_renyi(2000, 2400, seed=2)):
        _say(f"{g.name} cap 2")
        check_twins(g, cap=2)


def test_twin_batch_keeps_isolated_vertices_per_graph(spc):
    gs = [inputs.rmat(10, 4, seed=11), inputs.from_edges(6, np.array([(0, 1), (1, 2)]), name="p3+iso"),
          inputs.from_edges(4, np.zeros((0, 2)), name="iso4"), twin_graphs()[1], inputs.rmat(9, 8, seed=12)]
    ix = spc.build_index_batch(gs, opts=spc.BuildOptions(equivalence=True))
    for i, g in enumerate(gs):
        red = oracle.build_twin_reduced(g.off, g.adj, order=g.order, tie_key=g.tie_key)
        ex = ix.export_reduction(i)
        assert np.array_equal(ex["root"], red.rep), g.name
        ref = dataclasses.replace(red.labels, order=red.ids[red.labels.order])
        assert_labels_equal(ix.export(i), ref, g.name)
        s, t = all_pairs(g.n) if g.n <= 64 else inputs.queries(g.n, 5000, seed=i)
        d, c, f = gpu_query(ix, s, t, graph_id=i)
        rd, rc = red.query(s, t)
        assert np.array_equal(d, rd) and np.array_equal(c, rc), g.name


def test_class_weight_multiplies_counts(spc):
    # a 12x12 grid whose corner 0 reaches vertex x through 300 twins: every
    # shortest x-to-far-corner path picks one of the 300, so the count is
    # 300 times the grid's C(22, 11)
    from math import comb

    k = 12
    e = [(i * k + j, i * k + j + 1) for i in range(k) for j in range(k - 1)]
    e += [(i * k + j, (i + 1) * k + j) for i in range(k - 1) for j in range(k)]
    n0 = k * k
    x = n0 + 300
    e += [(0, n0 + i) for i in range(300)] + [(n0 + i, x) for i in range(300)]
    g = csr(n0 + 301, e, "grid_fan")
    ix, red = check_twins(g)
    assert ix.stats()["twin_vertices"] == 299
    d, c, f = gpu_query(ix, np.array([x, n0 + 5]), np.array([n0 - 1, n0 + 7]))
    assert (int(d[0]), int(c[0])) == (2 + 2 * (k - 1), 300 * comb(2 * (k - 1), k - 1))
    assert (int(d[1]), int(c[1])) == (2, 2)


def test_both_reductions_rejected(spc):
    g = inputs.rmat(8, 4, seed=1)
    with pytest.raises(spc.SpcError) as e:
        spc.build_graph(g, opts=spc.BuildOptions(one_shell=True, equivalence=True))
    assert e.value.code == 1
