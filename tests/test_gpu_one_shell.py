"""Builds with the 1-shell reduction (Section "Reduction by 1-Shell",
SPC_REDUCE_ONE_SHELL): the device's fringe, roots, depths and parents equal
the oracle's 1-shell; the core labels equal the oracle's labels of the core
subgraph; every answer equals the oracle's unreduced index (itself pinned to
path enumeration), including tree paths inside the fringe and tree
components; batches, explicit orders, tie keys and truncated builds."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests.gpu_util import all_pairs, assert_labels_equal, gpu_query

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spc():
    import torch

    assert torch.cuda.is_available()
    from paper_2212_00977_amd import spc as mod

    return mod


def _say(msg):
    print(f"[case] {msg}", flush=True)


def forest(n, seed, extra=0):
    rng = np.random.default_rng(seed)
    e = [(v, int(rng.integers(0, v))) for v in range(1, n) if rng.random() < 0.97]
    for _ in range(extra):
        a, b = (int(x) for x in rng.integers(0, n, 2))
        if a != b:
            e.append((a, b))
    e = sorted(set(tuple(sorted(x)) for x in e))
    return inputs.from_edges(n, np.array(e, dtype=np.int64).reshape(-1, 2), name=f"forest{n}")


def path(n):
    return inputs.from_edges(n, np.array([(i, i + 1) for i in range(n - 1)], dtype=np.int64).reshape(-1, 2),
                             name=f"path{n}")


CASES = [
    ("worked_example", inputs.worked_example),
    ("er2000_sparse", lambda: inputs.erdos_renyi(2000, 2400, seed=1)),
    ("er2000", lambda: inputs.erdos_renyi(2000, 8000, seed=1)),
    ("chunglu12", lambda: inputs.chung_lu(1 << 12, seed=2)),
    ("chunglu14", lambda: inputs.chung_lu(1 << 14, seed=3)),
    ("rmat11", lambda: inputs.rmat(11, 8, seed=4)),
    ("grid40", lambda: inputs.grid_lcc(40, 0.05, seed=3)),
    ("forest3000", lambda: forest(3000, 5)),
    ("forest_cycles3000", lambda: forest(3000, 6, extra=40)),
    ("path300", lambda: path(300)),
    ("path2", lambda: path(2)),
    ("single", lambda: inputs.from_edges(1, np.zeros((0, 2)), name="single")),
    ("isolated5", lambda: inputs.from_edges(5, np.zeros((0, 2)), name="isolated5")),
]


def check_reduced(spc, g, opts=None, queries=20000, order=None, tie_key=None, cap=0):
    from paper_2212_00977_amd import spc as S

    opts = opts or S.BuildOptions(one_shell=True, round_cap=cap)
    order = g.order if order is None else order
    tie_key = g.tie_key if tie_key is None else tie_key
    ix = S.build_index(g.off, g.adj, order=order, tie_key=tie_key, opts=opts)
    red = oracle.build_reduced(g.off, g.adj, order=order, tie_key=tie_key, depth_cap=cap)
    sh = red.shell
    ex = ix.export_reduction()
    assert np.array_equal(ex["root"], sh.root), f"{g.name}: roots differ"
    assert np.array_equal(ex["depth"], sh.depth), f"{g.name}: depths differ"
    assert np.array_equal(ex["parent"], sh.parent), f"{g.name}: parents differ"
    st = ix.stats()
    assert st["fringe_vertices"] == int((~sh.core).sum())
    assert st["fringe_depth"] == (int(sh.depth.max()) if g.n else 0)
    lab = ix.export()
    ref = dataclasses.replace(red.labels, order=red.core_ids[red.labels.order])  # core -> input ids
    assert_labels_equal(lab, ref, g.name)
    assert st["n"] == int(sh.core.sum()) and st["entries"] == ref.entries
    if g.n:
        if g.n * g.n <= 4 * queries:
            s, t = all_pairs(g.n)
        else:
            s, t = inputs.queries(g.n, queries, seed=5)
        d, c, f = gpu_query(ix, s, t)
        rd, rc = red.query(s, t)
        assert np.array_equal(d, rd), g.name
        assert np.array_equal(c, rc), g.name
        if not cap:  # the unreduced index answers the same
            full = oracle.build(g.off, g.adj, order=order, tie_key=tie_key)
            fd, fc = full.query(s, t)
            assert np.array_equal(d, fd) and np.array_equal(c, fc), g.name
            assert (f & 0x4).sum() == 0
        else:
            same = sh.root[s] == sh.root[t]
            core_d = rd.astype(np.int64) - sh.depth[s] - sh.depth[t]
            horizon = ~same & ((rd == oracle.INF) | (core_d > cap))
            assert np.array_equal((f & 0x4) != 0, horizon), g.name
    return ix, red


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_reduced_build_matches_oracle(spc, name, make):
    g = make()
    _say(f"{name} n={g.n} m={g.m}")
    ix, red = check_reduced(spc, g)
    red_fr = int((~red.shell.core).sum())
    _say(f"{name}: fringe {red_fr}, core entries {ix.stats()['entries']}")


def test_reduced_with_explicit_order_and_tie_keys(spc):
    g = inputs.chung_lu(1 << 12, seed=7)
    rng = np.random.default_rng(3)
    check_reduced(spc, g, order=rng.permutation(g.n).astype(np.uint32))
    check_reduced(spc, g, tie_key=rng.integers(0, 1 << 40, g.n).astype(np.uint64))
    order, _ = spc.hybrid_order(g.off, g.adj, 5)
    check_reduced(spc, g, order=order)


def test_reduced_truncated(spc):
    for g in (inputs.erdos_renyi(2000, 2400, seed=2), inputs.grid_lcc(40, 0.05, seed=3)):
        _say(f"{g.name} cap 3")
        check_reduced(spc, g, cap=3)


def test_reduced_batch(spc):
    gs = [inputs.erdos_renyi(1500, 1800, seed=11), forest(800, 12), inputs.chung_lu(1 << 11, seed=13),
          path(7), inputs.rmat(10, 4, seed=14)]
    ix = spc.build_index_batch(gs, opts=spc.BuildOptions(one_shell=True))
    for i, g in enumerate(gs):
        red = oracle.build_reduced(g.off, g.adj, order=g.order, tie_key=g.tie_key)
        ex = ix.export_reduction(i)
        assert np.array_equal(ex["root"], red.shell.root), g.name
        assert np.array_equal(ex["depth"], red.shell.depth), g.name
        assert np.array_equal(ex["parent"], red.shell.parent), g.name
        ref = dataclasses.replace(red.labels, order=red.core_ids[red.labels.order])
        assert_labels_equal(ix.export(i), ref, g.name)
        s, t = inputs.queries(g.n, 5000, seed=i)
        d, c, f = gpu_query(ix, s, t, graph_id=i)
        rd, rc = red.query(s, t)
        assert np.array_equal(d, rd) and np.array_equal(c, rc), g.name
        # ids past this graph's input size are invalid, even where the core is smaller
        d, c, f = gpu_query(ix, np.array([g.n]), np.array([0]), graph_id=i)
        assert f[0] == 0x8 and c[0] == 0


def test_fringe_depth_widens_outputs(spc):
    # a path's core is its centre: labels hold distance 0 only, but queries
    # reach 299, so the outputs are 16 bits wide
    g = path(300)
    ix = spc.build_graph(g, opts=spc.BuildOptions(one_shell=True))
    st = ix.stats()
    assert st["label_bits"] == 8 and st["max_dist"] == 0 and st["dist_bits"] == 16
    assert st["fringe_vertices"] == 299 and st["fringe_depth"] == 150
    d, c, f = gpu_query(ix, np.array([0, 0, 149, 299]), np.array([299, 149, 150, 298]))
    assert list(d) == [299, 149, 1, 1] and list(c) == [1, 1, 1, 1]


def test_long_queries_over_short_labels_widen_outputs(spc):
    # ranking a path from its centre outwards keeps every label distance at
    # most 200, yet the end-to-end query is 400 long: 8-bit labels, 16-bit
    # outputs
    n = 401
    g = path(n)
    c0 = n // 2
    order = np.array(sorted(range(n), key=lambda v: (abs(v - c0), v)), dtype=np.uint32)
    ix = spc.build_index(g.off, g.adj, order=order)
    st = ix.stats()
    assert st["label_bits"] == 8 and st["max_dist"] == 200 and st["dist_bits"] == 16
    ref = oracle.build(g.off, g.adj, order=order)
    assert_labels_equal(ix.export(), ref, "path401")
    s, t = all_pairs(n)
    d, c, f = gpu_query(ix, s, t)
    rd, rc = ref.query(s, t)
    assert np.array_equal(d, rd) and np.array_equal(c, rc)
    assert int(d.max()) == 400


def test_reduced_rejects_asymmetric_input(spc):
    off = np.array([0, 1, 1, 2], dtype=np.uint64)
    adj = np.array([1, 0], dtype=np.uint32)  # 0->1 and 2->0: not symmetric
    with pytest.raises(spc.SpcError) as e:
        spc.build_index(off, adj, opts=spc.BuildOptions(one_shell=True))
    assert e.value.code == 1
    with pytest.raises(spc.SpcError):
        spc.build_index(off, adj, opts=spc.BuildOptions())


def test_unreduced_index_reports_identity_shell(spc):
    g = inputs.erdos_renyi(300, 320, seed=9)
    ix = spc.build_graph(g)
    ex = ix.export_reduction()
    assert np.array_equal(ex["root"], np.arange(g.n)) and not ex["depth"].any()
    assert ix.stats()["fringe_vertices"] == 0


def test_export_reduction_to_device_memory(spc):
    g = forest(500, 21, extra=10)
    for opts in (spc.BuildOptions(one_shell=True), spc.BuildOptions(equivalence=True), spc.BuildOptions()):
        ix = spc.build_graph(g, opts=opts)
        host = ix.export_reduction()
        dev = ix.export_reduction_device()
        for k in ("root", "depth", "parent"):
            assert np.array_equal(dev[k].cpu().numpy().view(np.uint32), host[k]), k
        with pytest.raises(spc.SpcError):
            ix.export_reduction(1)
