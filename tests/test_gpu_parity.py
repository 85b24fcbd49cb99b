"""GPU parity: the HIP build and query against the CPU oracle, bit for bit.

Labels are compared entry by entry (order, offsets, hubs, distances,
counts); query answers pair by pair; per-round counters against the
oracle's PULL counters.  Every case prints its name before touching the GPU.
"""
import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests import brute
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


def check_graph(spc, g, method="pruned", queries=2000, opts=None, all_q=False):
    _say(f"{g.name} n={g.n} m={g.m}")
    ix = spc.build_graph(g, opts=opts)
    ref = oracle.build_graph(g, method=method,
                             depth_cap=(opts.round_cap if opts is not None else 0))
    assert_labels_equal(ix.export(), ref, g.name)
    if g.n:
        if all_q:
            s, t = all_pairs(g.n)
        else:
            s, t = inputs.queries(g.n, queries, seed=5)
        d, c, f = gpu_query(ix, s, t)
        rd, rc = ref.query(s, t)
        assert np.array_equal(d, rd), g.name
        assert np.array_equal(c, rc), g.name
    return ix, ref


def test_worked_example(spc):
    g = inputs.worked_example()
    ix, ref = check_graph(spc, g, all_q=True)
    st = ix.stats()
    assert st["entries"] == 35 and st["rounds"] == 4 and st["max_dist"] == 3
    nb = brute.adjacency(10, g.edges())
    s, t = all_pairs(10)
    d, c, f = gpu_query(ix, s, t)
    for i in range(100):
        assert (int(d[i]), int(c[i])) == brute.spc_brute(nb, int(s[i]), int(t[i]))
    d, c, f = gpu_query(ix, np.array([9]), np.array([6]))
    assert (int(d[0]), int(c[0])) == (3, 4)


def test_tiny_random_graphs(spc):
    rng = np.random.default_rng(123)
    for i in range(150):
        n = int(rng.integers(1, 41))
        p = float(rng.choice([0.05, 0.1, 0.2, 0.4, 0.8]))
        g = inputs.random_tiny(n, p, seed=5000 + i)
        if i % 3 == 0:
            g.order = rng.permutation(n).astype(np.uint32)
        check_graph(spc, g, method="definition", all_q=True)


def test_er2000_full(spc):
    """Erdos-Renyi n=2000 m=8000 seed 1: full labels, per-round counters and
    all 4M ordered pairs against BFS path counting."""
    g = inputs.erdos_renyi(2000, 8000, seed=1)
    ix, _ = check_graph(spc, g, queries=100000)
    pull = oracle.build_graph(g, method="pull")
    rs = ix.round_stats()
    R = ix.stats()["rounds"]
    assert R == pull.rounds
    for key in ("raw", "merged", "kept"):
        assert rs[key].tolist() == pull.stats[key].tolist(), key
    s, t = all_pairs(g.n)
    d, c, f = gpu_query(ix, s, t)
    for src in range(g.n):
        bd, bc = oracle.bfs_count(g.off, g.adj, src)
        sl = slice(src * g.n, (src + 1) * g.n)
        assert np.array_equal(d[sl], bd) and np.array_equal(c[sl], bc), src


@pytest.mark.parametrize("make", [
    lambda: inputs.chung_lu(1 << 13, seed=2),
    lambda: inputs.rmat(12, 8, seed=4),
    lambda: inputs.rmat(11, 16, seed=5),
    lambda: inputs.grid_lcc(48, 0.05, seed=3),
])
def test_family_instances(spc, make):
    check_graph(spc, make(), queries=20000)


def test_grid_saturating_counts(spc):
    """36x36 grid: corner-to-corner counts exceed 2^64-1 and saturate."""
    k = 36
    e = [(i * k + j, i * k + j + 1) for i in range(k) for j in range(k - 1)]
    e += [(i * k + j, (i + 1) * k + j) for i in range(k - 1) for j in range(k)]
    g = inputs.from_edges(k * k, np.array(e), name="grid36")
    ix, ref = check_graph(spc, g, queries=20000)
    assert ix.stats()["saturated_entries"] == int((ref.count == np.uint64(oracle.SAT)).sum()) > 0
    d, c, f = gpu_query(ix, np.array([0]), np.array([k * k - 1]))
    assert int(c[0]) == oracle.SAT and (int(f[0]) & 1)


def test_long_path_widens_to_16_bits(spc):
    n = 300
    g = inputs.from_edges(n, np.array([(i, i + 1) for i in range(n - 1)]), name="path300")
    ix, ref = check_graph(spc, g, queries=5000)
    assert ix.stats()["dist_bits"] == 16 and ix.stats()["max_dist"] == int(ref.dist.max()) > 254
    with pytest.raises(spc.SpcError) as e:
        spc.build_graph(g, opts=spc.BuildOptions(dist_bits=8))
    assert e.value.code == 4
    check_graph(spc, g, queries=5000, opts=spc.BuildOptions(dist_bits=16))


def test_edge_cases(spc):
    cases = [
        inputs.from_edges(1, np.zeros((0, 2)), name="single"),
        inputs.from_edges(5, np.zeros((0, 2)), name="isolated5"),
        inputs.from_edges(2, np.array([(0, 1)]), name="edge"),
        inputs.from_edges(30, np.array([(0, i) for i in range(1, 30)]), name="star"),
        inputs.from_edges(12, np.array([(i, j) for i in range(12) for j in range(i + 1, 12)]),
                          name="k12"),
        inputs.from_edges(40, np.array([(i, i + 1) for i in range(19)] +
                                       [(20 + i, 21 + i) for i in range(19)]), name="two_paths"),
        inputs.from_edges(9, np.array([(0, 1), (1, 2), (5, 6)]), name="sparse_isolated"),
    ]
    for g in cases:
        check_graph(spc, g, all_q=True)
    _say("empty graph")
    g = inputs.from_edges(0, np.zeros((0, 2)), name="empty")
    ix = spc.build_graph(g)
    assert ix.stats()["entries"] == 0
    d, c, f = gpu_query(ix, np.array([0]), np.array([0]))
    assert int(f[0]) == 8


def test_query_special_cases(spc):
    g = inputs.from_edges(10, np.array([(0, 1), (1, 2), (3, 4)]), name="q_special")
    ix = spc.build_graph(g)
    d, c, f = gpu_query(ix, np.array([2, 0, 3, 7, 10, 1]), np.array([2, 2, 0, 7, 1, 99]))
    assert (int(d[0]), int(c[0]), int(f[0])) == (0, 1, 0)      # s = t
    assert (int(d[1]), int(c[1])) == (2, 1)
    assert d[2] == oracle.INF and c[2] == 0 and f[2] == 2      # unreachable
    assert (int(d[3]), int(c[3])) == (0, 1)                    # isolated, s = t
    assert f[4] == 8 and f[5] == 8 and c[4] == 0               # invalid ids
    _say("empty query batch")
    d, c, f = gpu_query(ix, np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    assert d.shape[0] == 0


def test_invalid_graphs_rejected(spc):
    base = inputs.erdos_renyi(50, 120, seed=3)
    bad = []
    adj = base.adj.copy()
    adj[5] = 50                                  # id out of range
    bad.append(("id_range", base.off, adj, None))
    off = base.off.copy()
    adj = base.adj.copy()
    adj[0] = 0 if base.adj[0] != 0 else 1        # breaks symmetry / self loop
    bad.append(("asym", off, adj, None))
    e = base.edges()
    ee = np.concatenate([e, e[:1][:, ::-1]])      # duplicate edge in one direction
    src = np.concatenate([ee[:, 0], e[:, 1]])
    dst = np.concatenate([ee[:, 1], e[:, 0]])
    o = np.lexsort((dst, src))
    off2 = np.zeros(51, dtype=np.uint64)
    np.cumsum(np.bincount(src, minlength=50), out=off2[1:])
    bad.append(("dup", off2, dst[o].astype(np.uint32), None))
    off3 = base.off.copy()
    off3[10] = off3[11] + 1                      # offsets not monotone
    bad.append(("offsets", off3, base.adj, None))
    order = np.arange(50, dtype=np.uint32)
    order[3] = 4
    bad.append(("order_not_perm", base.off, base.adj, order))
    for name, off, adj, order in bad:
        _say(f"invalid {name}")
        with pytest.raises(spc.SpcError) as err:
            spc.build_index(off, adj, order=order)
        assert err.value.code == 1, name
    _say("memory budget")
    with pytest.raises(spc.SpcError) as err:
        spc.build_graph(base, opts=spc.BuildOptions(mem_budget=4096))
    assert err.value.code == 2


def test_determinism_and_validate_off(spc):
    g = inputs.rmat(11, 8, seed=9)
    _say(g.name)
    a = spc.build_graph(g).export()
    b = spc.build_graph(g, opts=spc.BuildOptions(validate=False)).export()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_round_cap(spc):
    g = inputs.grid_lcc(24, 0.05, seed=3)
    for cap in (1, 4, 9):
        opts = spc.BuildOptions(round_cap=cap)
        ix, ref = check_graph(spc, g, queries=3000, opts=opts)
        st = ix.stats()
        assert st["truncated"] == 1 and st["rounds"] == cap
        s, t = inputs.queries(g.n, 3000, seed=8)
        d, c, f = gpu_query(ix, s, t)
        full = oracle.build_graph(g)
        fd, fc = full.query(s, t)
        exact = d <= cap
        assert np.array_equal(d[exact], fd[exact]) and np.array_equal(c[exact], fc[exact])
        assert np.all((f[~exact] & 4) != 0)


def test_batch_equals_solo(spc):
    graphs = inputs.rmat_batch(6, seed=4, scale_lo=6, scale_hi=10)
    graphs.append(inputs.from_edges(3, np.zeros((0, 2)), name="edgeless3"))
    _say("batch of %d" % len(graphs))
    ix = spc.build_index_batch(graphs)
    assert ix.stats()["num_graphs"] == len(graphs)
    for gi, g in enumerate(graphs):
        ref = oracle.build_graph(g)
        assert_labels_equal(ix.export(gi), ref, g.name)
        s, t = inputs.queries(g.n, 2000, seed=gi)
        d, c, f = gpu_query(ix, s, t, graph_id=gi)
        rd, rc = ref.query(s, t)
        assert np.array_equal(d, rd) and np.array_equal(c, rc)
