"""Large query batches answered in locality order (grouped by the label row
the query kernel stages, the longer label of an undirected query): answers
pair for pair equal to the unordered launch (SPC_QUERY_ORDER=0) and to the
oracle's labels, with invalid ids, s == t and repeated pairs in the batch;
undirected, directed and 1-shell-reduced indexes."""
import os

import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests.gpu_util import gpu_query

pytestmark = pytest.mark.gpu

# at least the batch size the ordered path starts at, plus a ragged tail
NQ = (1 << 20) + 12345


@pytest.fixture(scope="module")
def spc():
    import torch

    assert torch.cuda.is_available()
    from paper_2212_00977_amd import spc as mod

    return mod


def _batch(n, seed):
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n, NQ, dtype=np.int64).astype(np.uint32)
    t = rng.integers(0, n, NQ, dtype=np.int64).astype(np.uint32)
    t[:1000] = s[:1000]                      # s == t
    s[1000:1100] = n + np.arange(100, dtype=np.uint32)  # invalid ids
    t[1100:1200] = 0xFFFFFFFF
    s[2000:3000] = s[5000]                   # one long run of a vertex
    return s, t


def _both(ix, s, t):
    out = gpu_query(ix, s, t)
    os.environ["SPC_QUERY_ORDER"] = "0"
    try:
        ref = gpu_query(ix, s, t)
    finally:
        os.environ.pop("SPC_QUERY_ORDER", None)
    for a, b, nm in zip(out, ref, ("dist", "count", "flags")):
        assert np.array_equal(a, b), nm
    return out


def _oracle_sample(ref, s, t, d, c, n, t_row=0, k=20000):
    sel = np.r_[np.arange(0, 3000), np.random.default_rng(1).integers(0, NQ, k)]
    ok = (s[sel] < n) & (t[sel] < n)
    sel = sel[ok]
    rk = np.zeros(n, dtype=np.uint32)
    rk[ref.order] = np.arange(n, dtype=np.uint32)
    rd, rc = oracle.query_arrays(ref.off, ref.hub, ref.dist, ref.count, rk[s[sel]],
                                 t_row + rk[t[sel]], threads=oracle.host_threads())
    assert np.array_equal(d[sel], rd) and np.array_equal(c[sel], rc)


def test_ordered_batch_undirected(spc):
    g = inputs.rmat(13, 8, seed=21)
    print(f"[case] ordered batch {g.name} nq={NQ}", flush=True)
    ix = spc.build_graph(g)
    s, t = _batch(g.n, 3)
    d, c, f = _both(ix, s, t)
    bad = (s >= g.n) | (t >= g.n)
    assert (f[bad] & 8).all() and not (f[~bad] & 8).any()  # SPC_FLAG_INVALID
    _oracle_sample(oracle.build_graph(g, method="pull"), s, t, d, c, g.n)
    ix.free()


def test_ordered_batch_directed(spc):
    g = inputs.rmat_digraph(12, 8, seed=22)
    print(f"[case] ordered batch directed {g.name} nq={NQ}", flush=True)
    ix = spc.build_index(g.off, g.adj, directed=True)
    s, t = _batch(g.n, 4)
    d, c, f = _both(ix, s, t)
    ref = oracle.build_directed(g.n, g.off, g.adj)
    _oracle_sample(ref, s, t, d, c, g.n, t_row=g.n)
    ix.free()


def test_ordered_batch_one_shell(spc):
    g = inputs.chung_lu(8192, seed=23, wmax=500.0)
    print(f"[case] ordered batch one-shell {g.name} nq={NQ}", flush=True)
    ix = spc.build_graph(g, opts=spc.BuildOptions(one_shell=True))
    s, t = _batch(g.n, 5)
    d, c, f = _both(ix, s, t)
    # against the unreduced oracle index of the same graph
    _oracle_sample(oracle.build_graph(g, method="pull"), s, t, d, c, g.n)
    ix.free()
