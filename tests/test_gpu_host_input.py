"""Builds from host-resident graphs (spc_graph.on_device = 0, plain host
pointers through the C ABI; the library stages them to the device), plain
and with either reduction, equal the oracle; a reduced build that exceeds
its memory budget fails cleanly and the next build works; reductions with
forced 16-bit labels."""
import ctypes as C
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests.gpu_util import assert_labels_equal, gpu_query

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spc():
    import torch

    assert torch.cuda.is_available()
    from paper_2212_00977_amd import spc as mod

    return mod


def build_host(spc, g, opts):
    import torch

    from paper_2212_00977_amd import native

    off = np.ascontiguousarray(g.off, dtype=np.uint64)
    adj = np.ascontiguousarray(g.adj, dtype=np.uint32)
    gs = native.SpcGraph()
    gs.n = g.n
    gs.nnz = int(adj.shape[0])
    gs.row_off = off.ctypes.data
    gs.col = adj.ctypes.data if adj.shape[0] else None
    keep = [off, adj]
    if g.order is not None:
        o = np.ascontiguousarray(g.order, dtype=np.uint32)
        keep.append(o)
        gs.order = o.ctypes.data
    if g.tie_key is not None:
        tk = np.ascontiguousarray(g.tie_key, dtype=np.uint64)
        keep.append(tk)
        gs.tie_key = tk.ctypes.data
    gs.on_device = 0
    h = C.c_void_p()
    o = opts.struct()
    rc = native.load().spc_build_index(C.byref(gs), C.byref(o), None, C.byref(h))
    if rc:
        raise spc.SpcError(rc, "spc_build_index")
    return spc.Index(h, torch.device("cuda", torch.cuda.current_device()), [g.n])


@pytest.mark.parametrize("kind", ["plain", "one_shell", "equivalence"])
def test_host_input_build(spc, kind):
    for g in (inputs.rmat(11, 8, seed=4), inputs.grid_lcc(32, 0.05, seed=3), inputs.worked_example()):
        print(f"[case] host input {kind}: {g.name}", flush=True)
        opts = spc.BuildOptions(**({} if kind == "plain" else {kind: True}))
        ix = build_host(spc, g, opts)
        if kind == "plain":
            red, ids = None, None
            ref = oracle.build_graph(g)
        elif kind == "one_shell":
            red = oracle.build_reduced(g.off, g.adj, order=g.order, tie_key=g.tie_key)
            ref = dataclasses.replace(red.labels, order=red.core_ids[red.labels.order])
        else:
            red = oracle.build_twin_reduced(g.off, g.adj, order=g.order, tie_key=g.tie_key)
            ref = dataclasses.replace(red.labels, order=red.ids[red.labels.order])
        assert_labels_equal(ix.export(), ref, g.name)
        s, t = inputs.queries(g.n, 5000, seed=3)
        d, c, f = gpu_query(ix, s, t)
        rd, rc = (red or ref).query(s, t)
        assert np.array_equal(d, rd) and np.array_equal(c, rc), g.name


@pytest.mark.parametrize("kind", ["one_shell", "equivalence"])
def test_reduced_budget_failure_then_success(spc, kind):
    g = inputs.rmat(11, 8, seed=4)
    with pytest.raises(spc.SpcError) as e:
        spc.build_graph(g, opts=spc.BuildOptions(mem_budget=1 << 16, **{kind: True}))
    assert e.value.code == 2
    ix = spc.build_graph(g, opts=spc.BuildOptions(**{kind: True}))
    s, t = inputs.queries(g.n, 5000, seed=4)
    d, c, f = gpu_query(ix, s, t)
    rd, rc = oracle.build_graph(g).query(s, t)
    assert np.array_equal(d, rd) and np.array_equal(c, rc)


@pytest.mark.parametrize("kind", ["one_shell", "equivalence"])
def test_reduced_with_16_bit_labels(spc, kind):
    g = inputs.chung_lu(1 << 11, seed=9)
    ix = spc.build_graph(g, opts=spc.BuildOptions(dist_bits=16, **{kind: True}))
    st = ix.stats()
    assert st["label_bits"] == 16 and st["dist_bits"] == 16
    if kind == "one_shell":
        red = oracle.build_reduced(g.off, g.adj)
        ids = red.core_ids
    else:
        red = oracle.build_twin_reduced(g.off, g.adj)
        ids = red.ids
    assert_labels_equal(ix.export(), dataclasses.replace(red.labels, order=ids[red.labels.order]), g.name)
    s, t = inputs.queries(g.n, 5000, seed=8)
    d, c, f = gpu_query(ix, s, t)
    rd, rc = red.query(s, t)
    assert np.array_equal(d, rd) and np.array_equal(c, rc)


def test_round_one_paths_agree(spc):
    # validated input takes the dedicated round-1 kernel, unvalidated input
    # the round kernel: same labels, same per-round counters
    for g in (inputs.rmat(12, 8, seed=2), inputs.chung_lu(1 << 12, seed=5), inputs.grid_lcc(24, 0.05, seed=3)):
        a = spc.build_graph(g, opts=spc.BuildOptions(validate=True))
        b = spc.build_graph(g, opts=spc.BuildOptions(validate=False))
        ea, eb = a.export(), b.export()
        for k in ("off", "hub", "dist", "count", "order"):
            assert np.array_equal(ea[k], eb[k]), (g.name, k)
        ra, rb = a.round_stats(), b.round_stats()
        for k in ("raw", "merged", "kept"):
            assert np.array_equal(ra[k], rb[k]), (g.name, k)
        assert assert_labels_equal(ea, oracle.build_graph(g), g.name) is None
