"""Helpers of the GPU parity tests: compare a built index with the CPU
oracle (labels entry for entry; query answers pair for pair)."""
from __future__ import annotations

import numpy as np

import oracle


def dist_as_u32(d: np.ndarray, bits: int) -> np.ndarray:
    """GPU distances (uint8 / uint16) with INF mapped to the oracle's INF."""
    d = d.astype(np.uint32)
    d[d == ((1 << bits) - 1)] = oracle.INF
    return d


def assert_labels_equal(ex: dict, ref: "oracle.Labels", what: str = ""):
    assert np.array_equal(ex["order"], ref.order), f"{what}: vertex order differs"
    assert np.array_equal(ex["off"], ref.off), f"{what}: label sizes differ"
    assert np.array_equal(ex["hub"], ref.hub), f"{what}: hubs differ"
    assert np.array_equal(ex["dist"].astype(np.uint32), ref.dist), f"{what}: distances differ"
    assert np.array_equal(ex["count"], ref.count), f"{what}: counts differ"


def gpu_query(ix, s, t, graph_id=0):
    import torch
    from paper_2212_00977_amd import spc

    d, c, f = ix.query(s, t, graph_id=graph_id)
    torch.cuda.synchronize()
    bits = ix.dist_bits
    return (dist_as_u32(spc.as_dist(d), bits), spc.as_u64(c), f.cpu().numpy())


def all_pairs(n):
    s, t = np.meshgrid(np.arange(n, dtype=np.uint32), np.arange(n, dtype=np.uint32),
                       indexing="ij")
    return s.ravel(), t.ravel()


def check_invariants_device(ex: dict, m: int, n: int):
    """Properties of any label index, on a device export: one distance-1
    entry per edge, the self entry (v, 0, 1) closing every label, hubs
    strictly increasing and never ranked below the owner.  Returns the
    distance histogram (numpy)."""
    import torch

    off, hub, dist, cnt = ex["off"], ex["hub"].long(), ex["dist"].long(), ex["count"]
    if n == 0:
        return np.zeros(1, dtype=np.int64)
    deg = off[1:] - off[:-1]
    assert bool((deg >= 1).all()), "a label without its self entry"
    rows = torch.repeat_interleave(torch.arange(n, device=off.device), deg)
    assert int((dist == 1).sum()) == m
    last = off[1:] - 1
    assert torch.equal(hub[last], torch.arange(n, device=off.device))
    assert int(dist[last].abs().sum()) == 0
    assert bool((cnt[last] == 1).all())
    assert bool((hub <= rows).all())
    same = rows[1:] == rows[:-1]
    assert bool((hub[1:][same] > hub[:-1][same]).all())
    return torch.bincount(dist).cpu().numpy()


def check_hub_column_device(ex: dict, roff, radj, w: int, depth_cap: int = 0):
    """Every entry with hub w equals the oracle's column from the
    trough-path definition (vertex, distance, count)."""
    import torch

    v, d, c = oracle.hub_column(roff, radj, int(w), depth_cap=depth_cap)
    off, hub = ex["off"], ex["hub"]
    idx = torch.nonzero(hub == int(w)).flatten()
    rows = torch.searchsorted(off[1:], idx, right=True)
    assert np.array_equal(rows.cpu().numpy().astype(np.uint32), v), w
    assert np.array_equal(ex["dist"][idx].cpu().numpy().astype(np.uint32), d), w
    assert np.array_equal(ex["count"][idx].cpu().numpy().view(np.uint64), c), w


def check_source_answers(ix, g, src: int, targets, graph_id: int = 0):
    """Answers (src, t) for the given targets against BFS path counting."""
    t = np.asarray(targets, dtype=np.uint32)
    s = np.full(t.shape[0], src, dtype=np.uint32)
    d, c, f = gpu_query(ix, s, t, graph_id=graph_id)
    bd, bc = oracle.bfs_count(g.off, g.adj, src)
    assert np.array_equal(d, bd[t]) and np.array_equal(c, bc[t]), (g.name, src)
