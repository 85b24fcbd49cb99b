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
