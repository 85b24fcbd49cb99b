"""Seeded synthetic inputs for the SPC label build and query.

This module only draws graphs, vertex tie keys and query pairs.  It holds no
part of the labelling method: no ordering, no BFS, no label arithmetic.  Both
the CPU oracle and the HIP path consume exactly what it returns.

Every generator returns a simple undirected graph as a symmetric CSR
(``off`` uint64[n+1], ``adj`` uint32[2m], each adjacency list sorted by id,
no self loops, no duplicate edges), which is the graph model of the paper's
Preliminaries section (unweighted, undirected).  The paper's datasets are
public SNAP/KONECT/LAW graphs that are not available here; these seeded
generators stand in for them with the shapes the workloads name.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

GEN_VERSION = 1


@dataclass
class Graph:
    n: int
    off: np.ndarray            # uint64[n+1]
    adj: np.ndarray            # uint32[2m]
    name: str = ""
    order: Optional[np.ndarray] = None     # explicit rank -> vertex order (uint32[n]) or None
    tie_key: Optional[np.ndarray] = None   # uint64[n] random tie keys or None
    meta: dict = field(default_factory=dict)
    directed: bool = False  # off/adj hold each arc once, in its tail's row

    @property
    def m(self) -> int:
        """Undirected edges, or arcs of a directed graph."""
        return int(self.adj.shape[0]) if self.directed else int(self.adj.shape[0]) // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.off).astype(np.int64)

    def edges(self) -> np.ndarray:
        """Undirected edges (u < v) as an int64 [m, 2] array."""
        deg = self.degrees()
        src = np.repeat(np.arange(self.n, dtype=np.int64), deg)
        dst = self.adj.astype(np.int64)
        keep = src < dst
        return np.stack([src[keep], dst[keep]], axis=1)


def csr_from_edges(n: int, e: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Symmetric CSR from an undirected edge array; drops loops and duplicates."""
    e = np.asarray(e, dtype=np.int64).reshape(-1, 2)
    if e.size:
        a = np.minimum(e[:, 0], e[:, 1])
        b = np.maximum(e[:, 0], e[:, 1])
        keep = a != b
        a, b = a[keep], b[keep]
        key = np.unique(a * np.int64(n) + b)
        a, b = key // n, key % n
    else:
        a = b = np.zeros(0, dtype=np.int64)
    # both directions, ordered by (source, target): one sort of the packed
    # pair (n * n < 2^63 for every n < 2^31)
    both = np.concatenate([a * np.int64(n) + b, b * np.int64(n) + a])
    both.sort()
    src, dst = (both // n, both % n) if both.size else (both, both)
    counts = np.bincount(src, minlength=n).astype(np.uint64)
    off = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(counts, out=off[1:])
    return off, dst.astype(np.uint32)


def from_edges(n: int, e, name: str = "", order=None, tie_key=None, **meta) -> Graph:
    off, adj = csr_from_edges(n, np.asarray(e, dtype=np.int64).reshape(-1, 2))
    return Graph(n, off, adj, name=name,
                 order=None if order is None else np.asarray(order, dtype=np.uint32),
                 tie_key=None if tie_key is None else np.asarray(tie_key, dtype=np.uint64),
                 meta=dict(meta))


# --------------------------------------------------------------------------
# Worked example of the paper (Fig. 2 graph, order and Table 2 labels).
# Vertex v_k is id k-1.  The 13 edges are exactly the distance-1 entries of
# Table 2: each edge appears once as (higher-ranked endpoint, 1, 1) in the
# label of its lower-ranked endpoint.
# --------------------------------------------------------------------------
WORKED_EDGES_1BASED = [(1, 3), (1, 4), (1, 5), (1, 10), (2, 4), (2, 10), (3, 6),
                       (4, 7), (5, 7), (6, 7), (7, 8), (8, 9), (9, 10)]
# Fig. 2 caption: v1 <= v7 <= v4 <= v10 <= v3 <= v5 <= v6 <= v2 <= v8 <= v9.
WORKED_ORDER_1BASED = [1, 7, 4, 10, 3, 5, 6, 2, 8, 9]


def worked_example() -> Graph:
    e = np.array(WORKED_EDGES_1BASED, dtype=np.int64) - 1
    order = np.array(WORKED_ORDER_1BASED, dtype=np.uint32) - 1
    return from_edges(10, e, name="worked_example", order=order)


# --------------------------------------------------------------------------
# Random families
# --------------------------------------------------------------------------
def _distinct_pairs_until(n: int, m: int, draw, rng, batch: int) -> np.ndarray:
    """Draw endpoint pairs with ``draw(rng, k)`` until exactly m distinct
    non-loop undirected pairs exist; keeps the first m in draw order."""
    keys = np.zeros(0, dtype=np.int64)
    first = np.zeros(0, dtype=np.int64)
    drawn = 0
    while True:
        a, b = draw(rng, batch)
        a = a.astype(np.int64)
        b = b.astype(np.int64)
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        ok = lo != hi
        k = lo[ok] * np.int64(n) + hi[ok]
        pos = np.nonzero(ok)[0].astype(np.int64) + drawn
        drawn += batch
        keys = np.concatenate([keys, k])
        first = np.concatenate([first, pos])
        uk, idx = np.unique(keys, return_index=True)
        keys, first = uk, first[idx]
        if keys.shape[0] >= m:
            sel = np.argsort(first, kind="stable")[:m]
            k = keys[sel]
            return np.stack([k // n, k % n], axis=1)


def erdos_renyi(n: int, m: int, seed: int) -> Graph:
    """G(n, m): exactly m distinct non-loop pairs, uniform."""
    rng = np.random.default_rng(seed)

    def draw(r, k):
        return r.integers(0, n, size=k), r.integers(0, n, size=k)

    e = _distinct_pairs_until(n, m, draw, rng, batch=max(1024, 2 * m))
    return from_edges(n, e, name=f"er_n{n}_m{m}_s{seed}", seed=seed)


def chung_lu(n: int, seed: int, exponent: float = 2.1, wmin: float = 2.0,
             wmax: float = 20000.0, mean_degree: float = 10.0) -> Graph:
    """Chung-Lu graph with truncated power-law expected degrees.

    Weights are i.i.d. from pdf ~ x^-exponent on [wmin, wmax] (inverse CDF).
    Endpoints are sampled independently in proportion to the weights until
    exactly n*mean_degree/2 distinct non-loop edges exist, so the realised
    mean degree is exactly ``mean_degree``.  Rescaling the weights to a
    target mean does not change proportional sampling, so none is applied.
    """
    rng = np.random.default_rng(seed)
    g1 = 1.0 - exponent
    u = rng.random(n)
    w = (wmin ** g1 + u * (wmax ** g1 - wmin ** g1)) ** (1.0 / g1)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    m = int(round(n * mean_degree / 2))

    def draw(r, k):
        a = np.searchsorted(cdf, r.random(k), side="right")
        b = np.searchsorted(cdf, r.random(k), side="right")
        return np.minimum(a, n - 1), np.minimum(b, n - 1)

    e = _distinct_pairs_until(n, m, draw, rng, batch=max(4096, int(1.3 * m)))
    return from_edges(n, e, name=f"chunglu_n{n}_s{seed}", seed=seed)


def rmat(scale: int, edge_factor: int, seed, a=0.57, b=0.19, c=0.19) -> Graph:
    """R-MAT: edge_factor * 2^scale sampled edges, no noise; symmetrised,
    deduplicated, loops dropped; all 2^scale vertices kept."""
    n = 1 << scale
    src, dst = _rmat_pairs(scale, edge_factor, seed, a, b, c)
    return from_edges(n, np.stack([src, dst], axis=1),
                      name=f"rmat_s{scale}_ef{edge_factor}", scale=scale)


def rmat_digraph(scale: int, edge_factor: int, seed, a=0.57, b=0.19, c=0.19) -> Graph:
    """The R-MAT draws of rmat() kept as arcs (source -> target):
    deduplicated, loops dropped, all 2^scale vertices kept."""
    n = 1 << scale
    src, dst = _rmat_pairs(scale, edge_factor, seed, a, b, c)
    return digraph_from_arcs(n, np.stack([src, dst], axis=1), name=f"rmat_dir_s{scale}_ef{edge_factor}")


def digraph_from_arcs(n: int, arcs, name: str = "") -> Graph:
    """Directed graph: each distinct non-loop arc (a, b) once, in row a,
    rows sorted by head."""
    e = np.asarray(arcs, dtype=np.int64).reshape(-1, 2)
    e = e[e[:, 0] != e[:, 1]]
    key = np.unique(e[:, 0] * np.int64(n) + e[:, 1]) if e.size else np.zeros(0, dtype=np.int64)
    src, dst = (key // n, key % n) if key.size else (key, key)
    off = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(np.bincount(src, minlength=n).astype(np.uint64), out=off[1:])
    return Graph(n, off, dst.astype(np.uint32), name=name, directed=True)


def random_digraph(n: int, m: int, seed: int) -> Graph:
    """m arcs drawn uniformly (with repeats, then deduplicated, loops dropped)."""
    rng = np.random.default_rng(seed)
    arcs = rng.integers(0, n, size=(m, 2)) if n else np.zeros((0, 2), dtype=np.int64)
    return digraph_from_arcs(n, arcs, name=f"digraph_n{n}_m{m}_s{seed}")


def _rmat_pairs(scale: int, edge_factor: int, seed, a=0.57, b=0.19, c=0.19):
    """The R-MAT draws: (source, target) of edge_factor * 2^scale samples.

    Edge i takes, at recursion level L, the uniform number at position
    L * k + i of the stream of ``default_rng(seed)`` (k sampled edges): the
    levels are drawn one after another, each as one block of k numbers.
    Large graphs draw their blocks in parallel, each worker jumping the
    PCG64 stream to its slice (one 64-bit output per double), so the graph
    is the same as with one sequential stream."""
    n = 1 << scale
    k = edge_factor * n
    src = np.zeros(k, dtype=np.int64)
    dst = np.zeros(k, dtype=np.int64)

    def fill(i0, i1, rng_at):
        s, d = src[i0:i1], dst[i0:i1]
        for level in range(scale):
            r = rng_at(level * k + i0).random(i1 - i0)
            bit = np.int64(1) << np.int64(scale - 1 - level)
            down = r >= a + b
            right = ((r >= a) & (r < a + b)) | (r >= a + b + c)
            np.add(s, bit, out=s, where=down)
            np.add(d, bit, out=d, where=right)

    base = np.random.default_rng(seed).bit_generator
    if k < (1 << 20):
        rng = np.random.Generator(base)
        fill(0, k, lambda pos: rng)  # sequential: the stream is at pos already
    else:
        from concurrent.futures import ThreadPoolExecutor

        state = base.state

        def rng_at(pos):
            bg = np.random.PCG64()
            bg.state = state
            bg.advance(pos)
            return np.random.Generator(bg)

        workers = max(1, min(16, os.cpu_count() or 1))
        chunk = -(-k // (4 * workers))
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(lambda i0: fill(i0, min(k, i0 + chunk), rng_at), range(0, k, chunk)))
    return src, dst


def grid_lcc(k: int, delete_frac: float, seed: int) -> Graph:
    """k x k 4-neighbour grid, delete round(delete_frac * |E|) edges chosen
    uniformly without replacement, keep the largest connected component
    (ids renumbered in increasing original id).  Tie keys for a random
    tie-break are drawn from the same stream."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    rng = np.random.default_rng(seed)
    ids = np.arange(k * k, dtype=np.int64).reshape(k, k)
    horiz = np.stack([ids[:, :-1].ravel(), ids[:, 1:].ravel()], axis=1)
    vert = np.stack([ids[:-1, :].ravel(), ids[1:, :].ravel()], axis=1)
    e = np.concatenate([horiz, vert])
    ndel = int(round(delete_frac * e.shape[0]))
    if ndel:
        drop = rng.choice(e.shape[0], size=ndel, replace=False)
        keep = np.ones(e.shape[0], dtype=bool)
        keep[drop] = False
        e = e[keep]
    nn = k * k
    mat = coo_matrix((np.ones(e.shape[0]), (e[:, 0], e[:, 1])), shape=(nn, nn))
    ncomp, lab = connected_components(mat, directed=False)
    big = np.argmax(np.bincount(lab))
    keepv = lab == big
    newid = -np.ones(nn, dtype=np.int64)
    newid[keepv] = np.arange(int(keepv.sum()))
    e = e[keepv[e[:, 0]] & keepv[e[:, 1]]]
    e = newid[e]
    n = int(keepv.sum())
    tie = rng.integers(0, np.iinfo(np.int64).max, size=n, dtype=np.int64).astype(np.uint64)
    return from_edges(n, e, name=f"grid{k}_del{delete_frac}_s{seed}", tie_key=tie,
                      k=k, deleted=ndel)


def rmat_batch(count: int, seed: int, scale_lo: int = 10, scale_hi: int = 16,
               edge_factor: int = 8) -> list[Graph]:
    """Independent R-MAT graphs with scales uniform in [scale_lo, scale_hi];
    graph i uses the seed sequence (seed, i)."""
    rng = np.random.default_rng(seed)
    scales = rng.integers(scale_lo, scale_hi + 1, size=count)
    out = []
    for i, s in enumerate(scales):
        g = rmat(int(s), edge_factor, np.random.SeedSequence([seed, i]))
        g.name = f"rmat_batch{seed}_{i}_s{int(s)}"
        out.append(g)
    return out


def random_tiny(n: int, p: float, seed: int) -> Graph:
    """Small G(n, p) graph for exhaustive checks."""
    rng = np.random.default_rng(seed)
    iu = np.triu_indices(n, 1)
    keep = rng.random(iu[0].shape[0]) < p
    e = np.stack([iu[0][keep], iu[1][keep]], axis=1)
    return from_edges(n, e, name=f"tiny_n{n}_p{p}_s{seed}")


def queries(n: int, q: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Uniform (s, t) pairs with replacement (s = t allowed)."""
    rng = np.random.default_rng(seed * 1000 + 1)
    s = rng.integers(0, n, size=q, dtype=np.int64).astype(np.uint32)
    t = rng.integers(0, n, size=q, dtype=np.int64).astype(np.uint32)
    return s, t


def poisson_requests(n_vertices: int, rate_per_s: float, count: int, seed: int,
                     max_batch: int = 65536, graph_id: int = 0) -> list:
    """Open-loop Poisson arrivals; batch sizes log-uniform in [1, max_batch];
    uniform (s, t) pairs.  Returns (id, s, t, arrival_s, graph_id) tuples."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    sizes = np.floor(np.exp(rng.uniform(0.0, np.log(max_batch + 1), size=count))).astype(np.int64)
    sizes = np.clip(sizes, 1, max_batch)
    reqs = []
    for i in range(count):
        s = rng.integers(0, n_vertices, size=sizes[i], dtype=np.int64).astype(np.uint32)
        t = rng.integers(0, n_vertices, size=sizes[i], dtype=np.int64).astype(np.uint32)
        reqs.append((i, s, t, float(arrivals[i]), graph_id))
    return reqs


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------
def workload(name: str, scale_down: int = 0) -> Graph:
    """Named workloads; ``scale_down`` shrinks the vertex count by 2^k with
    the same generator (for smaller same-family parity instances)."""
    if name == "er2000":
        return erdos_renyi(2000, 8000, seed=1)
    if name == "chunglu":
        n = 1 << (20 - scale_down)
        return chung_lu(n, seed=2)
    if name == "grid":
        k = 2048 >> scale_down
        return grid_lcc(k, 0.05, seed=3)
    if name == "rmat21":
        return rmat(21 - scale_down, 16, seed=5)
    raise KeyError(name)
