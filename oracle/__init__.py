"""CPU oracle for the SPC 2-hop label index (ctypes wrapper over spc_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product path never imports it.  It shares no
code with the GPU library.  Results are numpy arrays.

All builders take a graph in original ids plus an order (rank -> vertex),
relabel it into rank space (vertex id == rank, 0 = most important) and
return labels in rank space, sorted by hub within each vertex, together with
the order.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
INF = 0xFFFFFFFF
SAT = 0xFFFFFFFFFFFFFFFF

_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def build_oracle(force: bool = True) -> str:
    """Compile liboracle.so in-tree with gcc."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-Wall", "-Wextra",
               "-shared", "-fPIC", "-pthread", "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build_oracle()
    L = C.CDLL(_LIB)
    vp = C.c_void_p
    L.oracle_degree_order.argtypes = [C.c_uint32, _u64p, vp, _u32p]
    L.oracle_degree_order.restype = None
    L.oracle_relabel.argtypes = [C.c_uint32, _u64p, _u32p, _u32p, _u64p, _u32p]
    L.oracle_relabel.restype = None
    L.oracle_bfs_count.argtypes = [C.c_uint32, _u64p, _u32p, C.c_uint32, C.c_int, C.c_uint32,
                                   _u32p, _u64p]
    L.oracle_bfs_count.restype = None
    L.oracle_hub_column.argtypes = [C.c_uint32, _u64p, _u32p, C.c_uint32, C.c_uint32,
                                    _u32p, _u32p, _u64p]
    L.oracle_hub_column.restype = C.c_uint64
    for nm in ("oracle_build_definition", "oracle_build_pull"):
        f = getattr(L, nm)
        f.argtypes = [C.c_uint32, _u64p, _u32p, C.c_uint32]
        f.restype = vp
    L.oracle_build_pull_threads.argtypes = [C.c_uint32, _u64p, _u32p, C.c_uint32, C.c_uint32]
    L.oracle_build_pull_threads.restype = vp
    L.oracle_set_progress.argtypes = [C.c_int]
    L.oracle_set_progress.restype = None
    L.oracle_index_model_stats.argtypes = [vp, _u64p, _u64p, _u64p]
    L.oracle_index_model_stats.restype = None
    L.oracle_query_arrays_threads.argtypes = [_u64p, _u32p, _u32p, _u64p, C.c_uint64, _u32p,
                                              _u32p, _u32p, _u64p, C.c_uint32]
    L.oracle_query_arrays_threads.restype = None
    L.oracle_build_directed_definition.argtypes = [C.c_uint32, _u64p, _u32p, _u64p, _u32p]
    L.oracle_build_directed_definition.restype = vp
    L.oracle_label_hubs.argtypes = [C.c_uint32, _u64p, _u32p, C.c_uint32, _u32p, _u32p]
    L.oracle_label_hubs.restype = C.c_uint64
    L.oracle_build_definition_weighted.argtypes = [C.c_uint32, _u64p, _u32p, _u64p, C.c_uint32]
    L.oracle_build_definition_weighted.restype = vp
    L.oracle_build_pruned.argtypes = [C.c_uint32, _u64p, _u32p, C.c_uint32, C.c_uint32,
                                      C.c_double]
    L.oracle_build_pruned.restype = vp
    L.oracle_index_entries.argtypes = [vp]
    L.oracle_index_entries.restype = C.c_uint64
    L.oracle_index_rounds.argtypes = [vp]
    L.oracle_index_rounds.restype = C.c_uint32
    L.oracle_index_hubs_done.argtypes = [vp]
    L.oracle_index_hubs_done.restype = C.c_uint32
    L.oracle_index_export.argtypes = [vp, _u64p, _u32p, _u32p, _u64p]
    L.oracle_index_export.restype = None
    L.oracle_index_round_stats.argtypes = [vp, _u64p, _u64p, _u64p, _u64p]
    L.oracle_index_round_stats.restype = None
    L.oracle_index_free.argtypes = [vp]
    L.oracle_index_free.restype = None
    L.oracle_query_arrays.argtypes = [_u64p, _u32p, _u32p, _u64p, C.c_uint64, _u32p, _u32p,
                                      _u32p, _u64p]
    L.oracle_query_arrays.restype = None
    _lib = L
    return L


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def degree_order(off, tie_key=None) -> np.ndarray:
    """Rank -> vertex: degree descending, ties by tie_key then id."""
    off = _u64(off)
    n = off.shape[0] - 1
    order = np.zeros(n, dtype=np.uint32)
    tk = None if tie_key is None else _u64(tie_key)
    lib().oracle_degree_order(n, off, None if tk is None else tk.ctypes.data, order)
    return order


def relabel(off, adj, order):
    off, adj, order = _u64(off), _u32(adj), _u32(order)
    n = off.shape[0] - 1
    roff = np.zeros(n + 1, dtype=np.uint64)
    radj = np.zeros(adj.shape[0], dtype=np.uint32)
    lib().oracle_relabel(n, off, adj, order, roff, radj)
    return roff, radj


def bfs_count(off, adj, src: int, restricted: bool = False, depth_cap: int = 0):
    """Distances (uint32, INF unreached) and saturated path counts (uint64)."""
    off, adj = _u64(off), _u32(adj)
    n = off.shape[0] - 1
    d = np.zeros(n, dtype=np.uint32)
    s = np.zeros(n, dtype=np.uint64)
    lib().oracle_bfs_count(n, off, adj, int(src), int(restricted), int(depth_cap), d, s)
    return d, s


def hub_column(roff, radj, w: int, depth_cap: int = 0):
    """(vertex, dist, count) of every entry with hub w (rank space)."""
    roff, radj = _u64(roff), _u32(radj)
    n = roff.shape[0] - 1
    v = np.zeros(n, dtype=np.uint32)
    d = np.zeros(n, dtype=np.uint32)
    c = np.zeros(n, dtype=np.uint64)
    k = lib().oracle_hub_column(n, roff, radj, int(w), int(depth_cap), v, d, c)
    return v[:k].copy(), d[:k].copy(), c[:k].copy()


@dataclass
class Labels:
    """Labels in rank space: entries of vertex r at off[r]:off[r+1], by hub."""
    n: int
    off: np.ndarray
    hub: np.ndarray
    dist: np.ndarray
    count: np.ndarray
    order: np.ndarray        # rank -> original vertex
    rounds: int
    hubs_done: int
    stats: dict | None = None

    @property
    def entries(self) -> int:
        return int(self.off[-1])

    def rank_of(self) -> np.ndarray:
        r = np.zeros(self.n, dtype=np.uint32)
        r[self.order] = np.arange(self.n, dtype=np.uint32)
        return r

    def query(self, s, t):
        """SPC query with ORIGINAL vertex ids; returns (dist uint32, count uint64)."""
        rk = self.rank_of()
        s = _u32(rk[_u32(s)])
        t = _u32(rk[_u32(t)])
        return query_arrays(self.off, self.hub, self.dist, self.count, s, t)


def query_arrays(off, hub, dist, count, s, t, threads: int = 1):
    """Query over label arrays (ids in the labels' own space); `threads`
    splits the batch over that many host threads."""
    s, t = _u32(s), _u32(t)
    q = s.shape[0]
    od = np.zeros(q, dtype=np.uint32)
    oc = np.zeros(q, dtype=np.uint64)
    lib().oracle_query_arrays_threads(_u64(off), _u32(hub), _u32(dist), _u64(count), q, s, t,
                                      od, oc, max(1, int(threads)))
    return od, oc


def label_hubs(roff, radj, s: int):
    """Hubs of L(s) and their distances from the definition, without counts
    (rank-space graph): (hub uint32[], dist uint32[]) in hub order."""
    roff, radj = _u64(roff), _u32(radj)
    n = roff.shape[0] - 1
    h = np.zeros(max(n, 1), dtype=np.uint32)
    d = np.zeros(max(n, 1), dtype=np.uint32)
    k = lib().oracle_label_hubs(n, roff, radj, int(s), h, d)
    return h[:k].copy(), d[:k].copy()


def host_threads() -> int:
    """Threads the host offers this process (its CPU affinity)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _collect(h, n, order, with_stats: bool) -> Labels:
    L = lib()
    try:
        e = L.oracle_index_entries(h)
        off = np.zeros(n + 1, dtype=np.uint64)
        hub = np.zeros(e, dtype=np.uint32)
        dist = np.zeros(e, dtype=np.uint32)
        cnt = np.zeros(e, dtype=np.uint64)
        L.oracle_index_export(h, off, hub, dist, cnt)
        rounds = L.oracle_index_rounds(h)
        stats = None
        if with_stats:
            k = rounds + 1
            raw, mer, kept, scan, act, act_adj, staged = (np.zeros(k, dtype=np.uint64)
                                                          for _ in range(7))
            L.oracle_index_round_stats(h, raw, mer, kept, scan)
            L.oracle_index_model_stats(h, act, act_adj, staged)
            stats = dict(raw=raw, merged=mer, kept=kept, scanned=scan, active=act,
                         active_adj=act_adj, staged=staged)
        return Labels(n, off, hub, dist, cnt, order, int(rounds), int(L.oracle_index_hubs_done(h)),
                      stats)
    finally:
        L.oracle_index_free(h)


def _prep(off, adj, order, tie_key):
    off, adj = _u64(off), _u32(adj)
    if order is None:
        order = degree_order(off, tie_key)
    order = _u32(order)
    roff, radj = relabel(off, adj, order)
    return off.shape[0] - 1, roff, radj, order


def build(off, adj, order=None, tie_key=None, method: str = "pruned", depth_cap: int = 0,
          max_hubs: int = 0, time_limit_s: float = 0.0, threads: int = 1) -> Labels:
    """Build the label index; method in {"definition", "pruned", "pull"};
    `threads` spreads each PULL round's pullers over that many host
    threads (same result)."""
    n, roff, radj, order = _prep(off, adj, order, tie_key)
    L = lib()
    if method == "definition":
        h = L.oracle_build_definition(n, roff, radj, depth_cap)
    elif method == "pruned":
        h = L.oracle_build_pruned(n, roff, radj, depth_cap, max_hubs, time_limit_s)
    elif method == "pull":
        h = L.oracle_build_pull_threads(n, roff, radj, depth_cap, max(1, int(threads)))
    else:
        raise ValueError(method)
    return _collect(h, n, order, with_stats=(method == "pull"))


def pull_stats(off, adj, order=None, tie_key=None, depth_cap: int = 0, threads: int = 1) -> dict:
    """The threaded PULL build's per-round counters, entry count and rounds,
    without exporting the labels (for graphs whose index is too large to
    copy out once more)."""
    n, roff, radj, order = _prep(off, adj, order, tie_key)
    L = lib()
    h = L.oracle_build_pull_threads(n, roff, radj, depth_cap, max(1, int(threads)))
    try:
        rounds = int(L.oracle_index_rounds(h))
        k = rounds + 1
        raw, mer, kept, scan, act, act_adj, staged = (np.zeros(k, dtype=np.uint64)
                                                      for _ in range(7))
        L.oracle_index_round_stats(h, raw, mer, kept, scan)
        L.oracle_index_model_stats(h, act, act_adj, staged)
        return dict(n=n, entries=int(L.oracle_index_entries(h)), rounds=rounds, raw=raw,
                    merged=mer, kept=kept, scanned=scan, active=act, active_adj=act_adj,
                    staged=staged)
    finally:
        L.oracle_index_free(h)


def build_graph(g, method: str = "pruned", depth_cap: int = 0, **kw) -> Labels:
    """Build for an inputs.Graph (uses its explicit order or tie keys)."""
    return build(g.off, g.adj, order=g.order, tie_key=g.tie_key, method=method,
                 depth_cap=depth_cap, **kw)


def hybrid_order(off, adj, delta: int):
    """Hybrid vertex order (the paper's "Vertex Ordering Strategies": the
    road-network order from tree decomposition for the fringe, the degree
    order for the core), written out with Python sets.  Returns
    (order rank -> vertex, core size).

    Fringe: remove a vertex of least current degree (ties: smaller id) while
    that degree is <= delta, connecting its remaining neighbours pairwise;
    degrees are those of this elimination graph (the paper's update
    deg(u) + deg(u_0) - 1 counts shared neighbours twice; the elimination
    graph is what the tree decomposition it cites is built from).  Core: the
    rest, by input degree descending, ties by id, ranked first; then the
    fringe in reverse order of removal.  Small graphs only."""
    import heapq

    off, adj = _u64(off), _u32(adj)
    n = off.shape[0] - 1
    nbr = [set(int(w) for w in adj[off[v]:off[v + 1]] if int(w) != v) for v in range(n)]
    deg0 = [len(s) for s in nbr]
    removed = [False] * n
    heap = [(len(nbr[v]), v) for v in range(n) if len(nbr[v]) <= delta]
    heapq.heapify(heap)
    elim = []
    while heap:
        dg, v = heapq.heappop(heap)
        if removed[v] or dg != len(nbr[v]):
            continue
        removed[v] = True
        elim.append(v)
        ns = sorted(nbr[v])
        nbr[v] = set()
        for a in ns:
            nbr[a].discard(v)
        for i, a in enumerate(ns):
            for b in ns[i + 1:]:
                nbr[a].add(b)
                nbr[b].add(a)
        for a in ns:
            if len(nbr[a]) <= delta:
                heapq.heappush(heap, (len(nbr[a]), a))
    core = sorted((v for v in range(n) if not removed[v]), key=lambda v: (-deg0[v], v))
    order = np.array(core + elim[::-1], dtype=np.uint32)
    return order, len(core)


@dataclass
class Shell:
    """1-shell of a graph (per vertex, original ids)."""
    core: np.ndarray    # bool: vertex keeps a label
    root: np.ndarray    # shr(v): the core vertex v's tree hangs from (v itself in the core)
    depth: np.ndarray   # distance from v to root[v]
    parent: np.ndarray  # neighbour of v on the path to root[v] (v itself in the core)


def one_shell(off, adj) -> Shell:
    """The 1-shell of the paper's Section "Reduction by 1-Shell", written
    from its definitions with Python sets (small graphs only).

    The core is the 2-core: the largest subgraph in which every vertex has
    at least two neighbours, obtained by deleting vertices of degree below
    two until none is left.  Every other vertex is in the fringe, which is a
    forest; each of its trees is joined to the core by one edge, whose core
    end is the root shr(v) of the tree's vertices.  A component with an empty
    2-core is a tree: its centre (least eccentricity, the smaller id of two
    centres) stays in the core as the root of the rest.  depth and parent
    follow a breadth-first search from the roots through fringe vertices."""
    from collections import deque

    off, adj = _u64(off), _u32(adj)
    n = off.shape[0] - 1
    nbr = [sorted(set(int(w) for w in adj[off[v]:off[v + 1]] if int(w) != v)) for v in range(n)]
    deg = [len(x) for x in nbr]
    core = [True] * n
    stack = [v for v in range(n) if deg[v] < 2]
    while stack:
        v = stack.pop()
        if not core[v]:
            continue
        core[v] = False
        for w in nbr[v]:
            if core[w]:
                deg[w] -= 1
                if deg[w] < 2:
                    stack.append(w)

    def bfs(src):
        dist = {src: 0}
        q = deque([src])
        while q:
            v = q.popleft()
            for w in nbr[v]:
                if w not in dist:
                    dist[w] = dist[v] + 1
                    q.append(w)
        return dist

    seen = [False] * n
    for v in range(n):
        if seen[v]:
            continue
        comp = list(bfs(v))
        for x in comp:
            seen[x] = True
        if not any(core[x] for x in comp):
            ecc = {x: max(bfs(x).values()) for x in comp}
            centre = min(comp, key=lambda x: (ecc[x], x))
            core[centre] = True
    root = np.arange(n, dtype=np.uint32)
    depth = np.zeros(n, dtype=np.uint32)
    parent = np.arange(n, dtype=np.uint32)
    q = deque(v for v in range(n) if core[v])
    done = list(core)
    while q:
        v = q.popleft()
        for w in nbr[v]:
            if not done[w]:
                done[w] = True
                root[w], depth[w], parent[w] = root[v], depth[v] + 1, v
                q.append(w)
    return Shell(np.array(core, dtype=bool), root, depth, parent)


@dataclass
class ReducedIndex:
    """Labels of the core only, plus the 1-shell that answers the rest."""
    shell: Shell
    core_ids: np.ndarray  # core id -> original vertex (ascending)
    cid: np.ndarray       # original vertex -> core id (core vertices only)
    labels: Labels        # index of the core subgraph, ORIGINAL core ids in .order

    def query(self, s, t):
        """Query rule of the 1-shell reduction: when root(s) = root(t) the
        tree path is the only shortest path; otherwise the core query
        between the roots, with both depths added to the distance."""
        sh = self.shell
        s, t = _u32(s), _u32(t)
        rs, rt = sh.root[s], sh.root[t]
        d, c = self.labels.query(self.cid[rs], self.cid[rt])
        d = d.astype(np.uint64)
        far = d != INF
        d[far] += sh.depth[s][far].astype(np.uint64) + sh.depth[t][far]
        d = np.where(far, d, INF).astype(np.uint32)
        for i in np.nonzero(rs == rt)[0]:
            x, y = int(s[i]), int(t[i])
            dx, dy = int(sh.depth[x]), int(sh.depth[y])
            tot = dx + dy
            while dx > dy:
                x, dx = int(sh.parent[x]), dx - 1
            while dy > dx:
                y, dy = int(sh.parent[y]), dy - 1
            while x != y:
                x, y, dx = int(sh.parent[x]), int(sh.parent[y]), dx - 1
            d[i], c[i] = tot - 2 * dx, 1
        return d, c


def core_subgraph(off, adj, core, order=None, tie_key=None):
    """CSR of the subgraph induced by the core (core ids ascending with the
    original ids), the order restricted to it, and its tie keys."""
    off, adj = _u64(off), _u32(adj)
    core = np.asarray(core, dtype=bool)
    n = off.shape[0] - 1
    ids = np.nonzero(core)[0].astype(np.uint32)
    cid = np.full(n, INF, dtype=np.uint32)
    cid[ids] = np.arange(ids.shape[0], dtype=np.uint32)
    rows = []
    for v in ids:
        nb = adj[off[v]:off[v + 1]]
        rows.append(cid[nb[core[nb]]])
    coff = np.zeros(ids.shape[0] + 1, dtype=np.uint64)
    coff[1:] = np.cumsum([r.shape[0] for r in rows]) if rows else []
    cadj = np.concatenate(rows).astype(np.uint32) if rows else np.zeros(0, dtype=np.uint32)
    cord = None if order is None else cid[_u32(order)[core[_u32(order)]]]
    ctie = None if tie_key is None else _u64(tie_key)[ids]
    return coff, cadj, ids, cid, cord, ctie


def build_reduced(off, adj, order=None, tie_key=None, depth_cap: int = 0) -> ReducedIndex:
    """1-shell reduction, then the label index of the core subgraph (its own
    degree order unless an order is given, which is then restricted to the
    core; depth_cap > 0 keeps the distance-partial core labels)."""
    sh = one_shell(off, adj)
    coff, cadj, ids, cid, cord, ctie = core_subgraph(off, adj, sh.core, order, tie_key)
    lab = build(coff, cadj, order=cord, tie_key=ctie, depth_cap=depth_cap)
    return ReducedIndex(sh, ids, cid, lab)


def twin_classes(off, adj) -> np.ndarray:
    """Classes of the neighbourhood-equivalence relation of the paper's
    Section "Reduction by Equivalence Relation": u ~ v when
    nbr(u) minus {v} equals nbr(v) minus {u}.  For two vertices that are not
    adjacent this says nbr(u) = nbr(v); for adjacent ones, nbr(u) + {u} =
    nbr(v) + {v}; vertices are grouped by those two sets.  Returns rep[v]:
    the smallest vertex of v's class."""
    off, adj = _u64(off), _u32(adj)
    n = off.shape[0] - 1
    nbr = [frozenset(int(w) for w in adj[off[v]:off[v + 1]] if int(w) != v) for v in range(n)]
    rep = np.arange(n, dtype=np.uint32)
    first_open, first_closed = {}, {}
    for v in range(n):
        o = nbr[v]
        c = o | {v}
        if o in first_open:
            rep[v] = first_open[o]
        elif c in first_closed:
            rep[v] = first_closed[c]
        else:
            first_open[o] = v
            first_closed[c] = v
    return rep


def weighted_labels(off, adj, weight, order=None, tie_key=None, depth_cap: int = 0) -> Labels:
    """Label index of a graph whose vertices carry weights, from the
    definition (Python big integers, small graphs only).  An entry (h, d, c)
    of L(v) exists when some shortest v-h path has every vertex other than
    h ranked below h (a trough path); c sums, over those paths, the product
    of the weights of the path's inner vertices (both ends excluded),
    saturated at 2^64-1.  With every weight 1 this is the plain index."""
    from collections import deque

    off, adj = _u64(off), _u32(adj)
    n = off.shape[0] - 1
    if order is None:
        order = degree_order(off, tie_key)
    order = _u32(order)
    rank = np.zeros(n, dtype=np.int64)
    rank[order] = np.arange(n)
    nbr = [[int(w) for w in adj[off[v]:off[v + 1]]] for v in range(n)]
    w = [int(x) for x in weight]
    lab = [[] for _ in range(n)]  # per rank: (hub rank, dist, count)
    for hr in range(n):
        h = int(order[hr])
        full = {h: 0}
        q = deque([h])
        while q:
            u = q.popleft()
            for x in nbr[u]:
                if x not in full:
                    full[x] = full[u] + 1
                    q.append(x)
        dist, sig = {h: 0}, {h: 1}
        q = deque([h])
        while q:
            u = q.popleft()
            if depth_cap and dist[u] >= depth_cap:
                continue
            f = 1 if u == h else w[u]
            for x in nbr[u]:
                if rank[x] <= hr:
                    continue
                if x not in dist:
                    dist[x] = dist[u] + 1
                    sig[x] = 0
                    q.append(x)
                if dist[x] == dist[u] + 1:
                    sig[x] += sig[u] * f
        for v, dv in dist.items():
            if dv == full[v]:
                lab[int(rank[v])].append((hr, dv, min(sig[v], SAT)))
    offs = np.zeros(n + 1, dtype=np.uint64)
    offs[1:] = np.cumsum([len(x) for x in lab])
    ent = [e for x in lab for e in sorted(x)]
    hub = np.array([e[0] for e in ent], dtype=np.uint32)
    dst = np.array([e[1] for e in ent], dtype=np.uint32)
    cnt = np.array([e[2] for e in ent], dtype=np.uint64)
    return Labels(n, offs, hub, dst, cnt, order, int(dst.max()) + 1 if ent else 0, n)


def build_weighted(off, adj, weight, order=None, tie_key=None, depth_cap: int = 0) -> Labels:
    """weighted_labels in C (the definition, one BFS pair per hub), for
    graphs of a few thousand vertices; weight is per vertex (input ids)."""
    n, roff, radj, order = _prep(off, adj, order, tie_key)
    wr = np.zeros(max(n, 1), dtype=np.uint64)
    wr[:n] = _u64(weight)[order]
    h = lib().oracle_build_definition_weighted(n, roff, radj, wr, depth_cap)
    return _collect(h, n, order, with_stats=False)


def weighted_query(lab: Labels, weight_by_rank, rs, rt):
    """Query over weighted labels (rank-space ids): least d_s + d_t over
    common hubs; the count sums c_s c_t, times the hub's weight when the hub
    is inside the path (not s or t itself)."""
    out_d, out_c = [], []
    for a, b in zip((int(x) for x in rs), (int(x) for x in rt)):
        la = {int(h): (int(d), int(c)) for h, d, c in zip(lab.hub[lab.off[a]:lab.off[a + 1]],
                                                         lab.dist[lab.off[a]:lab.off[a + 1]],
                                                         lab.count[lab.off[a]:lab.off[a + 1]])}
        best, tot = INF, 0
        for h, d, c in zip(lab.hub[lab.off[b]:lab.off[b + 1]], lab.dist[lab.off[b]:lab.off[b + 1]],
                           lab.count[lab.off[b]:lab.off[b + 1]]):
            h = int(h)
            if h not in la:
                continue
            dd = la[h][0] + int(d)
            f = 1 if h in (a, b) else int(weight_by_rank[h])
            x = la[h][1] * int(c) * f
            if dd < best:
                best, tot = dd, x
            elif dd == best:
                tot += x
        out_d.append(best)
        out_c.append(min(tot, SAT))
    return np.array(out_d, dtype=np.uint32), np.array(out_c, dtype=np.uint64)


@dataclass
class TwinIndex:
    """Equivalence-reduced index: one representative per class, weighted by
    the class size, and the weighted labels of the quotient graph."""
    rep: np.ndarray       # input vertex -> its class's representative (smallest id)
    cid: np.ndarray       # input vertex -> quotient id (representatives only)
    ids: np.ndarray       # quotient id -> input vertex
    weight: np.ndarray    # quotient id -> class size
    clique: np.ndarray    # input vertex: its class is a clique (adjacent twins)
    degree: np.ndarray    # input degree
    labels: Labels        # weighted labels of the quotient graph (quotient ids)

    def query(self, s, t):
        """Query rule: s = t gives (0, 1); two members of one class are
        adjacent (1, 1) or share every neighbour (2, degree); otherwise the
        weighted query between the representatives, which equals the
        input graph's answer because a shortest path meets each class at
        most once and any member of a class can stand for the one used."""
        s, t = _u32(s), _u32(t)
        rank = self.labels.rank_of()
        wr = np.zeros(self.weight.shape[0], dtype=np.uint64)
        wr[rank] = self.weight
        d, c = weighted_query(self.labels, wr, rank[self.cid[self.rep[s]]], rank[self.cid[self.rep[t]]])
        for i in range(s.shape[0]):
            a, b = int(s[i]), int(t[i])
            if a == b:
                d[i], c[i] = 0, 1
            elif self.rep[a] == self.rep[b]:
                if self.clique[a]:
                    d[i], c[i] = 1, 1
                elif self.degree[a] == 0:
                    d[i], c[i] = INF, 0
                else:
                    d[i], c[i] = 2, int(self.degree[a])
        return d, c


def build_twin_reduced(off, adj, order=None, tie_key=None, depth_cap: int = 0) -> TwinIndex:
    """Neighbourhood-equivalence reduction, then the weighted labels of the
    quotient graph (the subgraph induced by the representatives; its own
    degree order unless an order is given, which is then restricted)."""
    off, adj = _u64(off), _u32(adj)
    n = off.shape[0] - 1
    rep = twin_classes(off, adj)
    keep = rep == np.arange(n)
    coff, cadj, ids, cid, cord, ctie = core_subgraph(off, adj, keep, order, tie_key)
    size = np.bincount(rep, minlength=n)[ids].astype(np.uint64)
    adjset = [set(int(w) for w in adj[off[v]:off[v + 1]]) for v in range(n)]
    # members of a class of adjacent twins are pairwise adjacent
    clique = np.array([any(rep[u] == rep[v] for u in adjset[v]) for v in range(n)], dtype=bool)
    deg = np.diff(off).astype(np.uint64)
    build_fn = weighted_labels if ids.shape[0] <= 400 else build_weighted
    lab = build_fn(coff, cadj, size, order=cord, tie_key=ctie, depth_cap=depth_cap)
    return TwinIndex(rep, cid, ids, size, clique, deg, lab)


@dataclass
class DirectedLabels:
    """In- and out-labels of a directed graph, per vertex (ORIGINAL ids):
    out[v] = {w: (sd(v, w), count)}, inn[v] = {w: (sd(w, v), count)}."""
    order: np.ndarray
    out: list
    inn: list

    def query(self, s, t):
        """Eq. con:spc1 / con:spc2 on L_out(s) and L_in(t)."""
        d_out, c_out = [], []
        for a, b in zip((int(x) for x in s), (int(x) for x in t)):
            best, tot = INF, 0
            lo, li = self.out[a], self.inn[b]
            for h, (da, ca) in lo.items():
                if h in li:
                    dd = da + li[h][0]
                    if dd < best:
                        best, tot = dd, ca * li[h][1]
                    elif dd == best:
                        tot += ca * li[h][1]
            d_out.append(best)
            c_out.append(min(tot, SAT))
        return np.array(d_out, dtype=np.uint32), np.array(c_out, dtype=np.uint64)


def directed_labels(n: int, arcs, order=None) -> DirectedLabels:
    """The 2-hop SPC labels of a directed graph (Section "2-Hop Labeling for
    Shortest Path Counting": an in-label and an out-label per vertex), from
    the definition, Python big integers, small graphs only.  For a hub w and
    a vertex v ranked at or below w, L_out(v) holds (w, sd(v, w), c) when
    some shortest v-to-w path has every vertex but w ranked below w, c
    counting those paths; L_in(v) likewise for paths from w to v.  order
    (rank -> vertex) defaults to total degree (in + out) descending, ties by
    id -- the paper does not fix the directed order."""
    from collections import deque

    fwd = [[] for _ in range(n)]
    rev = [[] for _ in range(n)]
    for a, b in arcs:
        a, b = int(a), int(b)
        if a != b and b not in fwd[a]:
            fwd[a].append(b)
            rev[b].append(a)
    if order is None:
        order = sorted(range(n), key=lambda v: (-(len(fwd[v]) + len(rev[v])), v))
    order = np.asarray(order, dtype=np.uint32)
    rank = np.zeros(n, dtype=np.int64)
    rank[order] = np.arange(n)

    def bfs(src, nbr, below):
        dist, sig = {src: 0}, {src: 1}
        q = deque([src])
        while q:
            u = q.popleft()
            for x in nbr[u]:
                if below is not None and rank[x] <= below:
                    continue
                if x not in dist:
                    dist[x] = dist[u] + 1
                    sig[x] = 0
                    q.append(x)
                if dist[x] == dist[u] + 1:
                    sig[x] += sig[u]
        return dist, sig

    out = [dict() for _ in range(n)]
    inn = [dict() for _ in range(n)]
    for hr in range(n):
        w = int(order[hr])
        # paths v -> w walk the reversed arcs from w; paths w -> v the arcs
        for nbr, lab in ((rev, out), (fwd, inn)):
            full, _ = bfs(w, nbr, None)
            dist, sig = bfs(w, nbr, hr)
            for v, dv in dist.items():
                if dv == full[v]:
                    lab[v][w] = (dv, min(sig[v], SAT))
    return DirectedLabels(order, out, inn)


def directed_order(n: int, off, adj) -> np.ndarray:
    """Rank -> vertex of a digraph given by out-arcs (CSR): total degree
    (out + in) descending, ties by id (the paper fixes no directed order)."""
    off, adj = _u64(off), _u32(adj)
    deg = np.diff(off).astype(np.int64) + np.bincount(adj.astype(np.int64), minlength=n)[:n]
    return np.lexsort((np.arange(n), -deg)).astype(np.uint32)


def build_directed(n: int, off, adj, order=None) -> Labels:
    """Directed labels from the definition (C): a Labels of 2n rows in rank
    space, row r = L_out of rank r, row n + r = L_in of rank r; `order` is
    rank -> vertex (default directed_order)."""
    off, adj = _u64(off), _u32(adj)
    if order is None:
        order = directed_order(n, off, adj)
    order = _u32(order)
    rank = np.zeros(n, dtype=np.uint32)
    rank[order] = np.arange(n, dtype=np.uint32)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(off).astype(np.int64))
    a, b = rank[src].astype(np.int64), rank[adj].astype(np.int64)

    def csr(x, y):
        o = np.lexsort((y, x))
        cnt = np.bincount(x, minlength=n).astype(np.uint64)
        ro = np.zeros(n + 1, dtype=np.uint64)
        np.cumsum(cnt, out=ro[1:])
        return ro, y[o].astype(np.uint32)

    roff, radj = csr(a, b)
    ioff, iadj = csr(b, a)
    h = lib().oracle_build_directed_definition(n, roff, radj, ioff, iadj)
    return _collect(h, 2 * n, order, with_stats=False)
