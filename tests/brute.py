"""Brute-force references used to pin the oracle (pure Python, big ints).

Independent of the oracle's C code: shortest paths are enumerated
explicitly, and the trough-path definition is applied to each path.
Only for tiny graphs.
"""
from __future__ import annotations

from collections import deque

SAT = (1 << 64) - 1


def adjacency(n, edges):
    nb = [set() for _ in range(n)]
    for a, b in edges:
        a, b = int(a), int(b)
        if a != b:
            nb[a].add(b)
            nb[b].add(a)
    return [sorted(x) for x in nb]


def bfs_dist(nb, s):
    d = [None] * len(nb)
    d[s] = 0
    q = deque([s])
    while q:
        v = q.popleft()
        for x in nb[v]:
            if d[x] is None:
                d[x] = d[v] + 1
                q.append(x)
    return d


def all_shortest_paths(nb, s, t):
    """Every shortest s-t path, as a tuple of vertices (explicit enumeration)."""
    dist = bfs_dist(nb, s)
    if dist[t] is None:
        return []
    dt = bfs_dist(nb, t)
    out = []

    def rec(path):
        v = path[-1]
        if v == t:
            out.append(tuple(path))
            return
        for x in nb[v]:
            if dist[x] == dist[v] + 1 and dt[x] == dt[v] - 1:
                rec(path + [x])

    rec([s])
    return out


def labels_by_definition(nb, rank):
    """{v: {w: (sd, tau)}} with tau = #shortest v-w paths whose vertices other
    than w all have a larger rank number than w (rank 0 = most important)."""
    n = len(nb)
    lab = {}
    for v in range(n):
        lab[v] = {}
        for w in range(n):
            if rank[w] > rank[v]:
                continue
            paths = all_shortest_paths(nb, v, w)
            tau = sum(1 for p in paths if all(rank[x] > rank[w] for x in p if x != w))
            if tau:
                lab[v][w] = (len(paths[0]) - 1, tau)
    return lab


def spc_brute(nb, s, t):
    paths = all_shortest_paths(nb, s, t)
    if not paths:
        return None, 0
    return len(paths[0]) - 1, len(paths)


def sigma_bfs_bigint(nb, s):
    """BFS path counts with exact Python integers."""
    n = len(nb)
    d = [None] * n
    c = [0] * n
    d[s], c[s] = 0, 1
    q = deque([s])
    while q:
        v = q.popleft()
        for x in nb[v]:
            if d[x] is None:
                d[x] = d[v] + 1
                c[x] = c[v]
                q.append(x)
            elif d[x] == d[v] + 1:
                c[x] += c[v]
    return d, c
