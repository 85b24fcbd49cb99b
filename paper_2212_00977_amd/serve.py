"""Serving SPC query batches from a resident index, with continuous batching.

Requests (batches of (s, t) pairs) arrive over time.  The server admits a
request when the device memory its inputs and outputs need fits the I/O
budget beside the requests already on the device, coalesces the admitted
requests waiting in arrival order into one query launch (up to a batch
limit), and keeps several launches in flight on separate streams, so work
that arrives while other work runs overlaps with it on the GPU.  Latency is
measured from each request's scheduled arrival time (open loop) to the host
observing its results.

Every query runs in the library's query kernel; this module only moves
inputs and outputs and decides what to launch when.
"""
from __future__ import annotations

import gc
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import native
from .spc import Index, _check, _stream_handle

BYTES_PER_QUERY_IO = 4 + 4 + 2 + 8 + 1  # s, t, dist (<= 2 B), count, flags


@dataclass
class Request:
    rid: int
    s: np.ndarray          # uint32
    t: np.ndarray          # uint32
    arrival: float         # seconds after the start of the run
    graph_id: int = 0


@dataclass
class Result:
    rid: int
    dist: np.ndarray       # uint16 (uint8 indexes are widened)
    count: np.ndarray      # uint64
    flags: np.ndarray      # uint8
    arrival: float
    done: float
    admitted: float

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class _Launch:
    reqs: list
    offsets: list
    nbytes: int
    event: object
    host_out: tuple
    keep: tuple
    admitted: float


@dataclass
class ServeStats:
    results: dict = field(default_factory=dict)
    makespan_s: float = 0.0
    queries: int = 0
    launches: int = 0
    deferred: int = 0          # requests that waited in the queue for memory

    def latencies(self) -> np.ndarray:
        return np.array([r.latency for r in self.results.values()])

    def summary(self) -> dict:
        lat = self.latencies()
        return {"requests": len(self.results), "queries": self.queries,
                "queries_per_s": self.queries / self.makespan_s if self.makespan_s else 0.0,
                "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else 0.0,
                "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else 0.0,
                "launches": self.launches, "deferred": self.deferred,
                "makespan_s": self.makespan_s}


def take_batch(queue, used: int, budget: int, any_inflight: bool, coalesce: bool, max_batch: int) -> int:
    """How many requests from the head of `queue` (arrival order) the next
    launch takes: while their inputs and outputs fit the I/O budget beside
    the `used` bytes in flight (a request larger than the whole budget still
    runs alone once nothing is in flight), all of one graph, at most
    max_batch queries together, one request when not coalescing.  0 means
    the head request waits for memory."""
    n, nb, nq = 0, 0, 0
    for r in queue:
        need = int(r.s.shape[0]) * BYTES_PER_QUERY_IO
        if used + nb + need > budget and (n or any_inflight):
            break
        if n and (not coalesce or nq + int(r.s.shape[0]) > max_batch or r.graph_id != queue[0].graph_id):
            break
        n += 1
        nb += need
        nq += int(r.s.shape[0])
    return n


class Server:
    """Continuous-batching query server over one resident index.

    io_budget_bytes: device memory for in-flight request inputs/outputs;
    streams: launches in flight at once; max_batch: queries per launch.
    """

    def __init__(self, index: Index, io_budget_bytes: int = 1 << 28, streams: int = 4,
                 max_batch: int = 1 << 18, coalesce: bool = True):
        import torch

        self.torch = torch
        self.ix = index
        self.budget = int(io_budget_bytes)
        self.max_batch = int(max_batch)
        self.coalesce = coalesce
        self.streams = [torch.cuda.Stream(device=index.device) for _ in range(max(1, streams))]
        self.wide = index.dist_bits != 8

    # ---- one launch ---------------------------------------------------------
    def _launch(self, reqs: list, stream, now: float) -> _Launch:
        torch = self.torch
        dev = self.ix.device
        sizes = [int(r.s.shape[0]) for r in reqs]
        offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        nq = int(offsets[-1])
        s_h = torch.from_numpy(np.concatenate([r.s for r in reqs]).view(np.int32)).pin_memory()
        t_h = torch.from_numpy(np.concatenate([r.t for r in reqs]).view(np.int32)).pin_memory()
        with torch.cuda.stream(stream):
            s_d = s_h.to(dev, non_blocking=True)
            t_d = t_h.to(dev, non_blocking=True)
            dist = torch.empty(max(nq, 1), dtype=torch.int16 if self.wide else torch.uint8, device=dev)
            cnt = torch.empty(max(nq, 1), dtype=torch.int64, device=dev)
            flg = torch.empty(max(nq, 1), dtype=torch.uint8, device=dev)
        gid = reqs[0].graph_id
        rc = native.load().spc_query_batch(self.ix.handle, gid, s_d.data_ptr(), t_d.data_ptr(), nq,
                                           dist.data_ptr(), cnt.data_ptr(), flg.data_ptr(),
                                           _stream_handle(stream))
        _check(rc, "spc_query_batch")
        with torch.cuda.stream(stream):
            dist_h = torch.empty(dist.shape, dtype=dist.dtype, pin_memory=True)
            cnt_h = torch.empty(cnt.shape, dtype=cnt.dtype, pin_memory=True)
            flg_h = torch.empty(flg.shape, dtype=flg.dtype, pin_memory=True)
            dist_h.copy_(dist, non_blocking=True)
            cnt_h.copy_(cnt, non_blocking=True)
            flg_h.copy_(flg, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        return _Launch(reqs, offsets.tolist(), nq * BYTES_PER_QUERY_IO, ev,
                       (dist_h, cnt_h, flg_h), (s_h, t_h, s_d, t_d, dist, cnt, flg), now)

    def _finish(self, L: _Launch, done: float, out: ServeStats):
        dist_h, cnt_h, flg_h = L.host_out
        d = dist_h.numpy()
        d = d.astype(np.uint16) if d.dtype == np.uint8 else d.view(np.uint16)
        c = cnt_h.numpy().view(np.uint64)
        f = flg_h.numpy()
        for i, r in enumerate(L.reqs):
            a, b = L.offsets[i], L.offsets[i + 1]
            out.results[r.rid] = Result(r.rid, d[a:b].copy(), c[a:b].copy(), f[a:b].copy(),
                                        r.arrival, done, L.admitted)

    # ---- open-loop run --------------------------------------------------------
    def run(self, requests: list) -> ServeStats:
        """Serve `requests` (arrival times relative to the start).  The
        interpreter's cyclic garbage collector is paused meanwhile, so its
        sweeps do not land in the latency tail."""
        was = gc.isenabled()
        gc.disable()
        try:
            return self._run(requests)
        finally:
            if was:
                gc.enable()

    def _run(self, requests: list) -> ServeStats:
        torch = self.torch
        out = ServeStats()
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        queue: deque = deque()
        inflight: list = []
        used = 0
        busy = [0] * len(self.streams)
        deferred = set()
        t0 = time.perf_counter()
        while pending or queue or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            # completions free their memory and stream
            still = []
            for k, L in inflight:
                if L.event.query():
                    self._finish(L, time.perf_counter() - t0, out)
                    used -= L.nbytes
                    busy[k] -= 1
                else:
                    still.append((k, L))
            inflight = still
            # admit in arrival order while memory and a stream are free
            while queue:
                k = min(range(len(self.streams)), key=lambda i: busy[i])
                if busy[k] >= 2:
                    break
                n = take_batch(queue, used, self.budget, bool(inflight), self.coalesce, self.max_batch)
                batch = [queue.popleft() for _ in range(n)]
                if not batch:
                    deferred.update(r.rid for r in queue)  # waiting for memory
                    break
                L = self._launch(batch, self.streams[k], time.perf_counter() - t0)
                inflight.append((k, L))
                used += L.nbytes
                busy[k] += 1
                out.launches += 1
                out.queries += sum(int(r.s.shape[0]) for r in batch)
            if not queue and not inflight and pending:
                wait = pending[0].arrival - (time.perf_counter() - t0)
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
        torch.cuda.synchronize()
        out.makespan_s = time.perf_counter() - t0
        out.deferred = len(deferred)
        return out


def requests_from(tuples) -> list:
    """Request objects from inputs.poisson_requests tuples."""
    return [Request(i, s, t, a, g) for (i, s, t, a, g) in tuples]


def fifo_baseline(index: Index, requests: list) -> ServeStats:
    """One request at a time on one stream, in arrival order, no overlap."""
    srv = Server(index, io_budget_bytes=1 << 62, streams=1, coalesce=False)
    out = ServeStats()
    t0 = time.perf_counter()
    for r in sorted(requests, key=lambda r: r.arrival):
        now = time.perf_counter() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        L = srv._launch([r], srv.streams[0], time.perf_counter() - t0)
        L.event.synchronize()
        srv._finish(L, time.perf_counter() - t0, out)
        out.launches += 1
        out.queries += int(r.s.shape[0])
    out.makespan_s = time.perf_counter() - t0
    return out
