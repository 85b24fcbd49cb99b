"""Python binding of the SPC label library: argument marshalling only.

Every step (ordering, distance rounds, counts, queries) runs in the HIP
kernels of libspc.so.  torch provides device memory and the stream.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import native

SPC_OK = 0
STATUS = {0: "SPC_OK", 1: "SPC_ERR_INVALID_ARG", 2: "SPC_ERR_OUT_OF_MEMORY", 3: "SPC_ERR_DEVICE",
          4: "SPC_ERR_DIST_RANGE", 5: "SPC_ERR_UNSUPPORTED"}
FLAG_SATURATED, FLAG_UNREACHABLE, FLAG_HORIZON, FLAG_INVALID = 1, 2, 4, 8


class SpcError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        lib = native.load()
        super().__init__(f"{where}: {STATUS.get(code, code)} "
                         f"({lib.spc_status_string(code).decode()})")


def _check(code: int, where: str):
    if code != SPC_OK:
        raise SpcError(code, where)


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(a, dtype_np, dtype_t, device):
    """Contiguous device tensor holding `a` (numpy array or tensor) with the
    bit pattern of dtype_np."""
    torch = _torch()
    if isinstance(a, torch.Tensor):
        t = a.to(device=device)
        if t.dtype != dtype_t:
            t = t.to(dtype_t)
        return t.contiguous()
    arr = np.ascontiguousarray(np.asarray(a, dtype=dtype_np))
    return torch.from_numpy(arr.view(_np_view(dtype_t))).to(device)


def _np_view(dtype_t):
    torch = _torch()
    return {torch.int32: np.int32, torch.int64: np.int64, torch.int16: np.int16,
            torch.uint8: np.uint8}[dtype_t]


def _graph_struct(off, adj, order, tie_key, device, keep, directed=False):
    torch = _torch()
    off_t = _dev(off, np.uint64, torch.int64, device)
    n = off_t.shape[0] - 1
    adj_t = _dev(adj, np.uint32, torch.int32, device) if int(np.asarray(adj.shape[0])) else \
        torch.zeros(1, dtype=torch.int32, device=device)
    nnz = int(adj.shape[0])
    g = native.SpcGraph()
    g.n = n
    g.nnz = nnz
    g.row_off = off_t.data_ptr()
    g.col = adj_t.data_ptr()
    keep += [off_t, adj_t]
    if order is not None:
        o = _dev(order, np.uint32, torch.int32, device)
        keep.append(o)
        g.order = o.data_ptr()
    if tie_key is not None:
        tk = _dev(tie_key, np.uint64, torch.int64, device)
        keep.append(tk)
        g.tie_key = tk.data_ptr()
    g.on_device = 1
    g.directed = 1 if directed else 0
    return g


@dataclass
class BuildOptions:
    dist_bits: int = 0
    round_cap: int = 0
    mem_budget: int = 0
    validate: bool = True
    one_shell: bool = False  # SPC_REDUCE_ONE_SHELL: label the 2-core only
    equivalence: bool = False  # SPC_REDUCE_EQUIVALENCE: one weighted vertex per class of twins
    propagation: str = "pull"  # "pull" (Alg. 2), "push" (Alg. 1) or "auto" (chosen per round)
    tune_cache: str | None = None  # on-disk tuning cache: query configuration and bucket threshold

    def struct(self):
        o = native.SpcBuildOpts()
        o.dist_bits = self.dist_bits
        o.round_cap = self.round_cap
        o.mem_budget = self.mem_budget
        o.validate = 1 if self.validate else 0
        o.reduce = (1 if self.one_shell else 0) | (2 if self.equivalence else 0)
        o.propagation = {"pull": 0, "push": 1, "auto": 2}[self.propagation]
        o.reserved = 0
        o.tune_cache = None if self.tune_cache is None else os.fsencode(self.tune_cache)
        return o


class Index:
    """A built SPC label index resident in device memory."""

    def __init__(self, handle: C.c_void_p, device, sizes=None):
        self._h = handle
        self.device = device
        self._stats = None
        self._sizes = sizes  # input vertex count of each graph

    def __del__(self):
        # at interpreter exit the module globals may already be gone; the
        # process's device memory goes with it then
        try:
            self.free()
        except (AttributeError, TypeError):
            pass

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            native.load().spc_free(self._h)
        self._h = None

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise RuntimeError("index freed")
        return self._h

    def stats(self) -> dict:
        st = native.SpcStats()
        _check(native.load().spc_index_stats(self.handle, C.byref(st)), "spc_index_stats")
        return {f: getattr(st, f) for f, _ in native.SpcStats._fields_}

    def round_stats(self) -> dict:
        R = self.stats()["rounds"] + 1
        arrs = {k: np.zeros(R, dtype=np.uint64) for k in ("raw", "merged", "kept", "scanned")}
        _check(native.load().spc_round_stats(self.handle, R, *(arrs[k].ctypes.data for k in
                                                                ("raw", "merged", "kept",
                                                                 "scanned"))),
               "spc_round_stats")
        return arrs

    def round_kernel_launches(self) -> int:
        return int(self.stats()["round_kernel_launches"])

    def round_profile(self) -> dict:
        R = self.stats()["rounds"] + 1
        ms = np.zeros(R, dtype=np.float64)
        arrs = {k: np.zeros(R, dtype=np.uint64) for k in ("staged", "row_bytes", "headers",
                                                           "mem_peak", "filter_bytes")}
        _check(native.load().spc_round_profile(self.handle, R, ms.ctypes.data,
                                               arrs["staged"].ctypes.data,
                                               arrs["row_bytes"].ctypes.data,
                                               arrs["headers"].ctypes.data,
                                               arrs["mem_peak"].ctypes.data,
                                               arrs["filter_bytes"].ctypes.data), "spc_round_profile")
        arrs["kernel_ms"] = ms
        return arrs

    def graph_entries(self, graph_id: int = 0):
        n = C.c_uint32()
        e = C.c_uint64()
        _check(native.load().spc_graph_entries(self.handle, graph_id, C.byref(n), C.byref(e)),
               "spc_graph_entries")
        return n.value, e.value

    def _outputs(self, nq, out, what):
        """Caller's output tensors, checked, or new ones (current stream)."""
        torch = _torch()
        bits = self.dist_bits
        if out is None:
            n = max(nq, 1)
            return (torch.empty(n, dtype=torch.uint8 if bits == 8 else torch.int16, device=self.device),
                    torch.empty(n, dtype=torch.int64, device=self.device),
                    torch.empty(n, dtype=torch.uint8, device=self.device))
        dist, cnt, flags = out
        if dist.element_size() * 8 != bits:
            raise ValueError(f"{what}: dist output holds {dist.element_size() * 8}-bit values, "
                             f"the index answers with {bits}-bit distances")
        if cnt.element_size() != 8 or (flags is not None and flags.element_size() != 1):
            raise ValueError(f"{what}: count must be 8-byte and flags 1-byte elements")
        for nm, x in (("dist", dist), ("count", cnt), ("flags", flags)):
            if x is None:
                continue
            if x.numel() < nq or not x.is_contiguous() or x.device.type != "cuda":
                raise ValueError(f"{what}: {nm} output must be a contiguous device tensor "
                                 f"of at least {nq} elements")
        return dist, cnt, flags

    def query(self, s, t, graph_id: int = 0, stream=None, out=None):
        """SPC(s, t) for vertex ids of graph `graph_id`.  Returns device
        tensors (dist uint8 / int16-as-uint16, count int64-as-uint64,
        flags uint8), written asynchronously on `stream`.  Inputs and new
        outputs are placed on `stream`, so they stay valid for the launch."""
        torch = _torch()
        strm = stream if stream is not None else torch.cuda.current_stream()
        with torch.cuda.stream(strm):
            s_t = _dev(s, np.uint32, torch.int32, self.device)
            t_t = _dev(t, np.uint32, torch.int32, self.device)
            nq = int(s_t.shape[0])
            if int(t_t.shape[0]) != nq:
                raise ValueError("s and t differ in length")
            dist, cnt, flags = self._outputs(nq, out, "Index.query")
        rc = native.load().spc_query_batch(self.handle, graph_id, s_t.data_ptr(), t_t.data_ptr(),
                                           nq, dist.data_ptr(), cnt.data_ptr(),
                                           flags.data_ptr() if flags is not None else None,
                                           _stream_handle(strm))
        _check(rc, "spc_query_batch")
        self._keep = (s_t, t_t)  # inputs stay alive until the next call
        return dist[:nq], cnt[:nq], (flags[:nq] if flags is not None else None)

    def query_multi(self, graph_ids, s, t, stream=None, out=None):
        """SPC(s[i], t[i]) on graph graph_ids[i] for every i, in one call
        (spc_query_batch_multi: bucketed by label length); graph_ids None =
        every query on graph 0.  Same outputs as query()."""
        torch = _torch()
        strm = stream if stream is not None else torch.cuda.current_stream()
        with torch.cuda.stream(strm):
            s_t = _dev(s, np.uint32, torch.int32, self.device)
            t_t = _dev(t, np.uint32, torch.int32, self.device)
            g_t = None if graph_ids is None else _dev(graph_ids, np.uint32, torch.int32, self.device)
            nq = int(s_t.shape[0])
            if int(t_t.shape[0]) != nq or (g_t is not None and int(g_t.shape[0]) != nq):
                raise ValueError("graph_ids, s and t differ in length")
            dist, cnt, flags = self._outputs(nq, out, "Index.query_multi")
        rc = native.load().spc_query_batch_multi(self.handle, None if g_t is None else g_t.data_ptr(),
                                                 s_t.data_ptr(), t_t.data_ptr(), nq, dist.data_ptr(),
                                                 cnt.data_ptr(),
                                                 flags.data_ptr() if flags is not None else None,
                                                 _stream_handle(strm))
        _check(rc, "spc_query_batch_multi")
        self._keep = (s_t, t_t, g_t)
        return dist[:nq], cnt[:nq], (flags[:nq] if flags is not None else None)

    def tune_query_buckets(self, graph_ids, s, t, stream=None) -> int:
        """Autotune the bucket threshold of query_multi on sample queries;
        returns the threshold kept (0 = no bucketing)."""
        torch = _torch()
        s_t = _dev(s, np.uint32, torch.int32, self.device)
        t_t = _dev(t, np.uint32, torch.int32, self.device)
        g_t = None if graph_ids is None else _dev(graph_ids, np.uint32, torch.int32, self.device)
        out = C.c_uint32()
        _check(native.load().spc_tune_query_buckets(self.handle, None if g_t is None else g_t.data_ptr(),
                                                    s_t.data_ptr(), t_t.data_ptr(), int(s_t.shape[0]),
                                                    _stream_handle(stream), C.byref(out)),
               "spc_tune_query_buckets")
        return out.value

    def set_query_buckets(self, small: int):
        _check(native.load().spc_set_query_buckets(self.handle, int(small)), "spc_set_query_buckets")

    def tune_queries(self, s, t, graph_id: int = 0, stream=None) -> int:
        """Autotune the query launch configuration on the sample pairs (s, t):
        every configuration is timed (and checked to agree); the fastest is
        kept for this index.  Returns its number."""
        torch = _torch()
        s_t = _dev(s, np.uint32, torch.int32, self.device)
        t_t = _dev(t, np.uint32, torch.int32, self.device)
        if int(s_t.shape[0]) != int(t_t.shape[0]):
            raise ValueError("s and t differ in length")
        cfg = C.c_uint32()
        _check(native.load().spc_tune_queries(self.handle, graph_id, s_t.data_ptr(), t_t.data_ptr(),
                                              int(s_t.shape[0]), _stream_handle(stream),
                                              C.byref(cfg)), "spc_tune_queries")
        return cfg.value

    def set_query_config(self, cfg: int):
        _check(native.load().spc_set_query_config(self.handle, int(cfg)), "spc_set_query_config")

    @property
    def query_config(self) -> int:
        return int(self.stats()["query_config"])

    @property
    def dist_bits(self) -> int:
        if self._stats is None:
            self._stats = self.stats()
        return self._stats["dist_bits"]

    def export(self, graph_id: int = 0):
        """Labels of one graph in its rank space, on the host (numpy):
        off, hub, dist (uint16), count (uint64), order (rank -> vertex)."""
        n, e = self.graph_entries(graph_id)
        off = np.zeros(n + 1, dtype=np.uint64)
        hub = np.zeros(max(e, 1), dtype=np.uint32)
        dist = np.zeros(max(e, 1), dtype=np.uint16)
        cnt = np.zeros(max(e, 1), dtype=np.uint64)
        order = np.zeros(max(n, 1), dtype=np.uint32)
        rc = native.load().spc_export_labels(self.handle, graph_id, off.ctypes.data,
                                             hub.ctypes.data, dist.ctypes.data, cnt.ctypes.data,
                                             order.ctypes.data, 0, _stream_handle(None))
        _check(rc, "spc_export_labels")
        nv = n // 2 if self.stats()["directed"] else n  # a directed index has 2n label rows
        return dict(off=off, hub=hub[:e], dist=dist[:e], count=cnt[:e], order=order[:nv])

    def export_reduction(self, graph_id: int = 0):
        """The 1-shell of one graph (host numpy, input vertex ids): root
        (shr), depth, parent per vertex; identity for an unreduced index."""
        n = self.input_vertices(graph_id)
        out = [np.zeros(max(n, 1), dtype=np.uint32) for _ in range(3)]
        rc = native.load().spc_export_reduction(self.handle, graph_id, *(a.ctypes.data for a in out),
                                                0, _stream_handle(None))
        _check(rc, "spc_export_reduction")
        return dict(root=out[0][:n], depth=out[1][:n], parent=out[2][:n])

    def export_reduction_device(self, graph_id: int = 0):
        """export_reduction into device tensors (int32 bit views)."""
        torch = _torch()
        n = self.input_vertices(graph_id)
        out = [torch.empty(max(n, 1), dtype=torch.int32, device=self.device) for _ in range(3)]
        rc = native.load().spc_export_reduction(self.handle, graph_id, *(a.data_ptr() for a in out), 1,
                                                _stream_handle(None))
        _check(rc, "spc_export_reduction")
        return dict(root=out[0][:n], depth=out[1][:n], parent=out[2][:n])

    def input_vertices(self, graph_id: int = 0) -> int:
        """Vertices of graph `graph_id` as given to the build."""
        if self._sizes is None:
            raise RuntimeError("input sizes unknown for this handle")
        # an id out of range is left to the library, which refuses it
        return self._sizes[graph_id] if 0 <= graph_id < len(self._sizes) else 0

    def export_device(self, graph_id: int = 0):
        """Same as export() into device tensors (int32/int16/int64 bit views)."""
        torch = _torch()
        n, e = self.graph_entries(graph_id)
        dev = self.device
        off = torch.empty(n + 1, dtype=torch.int64, device=dev)
        hub = torch.empty(max(e, 1), dtype=torch.int32, device=dev)
        dist = torch.empty(max(e, 1), dtype=torch.int16, device=dev)
        cnt = torch.empty(max(e, 1), dtype=torch.int64, device=dev)
        order = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        rc = native.load().spc_export_labels(self.handle, graph_id, off.data_ptr(), hub.data_ptr(),
                                             dist.data_ptr(), cnt.data_ptr(), order.data_ptr(), 1,
                                             _stream_handle(None))
        _check(rc, "spc_export_labels")
        return dict(off=off, hub=hub[:e], dist=dist[:e], count=cnt[:e], order=order[:n])


def build_index(off, adj, order=None, tie_key=None, opts: BuildOptions | None = None,
                device=None, stream=None, directed: bool = False) -> Index:
    """Build the SPC label index of one graph (symmetric CSR off/adj, numpy or
    torch; with directed=True, each arc once in its tail's row).  Inputs are
    placed in device memory first."""
    torch = _torch()
    device = device or torch.device("cuda", torch.cuda.current_device())
    keep = []
    g = _graph_struct(off, adj, order, tie_key, device, keep, directed=directed)
    o = (opts or BuildOptions()).struct()
    h = C.c_void_p()
    rc = native.load().spc_build_index(C.byref(g), C.byref(o), _stream_handle(stream), C.byref(h))
    _check(rc, "spc_build_index")
    return Index(h, device, [int(g.n)])


def build_graph(graph, opts: BuildOptions | None = None, device=None, stream=None) -> Index:
    """build_index for an inputs.Graph (its explicit order / tie keys)."""
    return build_index(graph.off, graph.adj, order=graph.order, tie_key=graph.tie_key, opts=opts,
                       device=device, stream=stream)


def build_index_batch(graphs, opts: BuildOptions | None = None, device=None, stream=None) -> Index:
    """One index over many independent graphs (inputs.Graph objects)."""
    torch = _torch()
    device = device or torch.device("cuda", torch.cuda.current_device())
    keep = []
    arr = (native.SpcGraph * len(graphs))()
    for i, g in enumerate(graphs):
        arr[i] = _graph_struct(g.off, g.adj, g.order, g.tie_key, device, keep)
    o = (opts or BuildOptions()).struct()
    h = C.c_void_p()
    rc = native.load().spc_build_index_batch(arr, len(graphs), C.byref(o), _stream_handle(stream),
                                             C.byref(h))
    _check(rc, "spc_build_index_batch")
    return Index(h, device, [int(g.n) for g in graphs])


def hybrid_order(off, adj, delta: int = 5):
    """Hybrid vertex order of a host CSR (numpy): (order rank -> vertex, core
    size); computed on the host by the library (spc_hybrid_order)."""
    off = np.ascontiguousarray(np.asarray(off, dtype=np.uint64))
    adj = np.ascontiguousarray(np.asarray(adj, dtype=np.uint32))
    n = off.shape[0] - 1
    g = native.SpcGraph()
    g.n = n
    g.nnz = int(adj.shape[0])
    g.row_off = off.ctypes.data
    g.col = adj.ctypes.data if adj.shape[0] else None
    g.on_device = 0
    order = np.zeros(max(n, 1), dtype=np.uint32)
    core = C.c_uint32()
    _check(native.load().spc_hybrid_order(C.byref(g), int(delta) & 0xFFFFFFFF, order.ctypes.data,
                                          C.byref(core)), "spc_hybrid_order")
    return order[:n], core.value


def query_configs() -> list:
    """(stage, tiles) of every query launch configuration, by number."""
    lib = native.load()
    out = []
    for i in range(lib.spc_query_config_count()):
        st, tl = C.c_uint32(), C.c_uint32()
        _check(lib.spc_query_config_info(i, C.byref(st), C.byref(tl)), "spc_query_config_info")
        out.append((st.value, tl.value))
    return out


def release_cached_memory():
    """Return the library's cached device blocks (freed build buffers) to
    the device allocator."""
    native.load().spc_release_cached_memory()


def set_cache_limit(nbytes=None):
    """Most freed device memory the library keeps per device after a build
    or a free (None: all of it, until release_cached_memory; 0: the default,
    a quarter of the device)."""
    native.load().spc_set_cache_limit((1 << 64) - 1 if nbytes is None else int(nbytes))


def as_u64(count_tensor) -> np.ndarray:
    """Host uint64 view of a count tensor (int64 bit pattern)."""
    return count_tensor.cpu().numpy().view(np.uint64)


def as_dist(dist_tensor) -> np.ndarray:
    """Host uint16 view of a dist tensor (uint8 or int16 bit pattern)."""
    a = dist_tensor.cpu().numpy()
    return a.astype(np.uint16) if a.dtype == np.uint8 else a.view(np.uint16)
