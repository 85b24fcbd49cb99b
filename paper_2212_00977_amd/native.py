"""Build and load ``libspc.so``, the gfx950 HIP library behind include/spc.h.

The library is compiled in-tree with hipcc for gfx950 only.  Loading fails
loudly when it is missing: there is no CPU fallback for any entry point.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(PKG, "lib")
LIBPATH = os.path.join(LIBDIR, "libspc.so")
SOURCES = ["memory.hip", "primitives.hip", "build.hip", "reduce.hip", "query.hip", "order.hip",
           "capi.hip"]
HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

EXPORTS = ["spc_build_index", "spc_build_index_batch", "spc_query_batch", "spc_free",
           "spc_index_stats", "spc_round_stats", "spc_round_profile", "spc_graph_entries", "spc_export_labels",
           "spc_status_string", "spc_release_cached_memory", "spc_query_config_count",
           "spc_query_config_info", "spc_tune_queries", "spc_set_query_config", "spc_hybrid_order",
           "spc_export_reduction", "spc_query_batch_multi", "spc_tune_query_buckets",
           "spc_set_query_buckets", "spc_query_batch_multi_noalloc", "spc_set_cache_limit"]


# A test build with tiny on-chip tables (8-bit hash of 128 slots for the
# puller's label, 256 distinct candidates per chunk) and 2^14 pulled
# entries per batch: small graphs then take the paths that only large labels
# and large rounds take in the default build (unstaged label parts, chunk
# overflow and narrowing, many chunks per puller, many batches per round,
# pullers with a buffer of their own) and a 16-pair list of filter hits (so
# the probes that search at once run too).
SMALL_TABLES = ["-DSPC_LBITS=7", "-DSPC_LBITS_LONG=7", "-DSPC_CBITS=9", "-DSPC_TEMP_LOG2=14",
                "-DSPC_TEMP_MAX_LOG2=14", "-DSPC_FILT_LIST=16"]
SMALL_TABLES_PATH = os.path.join(LIBDIR, "libspc_smalltab.so")


def build_library(verbose: bool = False, small_tables: bool = False) -> str:
    """Compile every HIP source into libspc.so (always recompiles); with
    small_tables, the test build libspc_smalltab.so."""
    os.makedirs(LIBDIR, exist_ok=True)
    out = SMALL_TABLES_PATH if small_tables else LIBPATH
    tmp = out + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, *(SMALL_TABLES if small_tables else []), "-I", INCLUDE,
           "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    if verbose:
        print(r.stderr)
    os.replace(tmp, out)
    return out


class SpcStats(C.Structure):
    _fields_ = [("n", C.c_uint32), ("num_graphs", C.c_uint32), ("m", C.c_uint64),
                ("entries", C.c_uint64), ("rounds", C.c_uint32), ("max_dist", C.c_uint32),
                ("dist_bits", C.c_uint32), ("truncated", C.c_uint32),
                ("saturated_entries", C.c_uint64), ("index_bytes", C.c_uint64),
                ("peak_build_bytes", C.c_uint64), ("ms_order", C.c_double),
                ("ms_rounds", C.c_double), ("ms_finalize", C.c_double), ("ms_total", C.c_double),
                ("ms_round_kernel", C.c_double), ("alg_bytes_round_kernel", C.c_uint64),
                ("round_kernel_launches", C.c_uint64), ("query_config", C.c_uint32),
                ("label_bits", C.c_uint32), ("fringe_vertices", C.c_uint64),
                ("fringe_depth", C.c_uint32), ("twin_vertices", C.c_uint32),
                ("directed", C.c_uint32), ("query_small", C.c_uint32), ("tune_cached", C.c_uint32)]


class SpcGraph(C.Structure):
    _fields_ = [("n", C.c_uint32), ("nnz", C.c_uint64), ("row_off", C.c_void_p),
                ("col", C.c_void_p), ("order", C.c_void_p), ("tie_key", C.c_void_p),
                ("on_device", C.c_int32), ("directed", C.c_int32)]


class SpcBuildOpts(C.Structure):
    _fields_ = [("dist_bits", C.c_uint32), ("round_cap", C.c_uint32),
                ("mem_budget", C.c_uint64), ("validate", C.c_uint32), ("reduce", C.c_uint32),
                ("propagation", C.c_uint32), ("reserved", C.c_uint32), ("tune_cache", C.c_char_p)]


_lib = None


def load(path: str | None = None):
    """Load libspc.so (torch is imported first so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (HIP runtime of the process)
    path = path or LIBPATH
    if not os.path.exists(path):
        raise RuntimeError(f"libspc.so not built ({path}); run __graft_entry__.build()")
    L = C.CDLL(path)
    vp, u32, u64, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32
    L.spc_build_index.argtypes = [C.POINTER(SpcGraph), C.POINTER(SpcBuildOpts), vp, C.POINTER(vp)]
    L.spc_build_index.restype = C.c_int
    L.spc_build_index_batch.argtypes = [C.POINTER(SpcGraph), u32, C.POINTER(SpcBuildOpts), vp,
                                        C.POINTER(vp)]
    L.spc_build_index_batch.restype = C.c_int
    L.spc_query_batch.argtypes = [vp, u32, vp, vp, u64, vp, vp, vp, vp]
    L.spc_query_batch.restype = C.c_int
    L.spc_free.argtypes = [vp]
    L.spc_free.restype = None
    L.spc_release_cached_memory.argtypes = []
    L.spc_release_cached_memory.restype = None
    L.spc_set_cache_limit.argtypes = [u64]
    L.spc_set_cache_limit.restype = None
    L.spc_index_stats.argtypes = [vp, C.POINTER(SpcStats)]
    L.spc_index_stats.restype = C.c_int
    L.spc_round_stats.argtypes = [vp, u32, vp, vp, vp, vp]
    L.spc_round_stats.restype = C.c_int
    L.spc_round_profile.argtypes = [vp, u32, vp, vp, vp, vp, vp, vp]
    L.spc_round_profile.restype = C.c_int
    L.spc_graph_entries.argtypes = [vp, u32, C.POINTER(u32), C.POINTER(u64)]
    L.spc_graph_entries.restype = C.c_int
    L.spc_export_labels.argtypes = [vp, u32, vp, vp, vp, vp, vp, i32, vp]
    L.spc_export_labels.restype = C.c_int
    L.spc_query_config_count.argtypes = []
    L.spc_query_config_count.restype = u32
    L.spc_query_config_info.argtypes = [u32, C.POINTER(u32), C.POINTER(u32)]
    L.spc_query_config_info.restype = C.c_int
    L.spc_tune_queries.argtypes = [vp, u32, vp, vp, u64, vp, C.POINTER(u32)]
    L.spc_tune_queries.restype = C.c_int
    L.spc_hybrid_order.argtypes = [C.POINTER(SpcGraph), u32, vp, C.POINTER(u32)]
    L.spc_hybrid_order.restype = C.c_int
    L.spc_export_reduction.argtypes = [vp, u32, vp, vp, vp, i32, vp]
    L.spc_export_reduction.restype = C.c_int
    L.spc_query_batch_multi.argtypes = [vp, vp, vp, vp, u64, vp, vp, vp, vp]
    L.spc_query_batch_multi.restype = C.c_int
    L.spc_query_batch_multi_noalloc.argtypes = [vp, vp, vp, vp, u64, vp, vp, vp, vp]
    L.spc_query_batch_multi_noalloc.restype = C.c_int
    L.spc_tune_query_buckets.argtypes = [vp, vp, vp, vp, u64, vp, C.POINTER(u32)]
    L.spc_tune_query_buckets.restype = C.c_int
    L.spc_set_query_buckets.argtypes = [vp, u32]
    L.spc_set_query_buckets.restype = C.c_int
    L.spc_set_query_config.argtypes = [vp, u32]
    L.spc_set_query_config.restype = C.c_int
    L.spc_status_string.argtypes = [C.c_int]
    L.spc_status_string.restype = C.c_char_p
    _lib = L
    return L
