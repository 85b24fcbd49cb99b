"""The C-ABI library loads and exports every entry point declared in
include/spc.h (CPU only: no compute call is made).  Host-side argument
checks that return before any device work are exercised too."""
import ctypes as C
import os
import re

import pytest

from paper_2212_00977_amd import native

HEADER = os.path.join(native.INCLUDE, "spc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spc_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(native.LIBPATH):
        native.build_library()
    return native.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("spc_build_index", "spc_query_batch", "spc_free"):
        assert required in names
    assert set(names) == set(native.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code in range(6):
        s = lib.spc_status_string(code)
        assert s and len(s) > 1
    assert lib.spc_status_string(99) == b"unknown status"


def test_null_arguments_rejected_on_host(lib):
    out = C.c_void_p()
    assert lib.spc_build_index(None, None, None, C.byref(out)) == 1
    assert lib.spc_build_index_batch(None, 0, None, None, C.byref(out)) == 1
    assert lib.spc_query_batch(None, 0, None, None, 1, None, None, None, None) == 1
    st = native.SpcStats()
    assert lib.spc_index_stats(None, C.byref(st)) == 1
    assert lib.spc_round_stats(None, 1, None, None, None, None) == 1
    assert lib.spc_round_profile(None, 1, None, None, None, None, None, None) == 1
    assert lib.spc_export_labels(None, 0, None, None, None, None, None, 0, None) == 1
    assert lib.spc_tune_queries(None, 0, None, None, 1, None, None) == 1
    assert lib.spc_set_query_config(None, 0) == 1
    lib.spc_free(None)  # no-op
    assert out.value is None


def test_bad_options_rejected_on_host(lib):
    g = native.SpcGraph()
    g.n = 4
    g.nnz = 3  # odd: cannot be a symmetric CSR
    g.row_off = 1
    g.col = 1
    o = native.SpcBuildOpts()
    out = C.c_void_p()
    assert lib.spc_build_index(C.byref(g), C.byref(o), None, C.byref(out)) == 1
    g.nnz = 2
    o.dist_bits = 12
    assert lib.spc_build_index(C.byref(g), C.byref(o), None, C.byref(out)) == 1
    o.dist_bits = 0
    o.reduce = 6  # one reduction at a time
    assert lib.spc_build_index(C.byref(g), C.byref(o), None, C.byref(out)) == 1
    o.reduce = 0
    o.propagation = 3  # pull, push or auto
    assert lib.spc_build_index(C.byref(g), C.byref(o), None, C.byref(out)) == 1
    o.propagation = 0
    o.reserved = 1
    assert lib.spc_build_index(C.byref(g), C.byref(o), None, C.byref(out)) == 1
    assert out.value is None


def test_query_configs_listed(lib):
    n = lib.spc_query_config_count()
    assert n >= 2
    seen = set()
    for i in range(n):
        st, tl = C.c_uint32(), C.c_uint32()
        assert lib.spc_query_config_info(i, C.byref(st), C.byref(tl)) == 0
        assert st.value >= 64 and st.value % 64 == 0 and tl.value >= 1
        seen.add((st.value, tl.value))
    assert len(seen) == n  # no duplicate configurations
    assert lib.spc_query_config_info(n, None, None) == 1
