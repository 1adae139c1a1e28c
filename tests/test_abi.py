"""The C-ABI library loads and exports every function include/graphvine.h
declares; argument checks that precede any device work behave as documented.
No GPU compute is called here."""
import ctypes as C
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "graphvine.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gv_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2306_08252_amd import graphvine as gv
    if not os.path.exists(gv.LIB_PATH):
        pytest.fail("libgraphvine.so is not built (run __graft_entry__.build())")
    return gv.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gv_graph_init", "gv_insert_edges", "gv_delete_edges", "gv_insert_vertices",
                 "gv_delete_vertices", "gv_edge_exists", "gv_get_adjacency",
                 "gv_memory_used", "gv_graph_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_and_host_side_argument_checks(lib):
    from paper_2306_08252_amd import graphvine as gv
    assert gv.gv_strerror(gv.GV_OK) == "ok"
    assert "memory" in gv.gv_strerror(gv.GV_ENOMEM)
    # checks that happen before any device call
    assert lib.gv_graph_init(None, 10, None, None, 0, None, None) == gv.GV_EINVAL
    h = C.c_void_p()
    cfg = gv.gv_config(12, 0, 0, 0, 0)  # block size not a power of two
    assert lib.gv_graph_init(C.byref(h), 10, None, None, 0, C.byref(cfg), None) == gv.GV_EINVAL
    cfg = gv.gv_config(8, 1, 0, 0, 0)  # reserved flags
    assert lib.gv_graph_init(C.byref(h), 10, None, None, 0, C.byref(cfg), None) == gv.GV_EINVAL
    assert lib.gv_graph_init(C.byref(h), (1 << 31) + 1, None, None, 0, None, None) == gv.GV_EINVAL
    assert lib.gv_graph_init(C.byref(h), 10, None, None, 5, None, None) == gv.GV_EINVAL
    st = gv.gv_batch_stats()
    assert lib.gv_insert_edges(None, None, None, 0, C.byref(st)) == gv.GV_EINVAL
    assert lib.gv_delete_edges(None, None, None, 0, None) == gv.GV_EINVAL
    assert lib.gv_edge_exists(None, None, None, 0, None) == gv.GV_EINVAL
    assert lib.gv_sync(None) == gv.GV_EINVAL
    lib.gv_graph_destroy(None)
