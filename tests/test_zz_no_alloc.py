"""gv_edge_exists_noalloc (collected last): the query batch with its temporaries in a fixed
device array (no device allocation in the call), against gv_edge_exists on the
same graph and inputs, and against the oracle.  Two calls in a row, the second
smaller, so the second runs on what the first left in the array."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_helpers import need_gpu, say
from oracle import pyoracle as O
from paper_2306_08252_amd import inputs as I

pytestmark = pytest.mark.gpu


def _noalloc(gv, g, s, d):
    L = gv.lib()
    f = L.gv_edge_exists_noalloc
    f.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p]
    f.restype = C.c_int
    st = gv.as_device_u32(s, g.device)
    dt = gv.as_device_u32(d, g.device)
    out = torch.full((max(st.numel(), 1),), 7, dtype=torch.uint8, device=g.device)
    rc = f(C.c_void_p(g.h), gv._ptr(st), gv._ptr(dt), st.numel(), gv._ptr(out))
    return rc, out[: st.numel()]


def test_noalloc_query_matches_the_allocating_entry_point():
    gv = need_gpu()
    w = I.RmatWorkload(14, 1 << 18, name="noalloc")
    g = gv.Graph(w.num_vertices, w.src, w.dst, block_slots=16)
    o = O.OracleGraph(w.num_vertices, w.src, w.dst, block_slots=16)
    for j, q in enumerate([60001, 4097, 1000]):
        say(f"noalloc query batch {q}")
        s, d = w.query_batch(q, j)
        rc, got = _noalloc(gv, g, s, d)
        assert rc == gv.GV_OK
        want = g.edge_exists(s, d)
        assert g.sync() == gv.GV_OK
        np.testing.assert_array_equal(got.cpu().numpy(), want.cpu().numpy(), err_msg=str(q))
        np.testing.assert_array_equal(got.cpu().numpy(), o.edge_exists(s, d), err_msg=str(q))
    # more pairs than the fixed array holds: refused before any device work
    big = (1 << 18) + 1
    s = torch.zeros(big, dtype=torch.int32, device=g.device)
    rc, _ = _noalloc(gv, g, s, s)
    assert rc == gv.GV_ERANGE
    # the graph is still usable
    s, d = w.query_batch(777, 9)
    rc, got = _noalloc(gv, g, s, d)
    assert rc == gv.GV_OK
    np.testing.assert_array_equal(got.cpu().numpy(), o.edge_exists(s, d))
    g.close()
