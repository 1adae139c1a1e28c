"""Failure handling of the batch sort, forced from the host.

The look-back waits of the batch sort are bounded; gv_debug_spin_limit(0)
makes every such wait give up at once (no stall is needed, every kernel exits
normally).  The batch must then change nothing and the call must report
GV_EDEVICE, never GV_OK with statistics; the graph stays unusable.  Batches of
at most 4096 pairs are sorted by one workgroup without look-back, so the same
setting leaves them untouched.
"""
import numpy as np
import pytest

from gpu_helpers import assert_same, need_gpu, say
from oracle import pyoracle as O
from paper_2306_08252_amd import inputs as I

pytestmark = pytest.mark.gpu


def _graph(gv, B=8):
    w = I.RmatWorkload(12, 1 << 15, name="fail")
    g = gv.Graph(w.num_vertices, w.src, w.dst, block_slots=B)
    o = O.OracleGraph(w.num_vertices, w.src, w.dst, block_slots=B)
    return w, g, o


@pytest.mark.parametrize("op,overlap", [("insert", 0), ("delete", 0), ("query", 0),
                                        ("async", 0), ("insert", 1), ("delete", 1),
                                        ("async", 1)])
def test_lookback_give_up_is_reported(op, overlap):
    """With the sort overlap on, the passes run on the side stream and take
    tickets; a wait that gives up there is reported the same way."""
    gv = need_gpu()
    say(f"forced look-back give-up: {op}, overlap {overlap}")
    w, g, o = _graph(gv)
    gv.gv_set_tuning(g.h, overlap=overlap)
    assert_same(g, o, "init")
    # a single-tile batch never waits: the setting leaves it untouched
    s, d = w.insert_batch(3000, 0)
    gv.gv_debug_spin_limit(g.h, 0)
    assert g.insert_edges(s, d) == o.insert_edges(s, d)[1]
    assert_same(g, o, "single-tile batch with spin limit 0")
    s, d = (w.insert_batch if op != "delete" else w.delete_batch)(50000, 1)
    with pytest.raises(gv.GraphVineError) as e:
        if op == "insert":
            g.insert_edges(s, d)
        elif op == "delete":
            g.delete_edges(s, d)
        elif op == "query":
            g.edge_exists(s, d)
            rc = g.sync()
            if rc:
                raise gv.GraphVineError(rc, "gv_sync")
        else:
            g.insert_edges(s, d, stats=False)
            rc = g.sync()
            if rc:
                raise gv.GraphVineError(rc, "gv_sync")
    assert e.value.code == gv.GV_EDEVICE
    # the graph is unusable from then on
    with pytest.raises(gv.GraphVineError) as e:
        g.insert_edges(s[:10], d[:10])
    assert e.value.code == gv.GV_EDEVICE
    g.close()


def test_default_spin_limit_still_sorts():
    gv = need_gpu()
    w, g, o = _graph(gv)
    gv.gv_debug_spin_limit(g.h, 1 << 24)
    s, d = w.insert_batch(50000, 2)
    assert g.insert_edges(s, d) == o.insert_edges(s, d)[1]
    assert_same(g, o, "multi-tile batch, default limit")
    s, d = w.delete_batch(50000, 2)
    assert g.delete_edges(s, d) == o.delete_edges(s, d)[1]
    assert_same(g, o, "multi-tile delete, default limit")
    g.close()
