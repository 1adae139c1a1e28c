"""Vertex delete against the oracle on adjacency shapes that take every path
of the sweep: degrees at and around the one-thread limit (64 slots) and the
one-unit limit (1024 slots), hubs of several units that lose slots below and
past their new degree, a hub that loses every slot, a deleted hub, and block
sizes from 1 to 64 slots.  After each delete (and after inserts that reuse
the freed blocks) the canonical dump, checksum, block accounting and audit
must equal the oracle's.
"""
import numpy as np
import pytest

from gpu_helpers import assert_same, need_gpu, say
from oracle import pyoracle as O
from paper_2306_08252_amd import inputs as I

pytestmark = pytest.mark.gpu


def shaped_graph(n, seed):
    """Vertices 0..9 with chosen degrees (distinct destinations), the rest
    uniform pairs."""
    rng = np.random.default_rng(seed)
    degs = [5000, 3000, 1024, 1025, 65, 64, 63, 700, 2049, 4096]
    src, dst = [], []
    for v, d in enumerate(degs):
        src.append(np.full(d, v, np.uint32))
        dst.append(rng.permutation(n)[:d].astype(np.uint32))
    s, d = I.uniform_pairs(I.stream_seed("vertex-shapes", seed), 30000, n)
    return np.concatenate(src + [s]), np.concatenate(dst + [d])


@pytest.mark.parametrize("B", [1, 2, 4, 16, 64])
def test_vertex_delete_paths_match_oracle(B):
    gv = need_gpu()
    n = 8192
    src, dst = shaped_graph(n, B)
    g = gv.Graph(n, src, dst, block_slots=B, vertex_capacity=n)
    o = O.OracleGraph(n, src, dst, block_slots=B, vertex_capacity=n)
    assert_same(g, o, "init")
    rng = np.random.default_rng(100 + B)
    # every destination of vertex 9 (so it keeps nothing), vertex 1 (a
    # deleted hub), and random vertices
    d9 = dst[src == 9]
    rounds = [np.concatenate([[1], rng.integers(10, n, 300)]).astype(np.uint32),
              np.unique(d9).astype(np.uint32),
              rng.integers(0, n, 40).astype(np.uint32)]
    for r, ids in enumerate(rounds):
        say(f"B={B} round {r}: delete {len(ids)} ids")
        assert g.delete_vertices(ids) == o.delete_vertices(ids)[1], r
        assert_same(g, o, f"delete round {r}")
        # the freed blocks are reused by new edges
        back = np.unique(ids).astype(np.uint32)
        assert g.insert_vertices(back) == o.insert_vertices(back)[1], r
        s, d = I.uniform_pairs(I.stream_seed("vertex-shapes-ins", B, r), 4000, n)
        s[:500] = 0
        s[500:900] = 3
        assert g.insert_edges(s, d) == o.insert_edges(s, d)[1], r
        assert_same(g, o, f"insert round {r}")
    assert g.sync() == 0
    g.close()


def test_vertex_delete_in_a_plan_matches_eager():
    """The recorded form sizes its lists for a full pool: the same deletes in
    a plan and eagerly give the same graph as the oracle."""
    gv = need_gpu()
    n, B = 8192, 8
    src, dst = shaped_graph(n, 7)
    ga = gv.Graph(n, src, dst, block_slots=B, vertex_capacity=n)
    gb = gv.Graph(n, src, dst, block_slots=B, vertex_capacity=n)
    o = O.OracleGraph(n, src, dst, block_slots=B, vertex_capacity=n)
    ids = np.array([0, 3, 77, 501, 4000], np.uint32)
    ops = [(3, ids, None), (2, ids, None)]
    plan = gv.Plan(gb.h, ops)
    plan.launch()
    gv.gv_apply_ops(ga.h, ops)
    o.delete_vertices(ids)
    o.insert_vertices(ids)
    assert ga.sync() == 0 and gb.sync() == 0
    assert_same(ga, o, "eager")
    assert_same(gb, o, "plan")
    plan.close()
    ga.close()
    gb.close()


def test_fit_table_vertex_insert_flag():
    """GV_OP_FIT_TABLE: a vertex insert through gv_apply_ops that neither
    grows the table nor reads the device back gives the plain insert's
    result when its ids fit; an id past the table leaves a sticky GV_ERANGE
    (the fitting ids are still inserted); the flag on another op kind, or an
    unknown flag, is GV_EINVAL."""
    gv = need_gpu()
    n, cap = 1000, 1024
    s0, d0 = I.uniform_pairs(I.stream_seed("fit-table", 1), 5000, n)
    g = gv.Graph(n, s0, d0, block_slots=8, vertex_capacity=cap)
    o = O.OracleGraph(n, s0, d0, block_slots=8, vertex_capacity=cap)
    dels = np.arange(0, 60, 3, dtype=np.uint32)
    g.delete_vertices(dels)
    o.delete_vertices(dels)
    ids = np.array([1023, 5, 3, 1001, 1023, 0xFFFFFFFF, 6], np.uint32)
    gv.gv_apply_ops(g.h, [(gv.OP_INSERT_VERTICES, ids, None, gv.OP_FIT_TABLE)], g.device)
    o.insert_vertices(ids)
    assert g.sync() == 0
    assert_same(g, o, "fitting ids")
    gv.gv_apply_ops(g.h, [(gv.OP_INSERT_VERTICES, np.array([2000, 9], np.uint32), None,
                           gv.OP_FIT_TABLE)], g.device)
    o.insert_vertices(np.array([9], np.uint32))
    assert g.sync() == gv.GV_ERANGE
    assert g.info()["vertex_capacity"] == cap
    assert_same(g, o, "an id past the table")
    s, d = np.array([1, 2], np.uint32), np.array([3, 4], np.uint32)
    for bad in ([(gv.OP_INSERT_EDGES, s, d, gv.OP_FIT_TABLE)],
                [(gv.OP_DELETE_VERTICES, s, None, gv.OP_FIT_TABLE)],
                [(gv.OP_INSERT_VERTICES, s, None, 2)]):
        with pytest.raises(gv.GraphVineError):
            gv.gv_apply_ops(g.h, bad, g.device)
    g.close()
