"""The paper-faithful ablation (complete binary tree of edge blocks, one
thread per vertex, Alg. 1-3) against the CPU oracle: canonical dump, batch
statistics and query answers after every batch, bit-exact."""
import numpy as np
import pytest

from gpu_helpers import need_gpu, say, u32
from oracle import pyoracle as O
from paper_2306_08252_amd import inputs as I

pytestmark = pytest.mark.gpu


def same(c, o, label):
    offs, dst, e = c.dump()
    ooffs, odst, _ = o.dump()
    assert e == o.num_edges, label
    np.testing.assert_array_equal(offs.cpu().numpy().astype(np.uint64), ooffs, err_msg=label)
    np.testing.assert_array_equal(u32(dst), odst, err_msg=label)


@pytest.mark.parametrize("B", [1, 4, 16])
def test_cbt_tiny_workload(B):
    gv = need_gpu()
    w = I.tiny_workload()
    n = w["num_vertices"]
    say(f"cbt tiny B={B}")
    c = gv.CbtGraph(n, *w["init"], block_slots=B)
    o = O.OracleGraph(n, *w["init"], block_slots=B)
    same(c, o, "init")
    q = w["query"]
    for j, (s, d) in enumerate(w["insert"]):
        assert c.insert_edges(s, d) == o.insert_edges(s, d)[1], f"insert {j}"
        same(c, o, f"insert {j}")
        np.testing.assert_array_equal(c.edge_exists(*q).cpu().numpy(), o.edge_exists(*q))
    for j, (s, d) in enumerate(w["delete"]):
        assert c.delete_edges(s, d) == o.delete_edges(s, d)[1], f"delete {j}"
        same(c, o, f"delete {j}")
        np.testing.assert_array_equal(c.edge_exists(*q).cpu().numpy(), o.edge_exists(*q))
    # inserting after deletes appends past the holes
    for j, (s, d) in enumerate(w["delete"][:2]):
        assert c.insert_edges(s, d) == o.insert_edges(s, d)[1], f"re-insert {j}"
        same(c, o, f"re-insert {j}")
    c.close()


@pytest.mark.parametrize("B", [8, 32])
def test_cbt_rmat_multitile(B):
    gv = need_gpu()
    w = I.RmatWorkload(14, 1 << 18, name="mt")
    say(f"cbt rmat B={B}")
    c = gv.CbtGraph(w.num_vertices, w.src, w.dst, block_slots=B)
    o = O.OracleGraph(w.num_vertices, w.src, w.dst, block_slots=B)
    same(c, o, "init")
    for j, k in enumerate([10000, 30001, 1, 65536, 4097]):
        s, d = w.insert_batch(k, j)
        assert c.insert_edges(s, d) == o.insert_edges(s, d)[1], f"insert {k}"
        same(c, o, f"insert {k}")
    for j, k in enumerate([10000, 30001, 1, 65536]):
        s, d = w.delete_batch(k, j)
        assert c.delete_edges(s, d) == o.delete_edges(s, d)[1], f"delete {k}"
        same(c, o, f"delete {k}")
    for j, q in enumerate([1, 777, 50001]):
        s, d = w.query_batch(q, j)
        np.testing.assert_array_equal(c.edge_exists(s, d).cpu().numpy(), o.edge_exists(s, d),
                                      err_msg=f"query {q}")
    c.close()


def test_cbt_ids_past_the_graph_and_queue_exhaustion():
    gv = need_gpu()
    rng = np.random.default_rng(7)
    n, B = 1000, 4
    s0 = rng.integers(0, n, 3000).astype(np.uint32)
    d0 = rng.integers(0, n, 3000).astype(np.uint32)
    c = gv.CbtGraph(n, s0, d0, block_slots=B)
    o = O.OracleGraph(n, s0, d0, block_slots=B)
    same(c, o, "init")
    s = rng.integers(0, n + 30, 2000).astype(np.uint32)  # some past the graph
    d = rng.integers(0, n, 2000).astype(np.uint32)
    s[-1] = d[-1] = n - 1
    assert c.insert_edges(s, d) == o.insert_edges(s, d)[1]
    same(c, o, "ids past the graph")
    c.close()
    # a queue with 10 blocks to spare: a batch needing more is refused whole
    spare = 10
    c = gv.CbtGraph(n, s0, d0, block_slots=B, pool_blocks=o.blocks_in_use + spare)
    o2 = O.OracleGraph(n, s0, d0, block_slots=B)
    used = c.blocks()
    big_s = np.repeat(np.arange(200, dtype=np.uint32), 40)
    big_d = np.tile(np.arange(40, dtype=np.uint32) + 500, 200)
    with pytest.raises(gv.GraphVineError) as e:
        c.insert_edges(big_s, big_d)
    assert e.value.code == gv.GV_ENOMEM
    assert c.blocks() == used
    same(c, o2, "after the refused batch")
    # a batch that fits still goes in
    assert c.insert_edges(big_s[:4], big_d[:4]) == o2.insert_edges(big_s[:4], big_d[:4])[1]
    same(c, o2, "after a fitting batch")
    c.close()
