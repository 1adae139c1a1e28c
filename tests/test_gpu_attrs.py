"""Edge attributes (entries of A words beside each slot) against the oracle.

Bar: bit-exact.  After every batch (inserts, deletes that compact, vertex
deletes that fill holes, attribute writes with repeated and absent pairs)
the words read back for every stored edge and for random pairs equal the
oracle's, as do the statistics of each write and the structure.  At R-MAT
2^16 every edge's words are set to a function of its pair; after deletes
that move entries through every compaction path (lane, wave, workgroup) and
vertex deletes, every remaining edge must still read that function, and new
edges zeros.
"""
import numpy as np
import pytest

from gpu_helpers import assert_same, gpu_dump, need_gpu, say, u32
from oracle import pyoracle as O
from paper_2306_08252_amd import inputs as I

pytestmark = pytest.mark.gpu


def all_edges(g):
    offs, dst, _, _ = gpu_dump(g)
    deg = np.diff(offs.astype(np.int64))
    return np.repeat(np.arange(len(deg), dtype=np.uint32), deg), dst


@pytest.mark.parametrize("B,A", [(4, 1), (16, 3), (1, 2)])
def test_attributes_match_oracle(B, A):
    gv = need_gpu()
    n = 512
    rng = np.random.default_rng(B * 10 + A)
    s0, d0 = I.uniform_pairs(I.stream_seed("attr-init", B, A), 4000, n)
    s0[:600] = 3  # a hub, so deletes take the wave and workgroup paths
    g = gv.Graph(n, s0, d0, block_slots=B, vertex_capacity=n, edge_attr_words=A)
    o = O.OracleGraph(n, s0, d0, block_slots=B, vertex_capacity=n)
    o.set_attr_words(A)

    def check(label):
        assert_same(g, o, label)
        es, ed = all_edges(g)
        qs = np.concatenate([es, rng.integers(0, n + 5, 300).astype(np.uint32)])
        qd = np.concatenate([ed, rng.integers(0, n + 5, 300).astype(np.uint32)])
        f, v = g.get_edge_attrs(qs, qd)
        fo, vo = o.get_edge_attrs(qs, qd)
        np.testing.assert_array_equal(f.cpu().numpy(), fo, err_msg=label)
        np.testing.assert_array_equal(u32(v).reshape(len(qs), A), vo, err_msg=label)

    check("init")
    for r in range(8):
        es, ed = all_edges(g)
        k = len(es)
        pick = rng.integers(0, k, 900)
        # writes: stored pairs (some twice), absent and invalid pairs
        ws = np.concatenate([es[pick], rng.integers(0, n + 5, 200).astype(np.uint32)])
        wd = np.concatenate([ed[pick], rng.integers(0, n + 5, 200).astype(np.uint32)])
        vals = rng.integers(0, 1 << 32, (len(ws), A), dtype=np.uint64).astype(np.uint32)
        assert g.set_edge_attrs(ws, wd, vals) == o.set_edge_attrs(ws, wd, vals)[1], r
        check(f"set {r}")
        # deletes that move entries: half of the hub, random stored pairs
        hub = es == 3
        ds = np.concatenate([es[hub][::2], es[pick[:300]]])
        dd = np.concatenate([ed[hub][::2], ed[pick[:300]]])
        assert g.delete_edges(ds, dd) == o.delete_edges(ds, dd)[1], r
        check(f"delete {r}")
        ids = rng.integers(0, n, 6).astype(np.uint32)
        assert g.delete_vertices(ids) == o.delete_vertices(ids)[1], r
        assert g.insert_vertices(ids) == o.insert_vertices(ids)[1], r
        check(f"vertex delete {r}")
        ins, ind = I.uniform_pairs(I.stream_seed("attr-ins", B, A, r), 1500, n)
        ins[:400] = 3
        assert g.insert_edges(ins, ind) == o.insert_edges(ins, ind)[1], r
        check(f"insert {r}")
    assert g.sync() == 0
    g.close()


def test_attribute_entry_point_errors():
    gv = need_gpu()
    g = gv.Graph(16, [1], [2], block_slots=4)  # no attribute words
    with pytest.raises(gv.GraphVineError):
        g.set_edge_attrs([1], [2], [[1]])
    with pytest.raises(gv.GraphVineError):
        gv.gv_graph_init(16, [1], [2], edge_attr_words=9)
    g.close()


def mix_words(s, d, A):
    """A words per pair, a function of the pair (SplitMix64 output function)."""
    z = (s.astype(np.uint64) << np.uint64(32)) | d.astype(np.uint64)
    out = []
    with np.errstate(over="ignore"):
        for k in range(A):
            x = z + np.uint64(k * 0x9E3779B97F4A7C15 & ((1 << 64) - 1))
            x = (x ^ (x >> np.uint64(30))) * np.uint64(0xbf58476d1ce4e5b9)
            x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94d049bb133111eb)
            x = x ^ (x >> np.uint64(31))
            out.append((x & np.uint64(0xffffffff)).astype(np.uint32))
    return np.stack(out, axis=1)


def test_attributes_follow_entries_at_rmat16():
    gv = need_gpu()
    scale, m, B, A = 16, 1 << 20, 16, 2
    n = 1 << scale
    src, dst = I.rmat_graph(I.stream_seed("attr-rmat", scale), scale, m)
    g = gv.Graph(n, src, dst, block_slots=B, vertex_capacity=n, edge_attr_words=A)
    es, ed = all_edges(g)
    say(f"R-MAT 2^16: {len(es)} edges get words of their pair")
    st = g.set_edge_attrs(es, ed, mix_words(es, ed, A))
    assert st == (len(es), 0, 0)
    rng = np.random.default_rng(16)
    deg = np.bincount(es, minlength=n)
    hubs = np.argsort(deg)[-8:]
    for r in range(3):
        es, ed = all_edges(g)
        # most of the hubs' edges (workgroup path) and a random fifth
        h = np.isin(es, hubs) & (rng.random(len(es)) < 0.7)
        rsel = rng.random(len(es)) < 0.2
        g.delete_edges(es[h | rsel], ed[h | rsel])
        ids = rng.integers(0, n, 200).astype(np.uint32)
        g.delete_vertices(ids)
        g.insert_vertices(ids)
        ns, nd = I.rmat_pairs(I.stream_seed("attr-rmat-ins", r), 50000, scale)
        bs, bd = all_edges(g)
        before = (bs.astype(np.uint64) << np.uint64(32)) | bd.astype(np.uint64)
        g.insert_edges(ns, nd)
        es, ed = all_edges(g)
        f, v = g.get_edge_attrs(es, ed)
        assert f.cpu().numpy().all()
        got = u32(v).reshape(len(es), A)
        old = np.isin((es.astype(np.uint64) << np.uint64(32)) | ed.astype(np.uint64), before)
        np.testing.assert_array_equal(got[old], mix_words(es[old], ed[old], A), err_msg=f"round {r}")
        assert not got[~old].any(), f"round {r}: new edges start at zero"
        # the new edges get their words too, for the next round
        g.set_edge_attrs(es[~old], ed[~old], mix_words(es[~old], ed[~old], A))
        assert g.audit() == 0
        say(f"round {r}: {int(old.sum())} moved or kept entries checked")
    assert g.sync() == 0
    g.close()


def test_block_size_changes_keep_edges_words_and_activity():
    """The block size re-laid over the graph's life (gv_set_block_slots,
    gv_adapt_block_slots) against the oracle: same edges, block accounting
    at the new size, attribute words and inactive vertices kept, plans made
    invalid, a size that does not fit the pool refused with the graph as it
    was."""
    gv = need_gpu()
    n, A = 2000, 2
    s0, d0 = I.uniform_pairs(I.stream_seed("relayout"), 9000, n)
    s0[:3000] = 7
    pool = 4 * 16 * 2400
    g = gv.Graph(n, s0, d0, block_slots=16, vertex_capacity=n, pool_bytes=pool,
                 edge_attr_words=A)
    o = O.OracleGraph(n, s0, d0, block_slots=16, vertex_capacity=n, pool_bytes=pool)
    o.set_attr_words(A)
    dead = np.arange(100, 140, dtype=np.uint32)
    assert g.delete_vertices(dead) == o.delete_vertices(dead)[1]
    es, ed = all_edges(g)
    g.set_edge_attrs(es, ed, mix_words(es, ed, A))
    o.set_edge_attrs(es, ed, mix_words(es, ed, A))
    plan = gv.Plan(g.h, [(0, np.array([1], np.uint32), np.array([2], np.uint32))])
    for B in (4, 1, 16):
        say(f"relayout to B={B}")
        g.set_block_slots(B)
        assert o.set_block_slots(B) == 0
        assert_same(g, o, f"B={B}")
        assert g.info()["block_slots"] == B
        f, v = g.get_edge_attrs(es, ed)
        fo, vo = o.get_edge_attrs(es, ed)
        np.testing.assert_array_equal(f.cpu().numpy(), fo)
        np.testing.assert_array_equal(u32(v).reshape(len(es), A), vo)
        # the deleted vertices stay inactive: their pairs are rejected
        st = g.insert_edges(dead[:5], dead[5:10])
        assert st == o.insert_edges(dead[:5], dead[5:10])[1] and st[1] == 5
        s, d = I.uniform_pairs(I.stream_seed("relayout-ins", B), 3000, n)
        assert g.insert_edges(s, d) == o.insert_edges(s, d)[1]
        assert g.delete_edges(s[::2], d[::2]) == o.delete_edges(s[::2], d[::2])[1]
        assert_same(g, o, f"after batches at B={B}")
    with pytest.raises(gv.GraphVineError) as e:
        plan.launch()
    assert e.value.code == gv.GV_EINVAL
    plan.close()
    b = g.adapt_block_slots()
    assert b == o.adapted_block_slots()
    assert o.set_block_slots(b) == 0
    assert_same(g, o, "adapted")
    # blocks of 1024 slots: 2000 vertices' worth does not fit the budget
    with pytest.raises(gv.GraphVineError) as e:
        g.set_block_slots(1024)
    assert e.value.code == gv.GV_ENOMEM
    assert o.set_block_slots(1024) != 0
    assert_same(g, o, "refused")
    assert g.sync() == 0
    g.close()
