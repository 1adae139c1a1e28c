"""GPU structure vs. CPU oracle, element by element, through the C ABI.

Bar: bit-exact (integer work).  Every case compares the canonical sorted
adjacency dump, the checksum, the batch statistics, block accounting, the
structural audit and query answers after every batch.
"""
import numpy as np
import pytest

from gpu_helpers import assert_same, gpu_dump, need_gpu, same_answers, say, u32
from oracle import pyoracle as O
from paper_2306_08252_amd import inputs as I

pytestmark = pytest.mark.gpu


# ---------------------------------------------------------------- tiny
@pytest.mark.parametrize("B", [1, 4, 8, 16, 64])
def test_tiny_workload_every_batch(B):
    gv = need_gpu()
    w = I.tiny_workload()
    n = w["num_vertices"]
    say(f"tiny workload B={B}")
    g = gv.Graph(n, *w["init"], block_slots=B)
    o = O.OracleGraph(n, *w["init"], block_slots=B)
    assert_same(g, o, "init")
    for j, (s, d) in enumerate(w["insert"]):
        assert g.insert_edges(s, d) == o.insert_edges(s, d)[1], f"insert {j}"
        assert_same(g, o, f"insert {j}")
        same_answers(g, o, *w["query"], f"query after insert {j}")
    for j, (s, d) in enumerate(w["delete"]):
        assert g.delete_edges(s, d) == o.delete_edges(s, d)[1], f"delete {j}"
        assert_same(g, o, f"delete {j}")
        same_answers(g, o, *w["query"], f"query after delete {j}")
    for v in (0, 1, 17, 513, 1023):
        np.testing.assert_array_equal(u32(g.get_adjacency(v)), o.get_adjacency(v))
    g.close()


# ---------------------------------------------------------------- multi-tile
@pytest.mark.parametrize("B", [8, 16, 32])
def test_rmat_multitile_ragged(B):
    gv = need_gpu()
    scale, m = 14, 1 << 18
    w = I.RmatWorkload(scale, m, name="mt")
    say(f"rmat scale={scale} m={m} B={B}")
    g = gv.Graph(w.num_vertices, w.src, w.dst, block_slots=B)
    o = O.OracleGraph(w.num_vertices, w.src, w.dst, block_slots=B)
    assert_same(g, o, "init")
    for j, k in enumerate([10000, 30001, 1, 65536, 4097]):
        s, d = w.insert_batch(k, j)
        assert g.insert_edges(s, d) == o.insert_edges(s, d)[1], f"insert {k}"
        assert_same(g, o, f"insert {k}")
    for j, k in enumerate([10000, 30001, 1, 65536]):
        s, d = w.delete_batch(k, j)
        assert g.delete_edges(s, d) == o.delete_edges(s, d)[1], f"delete {k}"
        assert_same(g, o, f"delete {k}")
    for j, q in enumerate([1, 777, 50001]):
        same_answers(g, o, *w.query_batch(q, j), f"query {q}")
    deg = np.diff(o.dump()[0].astype(np.int64))
    for v in list(np.argsort(deg)[-3:]) + [5, 1000]:
        np.testing.assert_array_equal(u32(g.get_adjacency(int(v))), o.get_adjacency(int(v)))
    g.close()


@pytest.mark.parametrize("B", [4, 16])
def test_adjacency_around_one_tile(B):
    """Adjacency reads on both sides of the one-workgroup sort (4096 slots)
    and past it, in ascending order, against the oracle."""
    gv = need_gpu()
    n = 1 << 14
    degs = {1: 1, 2: 2, 3: 4095, 4: 4096, 5: 4097, 6: 9000, 7: 0}
    rng = np.random.default_rng(B)
    src = np.concatenate([np.full(dg, v, np.uint32) for v, dg in degs.items()])
    dst = np.concatenate([rng.permutation(n)[:dg].astype(np.uint32) for dg in degs.values()])
    g = gv.Graph(n, src, dst, block_slots=B)
    o = O.OracleGraph(n, src, dst, block_slots=B)
    # deletes leave adjacencies out of order before the reads
    ds, dd = src[::3], dst[::3]
    assert g.delete_edges(ds, dd) == o.delete_edges(ds, dd)[1]
    for v in degs:
        np.testing.assert_array_equal(u32(g.get_adjacency(v)), o.get_adjacency(v),
                                      err_msg=f"vertex {v}")
    g.close()


# ---------------------------------------------------------------- mixed ops
def _ops(rng, n, steps):
    for _ in range(steps):
        kind = rng.choice(["ins", "del", "vins", "vdel", "q"], p=[.35, .3, .1, .1, .15])
        k = int(rng.integers(0, 4 * n))
        hi = 2 * n
        if kind in ("ins", "del", "q"):
            s = rng.integers(0, hi, k).astype(np.uint32)
            d = rng.integers(0, hi, k).astype(np.uint32)
            if k and kind != "q":
                rep = rng.integers(0, k, k // 4)
                s = np.concatenate([s, s[rep]])
                d = np.concatenate([d, d[rep]])
            if k and rng.random() < 0.2:
                s[0] = 0xFFFFFFFF
            yield kind, s, d
        else:
            ids = rng.integers(0, hi + n, int(rng.integers(1, max(2, n // 4)))).astype(np.uint32)
            if rng.random() < 0.2:
                ids[0] = 0xFFFFFFFF
            yield kind, ids, None


@pytest.mark.parametrize("n,B,seed", [(200, 2, 1), (300, 8, 2), (64, 1, 3)])
def test_random_mixed_ops_with_vertex_churn(n, B, seed):
    gv = need_gpu()
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n, 4 * n).astype(np.uint32)
    d = rng.integers(0, n, 4 * n).astype(np.uint32)
    say(f"mixed ops n={n} B={B} seed={seed}")
    g = gv.Graph(n, s, d, block_slots=B)
    o = O.OracleGraph(n, s, d, block_slots=B)
    assert_same(g, o, "init")
    for step, (kind, x, y) in enumerate(_ops(rng, n, 30)):
        label = f"step {step} {kind} len={len(x)}"
        if kind == "ins":
            assert g.insert_edges(x, y) == o.insert_edges(x, y)[1], label
        elif kind == "del":
            assert g.delete_edges(x, y) == o.delete_edges(x, y)[1], label
        elif kind == "vins":
            assert g.insert_vertices(x) == o.insert_vertices(x)[1], label
        elif kind == "vdel":
            assert g.delete_vertices(x) == o.delete_vertices(x)[1], label
        else:
            same_answers(g, o, x, y, label)
        assert_same(g, o, label)
    g.close()


@pytest.mark.parametrize("group,unroll,chunk", [(16, 2, 64), (16, 8, 4096), (64, 2, 128),
                                                 (64, 8, 256), (32, 8, 1024)])
def test_probe_shapes_match_oracle(group, unroll, chunk):
    """Every probe shape the tuning may pick gives the oracle's results: a
    hub of several thousand slots (items of `chunk` slots, long segments)
    and many small sources, through inserts, deletes, queries and vertex
    deletes."""
    gv = need_gpu()
    n, B = 3000, 8
    rng = np.random.default_rng(group * 100 + unroll)
    s = rng.integers(0, n, 6 * n).astype(np.uint32)
    d = rng.integers(0, n, 6 * n).astype(np.uint32)
    s[: 4 * n // 2] = 5  # the hub
    g = gv.Graph(n, s, d, block_slots=B, vertex_capacity=n)
    t = gv.gv_set_tuning(g.h, probe_group=group, probe_unroll=unroll, item_chunk=chunk)
    assert (t["probe_group"], t["probe_unroll"], t["item_chunk"]) == (group, unroll, chunk)
    o = O.OracleGraph(n, s, d, block_slots=B, vertex_capacity=n)
    say(f"probe shape {group}x{unroll}, chunk {chunk}")
    for step in range(6):
        x = rng.integers(0, n, 5000).astype(np.uint32)
        y = rng.integers(0, n, 5000).astype(np.uint32)
        x[:1500] = 5
        assert g.insert_edges(x, y) == o.insert_edges(x, y)[1], step
        same_answers(g, o, x[::3], y[::3], f"query {step}")
        x2, y2 = x[::2], y[::2]
        assert g.delete_edges(x2, y2) == o.delete_edges(x2, y2)[1], step
        ids = rng.integers(6, n, 20).astype(np.uint32)
        assert g.delete_vertices(ids) == o.delete_vertices(ids)[1], step
        assert_same(g, o, f"shape {group}x{unroll} chunk {chunk} step {step}")
    g.close()


# ---------------------------------------------------------------- failures
def test_pool_exhaustion_is_all_or_nothing():
    gv = need_gpu()
    rng = np.random.default_rng(7)
    n, B = 64, 4
    s = rng.integers(0, n, 100).astype(np.uint32)
    d = rng.integers(0, n, 100).astype(np.uint32)
    pool = 4 * B * 60
    g = gv.Graph(n, s, d, block_slots=B, pool_bytes=pool)
    o = O.OracleGraph(n, s, d, block_slots=B, pool_bytes=pool)
    assert g.memory_used()["pool_capacity_blocks"] == o.pool_blocks == 60
    hits = 0
    for step in range(40):
        x = rng.integers(0, n, 40).astype(np.uint32)
        y = rng.integers(0, n, 40).astype(np.uint32)
        rc, st = o.insert_edges(x, y)
        if rc == O.ENOMEM:
            hits += 1
            with pytest.raises(gv.GraphVineError) as e:
                g.insert_edges(x, y)
            assert e.value.code == gv.GV_ENOMEM
        else:
            assert g.insert_edges(x, y) == st, step
        assert_same(g, o, f"step {step}")
        if step % 3 == 2:
            assert g.delete_edges(y, x) == o.delete_edges(y, x)[1]
            assert_same(g, o, f"delete {step}")
    assert hits > 0
    g.close()


def test_async_error_is_sticky_until_sync():
    gv = need_gpu()
    n, B = 32, 4
    g = gv.Graph(n, [0, 1], [1, 2], block_slots=B, pool_bytes=4 * B * 3)
    o = O.OracleGraph(n, [0, 1], [1, 2], block_slots=B, pool_bytes=4 * B * 3)
    big_s = np.repeat(np.arange(8, dtype=np.uint32), 8)
    big_d = np.tile(np.arange(8, 16, dtype=np.uint32), 8)
    assert o.insert_edges(big_s, big_d)[0] == O.ENOMEM
    assert g.insert_edges(big_s, big_d, stats=False) is None  # asynchronous
    assert g.insert_edges([3], [4], stats=False) is None      # later batch still applies
    o.insert_edges([3], [4])
    assert g.sync() == gv.GV_ENOMEM
    assert g.sync() == gv.GV_OK
    assert_same(g, o, "after sticky error")
    g.close()


def test_init_errors_and_argument_checks():
    gv = need_gpu()
    with pytest.raises(gv.GraphVineError) as e:
        gv.Graph(10, [1, 10], [2, 3])
    assert e.value.code == gv.GV_ERANGE
    with pytest.raises(gv.GraphVineError) as e:
        gv.Graph(10, [1], [2], block_slots=12)
    assert e.value.code == gv.GV_EINVAL
    with pytest.raises(gv.GraphVineError) as e:
        gv.Graph(8, [0, 0, 0], [1, 2, 3], block_slots=2, pool_bytes=8)
    assert e.value.code == gv.GV_ENOMEM
    g = gv.Graph(10, [1, 1, 1], [5, 2, 7], block_slots=4)
    with pytest.raises(gv.GraphVineError) as e:
        g.get_adjacency(16)
    assert e.value.code == gv.GV_ERANGE
    import ctypes as C
    import torch
    small = torch.empty(2, dtype=torch.int32, device="cuda:0")
    deg = C.c_uint64()
    rc = gv.lib().gv_get_adjacency(C.c_void_p(g.h), 1, C.c_void_p(small.data_ptr()), 2,
                                   C.byref(deg))
    assert rc == gv.GV_ERANGE and deg.value == 3
    assert g.insert_edges([], []) == (0, 0, 0)
    assert g.delete_edges([], []) == (0, 0, 0)
    assert g.edge_exists([], []).numel() == 0
    g.close()


def test_paper_block_rule_matches_oracle():
    gv = need_gpu()
    w = I.RmatWorkload(12, 1 << 15, name="rule")
    g = gv.Graph(w.num_vertices, w.src, w.dst, block_slots=0)
    o = O.OracleGraph(w.num_vertices, w.src, w.dst, block_slots=0)
    assert g.info()["block_slots"] == o.block_slots
    assert_same(g, o, "paper rule")
    g.close()


# ---------------------------------------------------------------- edge cases
def test_edge_cases_block_boundaries_hubs_and_ids():
    gv = need_gpu()
    B, n = 8, 1 << 10
    g = gv.Graph(n - 3, [], [], block_slots=B, vertex_capacity=n)
    o = O.OracleGraph(n - 3, [], [], block_slots=B, vertex_capacity=n)
    assert_same(g, o, "empty graph")
    # segments of B-1, B and B+1 edges into fresh vertices, then top-ups that
    # cross block boundaries
    for v, k in ((1, B - 1), (2, B), (3, B + 1), (4, 3 * B)):
        s = np.full(k, v, np.uint32)
        d = np.arange(10, 10 + k, dtype=np.uint32)
        assert g.insert_edges(s, d) == o.insert_edges(s, d)[1]
    assert_same(g, o, "boundaries")
    for v in (1, 2, 3, 4):
        s = np.full(B + 1, v, np.uint32)
        d = np.arange(100, 100 + B + 1, dtype=np.uint32)
        assert g.insert_edges(s, d) == o.insert_edges(s, d)[1]
    assert_same(g, o, "top-ups")
    # an all-duplicate batch and a batch of already present edges
    s = np.full(50, 4, np.uint32)
    d = np.full(50, 10, np.uint32)
    assert g.insert_edges(s, d) == o.insert_edges(s, d)[1] == (0, 0, 49)
    # ids beyond the active range, at capacity - 1 (inactive) and 0xFFFFFFFF
    s = np.array([n - 1, n - 3, 0xFFFFFFFF, 5, n + 7], np.uint32)
    d = np.array([1, 2, 3, 0xFFFFFFFF, 1], np.uint32)
    assert g.insert_edges(s, d) == o.insert_edges(s, d)[1]
    assert_same(g, o, "bad ids")
    # make vertex n - 1 active and give it edges
    assert g.insert_vertices([n - 1, n - 2]) == o.insert_vertices([n - 1, n - 2])[1]
    s = np.full(20, n - 1, np.uint32)
    d = np.arange(20, dtype=np.uint32)
    assert g.insert_edges(s, d) == o.insert_edges(s, d)[1]
    assert_same(g, o, "top id")
    # a hub: insert 5000 edges, then delete its whole adjacency in one batch
    hub = 7
    s = np.full(5000, hub, np.uint32)
    d = (np.arange(5000, dtype=np.uint32) * 7919) % (n - 3)
    assert g.insert_edges(s, d) == o.insert_edges(s, d)[1]
    assert_same(g, o, "hub insert")
    adj = o.get_adjacency(hub)
    s = np.full(len(adj), hub, np.uint32)
    assert g.delete_edges(s, adj) == o.delete_edges(s, adj)[1]
    assert_same(g, o, "hub emptied")
    assert g.memory_used()["blocks_in_use"] == o.blocks_in_use
    # absent deletes and deletes of everything twice
    assert g.delete_edges(s, adj) == o.delete_edges(s, adj)[1] == (0, 0, 0)
    # growing the dictionary by a vertex insert beyond capacity
    assert g.insert_vertices([5000]) == o.insert_vertices([5000])[1]
    assert g.info()["vertex_capacity"] == o.capacity == 8192
    assert g.insert_edges([5000, 5000], [1, 2]) == o.insert_edges([5000, 5000], [1, 2])[1]
    assert_same(g, o, "grown dictionary")
    # vertex delete removes in- and out-edges; re-activated vertex is empty
    assert g.delete_vertices([1, 2, 5000]) == o.delete_vertices([1, 2, 5000])[1]
    assert_same(g, o, "vertex delete")
    assert g.insert_vertices([1]) == o.insert_vertices([1])[1]
    assert_same(g, o, "reactivated")
    g.close()


def test_directory_reuse_after_churn():
    """Vertices grow and shrink repeatedly so that freed blocks and directory
    segments are reused; accounting and the audit must stay exact."""
    gv = need_gpu()
    rng = np.random.default_rng(5)
    n, B = 512, 2
    g = gv.Graph(n, [], [], block_slots=B)
    o = O.OracleGraph(n, [], [], block_slots=B)
    for it in range(12):
        vs = rng.integers(0, 16, 3000).astype(np.uint32)
        ds = rng.integers(0, n, 3000).astype(np.uint32)
        assert g.insert_edges(vs, ds) == o.insert_edges(vs, ds)[1]
        assert_same(g, o, f"grow {it}")
        keep = rng.random(3000) < 0.9
        assert g.delete_edges(vs[keep], ds[keep]) == o.delete_edges(vs[keep], ds[keep])[1]
        assert_same(g, o, f"shrink {it}")
    g.close()


@pytest.mark.parametrize("B", [4, 16])
def test_segment_lengths_around_lds_stage(B):
    """Batch segments of lengths around the probe's LDS stage (128 entries)
    and its sampling strides, with repeated pairs, for every operation."""
    gv = need_gpu()
    rng = np.random.default_rng(17)
    n = 1 << 13
    base_s = rng.integers(0, n, 40000).astype(np.uint32)
    base_d = rng.integers(0, n, 40000).astype(np.uint32)
    g = gv.Graph(n, base_s, base_d, block_slots=B)
    o = O.OracleGraph(n, base_s, base_d, block_slots=B)
    lens = [1, 127, 128, 129, 255, 256, 257, 513, 1025, 4097]
    for rep in range(3):
        s_parts, d_parts = [], []
        for j, L in enumerate(lens):
            v = 11 * j + 3 + rep
            d = rng.integers(0, n, L).astype(np.uint32)
            q = L // 4
            if q:
                d[L - q:] = d[:q]  # repeats inside the segment
            s_parts.append(np.full(L, v, np.uint32))
            d_parts.append(d)
        s = np.concatenate(s_parts)
        d = np.concatenate(d_parts)
        perm = rng.permutation(len(s))
        s, d = s[perm], d[perm]
        same_answers(g, o, s, d, f"query rep {rep}")
        assert g.insert_edges(s, d) == o.insert_edges(s, d)[1]
        assert_same(g, o, f"insert rep {rep}")
        same_answers(g, o, s, d, f"query after insert rep {rep}")
        half = len(s) // 2
        assert g.delete_edges(s[:half], d[:half]) == o.delete_edges(s[:half], d[:half])[1]
        assert_same(g, o, f"delete rep {rep}")
        same_answers(g, o, s, d, f"query after delete rep {rep}")
    g.close()


@pytest.mark.parametrize("B", [4, 16])
def test_small_batches_touching_hubs(B):
    """Batches whose size is not a multiple of the 64-lane wave (1 to 127
    pairs) touching sources with tens of work items: the last wave of the
    work-item scan has lanes that do not take part, and every item of a hub
    must still be written (stale items there once sent the probe to wild
    addresses)."""
    gv = need_gpu()
    rng = np.random.default_rng(23)
    n = 1 << 15
    hubs = np.array([0, 5, 77, 4096], np.uint32)
    degs = [41 * 256 + 3, 20 * 256, 5 * 256 + 1, 9000]
    s0 = np.concatenate([np.full(k, h, np.uint32) for h, k in zip(hubs, degs)])
    d0 = np.concatenate([rng.permutation(n)[:k].astype(np.uint32) for k in degs])
    g = gv.Graph(n, s0, d0, block_slots=B)
    o = O.OracleGraph(n, s0, d0, block_slots=B)
    assert_same(g, o, "init")
    for j, size in enumerate([1, 2, 5, 31, 63, 65, 100, 127]):
        s = rng.choice(hubs, size).astype(np.uint32)
        s[: size // 3] = rng.integers(0, n, size // 3).astype(np.uint32)  # some light sources
        d = rng.integers(0, n, size).astype(np.uint32)
        known = rng.integers(0, len(s0), size)
        ds, dd = s.copy(), d.copy()
        ds[size // 2:], dd[size // 2:] = s0[known[size // 2:]], d0[known[size // 2:]]
        say(f"size {size} B={B}")
        same_answers(g, o, ds, dd, f"query {size}")
        assert g.insert_edges(s, d) == o.insert_edges(s, d)[1], f"insert {size}"
        assert_same(g, o, f"insert {size}")
        assert g.delete_edges(ds, dd) == o.delete_edges(ds, dd)[1], f"delete {size}"
        assert_same(g, o, f"delete {size}")
        same_answers(g, o, ds, dd, f"query after delete {size}")
    g.close()


@pytest.mark.parametrize("size", [4095, 4096, 4097, 8192, 12288, 12289])
def test_one_workgroup_sort_boundary(size):
    """Batches on both sides of the single-workgroup pack and sort (one tile
    in LDS, at most 4096 pairs) and a few tiles past it, with invalid pairs,
    repeated pairs and the largest valid key (both endpoints the last id of
    the table)."""
    gv = need_gpu()
    rng = np.random.default_rng(size)
    n, B = 1 << 12, 8
    s0 = rng.integers(0, n, 5 * n).astype(np.uint32)
    d0 = rng.integers(0, n, 5 * n).astype(np.uint32)
    g = gv.Graph(n, s0, d0, block_slots=B)
    o = O.OracleGraph(n, s0, d0, block_slots=B)
    for rep in range(2):
        s = rng.integers(0, n + 50, size).astype(np.uint32)  # some past the table
        d = rng.integers(0, n, size).astype(np.uint32)
        s[: size // 8], d[: size // 8] = s[size // 8: 2 * (size // 8)], d[size // 8: 2 * (size // 8)]
        s[-1] = d[-1] = n - 1
        same_answers(g, o, s, d, f"query {size} rep {rep}")
        assert g.insert_edges(s, d) == o.insert_edges(s, d)[1]
        assert_same(g, o, f"insert {size} rep {rep}")
        assert g.delete_edges(d, s) == o.delete_edges(d, s)[1]
        assert_same(g, o, f"delete {size} rep {rep}")
    g.close()


def test_heavy_grow_sources_are_grown_once():
    """Sources on the edge of the grow kernel's two paths: each needs 9 new
    blocks of B = 4 (grown by a whole wave) while its next 33 pairs would need
    only 8 (a lane's share).  The lane loop must skip them by the planning
    kernel's decision: a record re-read after a wave has grown it would look
    light and the source would be grown twice (degree + 2k, its new blocks
    listed twice).  The heavy sources have the largest ids, so their lane-loop
    visits come last, after millions of light sources (several lane-loop
    rounds per wave), while the first waves to leave the loop grow them.
    Exact comparison by set algebra after each batch."""
    gv = need_gpu()
    rng = np.random.default_rng(4242)
    n, B = 1 << 22, 4
    heavy = np.arange(n - 30000, n, dtype=np.uint32)
    light = rng.choice(n - 30000, 3_000_000, replace=False).astype(np.uint32)

    def rows(src_ids, deg, exclude=None):
        s = np.repeat(src_ids, deg)
        d = rng.integers(0, n, len(s)).astype(np.uint32)
        keys = np.unique((s.astype(np.uint64) << np.uint64(32)) | d.astype(np.uint64))
        if exclude is not None:
            keys = np.setdiff1d(keys, exclude)
        return keys

    def pick(keys, src_ids, per):
        # exactly `per` keys of every source in src_ids (keys sorted)
        s = (keys >> np.uint64(32)).astype(np.uint32)
        first = np.searchsorted(s, src_ids)
        cnt = np.searchsorted(s, src_ids, side="right") - first
        assert (cnt >= per).all()
        idx = (first[:, None] + np.arange(per)[None, :]).ravel()
        return keys[idx]

    def split(keys):
        return (keys >> np.uint64(32)).astype(np.uint32), (keys & np.uint64(0xffffffff)).astype(np.uint32)

    init = np.union1d(pick(rows(heavy, 48), heavy, 36), rows(light, 1))
    g = gv.Graph(n, *split(init), block_slots=B)
    have = init
    for rep in range(2):
        hnew = pick(rows(heavy, 48, have), heavy, 33)
        add = np.union1d(hnew, rows(light, 1, have))
        say(f"heavy grow: batch {rep} with {len(add)} new pairs")
        sh = rng.permutation(len(add))
        st = g.insert_edges(*split(add[sh]))
        assert st == (len(add), 0, 0)
        have = np.union1d(have, add)
        offs, dst, _, e = gpu_dump(g)
        deg = np.diff(offs.astype(np.int64))
        src = np.repeat(np.arange(len(deg), dtype=np.uint64), deg)
        got = (src << np.uint64(32)) | dst.astype(np.uint64)
        if e != len(have):
            twice = np.nonzero(deg[heavy] != 69)[0]
            raise AssertionError(f"batch {rep}: {e} edges, want {len(have)}; "
                                 f"{len(twice)} heavy sources off their degree 69")
        np.testing.assert_array_equal(got, have, err_msg=f"batch {rep}")
        m = g.memory_used()
        assert m["blocks_in_use"] == int(((deg + B - 1) // B).sum())
        assert g.audit() == 0
        # back to 36 entries per heavy source for the next batch
        st = g.delete_edges(*split(hnew))
        assert st[0] == len(hnew)
        have = np.setdiff1d(have, hnew)
    g.close()


@pytest.mark.parametrize("size", [131073, 262143, 262145, 524288, 524289])
def test_one_kernel_scan_boundary(size):
    """Batches on both sides of the one-kernel scans (at most 256 tiles, of
    2048 elements for most scans and 1024 for the work-item scan; 64 for the
    segment scan when it clears the batch counters) and the two-kernel
    scans beyond: inserts, deletes and queries against the oracle, element
    by element."""
    gv = need_gpu()
    rng = np.random.default_rng(size)
    n, B = 1 << 14, 8
    s0 = rng.integers(0, n, 4 * n).astype(np.uint32)
    d0 = rng.integers(0, n, 4 * n).astype(np.uint32)
    g = gv.Graph(n, s0, d0, block_slots=B)
    o = O.OracleGraph(n, s0, d0, block_slots=B)
    for rep in range(2):
        s = rng.integers(0, n, size).astype(np.uint32)
        d = rng.integers(0, n, size).astype(np.uint32)
        same_answers(g, o, s, d, f"query {size} rep {rep}")
        assert g.insert_edges(s, d) == o.insert_edges(s, d)[1]
        assert_same(g, o, f"insert {size} rep {rep}")
        assert g.delete_edges(d[: size // 2], s[: size // 2]) == \
            o.delete_edges(d[: size // 2], s[: size // 2])[1]
        assert_same(g, o, f"delete {size} rep {rep}")
    g.close()
