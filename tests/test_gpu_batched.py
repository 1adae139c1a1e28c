"""Batched form: a sequence of uneven batches recorded into one HIP graph
(gv_plan_*) against the same sequence applied one batch at a time
(gv_apply_ops) and against the oracle.

Bar: bit-exact.  A plan is launched several times, with the eager path and
synchronisations between launches; after every launch the planned graph,
the eagerly updated graph and the oracle agree (canonical dump, checksum,
block accounting, audit).
"""
import numpy as np
import pytest

from gpu_helpers import assert_same, gpu_dump, need_gpu, say
from oracle import pyoracle as O
from paper_2306_08252_amd import inputs as I

pytestmark = pytest.mark.gpu


def op_sequence(seed, n, count, max_pairs, vertex_share=0.1, known=None):
    """Seeded ops: sizes log-uniform in [1, max_pairs], inserts and deletes
    of edges in equal parts, vertex inserts/deletes at `vertex_share`."""
    draws = I.splitmix64(seed, 4 * count + 8)
    ops = []
    for j in range(count):
        u = float(draws[4 * j] >> np.uint64(11)) / float(1 << 53)
        size = max(1, int(round(np.exp(u * np.log(max_pairs)))))
        r = float(draws[4 * j + 1] >> np.uint64(11)) / float(1 << 53)
        sub = I.stream_seed("batched-op", seed, j)
        if r < vertex_share:
            ids = (I.splitmix64(sub, min(size, 64)) % np.uint64(n)).astype(np.uint32)
            kind = 2 if r < vertex_share / 2 else 3
            ops.append((kind, ids, None))
        else:
            s, d = I.uniform_pairs(sub, size, n)
            if r < (1 + vertex_share) / 2:
                ops.append((0, s, d))
            else:
                if known is not None and len(known[0]):
                    # half of a delete batch names stored pairs
                    idx = (I.splitmix64(sub + 1, size // 2) % np.uint64(len(known[0]))).astype(np.int64)
                    s = np.concatenate([known[0][idx], s[: size - size // 2]])
                    d = np.concatenate([known[1][idx], d[: size - size // 2]])
                ops.append((1, s, d))
    return ops


def oracle_apply(o, ops):
    for kind, a, b in ops:
        if kind == 0:
            o.insert_edges(a, b)
        elif kind == 1:
            o.delete_edges(a, b)
        elif kind == 2:
            o.insert_vertices(a)
        else:
            o.delete_vertices(a)


@pytest.mark.parametrize("B,coalesce,max_run", [(4, 0, 0), (16, 0, 0), (4, 1, 0), (16, 1, 0),
                                                 (16, 1, 1500)])
def test_plan_matches_eager_and_oracle(B, coalesce, max_run):
    """With coalescing, every run of edge batches is one mixed list (capped at
    max_run pairs); the result must still be the batches in order."""
    gv = need_gpu()
    n = 1024
    s0, d0 = I.uniform_pairs(I.stream_seed("batched-init", B), 6000, n)
    ops = op_sequence(I.stream_seed("batched-ops", B), n, 40, 700, known=(s0, d0))
    # a pair inserted then deleted, and deleted then inserted, within one run
    ops[1:1] = [(0, np.array([5, 6], np.uint32), np.array([7, 8], np.uint32)),
                (1, np.array([5, 9], np.uint32), np.array([7, 9], np.uint32)),
                (0, np.array([9], np.uint32), np.array([9], np.uint32)),
                (0, np.array([], np.uint32), np.array([], np.uint32))]
    say(f"plan vs eager vs oracle, B={B}, coalesce={coalesce}/{max_run}, {len(ops)} ops")
    ga = gv.Graph(n, s0, d0, block_slots=B, vertex_capacity=n)
    gb = gv.Graph(n, s0, d0, block_slots=B, vertex_capacity=n)
    for g in (ga, gb):
        t = gv.gv_set_tuning(g.h, coalesce=coalesce, max_run_pairs=max_run)
        assert t["coalesce"] == coalesce and gv.gv_get_tuning(g.h) == t
    o = O.OracleGraph(n, s0, d0, block_slots=B, vertex_capacity=n)
    plan = gv.Plan(gb.h, ops)
    for rnd in range(3):
        gv.gv_apply_ops(ga.h, ops)
        assert ga.sync() == 0
        plan.launch()
        assert gb.sync() == 0
        oracle_apply(o, ops)
        assert_same(ga, o, f"eager round {rnd}")
        assert_same(gb, o, f"plan round {rnd}")
    plan.close()
    ga.close()
    gb.close()


def test_plan_rmat_uneven_batches():
    """R-MAT 2^16 with batches of 10^0..10^5 pairs; the planned graph equals
    the eagerly updated one after each of two launches.  (Batches of a few
    pairs on hubs once left work items unwritten in a partial wave.)"""
    gv = need_gpu()
    scale, m, B = 16, 1 << 20, 16
    n = 1 << scale
    src, dst = I.rmat_graph(I.stream_seed("batched-rmat", scale), scale, m)
    ops = op_sequence(I.stream_seed("batched-rmat-ops"), n, 64, 10**5, known=(src, dst))
    say(f"rmat 2^{scale}: {len(ops)} ops, {sum(len(a) for _, a, _ in ops)} items")
    ga = gv.Graph(n, src, dst, block_slots=B, vertex_capacity=n)
    gb = gv.Graph(n, src, dst, block_slots=B, vertex_capacity=n)
    plan = gv.Plan(gb.h, ops)
    for rnd in range(2):
        gv.gv_apply_ops(ga.h, ops)
        plan.launch()
        assert ga.sync() == 0 and gb.sync() == 0
        oa, da, ca, ea = gpu_dump(ga)
        ob, db, cb, eb = gpu_dump(gb)
        assert ea == eb and ca == cb, rnd
        np.testing.assert_array_equal(oa, ob)
        np.testing.assert_array_equal(da, db)
        assert ga.memory_used() == gb.memory_used()
        assert gb.audit() == 0
    plan.close()
    ga.close()
    gb.close()


def test_plan_errors():
    gv = need_gpu()
    n = 256
    s0, d0 = I.uniform_pairs(I.stream_seed("batched-err"), 500, n)
    g = gv.Graph(n, s0, d0, block_slots=8, vertex_capacity=n)
    # a vertex insert past the fixed table fails the run, stickily
    plan = gv.Plan(g.h, [(2, np.array([n + 5], np.uint32), None)])
    plan.launch()
    with pytest.raises(gv.GraphVineError) as e:
        gv._check(g.sync(), "gv_sync")
    assert e.value.code == gv.GV_ERANGE
    assert g.sync() == 0  # reported once
    plan.close()
    # a plan with a vertex delete stays valid as the graph gains edges (its
    # buffers are sized for a full pool); the first batch of this size sizes
    # the scratch, so the second one reallocates nothing
    s, d = I.uniform_pairs(I.stream_seed("batched-err-more"), 300, n)
    g.insert_edges(s, d)
    o = O.OracleGraph(n, s0, d0, block_slots=8, vertex_capacity=n)
    o.insert_edges(s, d)
    plan = gv.Plan(g.h, [(3, np.array([1, 2], np.uint32), None)])
    s2, d2 = I.uniform_pairs(I.stream_seed("batched-err-more2"), 300, n)
    g.insert_edges(s2, d2)
    o.insert_edges(s2, d2)
    plan.launch()
    assert g.sync() == 0
    o.delete_vertices([1, 2])
    assert_same(g, o, "plan with a vertex delete after growth")
    plan.close()
    # buffers moved (a larger single batch grew the scratch): recreate
    plan = gv.Plan(g.h, [(0, s[:10], d[:10])])
    big_s, big_d = I.uniform_pairs(I.stream_seed("batched-err-big"), 200000, n)
    g.insert_edges(big_s, big_d)
    with pytest.raises(gv.GraphVineError) as e:
        plan.launch()
    assert e.value.code == gv.GV_EINVAL
    plan.close()
    g.close()


def test_tuning_rejects_bad_values():
    gv = need_gpu()
    g = gv.Graph(64, [1], [2], block_slots=8)
    with pytest.raises(gv.GraphVineError):
        gv.gv_set_tuning(g.h, coalesce=2)
    with pytest.raises(gv.GraphVineError):
        gv.gv_set_tuning(g.h, small_sort_max=4097)
    for bad in ({"probe_group": 8}, {"probe_unroll": 3}, {"item_chunk": 100},
                {"item_chunk": 8192}, {"overlap": 2}):
        with pytest.raises(gv.GraphVineError):
            gv.gv_set_tuning(g.h, **bad)
    assert gv.gv_get_tuning(g.h) == {"coalesce": 0, "max_run_pairs": 0, "small_sort_max": 4096,
                                     "probe_group": 32, "probe_unroll": 4, "item_chunk": 256,
                                     "overlap": 0}
    g.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("coalesce", [0, 1])
def test_plan_rmat22_full_size_against_set_algebra(coalesce):
    """The batched-form workload at its size: R-MAT 2^22 vertices / 2^26
    edges, 256 batches of log-uniform size in [10^2, 10^6] (45 / 45 / 10 edge
    inserts / edge deletes / vertex batches), recorded into one plan and
    launched once.  The whole edge set afterwards equals set algebra applying
    the batches in order (and the dump's checksum the sum computed from those
    keys); rows of sampled sources equal the CPU oracle applying the same
    batches restricted to those sources (vertex batches in full)."""
    gv = need_gpu()
    from gpu_helpers import EdgeSet, keys_of, mix64_sum, u32
    from paper_2306_08252_amd import inputs_torch as T
    from paper_2306_08252_amd import workloads as Wk
    scale, m, B = 22, 1 << 26, 16
    say("generate R-MAT 2^22 / 2^26 and 256 uneven batches on the GPU")
    w = T.RmatWorkload(scale, m, name="batched", device="cuda:0")
    n = w.num_vertices
    ops, pairs, vids = Wk.batched_ops(w, "batched", 256, "cuda:0")
    g = gv.Graph(n, w.src, w.dst, block_slots=B, vertex_capacity=n)
    gv.gv_set_tuning(g.h, coalesce=coalesce)
    plan = gv.Plan(g.h, ops)
    plan.launch()
    assert g.sync() == 0
    plan.close()
    say(f"plan applied: {pairs} pairs, {vids} vertex ids; set algebra")
    src, dst = u32(w.src), u32(w.dst)
    S = EdgeSet(n, src, dst)
    rng = np.random.default_rng(22)
    deg0 = np.bincount(src, minlength=n)
    sample = np.unique(np.concatenate([np.argsort(deg0)[-24:], rng.integers(0, n, 100)]))
    in_sample = np.zeros(n, bool)
    in_sample[sample] = True
    sel = in_sample[src]
    o = O.OracleGraph(n, src[sel], dst[sel], block_slots=B, vertex_capacity=n)
    for kind, a, b in ops:
        a = u32(a)
        if kind in (0, 1):
            b = u32(b)
            r = in_sample[a]
            if kind == 0:
                S.insert(a, b)
                o.insert_edges(a[r], b[r])
            else:
                S.delete(a, b)
                o.delete_edges(a[r], b[r])
        elif kind == 2:
            S.insert_vertices(a)
            o.insert_vertices(a)
        else:
            S.delete_vertices(a)
            o.delete_vertices(a)
    offs, gdst, ck, e = gpu_dump(g)
    deg = np.diff(offs.astype(np.int64))
    keys = keys_of(np.repeat(np.arange(len(deg), dtype=np.uint64), deg), gdst)
    assert e == len(S.E), f"{e} edges, want {len(S.E)}"
    np.testing.assert_array_equal(keys, S.E, err_msg="whole edge set")
    assert ck == mix64_sum(S.E)
    ooffs, odst, _ = o.dump()
    for v in sample:
        np.testing.assert_array_equal(gdst[offs[v]:offs[v + 1]], odst[ooffs[v]:ooffs[v + 1]],
                                      err_msg=f"row {v}")
    assert g.memory_used()["blocks_in_use"] == int(((deg + B - 1) // B).sum())
    assert g.audit() == 0
    g.close()
