"""Served form: mixed update lists (gv_apply_edge_ops) and continuous-batching
ticks against the oracle.

Bar: bit-exact.  A mixed list must leave the graph the oracle leaves after
applying its entries one at a time; a served run must give every query the
answer of the oracle replaying the server's commit order (each tick's writes
in arrival order, then its queries) and end in the same graph.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import assert_same, gpu_dump, need_gpu, say
from oracle import pyoracle as O
from paper_2306_08252_amd import inputs as I

pytestmark = pytest.mark.gpu


def mixed_list(rng, n, m, s0, d0, few=16):
    """Entries with recurring pairs, stored pairs, out-of-range ids and
    unknown op values."""
    s = rng.integers(0, 2 * n + 3, m).astype(np.uint32)
    d = rng.integers(0, 2 * n + 3, m).astype(np.uint32)
    hot = rng.integers(0, n, (few, 2))
    k = rng.integers(0, few, m)
    rec = rng.random(m) < 0.4
    s[rec], d[rec] = hot[k[rec], 0], hot[k[rec], 1]
    pk = rng.integers(0, len(s0), m)
    ex = rng.random(m) < 0.3
    s[ex], d[ex] = s0[pk[ex]], d0[pk[ex]]
    op = rng.choice(np.array([0, 1, 2], np.uint8), m, p=[0.45, 0.45, 0.1])
    return op, s, d


@pytest.mark.parametrize("n,B,seed", [(300, 4, 1), (5000, 16, 2), (1 << 14, 8, 3)])
def test_mixed_lists_match_oracle(n, B, seed):
    gv = need_gpu()
    rng = np.random.default_rng(seed)
    s0 = rng.integers(0, n, 6 * n).astype(np.uint32)
    d0 = rng.integers(0, n, 6 * n).astype(np.uint32)
    g = gv.Graph(n, s0, d0, block_slots=B, vertex_capacity=2 * n)
    o = O.OracleGraph(n, s0, d0, block_slots=B, vertex_capacity=2 * n)
    dead = rng.choice(n, n // 10, replace=False).astype(np.uint32)
    g.delete_vertices(dead)
    o.delete_vertices(dead)
    for rep, m in enumerate([1, 2, 63, 65, 4097, 3 * n]):
        op, s, d = mixed_list(rng, n, m, s0, d0)
        say(f"mixed n={n} B={B} m={m}")
        g.apply_edge_ops(op, s, d)
        assert g.sync() == 0
        o.apply_edge_ops(op, s, d)
        assert_same(g, o, f"mixed rep {rep} m {m}")
    g.close()


@pytest.mark.parametrize("n,B,seed", [(300, 4, 5), (5000, 16, 6)])
def test_mixed_request_stats_match_oracle(n, B, seed):
    """Per-request statistics of one mixed list equal the oracle applying each
    request alone, in order, with the single-batch calls: pairs recurring
    within and across requests, stored pairs, inactive and out-of-range ids,
    an unknown op value, empty requests."""
    gv = need_gpu()
    rng = np.random.default_rng(seed)
    s0 = rng.integers(0, n, 6 * n).astype(np.uint32)
    d0 = rng.integers(0, n, 6 * n).astype(np.uint32)
    g = gv.Graph(n, s0, d0, block_slots=B, vertex_capacity=2 * n)
    o = O.OracleGraph(n, s0, d0, block_slots=B, vertex_capacity=2 * n)
    dead = rng.choice(n, n // 10, replace=False).astype(np.uint32)
    g.delete_vertices(dead)
    o.delete_vertices(dead)
    for rep in range(4):
        reqs = []
        # the last list: a few large requests, each over many workgroups
        big = [int(rng.integers(9000, 30000)), 0, int(rng.integers(3000, 9000)), 2049]
        for r in range(60 if rep < 3 else len(big)):
            size = big[r] if rep == 3 else int(rng.integers(0, 200)) if r % 17 else 0
            op, s, d = mixed_list(rng, n, size, s0, d0, few=8)
            kind = 2 if r % 23 == 5 else int(rng.integers(0, 2))
            reqs.append((kind, s, d))
        op = np.concatenate([np.full(len(x[1]), x[0], np.uint8) for x in reqs])
        s = np.concatenate([x[1] for x in reqs])
        d = np.concatenate([x[2] for x in reqs])
        ends = np.cumsum([len(x[1]) for x in reqs])
        say(f"request stats n={n} B={B} rep {rep}: {len(op)} entries, {len(reqs)} requests")
        keep, st = g.apply_edge_ops_stats(op, s, d, ends)
        assert g.sync() == 0
        got = st.cpu().numpy()
        for r, (kind, a, b) in enumerate(reqs):
            if kind == 0:
                want = o.insert_edges(a, b)[1]
            elif kind == 1:
                want = o.delete_edges(a, b)[1]
            else:
                want = (0, len(a), 0)
            assert tuple(int(x) for x in got[r]) == tuple(want), f"rep {rep} request {r}"
        assert_same(g, o, f"request stats rep {rep}")
    g.close()


def test_served_ticks_match_oracle_replay():
    gv = need_gpu()
    from paper_2306_08252_amd import served as S
    scale, m, B = 12, 1 << 16, 8
    n = 1 << scale
    s0, d0 = I.rmat_graph(I.stream_seed("served-test", scale), scale, m)
    g = gv.Graph(n, s0, d0, block_slots=B, vertex_capacity=n)
    o = O.OracleGraph(n, s0, d0, block_slots=B, vertex_capacity=n)
    rng = np.random.default_rng(8)
    dev = g.device
    reqs, host = [], []
    for j in range(120):
        kind = int(rng.choice(5, p=[0.35, 0.35, 0.2, 0.05, 0.05]))
        size = int(np.exp(rng.random() * np.log(3000))) + 1
        if j == 90:
            # ids past the table: this vertex insert grows it, waiting for
            # the running ticks (the others are queued without a wait)
            host.append((S.VINSERT, np.array([n + 1, n + 7, 3], np.uint32), None))
        elif kind in (S.VINSERT, S.VDELETE):
            ids = rng.integers(0, n, min(size, 40)).astype(np.uint32)
            host.append((kind, ids, None))
        else:
            pk = rng.integers(0, len(s0), size)
            s = np.where(rng.random(size) < 0.6, s0[pk], rng.integers(0, n, size)).astype(np.uint32)
            d = np.where(rng.random(size) < 0.6, d0[pk], rng.integers(0, n, size)).astype(np.uint32)
            host.append((kind, s, d))
    for kind, a, b in host:
        ta = torch.from_numpy(a.view(np.int32)).to(dev)
        tb = None if b is None else torch.from_numpy(b.view(np.int32)).to(dev)
        reqs.append((kind, ta, tb))
    done, ticks, answers = S.serve(g, reqs, None, max_tick_pairs=6000, keep_answers=True)
    say(f"{len(reqs)} requests in {len(ticks)} ticks")
    assert len(ticks) > 10 and max(e - f for f, e in ticks) > 2  # ticks do mix requests
    for f, e in ticks:
        kinds = [host[i][0] for i in range(f, e)]
        if kinds[0] in (S.VINSERT, S.VDELETE):
            assert e == f + 1
            if kinds[0] == S.VINSERT:
                o.insert_vertices(host[f][1])
            else:
                o.delete_vertices(host[f][1])
            continue
        ws = [host[i] for i in range(f, e) if host[i][0] in (S.INSERT, S.DELETE)]
        if ws:
            op = np.concatenate([np.full(len(w[1]), w[0], np.uint8) for w in ws])
            o.apply_edge_ops(op, np.concatenate([w[1] for w in ws]),
                             np.concatenate([w[2] for w in ws]))
        for i in range(f, e):
            if host[i][0] == S.QUERY:
                np.testing.assert_array_equal(answers[i], o.edge_exists(host[i][1], host[i][2]),
                                              err_msg=f"query {i}")
    assert_same(g, o, "after the served run")
    assert np.all(np.diff(done) >= 0)
    g.close()


def test_mixed_list_past_the_pool_is_sticky_and_consistent():
    """A mixed list whose inserts do not fit: gv_sync reports GV_ENOMEM once,
    the deletes of the list are applied, the inserts are not, and the graph
    stays consistent."""
    gv = need_gpu()
    rng = np.random.default_rng(9)
    n, B = 64, 4
    s0 = rng.integers(0, n, 100).astype(np.uint32)
    d0 = rng.integers(0, n, 100).astype(np.uint32)
    pool = 4 * B * 60
    g = gv.Graph(n, s0, d0, block_slots=B, pool_bytes=pool)
    o = O.OracleGraph(n, s0, d0, block_slots=B, pool_bytes=pool)
    m = 600
    s = rng.integers(0, n, m).astype(np.uint32)
    d = rng.integers(0, n, m).astype(np.uint32)
    op = (rng.random(m) < 0.2).astype(np.uint8)  # mostly inserts: past the pool
    s[:40], d[:40], op[:40] = s0[:40], d0[:40], 1  # and some stored pairs deleted
    last = {}
    for i in range(m):
        last[(int(s[i]), int(d[i]))] = int(op[i])
    gone = [k for k, v in last.items() if v == 1]
    g.apply_edge_ops(op, s, d)
    with pytest.raises(gv.GraphVineError) as e:
        gv._check(g.sync(), "gv_sync")
    assert e.value.code == gv.GV_ENOMEM
    assert g.sync() == 0  # reported once
    o.delete_edges(np.array([k[0] for k in gone], np.uint32),
                   np.array([k[1] for k in gone], np.uint32))
    assert_same(g, o, "deletes applied, inserts not")
    g.close()


def test_served_admission_by_free_blocks():
    """A pool with little room: inserts wait for ticks whose bounds fit the
    free blocks, an insert too large for the whole free pool is rejected,
    no tick runs out of pool, and the graph equals the oracle replaying the
    admitted requests in commit order."""
    gv = need_gpu()
    from paper_2306_08252_amd import served as S
    rng = np.random.default_rng(10)
    n, B = 256, 4
    s0 = rng.integers(0, n, 600).astype(np.uint32)
    d0 = rng.integers(0, n, 600).astype(np.uint32)
    pool = 4 * B * 1200
    g = gv.Graph(n, s0, d0, block_slots=B, pool_bytes=pool, vertex_capacity=n)
    o = O.OracleGraph(n, s0, d0, block_slots=B, pool_bytes=pool, vertex_capacity=n)
    dev = g.device
    host = []
    for j in range(60):
        kind = int(rng.choice(3, p=[0.5, 0.3, 0.2]))
        size = int(rng.integers(1, 120))
        if j == 30:
            kind, size = S.INSERT, 5000  # bound past the whole pool
        s = rng.integers(0, n, size).astype(np.uint32)
        d = rng.integers(0, n, size).astype(np.uint32)
        if kind == S.DELETE:
            pk = rng.integers(0, len(s0), size)
            s, d = s0[pk], d0[pk]
        host.append((kind, s, d))
    reqs = [(k, torch.from_numpy(a.view(np.int32)).to(dev), torch.from_numpy(b.view(np.int32)).to(dev))
            for k, a, b in host]
    rejected = []
    done, ticks, answers = S.serve(g, reqs, None, max_tick_pairs=400, keep_answers=True,
                                   rejected=rejected)
    assert g.sync() == 0  # no tick ran out of pool
    assert 30 in rejected
    assert sum(e - f for f, e in ticks) + len(rejected) == len(reqs)
    for f, e in ticks:
        ws = [host[i] for i in range(f, e) if host[i][0] in (S.INSERT, S.DELETE)]
        if ws:
            op = np.concatenate([np.full(len(w[1]), w[0], np.uint8) for w in ws])
            o.apply_edge_ops(op, np.concatenate([w[1] for w in ws]),
                             np.concatenate([w[2] for w in ws]))
        for i in range(f, e):
            if host[i][0] == S.QUERY:
                np.testing.assert_array_equal(answers[i], o.edge_exists(host[i][1], host[i][2]))
    assert_same(g, o, "after admission-controlled serving")
    g.close()


def _requests(rng, n, count, s0, d0, dev, max_size, vertex_share=0.05):
    """Seeded requests of log-uniform size: edge inserts and deletes (60 % of
    their pairs stored ones), queries, vertex inserts and deletes."""
    from paper_2306_08252_amd import served as S
    host = []
    p = [0.4 - vertex_share / 2, 0.4 - vertex_share / 2, 0.2, vertex_share / 2, vertex_share / 2]
    for _ in range(count):
        kind = int(rng.choice(5, p=p))
        size = max(1, int(np.exp(rng.random() * np.log(max_size))))
        if kind in (S.VINSERT, S.VDELETE):
            host.append((kind, rng.integers(0, n, min(size, 200)).astype(np.uint32), None))
        else:
            pk = rng.integers(0, len(s0), size)
            own = rng.random(size) < 0.6
            s = np.where(own, s0[pk], rng.integers(0, n, size)).astype(np.uint32)
            d = np.where(own, d0[pk], rng.integers(0, n, size)).astype(np.uint32)
            host.append((kind, s, d))
    reqs = [(k, torch.from_numpy(a.view(np.int32)).to(dev),
             None if b is None else torch.from_numpy(b.view(np.int32)).to(dev))
            for k, a, b in host]
    return host, reqs


def test_served_request_alone_equals_in_the_mix():
    """Every request's result is the same alone as in the mix: a second
    graph, from the same initial state, applies the requests one at a time,
    each alone with the single-batch calls, in the server's commit order (a
    tick's writes in arrival order, then its queries); every query answered
    in a mixed tick equals the same query run alone on that graph at its
    commit point, every insert or delete request's statistics from its
    mixed tick equal those of the same request alone, and both graphs end
    equal.  The ticks overlap on the device (several in flight)."""
    gv = need_gpu()
    from paper_2306_08252_amd import served as S
    scale, m, B = 16, 1 << 20, 16
    n = 1 << scale
    s0, d0 = I.rmat_graph(I.stream_seed("served-alone", scale), scale, m)
    g = gv.Graph(n, s0, d0, block_slots=B, vertex_capacity=n)
    alone = gv.Graph(n, s0, d0, block_slots=B, vertex_capacity=n)
    rng = np.random.default_rng(11)
    host, reqs = _requests(rng, n, 300, s0, d0, g.device, 10**4)
    stats = {}
    done, ticks, answers = S.serve(g, reqs, None, max_tick_pairs=20000, keep_answers=True,
                                   max_inflight=3, stats=stats)
    assert g.sync() == 0
    say(f"{len(reqs)} requests in {len(ticks)} ticks")
    assert max(e - f for f, e in ticks) > 3  # ticks mix requests
    checked = 0
    for f, e in ticks:
        order = [i for i in range(f, e) if host[i][0] != S.QUERY] + \
                [i for i in range(f, e) if host[i][0] == S.QUERY]
        for i in order:
            kind, a, b = host[i]
            if kind == S.INSERT:
                assert stats[i] == tuple(alone.insert_edges(a, b)), f"insert request {i}"
            elif kind == S.DELETE:
                assert stats[i] == tuple(alone.delete_edges(a, b)), f"delete request {i}"
            elif kind == S.VINSERT:
                alone.insert_vertices(a)
            elif kind == S.VDELETE:
                alone.delete_vertices(a)
            else:
                np.testing.assert_array_equal(answers[i], alone.edge_exists(a, b).cpu().numpy(),
                                              err_msg=f"query request {i}")
                checked += 1
    assert checked > 30
    oa, da, ca, ea = gpu_dump(g)
    ob, db, cb, eb = gpu_dump(alone)
    assert ea == eb and ca == cb
    np.testing.assert_array_equal(oa, ob)
    np.testing.assert_array_equal(da, db)
    g.close()
    alone.close()


@pytest.mark.timeout(900)
def test_served_rmat20_against_oracle_replay():
    """The served form on R-MAT 2^20 vertices / 2^24 edges: requests of
    log-uniform size in [1, 10^5] (40 / 40 / 15 / 5 inserts / deletes /
    queries / vertex batches), overlapping ticks; every query answer and the
    final graph equal the CPU oracle replaying the server's commit order."""
    gv = need_gpu()
    from paper_2306_08252_amd import inputs_torch as T
    from paper_2306_08252_amd import served as S
    scale, m, B = 20, 1 << 24, 16
    say("generate R-MAT 2^20 / 2^24 on the GPU")
    w = T.RmatWorkload(scale, m, name="served-replay", device="cuda:0")
    n = w.num_vertices
    s0, d0 = gv_u32(w.src), gv_u32(w.dst)
    g = gv.Graph(n, w.src, w.dst, block_slots=B, vertex_capacity=n)
    rng = np.random.default_rng(20)
    host, reqs = _requests(rng, n, 200, s0, d0, g.device, 10**5)
    done, ticks, answers = S.serve(g, reqs, None, max_tick_pairs=1 << 20, keep_answers=True)
    assert g.sync() == 0
    say(f"{len(reqs)} requests in {len(ticks)} ticks; oracle replay")
    o = O.OracleGraph(n, s0, d0, block_slots=B, vertex_capacity=n)
    for f, e in ticks:
        if host[f][0] in (S.VINSERT, S.VDELETE):
            (o.insert_vertices if host[f][0] == S.VINSERT else o.delete_vertices)(host[f][1])
            continue
        ws = [host[i] for i in range(f, e) if host[i][0] in (S.INSERT, S.DELETE)]
        if ws:
            op = np.concatenate([np.full(len(x[1]), x[0], np.uint8) for x in ws])
            o.apply_edge_ops(op, np.concatenate([x[1] for x in ws]),
                             np.concatenate([x[2] for x in ws]))
        for i in range(f, e):
            if host[i][0] == S.QUERY:
                np.testing.assert_array_equal(answers[i], o.edge_exists(host[i][1], host[i][2]),
                                              err_msg=f"query request {i}")
    assert_same(g, o, "after the served run")
    g.close()


def gv_u32(t):
    return t.detach().cpu().numpy().view(np.uint32)
