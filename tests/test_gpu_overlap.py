"""Sort overlap (gv_tuning.overlap = 1): a large insert or delete batch packs
and sorts its pairs on the library's second stream while the graph's stream
still runs the batches queued before it.  The results must be the oracle's,
element by element (bit-exact), whatever is queued between the batches:
back-to-back edge batches (the two batch buffers alternate), buffers that
grow, small batches and queries on the graph's stream, vertex batches that
change the activity bitmap the packing reads, and profiling."""
import numpy as np
import pytest
import torch

from gpu_helpers import assert_same, need_gpu, say
from oracle import pyoracle as O
from paper_2306_08252_amd import inputs as I

pytestmark = pytest.mark.gpu


def _host(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("B", [4, 16])
def test_back_to_back_batches_match_oracle(B):
    gv = need_gpu()
    scale, m = 14, 1 << 17
    w = I.RmatWorkload(scale, m, name="ov")
    g = gv.Graph(w.num_vertices, w.src, w.dst, block_slots=B)
    assert gv.gv_set_tuning(g.h, overlap=1)["overlap"] == 1
    o = O.OracleGraph(w.num_vertices, w.src, w.dst, block_slots=B)
    # buffer 0 takes the inserts and buffer 1 the deletes; the 65536-pair
    # batch and the 70000-pair batch make both buffers grow mid-sequence
    sizes = [20000, 5000, 65536, 4097, 30001, 12000, 8000, 70000]
    ins = [tuple(gv.as_device_u32(a, g.device) for a in w.insert_batch(k, j))
           for j, k in enumerate(sizes)]
    dels = [tuple(gv.as_device_u32(a, g.device) for a in w.delete_batch(k, j))
            for j, k in enumerate(sizes)]
    torch.cuda.synchronize()
    say(f"overlap back-to-back B={B}")
    for j in range(len(sizes)):  # no host synchronisation between the calls
        g.insert_edges(*ins[j], stats=False)
        g.delete_edges(*dels[j], stats=False)
    assert g.sync() == 0
    for j in range(len(sizes)):
        o.insert_edges(*map(_host, ins[j]))
        o.delete_edges(*map(_host, dels[j]))
    assert_same(g, o, "after the back-to-back batches")
    # with statistics (a read-back after each batch)
    for j in range(3):
        s, d = w.insert_batch(9000 + j, 50 + j)
        assert g.insert_edges(s, d) == o.insert_edges(s, d)[1], f"insert {j}"
        s, d = w.delete_batch(9000 + j, 50 + j)
        assert g.delete_edges(s, d) == o.delete_edges(s, d)[1], f"delete {j}"
    assert_same(g, o, "after batches with statistics")
    g.close()


def test_interleaved_work_matches_oracle():
    """Queries, small batches and vertex batches between overlapped batches
    (the side stream then waits for the graph's stream), all queued without
    a host synchronisation; query answers are compared at the end with the
    oracle's answers at the same point of the sequence."""
    gv = need_gpu()
    n, B = 6000, 8
    rng = np.random.default_rng(7)
    s0 = rng.integers(0, n, 8 * n).astype(np.uint32)
    d0 = rng.integers(0, n, 8 * n).astype(np.uint32)
    g = gv.Graph(n, s0, d0, block_slots=B, vertex_capacity=2 * n)
    gv.gv_set_tuning(g.h, overlap=1)
    o = O.OracleGraph(n, s0, d0, block_slots=B, vertex_capacity=2 * n)
    say("overlap interleaved")
    answers = []
    ops = []
    for step in range(14):
        kind = ["ins", "del", "q", "small", "vdel", "vins", "ins", "del"][step % 8]
        if kind in ("ins", "del", "q", "small"):
            k = 300 if kind == "small" else int(rng.integers(5000, 40000))
            s = rng.integers(0, 2 * n, k).astype(np.uint32)
            d = rng.integers(0, 2 * n, k).astype(np.uint32)
            if kind != "q":
                rep = rng.integers(0, k, k // 4)  # duplicates within the batch
                s = np.concatenate([s, s[rep]])
                d = np.concatenate([d, d[rep]])
            ops.append((kind, gv.as_device_u32(s, g.device), gv.as_device_u32(d, g.device)))
        else:
            ids = rng.integers(0, 2 * n, 200).astype(np.uint32)
            ops.append((kind, gv.as_device_u32(ids, g.device), None))
    torch.cuda.synchronize()
    for kind, a, b in ops:
        if kind in ("ins", "small"):
            g.insert_edges(a, b, stats=False)
            o.insert_edges(_host(a), _host(b))
        elif kind == "del":
            g.delete_edges(a, b, stats=False)
            o.delete_edges(_host(a), _host(b))
        elif kind == "q":
            answers.append((g.edge_exists(a, b), o.edge_exists(_host(a), _host(b))))
        else:
            # vertex batches through the batched form: no read-back either
            code = gv.OP_DELETE_VERTICES if kind == "vdel" else gv.OP_INSERT_VERTICES
            gv.gv_apply_ops(g.h, [(code, a, None)], g.device)
            (o.delete_vertices if kind == "vdel" else o.insert_vertices)(_host(a))
    assert g.sync() == 0
    for j, (got, want) in enumerate(answers):
        np.testing.assert_array_equal(got.cpu().numpy(), want, err_msg=f"query {j}")
    assert_same(g, o, "after the interleaved sequence")
    g.close()


def test_batched_form_and_profiling_with_overlap():
    """gv_apply_ops runs its edge batches overlapped; a plan recorded with
    overlap on holds the side stream's work as parallel branches and gives
    the oracle's graph, launch after launch; the side stream's launches are
    timed with the graph's profiling."""
    gv = need_gpu()
    scale, m, B = 13, 1 << 16, 8
    w = I.RmatWorkload(scale, m, name="ovb")
    ops = []
    for j in range(6):
        ops.append((gv.OP_INSERT_EDGES, *w.insert_batch(6000 + 1000 * j, j)))
        ops.append((gv.OP_DELETE_EDGES, *w.delete_batch(5000 + 1000 * j, j)))
    ops.insert(5, (gv.OP_DELETE_VERTICES, np.arange(3, 40, 3, dtype=np.uint32), None))
    graphs = []
    for form in ("eager", "plan"):
        g = gv.Graph(w.num_vertices, w.src, w.dst, block_slots=B)
        gv.gv_set_tuning(g.h, overlap=1)
        say(f"overlap batched form {form}")
        if form == "eager":
            gv.gv_profile_enable(g.h, True)
            gv.gv_profile_only(g.h, "sort_pass")
            keep = gv.gv_apply_ops(g.h, ops, g.device)
            assert g.sync() == 0
            launches, ms = gv.gv_kernel_times(g.h, "sort_pass")
            gv.gv_profile_enable(g.h, False)
            del keep
            # 12 edge batches of 2 * 13 = 26-bit keys: 4 passes each
            assert launches == 12 * 4 and ms > 0
        else:
            # recorded with the side stream as a parallel branch; launched
            # twice (the second launch applies the same batches again)
            plan = gv.Plan(g.h, ops, g.device)
            plan.launch()
            plan.launch()
            assert g.sync() == 0
            plan.close()
        graphs.append(g)
    for g, label, times in zip(graphs, ("eager", "plan"), (1, 2)):
        o = O.OracleGraph(w.num_vertices, w.src, w.dst, block_slots=B)
        for _ in range(times):
            for kind, a, b in ops:
                if kind == gv.OP_INSERT_EDGES:
                    o.insert_edges(a, b)
                elif kind == gv.OP_DELETE_EDGES:
                    o.delete_edges(a, b)
                else:
                    o.delete_vertices(a)
        assert_same(g, o, label)
        g.close()


def test_pool_exhaustion_with_overlap_matches_oracle():
    """Overlapped insert batches against a pool that runs out: a batch that
    does not fit changes nothing and leaves a sticky GV_ENOMEM, later
    batches still apply (asynchronous calls), as in the oracle."""
    gv = need_gpu()
    n, B = 4096, 4
    rng = np.random.default_rng(11)
    s0 = rng.integers(0, n, 6000).astype(np.uint32)
    d0 = rng.integers(0, n, 6000).astype(np.uint32)
    pool = 4 * B * 9000
    g = gv.Graph(n, s0, d0, block_slots=B, pool_bytes=pool)
    gv.gv_set_tuning(g.h, overlap=1)
    o = O.OracleGraph(n, s0, d0, block_slots=B, pool_bytes=pool)
    batches = []
    for j in range(8):
        k = 6000 if j != 4 else 40000  # the fifth batch cannot fit
        x = rng.integers(0, n, k).astype(np.uint32)
        y = rng.integers(0, n, k).astype(np.uint32)
        batches.append((gv.as_device_u32(x, g.device), gv.as_device_u32(y, g.device), x, y))
    torch.cuda.synchronize()
    say("overlap pool exhaustion")
    failed = 0
    for j, (tx, ty, x, y) in enumerate(batches):
        g.insert_edges(tx, ty, stats=False)
        rc, _ = o.insert_edges(x, y)
        failed += rc == O.ENOMEM
        if j % 2:
            g.delete_edges(ty[:3000], tx[:3000], stats=False)
            o.delete_edges(y[:3000], x[:3000])
    assert failed >= 1
    assert g.sync() == gv.GV_ENOMEM
    assert g.sync() == gv.GV_OK
    assert_same(g, o, "after the overlapped batches")
    g.close()


def test_coalesced_runs_with_overlap_match_oracle():
    """Runs of edge batches coalesced into mixed lists with the overlap on:
    the gather, packing and sort of a list longer than one sort tile go to
    the side stream while the graph's stream applies the list before (and
    the vertex batch between them).  Vertex deletes and inserts between the
    runs change which entries count (the scan checks activity on the graph's
    stream), and one run names ids past the vertex table.  Eager calls, a
    plan launched around an eager call, all to the oracle's graph."""
    gv = need_gpu()
    scale, m, B = 13, 1 << 16, 8
    w = I.RmatWorkload(scale, m, name="ovc")
    n = w.num_vertices
    rng = np.random.default_rng(5)
    ops = []
    for j in range(7):
        for k in range(2 + j % 3):  # runs of 2 to 4 batches, some within one tile
            size = int(rng.integers(1500, 9000))
            if k % 2 == 0:
                ops.append((gv.OP_INSERT_EDGES, *w.insert_batch(size, 10 * j + k)))
            else:
                ops.append((gv.OP_DELETE_EDGES, *w.delete_batch(size, 10 * j + k)))
        ids = rng.integers(0, n, 60).astype(np.uint32)
        ops.append((gv.OP_DELETE_VERTICES if j % 2 == 0 else gv.OP_INSERT_VERTICES, ids, None))
    s = rng.integers(0, 2 * n, 7000).astype(np.uint32)
    d = rng.integers(0, 2 * n, 7000).astype(np.uint32)
    ops.append((gv.OP_INSERT_EDGES, s, d))
    ops.append((gv.OP_DELETE_EDGES, s[:3000], d[:3000]))
    ops.append((gv.OP_INSERT_EDGES, d[:5000], s[:5000]))

    def oracle(times):
        o = O.OracleGraph(n, w.src, w.dst, block_slots=B)
        for _ in range(times):
            for kind, a, b in ops:
                if kind == gv.OP_INSERT_EDGES:
                    o.insert_edges(a, b)
                elif kind == gv.OP_DELETE_EDGES:
                    o.delete_edges(a, b)
                elif kind == gv.OP_DELETE_VERTICES:
                    o.delete_vertices(a)
                else:
                    o.insert_vertices(a)
        return o

    g = gv.Graph(n, w.src, w.dst, block_slots=B)
    gv.gv_set_tuning(g.h, coalesce=1, overlap=1)
    say("overlap coalesced eager")
    for _ in range(2):
        keep = gv.gv_apply_ops(g.h, ops, g.device)
        assert g.sync() == 0
        del keep
    assert_same(g, oracle(2), "eager, two calls")
    g.close()

    g = gv.Graph(n, w.src, w.dst, block_slots=B)
    gv.gv_set_tuning(g.h, coalesce=1, overlap=1)
    say("overlap coalesced plan")
    plan = gv.Plan(g.h, ops, g.device)
    plan.launch()
    keep = gv.gv_apply_ops(g.h, ops, g.device)
    plan.launch()
    assert g.sync() == 0
    del keep
    plan.close()
    assert_same(g, oracle(3), "plan, eager call, plan")
    g.close()
