"""Full-size RMAT workload (2^20 vertices, 2^24 distinct edges, batches of
10^6) in the launch configuration the benchmark times (B = 16, default
pool).

Checks, after every operation:
  * the whole canonical dump equals the edge set given by plain set algebra
    on the input keys (union for insert, difference for delete), and the
    batch statistics equal the set sizes;
  * the rows of 256 sampled sources (the 64 largest hubs and 192 random
    vertices) equal the oracle's, run on the same inputs restricted to those
    sources (edges of different sources are independent under edge ops);
  * query answers equal set membership, and the oracle's for sampled sources.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import need_gpu, say, u32
from oracle import pyoracle as O
from paper_2306_08252_amd import inputs as I
from paper_2306_08252_amd import inputs_torch as T

pytestmark = pytest.mark.gpu


def keys_of(s, d):
    return (np.asarray(s, np.uint64) << np.uint64(32)) | np.asarray(d, np.uint64)


def dump_keys(g):
    offs, dst, ck, e = g.dump()
    offs = offs.cpu().numpy().astype(np.int64)
    src = np.repeat(np.arange(len(offs) - 1, dtype=np.uint64), np.diff(offs))
    return keys_of(src, u32(dst)), offs


def test_rmat20_full_size_batches():
    gv = need_gpu()
    scale, m, k = 20, 1 << 24, 10**6
    say("generate RMAT 2^20 / 2^24 on the GPU")
    w = T.RmatWorkload(scale, m, device="cuda:0")
    n = w.num_vertices
    g = gv.Graph(n, w.src, w.dst, block_slots=16)
    src_np, dst_np = u32(w.src), u32(w.dst)
    E = np.unique(keys_of(src_np, dst_np))
    assert len(E) == m

    rng = np.random.default_rng(20)
    deg = np.bincount(src_np, minlength=n)
    sample = np.unique(np.concatenate([np.argsort(deg)[-64:],
                                       rng.integers(0, n, 192)])).astype(np.uint32)
    in_sample = np.zeros(n, bool)
    in_sample[sample] = True
    sel = in_sample[src_np]
    o = O.OracleGraph(n, src_np[sel], dst_np[sel], block_slots=16)

    def check(label):
        say("check", label)
        got, offs = dump_keys(g)
        np.testing.assert_array_equal(got, E, err_msg=label)
        ooffs, odst, _ = o.dump()
        for v in sample:
            a, b = offs[v], offs[v + 1]
            want = odst[ooffs[v]:ooffs[v + 1]]
            np.testing.assert_array_equal((got[a:b] & np.uint64(0xFFFFFFFF)).astype(np.uint32),
                                          want, err_msg=f"{label} row {v}")
        mem = g.memory_used()
        assert mem["num_edges"] == len(E)
        assert g.audit() == 0, label

    check("init")
    s, d = w.insert_batch(k, 0)
    bs, bd = u32(s), u32(d)
    bk = keys_of(bs, bd)
    st = g.insert_edges(s, d)
    E2 = np.union1d(E, bk)
    assert st == (len(E2) - len(E), 0, k - len(np.unique(bk)))
    sel = in_sample[bs]
    o.insert_edges(bs[sel], bd[sel])
    E = E2
    check("insert 1e6")

    s, d = w.delete_batch(k, 0)
    bs, bd = u32(s), u32(d)
    bk = keys_of(bs, bd)
    st = g.delete_edges(s, d)
    E2 = np.setdiff1d(E, bk, assume_unique=False)
    assert st == (len(E) - len(E2), 0, k - len(np.unique(bk)))
    sel = in_sample[bs]
    o.delete_edges(bs[sel], bd[sel])
    E = E2
    check("delete 1e6")

    s, d = w.query_batch(k, 0)
    qs, qd = u32(s), u32(d)
    ans = g.edge_exists(s, d).cpu().numpy()
    np.testing.assert_array_equal(ans, np.isin(keys_of(qs, qd), E).astype(np.uint8))
    sel = in_sample[qs]
    np.testing.assert_array_equal(ans[sel], o.edge_exists(qs[sel], qd[sel]))
    g.close()


def test_batch_beyond_two_kernel_scan():
    """A batch of 2^24 + 12345 pairs: its scans have more tiles than the apply
    kernel adds up itself, so the partials are scanned by a middle kernel.
    Insert, then delete half: the dump equals the set algebra exactly."""
    gv = need_gpu()
    n, k = 1 << 16, (1 << 24) + 12345
    s, d = I.uniform_pairs(I.stream_seed("big-batch"), k, n)
    s0, d0 = I.uniform_pairs(I.stream_seed("big-batch-init"), 100000, n)
    say(f"batch of {k} pairs into 2^16 vertices")
    g = gv.Graph(n, s0, d0, block_slots=16)
    E = np.unique(keys_of(s0, d0))
    bk = keys_of(s, d)
    st = g.insert_edges(s, d)
    E2 = np.union1d(E, bk)
    assert st == (len(E2) - len(E), 0, k - len(np.unique(bk)))
    got, _ = dump_keys(g)
    np.testing.assert_array_equal(got, E2)
    assert g.audit() == 0
    half = k // 2
    st = g.delete_edges(s[:half], d[:half])
    E3 = np.setdiff1d(E2, bk[:half])
    assert st[0] == len(E2) - len(E3)
    got, _ = dump_keys(g)
    np.testing.assert_array_equal(got, E3)
    assert g.audit() == 0
    g.close()
