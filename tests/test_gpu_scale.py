"""Scale workloads: R-MAT with 2^24 vertices and 2^28 edges, and the road-like
4096 x 4096 lattice, with batches of 10^7 edges and of 10^4 vertices.

The whole edge set is checked after every operation, exactly: the expected
set is kept by set algebra on sorted uint64 keys (src << 32 | dst) -- union
with the valid new pairs of an insert, difference with a delete, removal of
every edge touching a deleted vertex, re-activation of an inserted vertex --
and the dump must equal it key for key; the dump's checksum must equal
sum(mix64(key)) mod 2^64 computed here from those keys (SplitMix64 output
function, written out in numpy).  Rows of sampled sources (the largest hubs
plus random vertices) are also compared with the CPU oracle run on the same
inputs restricted to those sources, and block accounting and the structural
audit are checked.
"""
import numpy as np
import pytest
from gpu_helpers import EdgeSet, keys_of, mix64_sum, need_gpu, say, u32
from oracle import pyoracle as O
from paper_2306_08252_amd import inputs as I
from paper_2306_08252_amd import inputs_torch as T

pytestmark = pytest.mark.gpu


class Checker:
    def __init__(self, g, n, src, dst, B, sample):
        self.g, self.n, self.B = g, n, B
        self.sample = sample
        self.in_sample = np.zeros(n, bool)
        self.in_sample[sample] = True
        sel = self.in_sample[src]
        self.o = O.OracleGraph(n, src[sel], dst[sel], block_slots=B)
        self.S = EdgeSet(n, src, dst)
        self.edges = None

    def restrict(self, s, d):
        sel = self.in_sample[s]
        return s[sel], d[sel]

    def check(self, label):
        say("check", label)
        g = self.g
        offs, dst, ck, e = g.dump()
        offs = offs.cpu().numpy().astype(np.int64)
        dst = u32(dst)
        deg = np.diff(offs)
        src = np.repeat(np.arange(len(deg), dtype=np.uint64), deg)
        keys = keys_of(src, dst)
        bad = np.nonzero(keys[1:] <= keys[:-1])[0]
        if len(bad):  # sorted, no duplicates; else say where
            u = (keys[bad[:8] + 1] >> np.uint64(32)).astype(np.int64)
            detail = [(int(v), int(keys[i + 1] & np.uint64(0xffffffff)), int(deg[v]))
                      for v, i in zip(u, bad[:8])]
            raise AssertionError(f"{label}: {len(bad)} order violations in {len(np.unique(u))}+ "
                                 f"rows; (src, dst, degree): {detail}; sync={g.sync()}")
        assert len(keys) == len(self.S.E), f"{label}: {len(keys)} edges, want {len(self.S.E)}"
        np.testing.assert_array_equal(keys, self.S.E, err_msg=f"{label}: whole edge set")
        assert ck == mix64_sum(self.S.E), f"{label}: checksum"
        mem = g.memory_used()
        assert mem["num_edges"] == e == len(dst)
        B = self.B
        assert mem["blocks_in_use"] == int(((deg + B - 1) // B).sum()), label
        assert g.audit() == 0, label
        ooffs, odst, _ = self.o.dump()
        for v in self.sample:
            np.testing.assert_array_equal(dst[offs[v]:offs[v + 1]],
                                          odst[ooffs[v]:ooffs[v + 1]], err_msg=f"{label} {v}")
        self.edges = e
        return keys


@pytest.mark.timeout(900)
def test_rmat24_scale():
    gv = need_gpu()
    scale, m, B = 24, 1 << 28, 16
    say("generate R-MAT 2^24 / 2^28 on the GPU")
    w = T.RmatWorkload(scale, m, name="scale", device="cuda:0")
    n = w.num_vertices
    g = gv.Graph(n, w.src, w.dst, block_slots=B)
    src, dst = u32(w.src), u32(w.dst)
    deg0 = np.bincount(src, minlength=n)
    rng = np.random.default_rng(24)
    sample = np.unique(np.concatenate([np.argsort(deg0)[-32:],
                                       rng.integers(0, n, 96)])).astype(np.uint32)
    C = Checker(g, n, src, dst, B, sample)
    C.check("init")
    assert C.edges == m
    k = 10**7
    s, d = w.insert_batch(k, 0)
    st = g.insert_edges(s, d)
    C.o.insert_edges(*C.restrict(u32(s), u32(d)))
    assert st[0] == C.S.insert(u32(s), u32(d))
    e0 = C.edges
    C.check("insert 1e7")
    assert C.edges == e0 + st[0] and st[1] == 0
    s, d = w.delete_batch(k, 0)
    st = g.delete_edges(s, d)
    C.o.delete_edges(*C.restrict(u32(s), u32(d)))
    assert st[0] == C.S.delete(u32(s), u32(d))
    e0 = C.edges
    C.check("delete 1e7")
    assert C.edges == e0 - st[0] and st[0] > 0
    # vertex batches of 10^4: delete (in- and out-edges), then re-insert
    ids = rng.choice(n, 10**4, replace=False).astype(np.uint32)
    ids[:8] = sample[:8]  # some sampled rows lose their out-edges
    st = g.delete_vertices(ids)
    assert st == C.o.delete_vertices(ids)[1]
    C.S.delete_vertices(ids)
    C.check("vertex delete 1e4")
    st = g.insert_vertices(ids)
    assert st == C.o.insert_vertices(ids)[1]
    C.S.insert_vertices(ids)
    C.check("vertex insert 1e4")
    qs, qd = w.query_batch(10**6, 0)
    ans = g.edge_exists(qs, qd).cpu().numpy()
    sel = C.in_sample[u32(qs)]
    np.testing.assert_array_equal(ans[sel], C.o.edge_exists(u32(qs)[sel], u32(qd)[sel]))
    # every answer against membership in the expected set
    qk = keys_of(u32(qs), u32(qd))
    pos = np.minimum(np.searchsorted(C.S.E, qk), len(C.S.E) - 1)
    np.testing.assert_array_equal(ans, (C.S.E[pos] == qk).astype(np.uint8), err_msg="queries")
    g.close()


@pytest.mark.timeout(900)
def test_lattice_road_scale():
    gv = need_gpu()
    side, B = 4096, 8
    n = side * side
    say("generate lattice 4096^2")
    src, dst = I.lattice_graph(I.stream_seed("road", side), side)
    g = gv.Graph(n, src, dst, block_slots=B)
    rng = np.random.default_rng(4096)
    sample = np.unique(rng.integers(0, n, 128)).astype(np.uint32)
    C = Checker(g, n, src, dst, B, sample)

    def symmetric(keys):
        rev = (keys << np.uint64(32)) | (keys >> np.uint64(32))
        return np.array_equal(keys, np.sort(rev))

    assert symmetric(C.check("init"))
    say("average degree", C.edges / n)
    k = 10**7 // 2  # each undirected update is stored in both directions
    a, b = I.uniform_pairs(I.stream_seed("road-ins", side), k, n)
    s, d = np.concatenate([a, b]), np.concatenate([b, a])
    st = g.insert_edges(s, d)
    C.o.insert_edges(*C.restrict(s, d))
    assert st[0] == C.S.insert(s, d)
    e0 = C.edges
    assert symmetric(C.check("insert 1e7"))
    assert C.edges == e0 + st[0]
    # delete half of the inserted pairs and a slice of the lattice, both ways
    a2, b2 = a[: k // 2], b[: k // 2]
    la, lb = src[: k // 2], dst[: k // 2]
    s = np.concatenate([a2, b2, la, lb])
    d = np.concatenate([b2, a2, lb, la])
    st = g.delete_edges(s, d)
    C.o.delete_edges(*C.restrict(s, d))
    assert st[0] == C.S.delete(s, d)
    e0 = C.edges
    assert symmetric(C.check("delete 1e7"))
    assert C.edges == e0 - st[0]
    ids = rng.choice(n, 10**4, replace=False).astype(np.uint32)
    assert g.delete_vertices(ids) == C.o.delete_vertices(ids)[1]
    C.S.delete_vertices(ids)
    assert symmetric(C.check("vertex delete 1e4"))
    assert g.insert_vertices(ids) == C.o.insert_vertices(ids)[1]
    C.S.insert_vertices(ids)
    C.check("vertex insert 1e4")
    g.close()
