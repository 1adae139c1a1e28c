"""Shared helpers for the GPU parity tests: compare the GPU structure, read
through the C ABI, with the CPU oracle."""
import numpy as np
import pytest
import torch

from oracle import pyoracle as O


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_08252_amd import graphvine as gv
    gv.lib()  # raises loudly if the HIP library is missing
    return gv


def say(*a):
    print(*a, flush=True)


def u32(t):
    return t.detach().cpu().numpy().view(np.uint32)


def gpu_dump(g):
    offs, dst, ck, e = g.dump()
    return offs.cpu().numpy().astype(np.uint64), u32(dst), ck, e


def assert_same(g, o, label=""):
    """Canonical dump, checksum, edge count, block accounting and the
    structural audit all agree with the oracle."""
    offs, dst, ck, e = gpu_dump(g)
    ooffs, odst, ock = o.dump()
    assert e == o.num_edges, label
    assert g.info()["vertex_capacity"] == o.capacity, label
    np.testing.assert_array_equal(offs, ooffs, err_msg=label)
    np.testing.assert_array_equal(dst, odst, err_msg=label)
    assert ck == ock, label
    m = g.memory_used()
    assert m["blocks_in_use"] == o.blocks_in_use, label
    assert m["num_edges"] == o.num_edges, label
    assert g.audit() == 0, label


def same_answers(g, o, s, d, label=""):
    got = g.edge_exists(s, d).cpu().numpy()
    want = o.edge_exists(s, d)
    np.testing.assert_array_equal(got, want, err_msg=label)


# ---------------------------------------------------------------- set algebra
def keys_of(s, d):
    return (np.asarray(s, np.uint64) << np.uint64(32)) | np.asarray(d, np.uint64)


def mix64_sum(keys):
    """sum of the SplitMix64 output function over keys, modulo 2^64."""
    total = np.uint64(0)
    c1, c2 = np.uint64(0xbf58476d1ce4e5b9), np.uint64(0x94d049bb133111eb)
    with np.errstate(over="ignore"):  # arithmetic modulo 2^64 is the definition
        for lo in range(0, len(keys), 1 << 24):
            z = keys[lo:lo + (1 << 24)].astype(np.uint64)
            z = (z ^ (z >> np.uint64(30))) * c1
            z = (z ^ (z >> np.uint64(27))) * c2
            z = z ^ (z >> np.uint64(31))
            total = total + np.sum(z, dtype=np.uint64)
    return int(total)


class EdgeSet:
    """The expected edge set by set algebra: sorted unique keys and the
    active vertices."""

    def __init__(self, n, src, dst):
        self.n = n
        self.active = np.ones(n, bool)
        self.E = np.unique(keys_of(src, dst))

    def _valid(self, s, d):
        s = np.asarray(s, np.uint64)
        d = np.asarray(d, np.uint64)
        ok = (s < self.n) & (d < self.n)
        ok[ok] &= self.active[s[ok].astype(np.int64)] & self.active[d[ok].astype(np.int64)]
        return keys_of(s[ok], d[ok])

    def insert(self, s, d):
        new = np.unique(self._valid(s, d))
        pos = np.searchsorted(self.E, new)
        have = pos < len(self.E)
        have[have] = self.E[pos[have]] == new[have]
        new = new[~have]
        self.E = np.insert(self.E, np.searchsorted(self.E, new), new)
        return len(new)

    def delete(self, s, d):
        k = np.unique(self._valid(s, d))
        pos = np.searchsorted(self.E, k)
        hit = pos < len(self.E)
        hit[hit] = self.E[pos[hit]] == k[hit]
        self.E = np.delete(self.E, pos[hit])
        return int(hit.sum())

    def delete_vertices(self, ids):
        dead = np.zeros(self.n, bool)
        ids = np.asarray(ids, np.int64)
        dead[ids[ids < self.n]] = True
        dead &= self.active
        src = (self.E >> np.uint64(32)).astype(np.int64)
        dst = (self.E & np.uint64(0xffffffff)).astype(np.int64)
        self.E = self.E[~(dead[src] | dead[dst])]
        self.active &= ~dead

    def insert_vertices(self, ids):
        ids = np.asarray(ids, np.int64)
        self.active[ids[ids < self.n]] = True
