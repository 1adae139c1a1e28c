"""Second, independent model of the graph operations: a dense boolean
adjacency matrix over the whole vertex dictionary, for tiny graphs only.

It is used to pin the ordered-set oracle.  It shares nothing with it: the
representation (matrix vs. ordered sets), the duplicate handling (numpy
unique vs. std::set) and the checksum (Python integers vs. C uint64) are all
written separately here.
"""
import numpy as np

MAX_CAPACITY = 1 << 31
MASK64 = (1 << 64) - 1


def py_mix64(z):
    """SplitMix64 output function in Python integer arithmetic."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def pow2_at_least(x):
    p = 1
    while p < x:
        p *= 2
    return p


def ceil_div(a, b):
    return -(-a // b)


class BruteGraph:
    def __init__(self, num_vertices, src, dst, vertex_capacity=0, block_slots=16,
                 pool_bytes=0):
        src = np.asarray(src, np.int64)
        dst = np.asarray(dst, np.int64)
        if len(src) and (src.max() >= num_vertices or dst.max() >= num_vertices):
            raise ValueError("id out of range")
        self.cap = pow2_at_least(max(num_vertices, vertex_capacity, 1))
        self.A = np.zeros((self.cap, self.cap), dtype=bool)
        self.active = np.zeros(self.cap, dtype=bool)
        self.active[:num_vertices] = True
        self.A[src, dst] = True
        assert block_slots > 0
        self.B = block_slots
        self.pool_bytes = pool_bytes
        self.pool_blocks = pool_bytes // (4 * block_slots) if pool_bytes else 0
        self.W = None  # attribute words per (src, dst), when enabled

    def set_attr_words(self, words):
        self.W = np.zeros((self.cap, self.cap, words), dtype=np.uint32)

    def set_block_slots(self, block_slots):
        pool = self.pool_bytes // (4 * block_slots) if self.pool_bytes else 0
        need = int(sum(ceil_div(int(x), block_slots) for x in self.A.sum(axis=1)))
        if pool and need > pool:
            return 3
        self.B, self.pool_blocks = block_slots, pool
        return 0

    def adapted_block_slots(self):
        deg = self.A.sum(axis=1)
        nz = int((deg > 0).sum())
        if nz == 0:
            return 8
        return max(8, min(64, pow2_at_least(ceil_div(int(deg.sum()), nz))))

    def set_edge_attrs(self, src, dst, vals):
        src = np.asarray(src, np.int64)
        dst = np.asarray(dst, np.int64)
        vals = np.asarray(vals, np.uint32).reshape(len(src), -1)
        inb = (src < self.cap) & (dst < self.cap)
        ok = np.zeros(len(src), dtype=bool)
        ok[inb] = self.active[src[inb]] & self.active[dst[inb]]
        idx = np.nonzero(ok)[0]
        code = src[idx] * self.cap + dst[idx]
        # the last row of each pair: first occurrence in the reversed order
        _, first_rev = np.unique(code[::-1], return_index=True)
        last = idx[::-1][first_rev]
        stored = self.A[src[last], dst[last]]
        keep = last[stored]
        self.W[src[keep], dst[keep]] = vals[keep]
        return 0, (int(stored.sum()), int((~ok).sum()), len(idx) - len(last))

    def get_edge_attrs(self, src, dst):
        found = self.edge_exists(src, dst)
        src = np.asarray(src, np.int64)
        dst = np.asarray(dst, np.int64)
        out = np.zeros((len(src), self.W.shape[2]), dtype=np.uint32)
        f = found.astype(bool)
        out[f] = self.W[src[f], dst[f]]
        return found, out

    # ---- helpers -------------------------------------------------------
    def _grow(self, cap):
        if cap <= self.cap:
            return
        A = np.zeros((cap, cap), dtype=bool)
        A[: self.cap, : self.cap] = self.A
        if self.W is not None:
            W = np.zeros((cap, cap, self.W.shape[2]), dtype=np.uint32)
            W[: self.cap, : self.cap] = self.W
            self.W = W
        act = np.zeros(cap, dtype=bool)
        act[: self.cap] = self.active
        self.A, self.active, self.cap = A, act, cap

    def _valid_pairs(self, src, dst):
        src = np.asarray(src, np.int64)
        dst = np.asarray(dst, np.int64)
        inb = (src < self.cap) & (dst < self.cap)
        ok = np.zeros(len(src), dtype=bool)
        ok[inb] = self.active[src[inb]] & self.active[dst[inb]]
        s, d = src[ok], dst[ok]
        uniq = np.unique(s * self.cap + d)
        return int((~ok).sum()), len(s) - len(uniq), uniq // self.cap, uniq % self.cap

    def blocks_in_use(self):
        return int(sum(ceil_div(int(x), self.B) for x in self.A.sum(axis=1)))

    # ---- operations ----------------------------------------------------
    def insert_edges(self, src, dst):
        rej, dup, s, d = self._valid_pairs(src, dst)
        new = ~self.A[s, d]
        if self.pool_blocks:
            A2 = self.A.copy()
            A2[s[new], d[new]] = True
            need = int(sum(ceil_div(int(x), self.B) for x in A2.sum(axis=1)))
            if need > self.pool_blocks:
                return 3, (0, 0, 0)
        self.A[s[new], d[new]] = True
        if self.W is not None:
            self.W[s[new], d[new]] = 0
        return 0, (int(new.sum()), rej, dup)

    def delete_edges(self, src, dst):
        rej, dup, s, d = self._valid_pairs(src, dst)
        hit = self.A[s, d]
        self.A[s[hit], d[hit]] = False
        if self.W is not None:
            self.W[s[hit], d[hit]] = 0
        return 0, (int(hit.sum()), rej, dup)

    def insert_vertices(self, ids):
        ids = np.asarray(ids, np.int64)
        ok = ids < MAX_CAPACITY
        good = ids[ok]
        if len(good):
            self._grow(pow2_at_least(int(good.max()) + 1))
        u = np.unique(good)
        fresh = ~self.active[u]
        self.active[u[fresh]] = True
        return 0, (int(fresh.sum()), int((~ok).sum()), len(good) - len(u))

    def delete_vertices(self, ids):
        ids = np.asarray(ids, np.int64)
        ok = ids < self.cap
        good = ids[ok]
        u = np.unique(good)
        gone = u[self.active[u]]
        self.A[gone, :] = False
        self.A[:, gone] = False
        if self.W is not None:
            self.W[gone, :] = 0
            self.W[:, gone] = 0
        self.active[gone] = False
        return 0, (len(gone), int((~ok).sum()), len(good) - len(u))

    def edge_exists(self, src, dst):
        src = np.asarray(src, np.int64)
        dst = np.asarray(dst, np.int64)
        out = np.zeros(len(src), dtype=np.uint8)
        inb = (src < self.cap) & (dst < self.cap)
        out[inb] = (self.active[src[inb]] & self.A[src[inb], dst[inb]]).astype(np.uint8)
        return out

    def get_adjacency(self, v):
        return np.nonzero(self.A[v])[0].astype(np.uint32)

    def dump(self):
        deg = self.A.sum(axis=1).astype(np.uint64)
        offs = np.zeros(self.cap + 1, dtype=np.uint64)
        offs[1:] = np.cumsum(deg)
        u, v = np.nonzero(self.A)  # row-major: ascending (u, v)
        h = 0
        for a, b in zip(u.tolist(), v.tolist()):
            h = (h + py_mix64((a << 32) | b)) & MASK64
        return offs, v.astype(np.uint32), h
