"""Seeded synthetic inputs for the dynamic-graph workloads.

This module only draws input data: edge lists, update batches and query
batches.  It holds none of the graph structure's arithmetic, so both the GPU
path and the CPU oracle can consume what it produces.

Every random number comes from SplitMix64 (Steele, Lea, Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014) used as a counter
based generator: draw i of stream s is mix64(s + (i + 1) * GAMMA).  Streams are
named; a name is hashed with FNV-1a 64 and then mixed, so every stream of every
workload is reproducible on any machine.

Workloads (stand-ins for the paper's DIMACS inputs, Sec. 5, Table 1, which are
not available here):
  * uniform random directed pairs without self-loops (tiny graph);
  * R-MAT (Chakrabarti, Zhan, Faloutsos 2004) with (a, b, c, d) =
    (0.57, 0.19, 0.19, 0.05): the skewed degree distribution of the
    co-papers graphs;
  * a 2-D lattice with 10 % of its edges removed and 1 % long-range edges
    added, stored in both directions: the mesh / road class.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK32 = np.uint64(0xFFFFFFFF)

RMAT_ABC = (0.57, 0.19, 0.19)


# --------------------------------------------------------------------------
# counter-based generator
# --------------------------------------------------------------------------
def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Draws start .. start+n-1 of the SplitMix64 sequence seeded with `seed`."""
    idx = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GAMMA
    return mix64(state)


def stream_seed(*names) -> int:
    """64-bit seed of a named stream: FNV-1a 64 of the joined name, mixed."""
    text = "/".join(str(x) for x in names).encode()
    h = 0xCBF29CE484222325
    for byte in text:
        h ^= byte
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return int(mix64(np.array([h], dtype=np.uint64))[0])


def _below(r32: np.ndarray, n: int) -> np.ndarray:
    """Map 32-bit uniforms to [0, n) by multiply-shift."""
    return ((r32 & _MASK32) * np.uint64(n)) >> np.uint64(32)


# --------------------------------------------------------------------------
# pair generators
# --------------------------------------------------------------------------
def uniform_pairs(seed: int, n: int, num_vertices: int, self_loops: bool = False):
    """n uniform directed pairs in [0, num_vertices)^2, in stream order.

    Draw i gives src from its high 32 bits and dst from its low 32 bits.
    Without self_loops, draws with src == dst are skipped."""
    out_s, out_d, have, start = [], [], 0, 0
    out_s.append(np.zeros(0, np.uint64))
    out_d.append(np.zeros(0, np.uint64))
    while have < n:
        want = (n - have) + (n - have) // 8 + 64
        r = splitmix64(seed, want, start)
        start += want
        s = _below(r >> np.uint64(32), num_vertices)
        d = _below(r, num_vertices)
        if not self_loops:
            keep = s != d
            s, d = s[keep], d[keep]
        s, d = s[: n - have], d[: n - have]
        out_s.append(s)
        out_d.append(d)
        have += len(s)
    return (np.concatenate(out_s).astype(np.uint32),
            np.concatenate(out_d).astype(np.uint32))


def rmat_thresholds(a=RMAT_ABC[0], b=RMAT_ABC[1], c=RMAT_ABC[2]):
    """Integer quadrant thresholds floor(p * 2^32) for cumulative a, a+b, a+b+c."""
    return (int(a * 2**32), int((a + b) * 2**32), int((a + b + c) * 2**32))


def rmat_pairs_raw(seed: int, n: int, scale: int, start: int = 0,
                   abc=RMAT_ABC):
    """Pairs start .. start+n-1 of the R-MAT stream (self-loops included).

    Pair i uses ceil(scale / 2) draws; level l (0 = most significant bit)
    reads the high half of draw l // 2 for even l and the low half for odd l.
    Quadrant q = [u >= t1] + [u >= t2] + [u >= t3] in 0..3, i.e.
    u < t1 -> (0,0); u < t2 -> (0,1); u < t3 -> (1,0); otherwise (1,1);
    the source bit is q >> 1 and the destination bit q & 1."""
    t1, t2, t3 = (np.uint32(t) for t in rmat_thresholds(*abc))
    w = (scale + 1) // 2
    src = np.zeros(n, dtype=np.uint32)
    dst = np.zeros(n, dtype=np.uint32)
    weights = (np.uint32(1) << np.arange(scale - 1, -1, -1, dtype=np.uint32))
    chunk = 1 << 21
    for c0 in range(0, n, chunk):
        m = min(chunk, n - c0)
        r = splitmix64(seed, m * w, (start + c0) * w).reshape(m, w)
        u = np.empty((m, 2 * w), dtype=np.uint32)
        u[:, 0::2] = (r >> np.uint64(32)).astype(np.uint32)
        u[:, 1::2] = (r & _MASK32).astype(np.uint32)
        u = u[:, :scale]
        q = ((u >= t1).astype(np.uint8) + (u >= t2).astype(np.uint8)
             + (u >= t3).astype(np.uint8))
        src[c0:c0 + m] = ((q >> 1).astype(np.uint32) * weights).sum(axis=1, dtype=np.uint32)
        dst[c0:c0 + m] = ((q & 1).astype(np.uint32) * weights).sum(axis=1, dtype=np.uint32)
    return src, dst


def rmat_pairs(seed: int, n: int, scale: int, abc=RMAT_ABC):
    """The first n R-MAT pairs of the stream that are not self-loops."""
    out_s, out_d, have, start = [], [], 0, 0
    out_s.append(np.zeros(0, np.uint32))
    out_d.append(np.zeros(0, np.uint32))
    while have < n:
        want = (n - have) + (n - have) // 16 + 64
        s, d = rmat_pairs_raw(seed, want, scale, start, abc)
        start += want
        keep = s != d
        s, d = s[keep][: n - have], d[keep][: n - have]
        out_s.append(s)
        out_d.append(d)
        have += len(s)
    return np.concatenate(out_s), np.concatenate(out_d)


def rmat_graph(seed: int, scale: int, m: int, abc=RMAT_ABC):
    """The first m distinct, non-self-loop pairs of the R-MAT stream, in
    stream order (a deduplicated directed R-MAT graph with m edges)."""
    total = m + m // 4 + 1024
    while True:
        s, d = rmat_pairs_raw(seed, total, scale, 0, abc)
        keys = (s.astype(np.uint64) << np.uint64(32)) | d.astype(np.uint64)
        ok = np.nonzero(s != d)[0]
        _, first = np.unique(keys[ok], return_index=True)
        if len(first) >= m:
            pos = ok[np.sort(first)[:m]]
            return s[pos].copy(), d[pos].copy()
        total += total // 2


def permutation(seed: int, n: int) -> np.ndarray:
    """A seeded permutation of range(n): indices ordered by their draw."""
    return np.argsort(splitmix64(seed, n), kind="stable")


def lattice_graph(seed: int, side: int, remove_frac: float = 0.10,
                  long_frac: float = 0.01):
    """Road-like graph: side x side 4-neighbour lattice, exactly
    floor(remove_frac * E) of its undirected edges removed (those with the
    smallest draws), then floor(long_frac * kept) distinct uniform long-range
    undirected edges that are neither self-loops nor lattice neighbours.
    Returned as directed pairs, both directions of every undirected edge."""
    n = side * side
    r = np.arange(side, dtype=np.int64)
    rr, cc = np.meshgrid(r, r, indexing="ij")
    v = (rr * side + cc)
    h_u, h_v = v[:, :-1].ravel(), v[:, 1:].ravel()
    v_u, v_v = v[:-1, :].ravel(), v[1:, :].ravel()
    eu = np.concatenate([h_u, v_u])
    ev = np.concatenate([h_v, v_v])
    e0 = len(eu)
    drop = int(remove_frac * e0)
    order = permutation(stream_seed(seed, "lattice-remove"), e0)
    kept = np.sort(order[drop:])
    eu, ev = eu[kept], ev[kept]
    want = int(long_frac * len(eu))
    lu_all, lv_all = [], []
    have, start_batch = 0, 0
    seen = np.zeros(0, dtype=np.uint64)
    while have < want:
        k = (want - have) * 2 + 1024
        a, b = uniform_pairs(stream_seed(seed, "lattice-long", start_batch), k, n)
        start_batch += 1
        a = a.astype(np.int64)
        b = b.astype(np.int64)
        ra, ca = a // side, a % side
        rb, cb = b // side, b % side
        neighbour = (np.abs(ra - rb) + np.abs(ca - cb)) == 1
        a, b = a[~neighbour], b[~neighbour]
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        key = (lo.astype(np.uint64) << np.uint64(32)) | hi.astype(np.uint64)
        # keep first occurrences in stream order, and nothing seen before
        _, first = np.unique(key, return_index=True)
        first = np.sort(first)
        key, lo, hi = key[first], lo[first], hi[first]
        fresh = ~np.isin(key, seen)
        key, lo, hi = key[fresh], lo[fresh], hi[fresh]
        take = min(want - have, len(key))
        lu_all.append(lo[:take])
        lv_all.append(hi[:take])
        seen = np.concatenate([seen, key[:take]])
        have += take
    lu = np.concatenate(lu_all) if lu_all else np.zeros(0, np.int64)
    lv = np.concatenate(lv_all) if lv_all else np.zeros(0, np.int64)
    uu = np.concatenate([eu, lu])
    vv = np.concatenate([ev, lv])
    src = np.concatenate([uu, vv]).astype(np.uint32)
    dst = np.concatenate([vv, uu]).astype(np.uint32)
    return src, dst


# --------------------------------------------------------------------------
# batch builders
# --------------------------------------------------------------------------
def shuffle_pairs(seed: int, src: np.ndarray, dst: np.ndarray):
    p = permutation(seed, len(src))
    return src[p], dst[p]


def pick(seed: int, n: int, src: np.ndarray, dst: np.ndarray):
    """n pairs drawn with replacement from the list (src, dst)."""
    idx = _below(splitmix64(seed, n) >> np.uint64(32), len(src)).astype(np.int64)
    return src[idx], dst[idx]


def absent_uniform(seed: int, n: int, num_vertices: int, known_keys: np.ndarray):
    """n uniform non-self-loop pairs whose (src << 32 | dst) key is not in the
    sorted array known_keys (draws that hit it are skipped)."""
    out_s, out_d, have, part = [], [], 0, 0
    while have < n:
        s, d = uniform_pairs(stream_seed(seed, part), 2 * (n - have) + 64, num_vertices)
        part += 1
        k = (s.astype(np.uint64) << np.uint64(32)) | d.astype(np.uint64)
        pos = np.searchsorted(known_keys, k)
        pos = np.minimum(pos, max(len(known_keys) - 1, 0))
        hit = (known_keys[pos] == k) if len(known_keys) else np.zeros(len(k), bool)
        s, d = s[~hit][: n - have], d[~hit][: n - have]
        out_s.append(s)
        out_d.append(d)
        have += len(s)
    return np.concatenate(out_s), np.concatenate(out_d)


def pair_keys(src, dst):
    return (np.asarray(src, np.uint64) << np.uint64(32)) | np.asarray(dst, np.uint64)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
def tiny_workload(seed: int = 0, num_vertices: int = 1024, num_edges: int = 8192,
                  batches: int = 4, batch: int = 1024, queries: int = 1024):
    """Tiny directed graph: uniform pairs without self-loops (duplicates kept
    in the raw list), insert batches of uniform pairs, delete batches that are
    half drawn from known pairs and half absent pairs, and a query batch that
    is half known pairs and half uniform pairs."""
    w = {"num_vertices": num_vertices}
    w["init"] = uniform_pairs(seed, num_edges, num_vertices)
    w["insert"] = [uniform_pairs(stream_seed("tiny", seed, "insert", j), batch,
                                 num_vertices) for j in range(batches)]
    known_s = np.concatenate([w["init"][0]] + [b[0] for b in w["insert"]])
    known_d = np.concatenate([w["init"][1]] + [b[1] for b in w["insert"]])
    known = np.unique(pair_keys(known_s, known_d))
    dels = []
    for j in range(batches):
        es, ed = pick(stream_seed("tiny", seed, "delete-existing", j), batch // 2,
                      known_s, known_d)
        as_, ad = absent_uniform(stream_seed("tiny", seed, "delete-absent", j),
                                 batch - batch // 2, num_vertices, known)
        dels.append(shuffle_pairs(stream_seed("tiny", seed, "delete-mix", j),
                                  np.concatenate([es, as_]), np.concatenate([ed, ad])))
    w["delete"] = dels
    qs, qd = pick(stream_seed("tiny", seed, "query-existing"), queries // 2,
                  known_s, known_d)
    us, ud = uniform_pairs(stream_seed("tiny", seed, "query-uniform"),
                           queries - queries // 2, num_vertices)
    w["query"] = shuffle_pairs(stream_seed("tiny", seed, "query-mix"),
                               np.concatenate([qs, us]), np.concatenate([qd, ud]))
    return w


class RmatWorkload:
    """Directed R-MAT graph of 2^scale vertices and m distinct edges, with
    insert batches drawn from the same R-MAT distribution, delete batches of
    which `exist_frac` are edges of the initial graph (disjoint across batches
    while they last) and the rest uniform pairs, and query batches half
    initial edges and half uniform pairs."""

    def __init__(self, scale: int = 20, m: int = 1 << 24, name: str = "rmat",
                 exist_frac: float = 0.8):
        self.scale = scale
        self.num_vertices = 1 << scale
        self.m = m
        self.name = f"{name}{scale}-{m}"
        self.exist_frac = exist_frac
        self.src, self.dst = rmat_graph(stream_seed(self.name, "graph"), scale, m)
        self._perm = None
        self._perm_pos = 0

    def insert_batch(self, k: int, j: int):
        return rmat_pairs(stream_seed(self.name, "insert", k, j), k, self.scale)

    def _take_existing(self, n: int):
        if self._perm is None:
            self._perm = permutation(stream_seed(self.name, "delete-order"), self.m)
        idx = np.take(self._perm, np.arange(self._perm_pos, self._perm_pos + n) % self.m)
        self._perm_pos += n
        return self.src[idx], self.dst[idx]

    def delete_batch(self, k: int, j: int):
        ne = int(round(self.exist_frac * k))
        es, ed = self._take_existing(ne)
        us, ud = uniform_pairs(stream_seed(self.name, "delete-uniform", k, j), k - ne,
                               self.num_vertices)
        return shuffle_pairs(stream_seed(self.name, "delete-mix", k, j),
                             np.concatenate([es, us]), np.concatenate([ed, ud]))

    def query_batch(self, q: int, j: int):
        es, ed = pick(stream_seed(self.name, "query-existing", q, j), q // 2,
                      self.src, self.dst)
        us, ud = uniform_pairs(stream_seed(self.name, "query-uniform", q, j), q - q // 2,
                               self.num_vertices)
        return shuffle_pairs(stream_seed(self.name, "query-mix", q, j),
                             np.concatenate([es, us]), np.concatenate([ed, ud]))
