"""ctypes wrapper around the CPU oracle (oracle/libgv_oracle.so).

TEST INFRASTRUCTURE ONLY.  Inputs are numpy arrays in host memory.  Each
method maps one-to-one onto a function of gv_oracle.h, which states the
definition it follows.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgv_oracle.so")

OK, EINVAL, ERANGE, ENOMEM = 0, 1, 2, 3

_lib = None


class Stats(C.Structure):
    _fields_ = [("applied", C.c_uint64), ("rejected", C.c_uint64),
                ("batch_duplicates", C.c_uint64)]

    def as_tuple(self):
        return (self.applied, self.rejected, self.batch_duplicates)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        u32p, u64p, u8p = (C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
                           C.POINTER(C.c_uint8))
        L.orc_next_pow2.restype = C.c_uint64
        L.orc_next_pow2.argtypes = [C.c_uint64]
        L.orc_paper_block_slots.restype = C.c_uint32
        L.orc_paper_block_slots.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_mix64.restype = C.c_uint64
        L.orc_mix64.argtypes = [C.c_uint64]
        L.orc_graph_init.restype = C.c_int
        L.orc_graph_init.argtypes = [C.POINTER(C.c_void_p), C.c_uint64, u32p, u32p,
                                     C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint64]
        L.orc_graph_destroy.restype = None
        L.orc_graph_destroy.argtypes = [C.c_void_p]
        for name in ("orc_insert_edges", "orc_delete_edges"):
            f = getattr(L, name)
            f.restype = C.c_int
            f.argtypes = [C.c_void_p, u32p, u32p, C.c_uint64, C.POINTER(Stats)]
        L.orc_apply_edge_ops.restype = C.c_int
        L.orc_apply_edge_ops.argtypes = [C.c_void_p, u8p, u32p, u32p, C.c_uint64]
        for name in ("orc_insert_vertices", "orc_delete_vertices"):
            f = getattr(L, name)
            f.restype = C.c_int
            f.argtypes = [C.c_void_p, u32p, C.c_uint64, C.POINTER(Stats)]
        L.orc_edge_exists.restype = C.c_int
        L.orc_edge_exists.argtypes = [C.c_void_p, u32p, u32p, C.c_uint64, u8p]
        L.orc_get_adjacency.restype = C.c_int
        L.orc_get_adjacency.argtypes = [C.c_void_p, C.c_uint32, u32p, C.c_uint64, u64p]
        L.orc_dump_canonical.restype = C.c_int
        L.orc_dump_canonical.argtypes = [C.c_void_p, u64p, u32p, C.c_uint64, u64p]
        for name, rt in (("orc_capacity", C.c_uint64), ("orc_num_edges", C.c_uint64),
                         ("orc_block_slots", C.c_uint32), ("orc_pool_blocks", C.c_uint64),
                         ("orc_blocks_in_use", C.c_uint64)):
            f = getattr(L, name)
            f.restype = rt
            f.argtypes = [C.c_void_p]
        L.orc_is_active.restype = C.c_int
        L.orc_is_active.argtypes = [C.c_void_p, C.c_uint32]
        L.orc_degree.restype = C.c_uint64
        L.orc_degree.argtypes = [C.c_void_p, C.c_uint32]
        L.orc_set_attr_words.restype = C.c_int
        L.orc_set_attr_words.argtypes = [C.c_void_p, C.c_uint32]
        L.orc_attr_words.restype = C.c_uint32
        L.orc_attr_words.argtypes = [C.c_void_p]
        L.orc_set_edge_attrs.restype = C.c_int
        L.orc_set_edge_attrs.argtypes = [C.c_void_p, u32p, u32p, u32p, C.c_uint64,
                                         C.POINTER(Stats)]
        L.orc_get_edge_attrs.restype = C.c_int
        L.orc_get_edge_attrs.argtypes = [C.c_void_p, u32p, u32p, C.c_uint64, u8p, u32p]
        L.orc_set_block_slots.restype = C.c_int
        L.orc_set_block_slots.argtypes = [C.c_void_p, C.c_uint32]
        L.orc_adapted_block_slots.restype = C.c_uint32
        L.orc_adapted_block_slots.argtypes = [C.c_void_p]
        _lib = L
    return _lib


def _u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(C.POINTER(C.c_uint32))


def next_pow2(x):
    return int(lib().orc_next_pow2(int(x)))


def paper_block_slots(edges, nonzero):
    return int(lib().orc_paper_block_slots(int(edges), int(nonzero)))


def mix64(z):
    return int(lib().orc_mix64(int(z)))


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


class OracleGraph:
    """Per-vertex ordered sets; see gv_oracle.h for every definition."""

    def __init__(self, num_vertices, src, dst, vertex_capacity=0, block_slots=16,
                 pool_bytes=0):
        L = lib()
        s, sp = _u32(src)
        d, dp = _u32(dst)
        if len(s) != len(d):
            raise ValueError("src/dst length mismatch")
        h = C.c_void_p()
        rc = L.orc_graph_init(C.byref(h), int(num_vertices), sp, dp, len(s),
                              int(vertex_capacity), int(block_slots), int(pool_bytes))
        if rc != OK:
            raise OracleError(rc, "orc_graph_init")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _edges(self, fn, src, dst):
        s, sp = _u32(src)
        d, dp = _u32(dst)
        if len(s) != len(d):
            raise ValueError("src/dst length mismatch")
        st = Stats()
        rc = fn(self._h, sp, dp, len(s), C.byref(st))
        return rc, st.as_tuple()

    def insert_edges(self, src, dst):
        """Returns (rc, (applied, rejected, batch_duplicates))."""
        return self._edges(lib().orc_insert_edges, src, dst)

    def delete_edges(self, src, dst):
        return self._edges(lib().orc_delete_edges, src, dst)

    def apply_edge_ops(self, op, src, dst):
        """Entry i inserts (op 0) or deletes (op 1) (src[i], dst[i]), one at a
        time in order.  Returns rc."""
        o = np.ascontiguousarray(np.asarray(op, dtype=np.uint8))
        s, sp = _u32(src)
        d, dp = _u32(dst)
        if not (len(o) == len(s) == len(d)):
            raise ValueError("op/src/dst length mismatch")
        return lib().orc_apply_edge_ops(self._h, o.ctypes.data_as(C.POINTER(C.c_uint8)),
                                        sp, dp, len(s))

    def set_attr_words(self, words):
        rc = lib().orc_set_attr_words(self._h, int(words))
        if rc != OK:
            raise OracleError(rc, "orc_set_attr_words")

    @property
    def attr_words(self):
        return int(lib().orc_attr_words(self._h))

    def set_edge_attrs(self, src, dst, vals):
        """vals: n x A rows.  Returns (rc, (applied, rejected, batch_duplicates))."""
        s, sp = _u32(src)
        d, dp = _u32(dst)
        v, vp = _u32(np.asarray(vals, np.uint32).reshape(-1))
        st = Stats()
        rc = lib().orc_set_edge_attrs(self._h, sp, dp, vp, len(s), C.byref(st))
        return rc, st.as_tuple()

    def get_edge_attrs(self, src, dst):
        """Returns (found uint8[n], vals uint32[n, A])."""
        s, sp = _u32(src)
        d, dp = _u32(dst)
        A = self.attr_words
        found = np.zeros(max(len(s), 1), dtype=np.uint8)
        vals = np.zeros((max(len(s), 1), max(A, 1)), dtype=np.uint32)
        rc = lib().orc_get_edge_attrs(self._h, sp, dp, len(s),
                                      found.ctypes.data_as(C.POINTER(C.c_uint8)),
                                      vals.ctypes.data_as(C.POINTER(C.c_uint32)))
        if rc != OK:
            raise OracleError(rc, "orc_get_edge_attrs")
        return found[: len(s)], vals[: len(s), :A]

    def set_block_slots(self, block_slots):
        return int(lib().orc_set_block_slots(self._h, int(block_slots)))

    def adapted_block_slots(self):
        return int(lib().orc_adapted_block_slots(self._h))

    def _verts(self, fn, ids):
        a, ap = _u32(ids)
        st = Stats()
        rc = fn(self._h, ap, len(a), C.byref(st))
        return rc, st.as_tuple()

    def insert_vertices(self, ids):
        return self._verts(lib().orc_insert_vertices, ids)

    def delete_vertices(self, ids):
        return self._verts(lib().orc_delete_vertices, ids)

    def edge_exists(self, src, dst):
        s, sp = _u32(src)
        d, dp = _u32(dst)
        out = np.zeros(len(s), dtype=np.uint8)
        rc = lib().orc_edge_exists(self._h, sp, dp, len(s),
                                   out.ctypes.data_as(C.POINTER(C.c_uint8)))
        if rc != OK:
            raise OracleError(rc, "orc_edge_exists")
        return out

    def get_adjacency(self, v):
        deg = C.c_uint64()
        rc = lib().orc_get_adjacency(self._h, int(v), None, 0, C.byref(deg))
        if rc == ERANGE and deg.value == 0 and int(v) >= self.capacity:
            raise OracleError(rc, "orc_get_adjacency")
        out = np.zeros(max(deg.value, 1), dtype=np.uint32)
        rc = lib().orc_get_adjacency(self._h, int(v),
                                     out.ctypes.data_as(C.POINTER(C.c_uint32)),
                                     len(out), C.byref(deg))
        if rc != OK:
            raise OracleError(rc, "orc_get_adjacency")
        return out[: deg.value]

    def dump(self):
        """Canonical CSR: (offsets uint64[capacity+1], dst uint32[E], checksum)."""
        L = lib()
        cap = self.capacity
        e = self.num_edges
        offs = np.zeros(cap + 1, dtype=np.uint64)
        dst = np.zeros(max(e, 1), dtype=np.uint32)
        ck = C.c_uint64()
        rc = L.orc_dump_canonical(self._h, offs.ctypes.data_as(C.POINTER(C.c_uint64)),
                                  dst.ctypes.data_as(C.POINTER(C.c_uint32)), len(dst),
                                  C.byref(ck))
        if rc != OK:
            raise OracleError(rc, "orc_dump_canonical")
        return offs, dst[:e], ck.value

    def checksum(self):
        ck = C.c_uint64()
        rc = lib().orc_dump_canonical(self._h, None, None, 0, C.byref(ck))
        if rc != OK:
            raise OracleError(rc, "orc_dump_canonical")
        return ck.value

    @property
    def capacity(self):
        return int(lib().orc_capacity(self._h))

    @property
    def num_edges(self):
        return int(lib().orc_num_edges(self._h))

    @property
    def block_slots(self):
        return int(lib().orc_block_slots(self._h))

    @property
    def pool_blocks(self):
        return int(lib().orc_pool_blocks(self._h))

    @property
    def blocks_in_use(self):
        return int(lib().orc_blocks_in_use(self._h))

    def is_active(self, v):
        return bool(lib().orc_is_active(self._h, int(v)))

    def degree(self, v):
        return int(lib().orc_degree(self._h, int(v)))
