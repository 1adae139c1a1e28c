"""Python binding of libgraphvine.so (include/graphvine.h).

Argument marshalling only: every function below forwards to the C function of
the same name, passing device pointers of torch tensors and the current HIP
stream.  All work runs in the library's HIP kernels.  There is no fallback:
if the library has not been built, importing a function raises.

Id arrays are 32-bit tensors (torch.int32 or torch.uint32, holding the
uint32 bit patterns) on the graph's GPU; numpy arrays are copied to the GPU
first.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgraphvine.so")

GV_OK, GV_EINVAL, GV_ERANGE, GV_ENOMEM, GV_EDEVICE = 0, 1, 2, 3, 4


class gv_config(C.Structure):
    _fields_ = [("block_slots", C.c_uint32), ("flags", C.c_uint32),
                ("pool_bytes", C.c_uint64), ("vertex_capacity", C.c_uint64),
                ("directory_entries", C.c_uint64), ("edge_attr_words", C.c_uint32),
                ("reserved", C.c_uint32)]


class gv_batch_stats(C.Structure):
    _fields_ = [("applied", C.c_uint64), ("rejected", C.c_uint64),
                ("batch_duplicates", C.c_uint64)]

    def as_tuple(self):
        return (self.applied, self.rejected, self.batch_duplicates)


class gv_mem(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "block_bytes", "pool_capacity_blocks", "blocks_in_use", "free_list_blocks",
        "bump_blocks", "vertex_capacity", "vertex_table_bytes", "directory_entries_in_use",
        "directory_bytes", "live_bytes", "num_edges", "reserved_bytes")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class gv_info(C.Structure):
    _fields_ = [("vertex_capacity", C.c_uint64), ("block_slots", C.c_uint32),
                ("device", C.c_uint32)]


class gv_counters(C.Structure):
    _fields_ = [("batches", C.c_uint64 * 3), ("pairs", C.c_uint64 * 3),
                ("touched", C.c_uint64 * 3), ("scanned_slots", C.c_uint64 * 3),
                ("new_blocks", C.c_uint64), ("freed_blocks", C.c_uint64),
                ("written_slots", C.c_uint64), ("moved_slots", C.c_uint64)]

    def as_dict(self):
        out = {}
        for n, _ in self._fields_:
            v = getattr(self, n)
            out[n] = list(v) if not isinstance(v, int) else v
        return out


TUNING_FIELDS = ("coalesce", "max_run_pairs", "small_sort_max", "probe_group", "probe_unroll",
                 "item_chunk", "overlap")


class gv_tuning(C.Structure):
    _fields_ = [(f, C.c_uint32) for f in TUNING_FIELDS] + [("reserved", C.c_uint32)]

    def as_dict(self):
        return {f: getattr(self, f) for f in TUNING_FIELDS}


class gv_op(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("flags", C.c_uint32), ("a", C.c_void_p),
                ("b", C.c_void_p), ("n", C.c_uint64)]


OP_INSERT_EDGES, OP_DELETE_EDGES, OP_INSERT_VERTICES, OP_DELETE_VERTICES = 0, 1, 2, 3
OP_FIT_TABLE = 1  # gv_op.flags: a vertex insert whose ids fit the table (no host wait)

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        vp, u32p, u64p = C.c_void_p, C.c_void_p, C.POINTER(C.c_uint64)
        sig = {
            "gv_graph_init": [C.POINTER(C.c_void_p), C.c_uint64, u32p, u32p, C.c_uint64,
                              C.POINTER(gv_config), vp],
            "gv_insert_edges": [vp, u32p, u32p, C.c_uint64, C.POINTER(gv_batch_stats)],
            "gv_delete_edges": [vp, u32p, u32p, C.c_uint64, C.POINTER(gv_batch_stats)],
            "gv_insert_vertices": [vp, u32p, C.c_uint64, C.POINTER(gv_batch_stats)],
            "gv_delete_vertices": [vp, u32p, C.c_uint64, C.POINTER(gv_batch_stats)],
            "gv_edge_exists": [vp, u32p, u32p, C.c_uint64, vp],
            "gv_apply_edge_ops": [vp, vp, u32p, u32p, C.c_uint64],
            "gv_set_edge_attrs": [vp, u32p, u32p, u32p, C.c_uint64, vp],
            "gv_set_block_slots": [vp, C.c_uint32],
            "gv_adapt_block_slots": [vp, C.POINTER(C.c_uint32)],
            "gv_get_edge_attrs": [vp, u32p, u32p, C.c_uint64, vp, u32p],
            "gv_apply_edge_ops_stats": [vp, vp, u32p, u32p, C.c_uint64, vp, C.c_uint64, vp],
            "gv_get_adjacency": [vp, C.c_uint32, u32p, C.c_uint64, u64p],
            "gv_memory_used": [vp, C.POINTER(gv_mem)],
            "gv_dump_canonical": [vp, vp, u32p, C.c_uint64, u64p, u64p],
            "gv_audit": [vp, u64p],
            "gv_graph_info": [vp, C.POINTER(gv_info)],
            "gv_get_counters": [vp, C.POINTER(gv_counters)],
            "gv_profile_enable": [vp, C.c_int],
            "gv_profile_reset": [vp],
            "gv_profile_only": [vp, C.c_char_p],
            "gv_kernel_times": [vp, C.c_char_p, u64p, C.POINTER(C.c_double)],
            "gv_kernel_names": [vp, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)],
            "gv_set_stream": [vp, vp],
            "gv_debug_spin_limit": [vp, C.c_uint32],
            "gv_set_tuning": [vp, C.POINTER(gv_tuning)],
            "gv_get_tuning": [vp, C.POINTER(gv_tuning)],
            "gv_cbt_init": [C.POINTER(C.c_void_p), C.c_uint64, u32p, u32p, C.c_uint64,
                            C.c_uint32, C.c_uint64, vp],
            "gv_cbt_insert_edges": [vp, u32p, u32p, C.c_uint64, C.POINTER(gv_batch_stats)],
            "gv_cbt_delete_edges": [vp, u32p, u32p, C.c_uint64, C.POINTER(gv_batch_stats)],
            "gv_cbt_edge_exists": [vp, u32p, u32p, C.c_uint64, vp],
            "gv_cbt_dump": [vp, vp, u32p, C.c_uint64, u64p],
            "gv_cbt_blocks": [vp, u64p],
            "gv_cbt_set_stream": [vp, vp],
            "gv_cbt_bitstring": [C.c_uint64, C.c_char_p, C.c_uint64],
            "gv_sync": [vp],
            "gv_apply_ops": [vp, C.POINTER(gv_op), C.c_uint64],
            "gv_plan_create": [vp, C.POINTER(gv_op), C.c_uint64, C.POINTER(C.c_void_p)],
            "gv_plan_launch": [vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.gv_strerror.argtypes = [C.c_int]
        L.gv_strerror.restype = C.c_char_p
        L.gv_last_error.argtypes = []
        L.gv_last_error.restype = C.c_char_p
        L.gv_graph_destroy.argtypes = [vp]
        L.gv_graph_destroy.restype = None
        L.gv_plan_destroy.argtypes = [vp]
        L.gv_plan_destroy.restype = None
        L.gv_cbt_destroy.argtypes = [vp]
        L.gv_cbt_destroy.restype = None
        _lib = L
    return _lib


class GraphVineError(RuntimeError):
    def __init__(self, code, fn):
        detail = lib().gv_last_error().decode() if code in (GV_ENOMEM, GV_EDEVICE) else ""
        super().__init__(f"{fn}: {gv_strerror(code)} (code {code})" +
                         (f" [{detail}]" if detail else ""))
        self.code = code


def gv_strerror(code: int) -> str:
    return lib().gv_strerror(int(code)).decode()


def _check(rc, fn):
    if rc != GV_OK:
        raise GraphVineError(rc, fn)


def _stream_ptr(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def as_device_u32(x, device) -> torch.Tensor:
    """A contiguous 32-bit tensor holding the uint32 ids of x on `device`."""
    if isinstance(x, torch.Tensor):
        if x.dtype not in (torch.int32, torch.uint32):
            raise TypeError("id tensors must be int32 or uint32")
        if x.device != torch.device(device):
            raise ValueError(f"tensor on {x.device}, graph on {device}")
        return x.contiguous()
    a = np.ascontiguousarray(np.asarray(x, dtype=np.uint32)).view(np.int32)
    return torch.from_numpy(a).to(device)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() else C.c_void_p(0)


# ------------------------------------------------------------------ C names
def gv_graph_init(num_vertices, src, dst, block_slots=0, pool_bytes=0, vertex_capacity=0,
                  directory_entries=0, device="cuda:0", edge_attr_words=0):
    """Returns an opaque graph handle (int).  See gv_graph_init in graphvine.h."""
    s = as_device_u32(src, device)
    d = as_device_u32(dst, device)
    if s.numel() != d.numel():
        raise ValueError("src/dst length mismatch")
    cfg = gv_config(int(block_slots), 0, int(pool_bytes), int(vertex_capacity),
                    int(directory_entries), int(edge_attr_words), 0)
    h = C.c_void_p()
    with torch.cuda.device(torch.device(device)):
        rc = lib().gv_graph_init(C.byref(h), int(num_vertices), _ptr(s), _ptr(d), s.numel(),
                                 C.byref(cfg), _stream_ptr(device))
    _check(rc, "gv_graph_init")
    return h.value


def _edges(fn, name, g, src, dst, device, stats):
    s = as_device_u32(src, device)
    d = as_device_u32(dst, device)
    if s.numel() != d.numel():
        raise ValueError("src/dst length mismatch")
    st = gv_batch_stats()
    rc = fn(C.c_void_p(g), _ptr(s), _ptr(d), s.numel(), C.byref(st) if stats else None)
    _check(rc, name)
    return st.as_tuple() if stats else None


def gv_insert_edges(g, src, dst, device="cuda:0", stats=True):
    return _edges(lib().gv_insert_edges, "gv_insert_edges", g, src, dst, device, stats)


def gv_delete_edges(g, src, dst, device="cuda:0", stats=True):
    return _edges(lib().gv_delete_edges, "gv_delete_edges", g, src, dst, device, stats)


def _verts(fn, name, g, ids, device):
    a = as_device_u32(ids, device)
    st = gv_batch_stats()
    _check(fn(C.c_void_p(g), _ptr(a), a.numel(), C.byref(st)), name)
    return st.as_tuple()


def gv_insert_vertices(g, ids, device="cuda:0"):
    return _verts(lib().gv_insert_vertices, "gv_insert_vertices", g, ids, device)


def gv_delete_vertices(g, ids, device="cuda:0"):
    return _verts(lib().gv_delete_vertices, "gv_delete_vertices", g, ids, device)


def gv_edge_exists(g, src, dst, device="cuda:0", out=None):
    s = as_device_u32(src, device)
    d = as_device_u32(dst, device)
    if s.numel() != d.numel():
        raise ValueError("src/dst length mismatch")
    if out is None:
        out = torch.empty(s.numel(), dtype=torch.uint8, device=device)
    _check(lib().gv_edge_exists(C.c_void_p(g), _ptr(s), _ptr(d), s.numel(), _ptr(out)),
           "gv_edge_exists")
    return out


def as_device_u8(x, device) -> torch.Tensor:
    """A contiguous uint8 tensor holding x on `device`."""
    if isinstance(x, torch.Tensor):
        if x.dtype != torch.uint8:
            raise TypeError("op tensors must be uint8")
        if x.device != torch.device(device):
            raise ValueError(f"tensor on {x.device}, graph on {device}")
        return x.contiguous()
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.uint8))).to(device)


def gv_apply_edge_ops(g, op, src, dst, device="cuda:0"):
    """Entry i inserts (op 0) or deletes (op 1) (src[i], dst[i]); the result is
    that of applying the entries one at a time in order.  Asynchronous."""
    o = as_device_u8(op, device)
    s = as_device_u32(src, device)
    d = as_device_u32(dst, device)
    if not (o.numel() == s.numel() == d.numel()):
        raise ValueError("op/src/dst length mismatch")
    _check(lib().gv_apply_edge_ops(C.c_void_p(g), _ptr(o), _ptr(s), _ptr(d), s.numel()),
           "gv_apply_edge_ops")
    return o, s, d


def gv_apply_edge_ops_stats(g, op, src, dst, req_end, device="cuda:0", stats=None):
    """gv_apply_edge_ops with per-request statistics: request r is entries
    [req_end[r-1], req_end[r]).  req_end: device int64 tensor or a host
    sequence (copied through pinned memory without a host wait).  Returns
    (tensors to keep alive until the call completes, stats: device int64
    (n_req, 3) of applied, rejected, batch duplicates, valid after sync)."""
    o = as_device_u8(op, device)
    s = as_device_u32(src, device)
    d = as_device_u32(dst, device)
    if not (o.numel() == s.numel() == d.numel()):
        raise ValueError("op/src/dst length mismatch")
    if not (torch.is_tensor(req_end) and req_end.is_cuda):
        req_end = torch.tensor(np.asarray(req_end, np.int64)).pin_memory().to(device,
                                                                               non_blocking=True)
    e = req_end.to(torch.int64).contiguous()
    if stats is None:
        stats = torch.empty((e.numel(), 3), dtype=torch.int64, device=device)
    _check(lib().gv_apply_edge_ops_stats(C.c_void_p(g), _ptr(o), _ptr(s), _ptr(d), s.numel(),
                                         _ptr(e), e.numel(), _ptr(stats)),
           "gv_apply_edge_ops_stats")
    return (o, s, d, e), stats


def gv_set_edge_attrs(g, src, dst, attr, device="cuda:0", stats=True):
    """attr: n x A uint32 (rows per pair).  Returns stats if requested."""
    s = as_device_u32(src, device)
    d = as_device_u32(dst, device)
    a = as_device_u32(np.asarray(attr, np.uint32).reshape(-1) if not torch.is_tensor(attr)
                      else attr.reshape(-1), device)
    if s.numel() != d.numel():
        raise ValueError("src/dst length mismatch")
    st = gv_batch_stats()
    _check(lib().gv_set_edge_attrs(C.c_void_p(g), _ptr(s), _ptr(d), _ptr(a), s.numel(),
                                   C.byref(st) if stats else None), "gv_set_edge_attrs")
    return st.as_tuple() if stats else (s, d, a)


def gv_get_edge_attrs(g, src, dst, words, device="cuda:0"):
    """Returns (found uint8 [n], attrs int32 [n, words]) device tensors."""
    s = as_device_u32(src, device)
    d = as_device_u32(dst, device)
    if s.numel() != d.numel():
        raise ValueError("src/dst length mismatch")
    found = torch.empty(max(s.numel(), 1), dtype=torch.uint8, device=device)
    out = torch.empty((max(s.numel(), 1), max(words, 1)), dtype=torch.int32, device=device)
    _check(lib().gv_get_edge_attrs(C.c_void_p(g), _ptr(s), _ptr(d), s.numel(), _ptr(found),
                                   _ptr(out)), "gv_get_edge_attrs")
    return found[: s.numel()], out[: s.numel()]


def gv_get_adjacency(g, v, device="cuda:0", out=None):
    deg = C.c_uint64()
    if out is None:
        rc = lib().gv_get_adjacency(C.c_void_p(g), int(v), C.c_void_p(0), 0, C.byref(deg))
        if rc not in (GV_OK, GV_ERANGE) or (rc == GV_ERANGE and deg.value == 0
                                            and int(v) >= gv_graph_info(g)["vertex_capacity"]):
            _check(rc, "gv_get_adjacency")
        out = torch.empty(max(deg.value, 1), dtype=torch.int32, device=device)
    rc = lib().gv_get_adjacency(C.c_void_p(g), int(v), _ptr(out), out.numel(), C.byref(deg))
    _check(rc, "gv_get_adjacency")
    return out[: deg.value]


def gv_memory_used(g):
    m = gv_mem()
    _check(lib().gv_memory_used(C.c_void_p(g), C.byref(m)), "gv_memory_used")
    return m.as_dict()


def gv_dump_canonical(g, device="cuda:0", checksum_only=False):
    """(offsets int64[capacity+1], dst int32[E], checksum, E); arrays are None
    when checksum_only."""
    ck, e = C.c_uint64(), C.c_uint64()
    L = lib()
    if checksum_only:
        _check(L.gv_dump_canonical(C.c_void_p(g), None, None, 0, C.byref(ck), C.byref(e)),
               "gv_dump_canonical")
        return None, None, ck.value, e.value
    cap = gv_graph_info(g)["vertex_capacity"]
    _check(L.gv_dump_canonical(C.c_void_p(g), None, None, 0, C.byref(ck), C.byref(e)),
           "gv_dump_canonical")
    offs = torch.empty(cap + 1, dtype=torch.int64, device=device)
    dst = torch.empty(max(e.value, 1), dtype=torch.int32, device=device)
    _check(L.gv_dump_canonical(C.c_void_p(g), _ptr(offs), _ptr(dst), dst.numel(), C.byref(ck),
                               C.byref(e)), "gv_dump_canonical")
    return offs, dst[: e.value], ck.value, e.value


def gv_audit(g):
    bad = C.c_uint64()
    _check(lib().gv_audit(C.c_void_p(g), C.byref(bad)), "gv_audit")
    return bad.value


def gv_graph_info(g):
    i = gv_info()
    _check(lib().gv_graph_info(C.c_void_p(g), C.byref(i)), "gv_graph_info")
    return {"vertex_capacity": i.vertex_capacity, "block_slots": i.block_slots,
            "device": i.device}


def gv_get_counters(g):
    c = gv_counters()
    _check(lib().gv_get_counters(C.c_void_p(g), C.byref(c)), "gv_get_counters")
    return c.as_dict()


def gv_profile_enable(g, enable=True):
    _check(lib().gv_profile_enable(C.c_void_p(g), int(bool(enable))), "gv_profile_enable")


def gv_profile_only(g, name=None):
    _check(lib().gv_profile_only(C.c_void_p(g), name.encode() if name else None),
           "gv_profile_only")


def gv_profile_reset(g):
    _check(lib().gv_profile_reset(C.c_void_p(g)), "gv_profile_reset")


def gv_kernel_times(g, name):
    n, ms = C.c_uint64(), C.c_double()
    _check(lib().gv_kernel_times(C.c_void_p(g), name.encode(), C.byref(n), C.byref(ms)),
           "gv_kernel_times")
    return n.value, ms.value


def gv_kernel_names(g):
    need = C.c_size_t()
    rc = lib().gv_kernel_names(C.c_void_p(g), None, 0, C.byref(need))
    if rc not in (0, GV_ERANGE):
        _check(rc, "gv_kernel_names")
    buf = C.create_string_buffer(need.value)
    _check(lib().gv_kernel_names(C.c_void_p(g), buf, need.value, C.byref(need)),
           "gv_kernel_names")
    text = buf.value.decode()
    return text.split(",") if text else []


def gv_set_stream(g, stream_ptr):
    _check(lib().gv_set_stream(C.c_void_p(g), C.c_void_p(stream_ptr)), "gv_set_stream")


def gv_sync(g):
    return lib().gv_sync(C.c_void_p(g))


def gv_set_tuning(g, **fields):
    """Sets the given fields of the graph's gv_tuning (others unchanged)."""
    t = gv_tuning()
    _check(lib().gv_get_tuning(C.c_void_p(g), C.byref(t)), "gv_get_tuning")
    for k, val in fields.items():
        if k not in TUNING_FIELDS:
            raise TypeError(f"unknown tuning field {k}")
        if val is not None:
            setattr(t, k, int(val))
    _check(lib().gv_set_tuning(C.c_void_p(g), C.byref(t)), "gv_set_tuning")
    return t.as_dict()


def gv_get_tuning(g):
    t = gv_tuning()
    _check(lib().gv_get_tuning(C.c_void_p(g), C.byref(t)), "gv_get_tuning")
    return t.as_dict()


def gv_debug_spin_limit(g, limit):
    _check(lib().gv_debug_spin_limit(C.c_void_p(g), int(limit)), "gv_debug_spin_limit")


def gv_graph_destroy(g):
    lib().gv_graph_destroy(C.c_void_p(g))


# ------------------------------------------------------------------ wrapper
class Graph:
    """Owning wrapper over a gv_graph handle on one GPU."""

    def __init__(self, num_vertices, src=(), dst=(), block_slots=16, pool_bytes=0,
                 vertex_capacity=0, directory_entries=0, device="cuda:0", edge_attr_words=0):
        self.device = torch.device(device)
        self.attr_words = int(edge_attr_words)
        self.h = gv_graph_init(num_vertices, src, dst, block_slots, pool_bytes, vertex_capacity,
                               directory_entries, self.device, edge_attr_words)

    def close(self):
        if getattr(self, "h", None):
            gv_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert_edges(self, src, dst, stats=True):
        return gv_insert_edges(self.h, src, dst, self.device, stats)

    def delete_edges(self, src, dst, stats=True):
        return gv_delete_edges(self.h, src, dst, self.device, stats)

    def insert_vertices(self, ids):
        return gv_insert_vertices(self.h, ids, self.device)

    def delete_vertices(self, ids):
        return gv_delete_vertices(self.h, ids, self.device)

    def edge_exists(self, src, dst, out=None):
        return gv_edge_exists(self.h, src, dst, self.device, out)

    def apply_edge_ops(self, op, src, dst):
        return gv_apply_edge_ops(self.h, op, src, dst, self.device)

    def set_block_slots(self, block_slots):
        _check(lib().gv_set_block_slots(C.c_void_p(self.h), int(block_slots)),
               "gv_set_block_slots")

    def adapt_block_slots(self):
        b = C.c_uint32()
        _check(lib().gv_adapt_block_slots(C.c_void_p(self.h), C.byref(b)),
               "gv_adapt_block_slots")
        return b.value

    def set_edge_attrs(self, src, dst, attr, stats=True):
        return gv_set_edge_attrs(self.h, src, dst, attr, self.device, stats)

    def get_edge_attrs(self, src, dst):
        return gv_get_edge_attrs(self.h, src, dst, self.attr_words, self.device)

    def apply_edge_ops_stats(self, op, src, dst, req_end):
        return gv_apply_edge_ops_stats(self.h, op, src, dst, req_end, self.device)

    def get_adjacency(self, v):
        return gv_get_adjacency(self.h, v, self.device)

    def memory_used(self):
        return gv_memory_used(self.h)

    def dump(self, checksum_only=False):
        return gv_dump_canonical(self.h, self.device, checksum_only)

    def audit(self):
        return gv_audit(self.h)

    def info(self):
        return gv_graph_info(self.h)

    def counters(self):
        return gv_get_counters(self.h)

    def sync(self):
        return gv_sync(self.h)


# ------------------------------------------------------------------ batched form
def _ops(ops, device):
    """[(kind, a, b or None[, flags])] -> (gv_op array, device tensors kept
    alive)."""
    arr = (gv_op * max(len(ops), 1))()
    keep = []
    for i, op in enumerate(ops):
        kind, a, b = op[:3]
        ta = as_device_u32(a, device)
        keep.append(ta)
        arr[i].kind = kind
        arr[i].flags = op[3] if len(op) > 3 else 0
        arr[i].a = ta.data_ptr() if ta.numel() else None
        arr[i].n = ta.numel()
        if kind in (OP_INSERT_EDGES, OP_DELETE_EDGES):
            tb = as_device_u32(b, device)
            if tb.numel() != ta.numel():
                raise ValueError("src/dst length mismatch")
            keep.append(tb)
            arr[i].b = tb.data_ptr() if tb.numel() else None
    return arr, keep


def gv_apply_ops(g, ops, device="cuda:0"):
    arr, keep = _ops(ops, device)
    _check(lib().gv_apply_ops(C.c_void_p(g), arr, len(ops)), "gv_apply_ops")
    return keep


class Plan:
    """A recorded sequence of batches (gv_plan_*); holds its input tensors."""

    def __init__(self, g, ops, device="cuda:0"):
        self.h = None
        self.arr, self.keep = _ops(ops, device)
        h = C.c_void_p()
        _check(lib().gv_plan_create(C.c_void_p(g), self.arr, len(ops), C.byref(h)),
               "gv_plan_create")
        self.h = h.value

    def launch(self):
        _check(lib().gv_plan_launch(C.c_void_p(self.h)), "gv_plan_launch")

    def close(self):
        if self.h:
            lib().gv_plan_destroy(C.c_void_p(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ paper-faithful ablation
def gv_cbt_bitstring(k: int) -> str:
    """Bit string of level-order position k >= 1 (computed by the library)."""
    buf = C.create_string_buffer(72)
    _check(lib().gv_cbt_bitstring(int(k), buf, 72), "gv_cbt_bitstring")
    return buf.value.decode()


class CbtGraph:
    """The paper's own layout (complete binary tree of edge blocks, one thread
    per vertex) through gv_cbt_*; all calls synchronous."""

    def __init__(self, num_vertices, src=(), dst=(), block_slots=16, pool_blocks=None,
                 device="cuda:0"):
        self.device = torch.device(device)
        s = as_device_u32(src, self.device)
        d = as_device_u32(dst, self.device)
        if s.numel() != d.numel():
            raise ValueError("src/dst length mismatch")
        if pool_blocks is None:
            pool_blocks = 4 * (s.numel() // block_slots + 1) + 2 * int(num_vertices) + (1 << 16)
        self.h = None
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            rc = lib().gv_cbt_init(C.byref(h), int(num_vertices), _ptr(s), _ptr(d), s.numel(),
                                   int(block_slots), int(pool_blocks), _stream_ptr(self.device))
        _check(rc, "gv_cbt_init")
        self.h = h.value
        cap = 1
        while cap < int(num_vertices):
            cap <<= 1
        self.capacity = cap

    def close(self):
        if getattr(self, "h", None):
            lib().gv_cbt_destroy(C.c_void_p(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _edges(self, fn, name, src, dst):
        s = as_device_u32(src, self.device)
        d = as_device_u32(dst, self.device)
        if s.numel() != d.numel():
            raise ValueError("src/dst length mismatch")
        st = gv_batch_stats()
        _check(fn(C.c_void_p(self.h), _ptr(s), _ptr(d), s.numel(), C.byref(st)), name)
        return st.as_tuple()

    def insert_edges(self, src, dst):
        return self._edges(lib().gv_cbt_insert_edges, "gv_cbt_insert_edges", src, dst)

    def delete_edges(self, src, dst):
        return self._edges(lib().gv_cbt_delete_edges, "gv_cbt_delete_edges", src, dst)

    def edge_exists(self, src, dst):
        s = as_device_u32(src, self.device)
        d = as_device_u32(dst, self.device)
        out = torch.empty(max(s.numel(), 1), dtype=torch.uint8, device=self.device)
        _check(lib().gv_cbt_edge_exists(C.c_void_p(self.h), _ptr(s), _ptr(d), s.numel(),
                                        _ptr(out)), "gv_cbt_edge_exists")
        return out[: s.numel()]

    def dump(self):
        """(offsets int64[capacity+1], dst int32[E], E)"""
        e = C.c_uint64()
        L = lib()
        _check(L.gv_cbt_dump(C.c_void_p(self.h), None, None, 0, C.byref(e)), "gv_cbt_dump")
        offs = torch.empty(self.capacity + 1, dtype=torch.int64, device=self.device)
        dst = torch.empty(max(e.value, 1), dtype=torch.int32, device=self.device)
        _check(L.gv_cbt_dump(C.c_void_p(self.h), _ptr(offs), _ptr(dst), dst.numel(),
                             C.byref(e)), "gv_cbt_dump")
        return offs, dst[: e.value], e.value

    def blocks(self):
        b = C.c_uint64()
        _check(lib().gv_cbt_blocks(C.c_void_p(self.h), C.byref(b)), "gv_cbt_blocks")
        return b.value
