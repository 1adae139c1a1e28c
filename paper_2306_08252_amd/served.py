"""The served form: continuous batching of update and query requests over one
graph, on the host side of the C ABI (every step of a tick runs in the
library's kernels).

A tick takes every request that has arrived, in arrival order, up to a pair
budget.  Its edge inserts and deletes go to the device as one mixed list
(gv_apply_edge_ops_stats), whose last-writer reduction gives the result of
applying them one pair at a time in arrival order, with each request's
statistics (applied, rejected, duplicates) as if it ran alone at its place
in that order; then the tick's queries are answered (gv_edge_exists).  So the commit order is: a tick's writes in
arrival order, then its queries.  Ticks overlap: a tick is queued as soon as
it is formed, while earlier ones still run on the device (a few at most),
and its answers come back by an asynchronous copy; requests that arrive
meanwhile form the next tick.  Vertex requests end a tick and run alone: a
vertex delete is queued in stream order like a tick (it only frees blocks,
so the host's free-block count stays a lower bound, and the library sizes
its lists without reading the device back); so is a vertex insert whose ids
all fit the vertex table (checked on a second stream, which waits for
nothing queued after the server started), queued with GV_OP_FIT_TABLE so
that it never reads the device back; one with an id past the table waits
for the running ticks (it grows the dictionary).  A request completes when its
tick's event has passed; latency is completion time minus scheduled arrival
time (open loop, so a late server does not lower the arrival rate).

Admission by free blocks: an edge-insert request of k pairs may need up to
ceil(k / B) + min(k, V) new blocks (its pairs packed into full blocks, plus
one partly filled block per touched source, at most V sources).  A tick
admits requests, in arrival order, while their bounds fit in the pool's
free blocks, so a tick's insert batch cannot run out of pool; the rest wait
for a later tick.  The free count is kept on the host as a lower bound (each
tick subtracts its bounds; deletes only add) and read back from the device
only when a request does not fit.  The directory arena is not part of the
bound: by default it holds four entries per pool block, and a segment holds
at most twice its vertex's blocks, but a directory shortfall would still
fail a tick's inserts with GV_ENOMEM (sticky, reported by gv_sync).  A request whose bound exceeds
the free blocks of an empty tick is rejected (it could fail the whole
tick's inserts) and reported as such.
"""
import math
import time

import numpy as np
import torch

from . import graphvine as gv

INSERT, DELETE, QUERY, VINSERT, VDELETE = 0, 1, 2, 3, 4
VINSERT_OP, VDELETE_OP = 2, 3  # their gv_op kinds


def _size(req):
    return int(req[1].numel())


def insert_block_bound(k, block_slots, vertex_capacity):
    """New blocks an insert of k pairs can take at most."""
    return -(-k // block_slots) + min(k, vertex_capacity)


def free_blocks(graph):
    m = graph.memory_used()
    return m["pool_capacity_blocks"] - m["blocks_in_use"]


class _PinnedRing:
    """Pinned host buffers reused by the ticks in turn (a slot is taken again
    only after its tick has completed: the ring has more slots than ticks in
    flight), so that no tick waits on a pinned allocation; a slot grows by
    doubling when a tick needs more."""

    def __init__(self, slots):
        self.slots = [{} for _ in range(slots)]
        self.next = 0

    def take(self):
        s = self.slots[self.next]
        self.next = (self.next + 1) % len(self.slots)
        return s

    @staticmethod
    def buf(slot, name, count, dtype):
        b = slot.get(name)
        if b is None or b.numel() < count:
            b = torch.empty(max(count, 2 * (0 if b is None else b.numel()), 64), dtype=dtype,
                            pin_memory=True)
            slot[name] = b
        return b[:count]


def _one_or_cat(parts):
    return parts[0] if len(parts) == 1 else torch.cat(parts)


def _enqueue_tick(graph, requests, i, j, dev, slot, codes):
    """Queues one tick's work on the graph's stream without waiting: the
    tick's edge inserts and deletes as one mixed list, then its queries as
    one batch whose answers are copied to pinned host memory (`slot` of the
    ring).  `codes` holds a row of insert op codes and a row of delete op
    codes, as long as the longest request, so that a request's op array is a
    view and a tick of one request copies nothing.  Returns the tick record
    (its tensors stay referenced until it completes)."""
    ws = [(m, r) for m, r in enumerate(requests[i:j], start=i) if r[0] in (INSERT, DELETE)]
    qs = [(m, r) for m, r in enumerate(requests[i:j], start=i) if r[0] == QUERY]
    keep = []
    wstats = None
    if ws:
        op = _one_or_cat([codes[r[0], :_size(r)] for _, r in ws])
        src = _one_or_cat([r[1] for _, r in ws])
        dst = _one_or_cat([r[2] for _, r in ws])
        ends_h = _PinnedRing.buf(slot, "ends", len(ws), torch.int64)
        ends_h.copy_(torch.from_numpy(np.cumsum([_size(r) for _, r in ws]).astype(np.int64)))
        ends = ends_h.to(dev, non_blocking=True)
        k, st = gv.gv_apply_edge_ops_stats(graph.h, op, src, dst, ends, dev)
        keep += list(k) + [st]
        wstats = _PinnedRing.buf(slot, "stats", st.numel(), st.dtype).view(st.shape)
        wstats.copy_(st, non_blocking=True)
    host = None
    if qs:
        out = graph.edge_exists(_one_or_cat([r[1] for _, r in qs]),
                                _one_or_cat([r[2] for _, r in qs]))
        host = _PinnedRing.buf(slot, "answers", out.numel(), out.dtype)
        host.copy_(out, non_blocking=True)
        keep.append(out)
    ev = torch.cuda.Event()
    ev.record(torch.cuda.current_stream(dev))
    return {"range": (i, j), "event": ev, "queries": qs, "answers": host, "keep": keep,
            "writes": [m for m, _ in ws], "stats": wstats}


def serve(graph, requests, arrivals=None, max_tick_pairs=1 << 20, keep_answers=False,
          clock=time.perf_counter, rejected=None, max_inflight=3, stats=None):
    """Runs `requests` [(kind, a, b)] (device id tensors; b is None for vertex
    requests) against `graph` (a graphvine.Graph).  `arrivals[i]` is request
    i's scheduled time in seconds from the start (None: all at time 0).
    Ticks overlap: a tick is queued on the graph's stream as soon as it is
    formed, while up to `max_inflight - 1` earlier ticks are still running,
    so requests that arrive meanwhile form the next tick and run right after
    (stream order keeps the commit order); a tick's requests complete when
    its event has passed.  A vertex insert whose ids fit the vertex table,
    and a vertex delete, are queued like a tick; a vertex insert that grows
    the table waits for every running tick.
    Returns (completion times, ticks as (first, end) request ranges, answers
    of the query requests by index if keep_answers).  Indices of requests
    rejected by admission are appended to `rejected` (a list) if given; a
    rejected request is not in any tick.  `stats` (a dict), if given,
    receives (applied, rejected, duplicates) for every edge insert / delete
    request, as if the request ran alone at its place in the commit order."""
    n = len(requests)
    arr = np.zeros(n) if arrivals is None else np.asarray(arrivals, np.float64)
    if n and np.any(np.diff(arr) < 0):
        raise ValueError("arrivals must be in order")
    dev = graph.device
    info = graph.info()
    bs, vcap = info["block_slots"], info["vertex_capacity"]
    free = free_blocks(graph)
    done = np.zeros(n)
    ticks = []
    answers = {}
    flight = []
    ring = _PinnedRing(max_inflight + 1)
    # op codes of every write request as views: row INSERT of zeros, row
    # DELETE of ones
    longest = max([_size(r) for r in requests if r[0] in (INSERT, DELETE)], default=1)
    codes = torch.zeros((2, max(longest, 1)), dtype=torch.uint8, device=dev)
    codes[DELETE].fill_(1)
    # the id check of vertex inserts runs on a second stream (default
    # priority), after the work queued before the server started (which made
    # the requests) and independent of the ticks queued since
    side = torch.cuda.Stream(device=dev)
    start = torch.cuda.Event()
    start.record(torch.cuda.current_stream(dev))
    side.wait_event(start)

    def fits_table(ids):
        if ids.numel() == 0:
            return True
        with torch.cuda.stream(side):
            top = int((ids.to(torch.int64) & 0xFFFFFFFF).max())  # waits on `side` only
        return top < vcap

    t0 = clock()

    def retire(block):
        # completes the ticks whose events have passed (all of them if block)
        while flight and (block or flight[0]["event"].query()):
            tk = flight.pop(0)
            tk["event"].synchronize()
            t = clock() - t0
            f, e = tk["range"]
            done[f:e] = t
            if stats is not None and tk["writes"]:
                st = tk["stats"].numpy()
                for row, m in enumerate(tk["writes"]):
                    stats[m] = tuple(int(x) for x in st[row])
            if keep_answers and tk["queries"]:
                out = tk["answers"].numpy()
                o = 0
                for m, r in tk["queries"]:
                    answers[m] = out[o:o + _size(r)].copy()
                    o += _size(r)

    i = 0
    while i < n:
        retire(False)
        now = clock() - t0
        if arr[i] > now or len(flight) >= max_inflight:
            if flight:
                continue  # poll the running ticks
            while clock() - t0 < arr[i]:
                pass
            now = clock() - t0
        kind = requests[i][0]
        if kind == VDELETE:
            # queued behind the running ticks, no host wait
            keep = gv.gv_apply_ops(graph.h, [(VDELETE_OP, requests[i][1], None)], dev)
            ev = torch.cuda.Event()
            ev.record(torch.cuda.current_stream(dev))
            flight.append({"range": (i, i + 1), "event": ev, "queries": [], "answers": None,
                           "keep": keep, "writes": [], "stats": None})
            ticks.append((i, i + 1))
            i += 1
            continue
        if kind == VINSERT and fits_table(requests[i][1]):
            keep = gv.gv_apply_ops(graph.h, [(VINSERT_OP, requests[i][1], None,
                                              gv.OP_FIT_TABLE)], dev)
            ev = torch.cuda.Event()
            ev.record(torch.cuda.current_stream(dev))
            flight.append({"range": (i, i + 1), "event": ev, "queries": [], "answers": None,
                           "keep": keep, "writes": [], "stats": None})
            ticks.append((i, i + 1))
            i += 1
            continue
        if kind == VINSERT:
            retire(True)
            graph.insert_vertices(requests[i][1])
            torch.cuda.synchronize(dev)
            done[i] = clock() - t0
            ticks.append((i, i + 1))
            free = free_blocks(graph)
            vcap = graph.info()["vertex_capacity"]  # the table may have grown
            i += 1
            continue
        j, pairs, need, fresh = i, 0, 0, False
        while j < n and arr[j] <= now and requests[j][0] in (INSERT, DELETE, QUERY):
            k = _size(requests[j])
            b = insert_block_bound(k, bs, vcap) if requests[j][0] == INSERT else 0
            if j > i and pairs + k > max_tick_pairs:
                break
            if need + b > free and not fresh:
                retire(True)
                free = free_blocks(graph)  # every queued tick has completed
                fresh = True
            if need + b > free:
                break  # waits for a later tick (or, alone, is rejected)
            pairs += k
            need += b
            j += 1
        if j == i:
            if rejected is not None:
                rejected.append(i)
            done[i] = clock() - t0
            i += 1
            continue
        flight.append(_enqueue_tick(graph, requests, i, j, dev, ring.take(), codes))
        ticks.append((i, j))
        free -= need
        i = j
    retire(True)
    return done, ticks, answers


def nearest_rank(x, p):
    """The p-quantile by nearest rank (p in (0, 1])."""
    s = np.sort(np.asarray(x))
    return float(s[max(0, math.ceil(p * len(s)) - 1)])


def poisson_arrivals(seed_draws, rate):
    """Arrival times of a Poisson process of `rate` per second from uniform
    draws (uint64): exponential gaps -ln(u) / rate."""
    u = ((np.asarray(seed_draws, np.uint64) >> np.uint64(11)).astype(np.float64) + 0.5) / float(1 << 53)
    return np.cumsum(-np.log(u) / rate)
