"""The served form: continuous batching of update and query requests over one
graph, on the host side of the C ABI (every step of a tick runs in the
library's kernels).

A tick takes every request that has arrived, in arrival order, up to a pair
budget.  Its edge inserts and deletes go to the device as one mixed list
(gv_apply_edge_ops), whose last-writer reduction gives the result of
applying them one pair at a time in arrival order; then the tick's queries
are answered (gv_edge_exists).  So the commit order is: a tick's writes in
arrival order, then its queries.  Vertex requests are barriers: a tick ends
before one, and it runs alone.  A request completes when its tick has
synchronised; latency is completion time minus scheduled arrival time (open
loop, so a late server does not lower the arrival rate).

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


def _size(req):
    return int(req[1].numel())


def insert_block_bound(k, block_slots, vertex_capacity):
    """New blocks an insert of k pairs can take at most."""
    return -(-k // block_slots) + min(k, vertex_capacity)


def free_blocks(graph):
    m = graph.memory_used()
    return m["pool_capacity_blocks"] - m["blocks_in_use"]


def serve(graph, requests, arrivals=None, max_tick_pairs=1 << 20, keep_answers=False,
          clock=time.perf_counter, rejected=None):
    """Runs `requests` [(kind, a, b)] (device id tensors; b is None for vertex
    requests) against `graph` (a graphvine.Graph).  `arrivals[i]` is request
    i's scheduled time in seconds from the start (None: all at time 0).
    Returns (completion times, ticks as (first, end) request ranges, answers
    of the query requests by index if keep_answers).  Indices of requests
    rejected by admission are appended to `rejected` (a list) if given; a
    rejected request is not in any tick."""
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
    t0 = clock()
    i = 0
    while i < n:
        now = clock() - t0
        if arr[i] > now:
            while clock() - t0 < arr[i]:
                pass
            now = clock() - t0
        kind = requests[i][0]
        if kind in (VINSERT, VDELETE):
            ids = requests[i][1]
            if kind == VINSERT:
                graph.insert_vertices(ids)
            else:
                graph.delete_vertices(ids)
            torch.cuda.synchronize(dev)
            done[i] = clock() - t0
            ticks.append((i, i + 1))
            i += 1
            continue
        j, pairs, need, fresh = i, 0, 0, False
        while j < n and arr[j] <= now and requests[j][0] in (INSERT, DELETE, QUERY):
            k = _size(requests[j])
            b = insert_block_bound(k, bs, vcap) if requests[j][0] == INSERT else 0
            if j > i and pairs + k > max_tick_pairs:
                break
            if need + b > free and not fresh:
                free = free_blocks(graph)  # the last tick has synchronised
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
        ws = [r for r in requests[i:j] if r[0] in (INSERT, DELETE)]
        qs = [(m, r) for m, r in enumerate(requests[i:j], start=i) if r[0] == QUERY]
        if ws:
            op = torch.cat([torch.full((_size(r),), r[0], dtype=torch.uint8, device=dev)
                            for r in ws])
            src = torch.cat([r[1] for r in ws])
            dst = torch.cat([r[2] for r in ws])
            gv.gv_apply_edge_ops(graph.h, op, src, dst, dev)
        if qs:
            out = graph.edge_exists(torch.cat([r[1] for _, r in qs]),
                                    torch.cat([r[2] for _, r in qs]))
        torch.cuda.synchronize(dev)
        t = clock() - t0
        done[i:j] = t
        if qs and keep_answers:
            o = 0
            out = out.cpu().numpy()
            for m, r in qs:
                answers[m] = out[o:o + _size(r)]
                o += _size(r)
        ticks.append((i, j))
        free -= need
        i = j
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
