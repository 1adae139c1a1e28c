"""Autotuner of the batched form.

For a workload it measures the hot path with each setting it tries and
keeps the fastest; the result goes to tuning.json beside this file, keyed by
workload, with the times it measured.  Two workloads:
  batched  a graph and a sequence of uneven batches (the batched form); knobs:
           block size B (8, 16, 32, 64 slots), coalescing of runs of edge
           batches into mixed lists, the longest run coalesced (pairs), the
           largest batch sorted by one workgroup, and the probe's shape;
  steps    insert + delete steps of equal batches on one graph (the
           benchmark's step, block size fixed by the workload); knobs: the
           probe's shape (lanes per work item, slots per lane per step) and
           the adjacency slots per work item.  Every setting is timed eagerly
(gv_apply_ops, coalescing as set) on a fresh copy of the same graph after
the same warm-up, and every run must end in the same graph (checksum and
edge count), so a setting cannot win by computing something else.

    python -m paper_2306_08252_amd.tuner                    # the batched workload
    python -m paper_2306_08252_amd.tuner --workload steps   # the benchmark's step
"""
import argparse
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_JSON = os.path.join(HERE, "tuning.json")


def workload_key(scale, edges, nbatch, seed_name):
    return f"rmat{scale}_e{edges}_batched{nbatch}_{seed_name}"


def load(key):
    """The stored setting for a workload, or None."""
    try:
        with open(TUNING_JSON) as f:
            return json.load(f).get(key)
    except (OSError, ValueError):
        return None


def store(key, entry):
    try:
        with open(TUNING_JSON) as f:
            t = json.load(f)
    except (OSError, ValueError):
        t = {}
    t[key] = entry
    with open(TUNING_JSON + ".tmp", "w") as f:
        json.dump(t, f, indent=1, sort_keys=True)
    os.replace(TUNING_JSON + ".tmp", TUNING_JSON)


def measure(gv, w, ops, dev, bs, tuning, warm, form="plan"):
    """Seconds for `ops` on a fresh graph with block size bs and the given
    tuning, and the resulting (checksum, edges).  form "plan": the ops
    recorded into one plan (recording not timed) and launched once; "eager":
    gv_apply_ops."""
    import torch
    g = gv.Graph(w.num_vertices, w.src, w.dst, block_slots=bs, device=dev)
    gv.gv_set_tuning(g.h, **tuning)
    warm(g)
    plan = gv.Plan(g.h, ops, dev) if form == "plan" else None
    arr, keep = gv._ops(ops, dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if plan is not None:
        plan.launch()
    else:
        gv._check(gv.lib().gv_apply_ops(gv.C.c_void_p(g.h), arr, len(ops)), "gv_apply_ops")
    rc = g.sync()
    el = time.perf_counter() - t0
    if plan is not None:
        plan.close()
    if rc != 0:
        raise RuntimeError(f"tuner: {gv.gv_strerror(rc)}")
    ck, e = gv.C.c_uint64(), gv.C.c_uint64()
    gv._check(gv.lib().gv_dump_canonical(gv.C.c_void_p(g.h), None, None, 0, gv.C.byref(ck),
                                         gv.C.byref(e)), "gv_dump_canonical")
    g.close()
    return el, (ck.value, e.value)


PROBE_SPACE = [("probe_group", [16, 32, 64]), ("probe_unroll", [2, 4, 8]),
               ("item_chunk", [64, 128, 256, 512, 1024, 2048, 4096])]
DEFAULT_PROBE = {"probe_group": 32, "probe_unroll": 4, "item_chunk": 256}


def descend(best, space, run):
    """Coordinate descent: each knob in turn takes its fastest value."""
    run(best)
    for knob, values in space:
        for v in values:
            cand = dict(best, **{knob: v})
            if run(cand) < run(best):
                best = cand
    return best


def tune(gv, w, ops, dev, warm, log=print, form="plan"):
    """Coordinate descent over the knobs, starting from the defaults, timing
    `form`; returns (best setting, all measured points in ms)."""
    best = dict({"block_slots": 16, "coalesce": 0, "max_run_pairs": 0, "small_sort_max": 4096,
                 "overlap": 0}, **DEFAULT_PROBE)
    space = [("block_slots", [8, 16, 32, 64]), ("coalesce", [0, 1]), ("overlap", [0, 1]),
             ("max_run_pairs", [0, 1 << 18, 1 << 20, 1 << 22]),
             ("small_sort_max", [0, 4096])] + PROBE_SPACE + [("block_slots", [8, 16, 32, 64])]
    points, want = {}, None

    def run(s):
        k = json.dumps(s, sort_keys=True)
        if k not in points:
            t = {x: s[x] for x in s if x != "block_slots"}
            el, dig = measure(gv, w, ops, dev, s["block_slots"], t, warm, form)
            nonlocal want
            if want is None:
                want = dig
            elif dig != want:
                raise RuntimeError(f"tuner: setting {s} changed the result")
            points[k] = el
            log(f"tuner: {s} -> {el * 1e3:.2f} ms")
        return points[k]

    best = descend(best, space, run)
    return best, {k: round(v * 1e3, 3) for k, v in points.items()}


def measure_steps(gv, w, ins, dels, dev, B, tuning, warmup=2, steps=10):
    """ms per insert + delete step on a fresh graph with the given tuning
    (the same batches for every setting), and the resulting (checksum, edges)."""
    import torch
    g = gv.Graph(w.num_vertices, w.src, w.dst, block_slots=B, device=dev)
    gv.gv_set_tuning(g.h, **tuning)
    for j in range(warmup):
        g.insert_edges(*ins[j], stats=False)
        g.delete_edges(*dels[j], stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(warmup, warmup + steps):
        g.insert_edges(*ins[j], stats=False)
        g.delete_edges(*dels[j], stats=False)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    rc = g.sync()
    if rc != 0:
        raise RuntimeError(f"tuner: {gv.gv_strerror(rc)}")
    _, _, ck, e = g.dump(checksum_only=True)
    g.close()
    return el, (ck, e)


def tune_steps(gv, w, ins, dels, dev, B, log=print):
    """Coordinate descent over the sort overlap, the probe's shape and the
    work-item size for the benchmark's step; returns (best setting, measured
    points in ms)."""
    points, want = {}, None

    def run(s):
        nonlocal want
        k = json.dumps(s, sort_keys=True)
        if k not in points:
            el, dig = measure_steps(gv, w, ins, dels, dev, B, s)
            if want is None:
                want = dig
            elif dig != want:
                raise RuntimeError(f"tuner: setting {s} changed the result")
            points[k] = el
            log(f"tuner: {s} -> {el * 1e3:.3f} ms per step")
        return points[k]

    space = [("overlap", [0, 1])] + PROBE_SPACE + PROBE_SPACE[:2]
    best = descend(dict(DEFAULT_PROBE, overlap=0), space, run)
    return best, {k: round(v * 1e3, 4) for k, v in points.items()}


def steps_key(scale, edges, batch, B):
    return f"rmat{scale}_e{edges}_steps{batch}_b{B}"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=("batched", "steps"), default="batched")
    ap.add_argument("--scale", type=int, default=None)
    ap.add_argument("--edges", type=int, default=None)
    ap.add_argument("--batches", type=int, default=256)
    ap.add_argument("--batch", type=int, default=10**6)
    ap.add_argument("--block-slots", type=int, default=16)
    ap.add_argument("--seed-name", default="batched")
    args = ap.parse_args()
    import torch

    from . import graphvine as gv
    from . import inputs_torch as T
    from . import workloads as Wk
    dev = torch.device("cuda:0")
    if args.workload == "steps":
        scale = args.scale or 20
        edges = args.edges or 1 << 24
        w = T.RmatWorkload(scale, edges, device=dev)
        ins = [w.insert_batch(args.batch, 1000 + j) for j in range(12)]
        dels = [w.delete_batch(args.batch, 1000 + j) for j in range(12)]
        best, points = tune_steps(gv, w, ins, dels, dev, args.block_slots)
        key = steps_key(scale, edges, args.batch, args.block_slots)
        store(key, {"setting": best, "ms": points[json.dumps(best, sort_keys=True)],
                    "measured_ms": points})
        print(json.dumps({"key": key, "best": best}))
        return
    args.scale = args.scale or 22
    args.edges = args.edges or 1 << 26
    w = T.RmatWorkload(args.scale, args.edges, name=args.seed_name, device=dev)
    ops, pairs, vids = Wk.batched_ops(w, args.seed_name, args.batches, dev)
    warm = Wk.batched_warmup(ops)
    best, points = tune(gv, w, ops, dev, warm)
    key = workload_key(args.scale, args.edges, args.batches, args.seed_name)
    store(key, {"setting": best, "ms": points[json.dumps(best, sort_keys=True)],
                "measured_ms": points, "pairs": pairs, "vertex_ids": vids})
    print(json.dumps({"key": key, "best": best}))


if __name__ == "__main__":
    main()
