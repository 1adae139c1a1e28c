#!/usr/bin/env python3
"""Benchmark of the GraphVine hot path on one MI355X.

Workload: directed R-MAT graph (a, b, c, d) = (0.57, 0.19, 0.19, 0.05) with
2^20 vertices and 2^24 distinct edges, block size B = 16, drawn on the GPU
from the seeded streams of paper_2306_08252_amd.inputs.  A step is one
batched edge insert of 10^6 R-MAT pairs followed by one batched edge delete
of 10^6 pairs (80 % existing edges, 20 % uniform pairs), both applied to the
resident graph through the C ABI with inputs already in HBM.

value = (insert pairs + delete pairs) per second over the timed steps.  The
same run also times, each in its own loop: bulk build from COO (init
edges/s), batched edge queries, vertex insert/delete batches, an adjacency
read of the largest hub and the memory report.

roofline: the kernel with the largest share of the step's GPU time, its
algorithmic bytes per launch over its average launch time.  Algorithmic bytes
follow the bytes-touched model M1 (counted once per batch): the grouping of a
batch is 16 B per pair (one write and one read of the packed pairs) however
many radix passes it takes, so a pass is credited 16 B per pair / passes; a
probe is credited the touched adjacency (4 B per slot, block granular).  The
launch time comes from HIP events on the kernel's stream in a second run of
the same steps with the sort overlap off, so that the kernel runs alone on
the device (under the overlap a pass shares it with the other stream's
kernels, and its events would also time its wait for compute units), one
event pair per run of consecutive launches of the kernel (the passes of one
sort share a pair, so the events' own cost is spread over them); the
committed kernel-trace summary of the same command gives the durations
without events.

cpu_baseline: the CPU oracle (ordered sets, one thread) applying the same
batches restricted to a quarter of the sources (those whose SplitMix64 hash
is 0 mod 4) to the same graph restricted the same way.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CPU_STEPS = 12  # batch pairs the oracle replays (about 10 s of one core)
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_JSON = os.path.join(PROFILES, "traffic_rmat20_b16_batch1e6.json")


def sources_digest():
    """SHA-256 over the kernel sources; a stored counter reading is used only
    while it matches (the kernels have not changed since it was taken)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2306_08252_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when there is none for it or the kernel sources changed since."""
    try:
        with open(TRAFFIC_JSON) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256") != sources_digest():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else int(k["fetch_bytes"] + k["write_bytes"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_model(name, per_launch):
    """Algorithmic bytes of one launch of `name` (counted once, at any cache
    level).  per_launch holds the averages of the batch quantities:
    k (pairs), T (touched sources), S (block-granular slots of the touched
    adjacencies), NB (blocks per touched adjacency, S / B), W (slots written),
    M (slots moved), NEW / FREED (blocks)."""
    k, T, S, NBLK = per_launch["k"], per_launch["T"], per_launch["S"], per_launch["NB"]
    P = per_launch.get("passes", 5)
    if name in ("probe_insert", "probe_delete", "probe_query"):
        # M1: the touched adjacency, scanned once (block-granular slots)
        return 4 * S
    tiles = (k + 4095) // 4096
    groups = min(tiles, 256)
    if name == "sort_pass":
        # M1: grouping is one write and one read of the packed pairs per
        # batch (16 B per pair), shared by the batch's radix passes
        return 16 * k / P
    if name == "sort_hist":
        # insert / delete batches: add the per-group digit counts of the
        # packing kernel (and the valid-pair counts) into the pass histograms
        return 4 * 256 * P * (groups + 1) + 4 * groups
    if name == "pack":
        # pairs in, keys and mark bytes out, the batch's look-back state
        # cleared, per-group digit counts out
        return 8 * k + 8 * k + k + 4 * (64 + P * tiles * 256 + P * ((tiles + 15) // 16) * 256) \
            + 4 * 256 * P * groups
    if name == "segments":
        return 8 * k + k + 4 * k + 8 * T  # keys in; flags, ranks, segment starts out
    if name == "items":
        return 8 * T + 16 * T + 32 * T  # segment list, vertex records, items out
    if name == "append":
        return k + k + 4 * k + 4 * per_launch["W"] + 16 * T
    if name == "compact":
        return 8 * per_launch["M"] + 16 * T + 4 * per_launch["FREED"]
    return None


def counter_delta(c0, c1):
    import numpy as np
    return {key: (np.array(c1[key]) - np.array(c0[key])) for key in c1}


def m1_bytes(pairs, d):
    """Bytes model M1 of edge batches (pairs read, one grouping pass, touched
    adjacency scan, slot writes, vertex records, block bookkeeping) from the
    library's counter deltas `d`."""
    return pairs * (8 + 16) + 4 * int(d["scanned_slots"][0] + d["scanned_slots"][1]) \
        + 4 * int(d["written_slots"]) + 16 * int(d["touched"][0] + d["touched"][1]) \
        + 8 * int(d["new_blocks"]) + 8 * int(d["moved_slots"]) + 4 * int(d["freed_blocks"])


def config3_form(gv, I, T, dev, k=10**7, nv=10**4):
    """Large graphs: R-MAT 2^24 vertices / 2^28 edges (B = 16) and the
    road-like 4096 x 4096 lattice (B = 8), each with one insert and one
    delete batch of 10^7 edges (R-MAT: R-MAT pairs, then 80 % stored and 20 %
    uniform pairs; lattice: 5 * 10^6 uniform undirected pairs stored both
    ways, then half of them and a slice of the lattice, both ways), then a
    vertex delete and re-insert batch of 10^4 uniform ids.  Each graph first
    takes an untimed insert and delete of other batches of the same sizes,
    and the vertex batches an untimed delete and re-insert of other ids
    (sizes the buffers).  Per batch: edges/s and the M1 fraction of HBM
    peak from the library's counters."""
    import numpy as np
    import torch

    def timed(g, fn, *a):
        torch.cuda.synchronize()
        c0 = g.counters()
        t0 = time.perf_counter()
        st = fn(*a)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        return st, el, counter_delta(c0, g.counters())

    def edge_row(g, fn, s, d, label):
        st, el, dd = timed(g, fn, s, d)
        m1 = m1_bytes(int(s.numel() if hasattr(s, "numel") else len(s)), dd)
        return {"pairs": int(len(s)), "ms": round(el * 1e3, 3),
                "edges_per_s": round(len(s) / el, 1), "applied": int(st[0]),
                "pct_hbm_m1": round(m1 / el / (HBM_PEAK_GBS * 1e9), 5), "op": label}

    def vertex_rows(g, n, tag):
        def draw(*name):
            return torch.from_numpy((I.splitmix64(I.stream_seed(tag, *name), nv) % np.uint64(n))
                                    .astype(np.uint32).view(np.int32)).to(dev)
        warm = draw("warm")  # untimed: sizes the buffers
        g.delete_vertices(warm)
        g.insert_vertices(warm)
        ids = draw("vertices")
        st, el_d, _ = timed(g, g.delete_vertices, ids)
        st2, el_i, _ = timed(g, g.insert_vertices, ids)
        return {"ids": nv, "delete_ms": round(el_d * 1e3, 3), "insert_ms": round(el_i * 1e3, 3),
                "delete_stats": st, "insert_stats": st2}

    out = {}
    w = T.RmatWorkload(24, 1 << 28, name="scale", device=dev)
    g = gv.Graph(w.num_vertices, w.src, w.dst, block_slots=16, device=dev)
    g.insert_edges(*w.insert_batch(k, 7), stats=False)
    g.delete_edges(*w.delete_batch(k, 7), stats=False)
    ins = edge_row(g, g.insert_edges, *w.insert_batch(k, 0), "insert")
    dele = edge_row(g, g.delete_edges, *w.delete_batch(k, 0), "delete")
    out["rmat24_e2^28_b16"] = {"insert_1e7": ins, "delete_1e7": dele,
                               "vertex_1e4": vertex_rows(g, w.num_vertices, "config3-rmat"),
                               "edges_after": g.memory_used()["num_edges"]}
    g.close()
    del w
    torch.cuda.empty_cache()
    side = 4096
    n = side * side
    src, dst = I.lattice_graph(I.stream_seed("road", side), side)
    g = gv.Graph(n, src, dst, block_slots=8, device=dev)

    def both(a, b):
        return (torch.from_numpy(np.concatenate([a, b]).view(np.int32)).to(dev),
                torch.from_numpy(np.concatenate([b, a]).view(np.int32)).to(dev))
    wa, wb = I.uniform_pairs(I.stream_seed("road-warm", side), k // 2, n)
    g.insert_edges(*both(wa, wb), stats=False)
    g.delete_edges(*both(wa, wb), stats=False)
    a, b = I.uniform_pairs(I.stream_seed("road-ins", side), k // 2, n)
    ins = edge_row(g, g.insert_edges, *both(a, b), "insert")
    da = np.concatenate([a[: k // 4], src[: k // 4]])
    db = np.concatenate([b[: k // 4], dst[: k // 4]])
    dele = edge_row(g, g.delete_edges, *both(da, db), "delete")
    out["lattice4096_b8"] = {"insert_1e7": ins, "delete_1e7": dele,
                             "vertex_1e4": vertex_rows(g, n, "config3-road"),
                             "edges_after": g.memory_used()["num_edges"]}
    rc = g.sync()
    g.close()
    if rc != 0:
        raise RuntimeError(f"config3: {gv.gv_strerror(rc)}")
    return out


def implementation_bytes(name, per_launch):
    """What the kernel itself must move per launch (not M1): a radix pass
    reads and writes every key; a probe also reads directory entries, work
    items, the batch keys and writes marks."""
    k, T, S, NBLK = per_launch["k"], per_launch["T"], per_launch["S"], per_launch["NB"]
    if name == "sort_pass":
        return 16 * k
    if name in ("probe_insert", "probe_delete", "probe_query"):
        return 4 * S + 4 * NBLK + 32 * T + 8 * k + k
    return None


def host_cpu():
    """CPU model (from /proc/cpuinfo) and the number of logical CPUs."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_available": avail}


def summarize_counters(pmc_dir, out_md, command, title):
    """Per-kernel averages of every counter in a rocprofv3 --pmc run (library
    kernels, grouped by kernel and grid size)."""
    import statistics
    acc = {}
    for r in _rows(pmc_dir, "counter_collection"):
        if "gv::" not in r["Kernel_Name"]:
            continue
        wg = int(r["Grid_Size"]) // max(1, int(r["Workgroup_Size"]))
        acc.setdefault((_short(r["Kernel_Name"]), wg), {}).setdefault(
            r["Counter_Name"], []).append(float(r["Counter_Value"]))
    names = sorted({c for v in acc.values() for c in v})
    lines = ["| kernel | grid (WGs) | dispatches | " + " | ".join(names) + " |",
             "|---|---|---|" + "---|" * len(names)]
    for (k, wg), cs in sorted(acc.items(), key=lambda kv: kv[0]):
        nd = max(len(v) for v in cs.values())
        vals = [f"{statistics.mean(cs[c]):.0f}" if c in cs else "" for c in names]
        lines.append(f"| `{k}` | {wg} | {nd} | " + " | ".join(vals) + " |")
    with open(out_md, "w") as f:
        f.write(f"# {title}\n\nCommand (repo root as $R):\n\n```\n{command}\n```\n\n"
                "Average counter value per dispatch, library kernels only:\n\n" +
                "\n".join(lines) + "\n")


# library launch names -> kernel symbol prefix in rocprofv3 output
KERNEL_SYMBOLS = {
    "sort_pass": "gv::k_os_pass<unsigned long, false>",
    "sort_hist": "gv::k_os_hist_sum",
    "pack": "gv::k_pack_hist(",
    "probe_insert": "gv::k_probe<0,",
    "probe_delete": "gv::k_probe<1,",
    "probe_query": "gv::k_probe<2,",
    "compact": "gv::k_compact(",
    "append": "gv::k_append(",
}


def _rows(csv_dir, kind):
    import csv
    import glob
    files = glob.glob(os.path.join(csv_dir, "**", f"*{kind}.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no *{kind}.csv under {csv_dir}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _short(name):
    return name.replace("void ", "").split("(")[0]


def summarize_trace(trace_dir, out_md, command):
    """Per-kernel launch counts and durations of the library kernels."""
    import statistics
    agg = {}
    for r in _rows(trace_dir, "kernel_trace"):
        if "gv::" not in r["Kernel_Name"]:
            continue
        wg = int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"]))
        key = (_short(r["Kernel_Name"]), wg)
        agg.setdefault(key, []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    lines = ["| kernel | grid (WGs) | launches | avg us | total us |", "|---|---|---|---|---|"]
    for (k, wg), v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| `{k}` | {wg} | {len(v)} | {statistics.mean(v) / 1e3:.2f} | "
                     f"{sum(v) / 1e3:.1f} |")
    with open(out_md, "w") as f:
        f.write(f"# Kernel trace: {os.path.basename(out_md)[:-3]}\n\nCommand (repo root "
                f"as $R):\n\n```\n{command}\n```\n\nDurations from the kernel trace (ns -> "
                f"us), library kernels only:\n\n" + "\n".join(lines) + "\n")


def summarize_traffic(fetch_dir, write_dir, cfetch_dir, cwrite_dir, grid_wgs, out_md, commands):
    """HBM bytes per dispatch from FETCH_SIZE / WRITE_SIZE (KiB per dispatch),
    scaled by what the same counters read for a plain 1 GiB device copy."""
    import statistics

    def per_kernel(d, counter, pick):
        acc = {}
        for r in _rows(d, "counter_collection"):
            if r["Counter_Name"] != counter or not pick(r):
                continue
            wg = int(r["Grid_Size"]) // max(1, int(r["Workgroup_Size"]))
            acc.setdefault((r["Kernel_Name"], wg), []).append(float(r["Counter_Value"]) * 1024)
        return acc

    copy = lambda r: "gv::" not in r["Kernel_Name"] and "copy" in r["Kernel_Name"].lower()
    cf = per_kernel(cfetch_dir, "FETCH_SIZE", copy)
    cw = per_kernel(cwrite_dir, "WRITE_SIZE", copy)
    gib = float(1 << 30)
    f_factor = gib / statistics.mean(max(cf.values(), key=len))
    w_factor = gib / statistics.mean(max(cw.values(), key=len))
    kf = per_kernel(fetch_dir, "FETCH_SIZE", lambda r: "gv::" in r["Kernel_Name"])
    kw = per_kernel(write_dir, "WRITE_SIZE", lambda r: "gv::" in r["Kernel_Name"])
    kernels = {}
    lines = ["| launch name | kernel | grid (WGs) | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB "
             "| HBM read B (scaled) | HBM write B (scaled) |", "|---|---|---|---|---|---|---|---|"]
    for name, sym in KERNEL_SYMBOLS.items():
        wg = grid_wgs.get(name)
        # a symbol ending in "," names every shape of a templated kernel
        same = lambda k, g: (_short(k) == sym.rstrip("(") or
                             (sym.endswith(",") and _short(k).startswith(sym))) \
            and (wg is None or g == wg)
        fk = [v for (k, g), v in kf.items() if same(k, g)]
        wk = [v for (k, g), v in kw.items() if same(k, g)]
        if not fk or not wk:
            continue
        fv = max(fk, key=len)
        wv = max(wk, key=len)
        fb = statistics.mean(fv) / 1024
        wb = statistics.mean(wv) / 1024
        kernels[name] = {"fetch_bytes": round(fb * 1024 * f_factor), "write_bytes":
                         round(wb * 1024 * w_factor), "dispatches": len(fv)}
        lines.append(f"| {name} | `{sym.rstrip('(')}` | {wg} | {len(fv)} | {fb:.0f} | {wb:.0f} | "
                     f"{kernels[name]['fetch_bytes']} | {kernels[name]['write_bytes']} |")
    t = {"sources_sha256": sources_digest(), "fetch_factor": f_factor, "write_factor": w_factor,
         "kernels": kernels}
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(t, f, indent=1)
    with open(out_md, "w") as f:
        f.write("# HBM traffic per dispatch: R-MAT 2^20 / 2^24 edges, B=16, batches of 10^6\n\n"
                "Commands (repo root as $R):\n\n```\n" + "\n".join(commands) +
                "\n```\n\nCalibration: a plain 1 GiB device copy reads "
                f"{1 / f_factor:.3f} GiB by FETCH_SIZE and writes {1 / w_factor:.3f} GiB by "
                f"WRITE_SIZE, so FETCH_SIZE is scaled by {f_factor:.3f} and WRITE_SIZE by "
                f"{w_factor:.3f}.  The scaled bytes per dispatch are stored in "
                f"`{os.path.basename(TRAFFIC_JSON)}` with the SHA-256 of the kernel sources "
                "they were measured on; `bench.py` reports them as `roofline.traffic` only "
                "while the sources match.\n\n" + "\n".join(lines) + "\n")


def cbt_form(gv, w, dev, B, ins, dels, first, steps=2):
    """The paper's own layout and algorithms (complete binary tree of edge
    blocks, one thread per vertex, Alg. 1-3; gv_cbt_*) on the same graph and
    the same insert + delete batches as the timed steps: build, one untimed
    step, then `steps` timed ones."""
    import torch
    n = w.num_vertices
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c = gv.CbtGraph(n, w.src, w.dst, block_slots=B, device=dev)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t0
    c.insert_edges(*ins[first - 1])
    c.delete_edges(*dels[first - 1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pairs = 0
    for j in range(first, first + steps):
        c.insert_edges(*ins[j])
        c.delete_edges(*dels[j])
        pairs += int(ins[j][0].numel()) + int(dels[j][0].numel())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    blocks = c.blocks()
    c.close()
    return {"form": "complete binary tree of edge blocks, bit-string placement, one thread "
                    "per vertex for insert and delete (Alg. 1-2), holes left by deletes",
            "steps": steps, "ms_per_step": round(el / steps * 1e3, 3),
            "edges_per_s": round(pairs / el, 1), "init_ms": round(init_s * 1e3, 3),
            "blocks_handed_out": blocks}


def block_size_sweep(gv, w, dev, ks=(10**4, 10**5, 10**6), block_slots=(8, 16, 32, 64),
                     steps=4):
    """Insert + delete edges/s on the same R-MAT graph for every block size
    and batch size (a fresh graph per block size; one untimed step, then
    `steps` timed ones per batch size, in order of batch size)."""
    import torch
    out = []
    for bs in block_slots:
        g = gv.Graph(w.num_vertices, w.src, w.dst, block_slots=bs, device=dev)
        for k in ks:
            ins = [w.insert_batch(k, 90000 + j) for j in range(steps + 1)]
            dels = [w.delete_batch(k, 90000 + j) for j in range(steps + 1)]
            gv.gv_insert_edges(g.h, *ins[0], dev, stats=False)
            gv.gv_delete_edges(g.h, *dels[0], dev, stats=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for j in range(1, steps + 1):
                gv.gv_insert_edges(g.h, *ins[j], dev, stats=False)
                gv.gv_delete_edges(g.h, *dels[j], dev, stats=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            out.append({"block_slots": bs, "batch": k,
                        "edges_per_s": round(2 * k * steps / el, 1)})
        rc = g.sync()
        g.close()
        if rc != 0:
            raise RuntimeError(f"block-size sweep: {gv.gv_strerror(rc)}")
    return out


def batch_latency(gv, w, dev, tuning, ks=(10**3, 10**4, 10**5), nb=20):
    """Time per batch of small insert / delete batches on the headline graph
    (B = 16), alternating inserts and deletes: queued one call at a time
    (eager), and recorded into one plan launched three times (no host work
    per batch), each with the sort overlap off and on (other knobs from
    `tuning`); a fresh graph per form."""
    import torch
    out = []
    for k in ks:
        ins = [w.insert_batch(k, 5000 + j) for j in range(2 * nb)]
        dels = [w.delete_batch(k, 5000 + j) for j in range(2 * nb)]
        torch.cuda.synchronize()
        row = {"batch": k}
        for form in ("eager", "plan"):
            for ov in (0, 1):
                g = gv.Graph(w.num_vertices, w.src, w.dst, block_slots=16, device=dev)
                gv.gv_set_tuning(g.h, **dict(tuning, overlap=ov))
                if form == "eager":
                    for j in range(3):
                        gv.gv_insert_edges(g.h, *ins[j], dev, stats=False)
                        gv.gv_delete_edges(g.h, *dels[j], dev, stats=False)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for j in range(nb):
                        gv.gv_insert_edges(g.h, *ins[j], dev, stats=False)
                        gv.gv_delete_edges(g.h, *dels[j], dev, stats=False)
                    torch.cuda.synchronize()
                    el = (time.perf_counter() - t0) / (2 * nb)
                else:
                    ops = []
                    for j in range(nb, 2 * nb):
                        ops.append((gv.OP_INSERT_EDGES, *ins[j]))
                        ops.append((gv.OP_DELETE_EDGES, *dels[j]))
                    plan = gv.Plan(g.h, ops, dev)
                    plan.launch()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(3):
                        plan.launch()
                    torch.cuda.synchronize()
                    el = (time.perf_counter() - t0) / (3 * 2 * nb)
                    plan.close()
                rc = g.sync()
                g.close()
                if rc != 0:
                    raise RuntimeError(f"batch latency: {gv.gv_strerror(rc)}")
                row[f"{form}_overlap{ov}_us"] = round(el * 1e6, 2)
        out.append(row)
    return out


def batched_form(gv, I, T, dev, scale=22, edges=1 << 26, nbatch=256, seed_name="batched"):
    """The batched form: `nbatch` batches of log-uniform size in [10^2, 10^6],
    45 % edge inserts (R-MAT pairs), 45 % edge deletes (80 % stored pairs, 20 %
    uniform), 10 % vertex batches (min(size, 10^4) uniform ids, insert or
    delete alike), applied in order.  Baseline: gv_apply_ops at the default
    settings (B = 16, no coalescing), one launch sequence per batch.  Tuned:
    the setting the autotuner stored for this workload in tuning.json (block
    size, coalescing of edge-batch runs into mixed lists, run cap, small-sort
    cutoff; tuned here when none is stored), first eagerly, then recorded
    into one HIP graph (gv_plan_create, not timed) and launched once.  Each
    run starts from a fresh copy of the graph after the same warm-up (which
    sizes the scratch buffers); every run must end with the same checksum
    and edge count."""
    import torch
    from paper_2306_08252_amd import tuner as Tu
    from paper_2306_08252_amd import workloads as Wk
    w = T.RmatWorkload(scale, edges, name=seed_name, device=dev)
    ops, pairs, vids = Wk.batched_ops(w, seed_name, nbatch, dev)
    warm = Wk.batched_warmup(ops)
    key = Tu.workload_key(scale, edges, nbatch, seed_name)
    stored = Tu.load(key)
    if stored is None:
        best, points = Tu.tune(gv, w, ops, dev, warm, log=lambda *a: None)
        source = "tuned in this run"
    else:
        best, points = stored["setting"], stored["measured_ms"]
        source = "tuning.json"
    knobs = {k: v for k, v in best.items() if k != "block_slots"}
    base = dict({"coalesce": 0, "max_run_pairs": 0, "small_sort_max": 4096}, **Tu.DEFAULT_PROBE)
    el_base, want = Tu.measure(gv, w, ops, dev, 16, base, warm, "eager")
    el_eager, got_e = Tu.measure(gv, w, ops, dev, best["block_slots"], knobs, warm, "eager")
    el_plan, got_p = Tu.measure(gv, w, ops, dev, best["block_slots"], knobs, warm, "plan")
    if got_e != want or got_p != want:
        raise RuntimeError(f"batched form: results differ: {want} {got_e} {got_p}")
    torch.cuda.synchronize()
    return {"workload": f"rmat{scale} {edges} edges, {nbatch} batches of log-uniform "
                        "size in [1e2, 1e6], 45/45/10 insert/delete/vertex",
            "pairs": pairs, "vertex_ids": vids,
            "baseline_form": "one launch sequence per batch, B=16, no coalescing",
            "ms": round(el_base * 1e3, 3), "edges_per_s": round(pairs / el_base, 1),
            "tuned_setting": best, "tuning_source": source,
            "tuner_points_ms": points,
            "tuned_eager_ms": round(el_eager * 1e3, 3),
            "plan_ms": round(el_plan * 1e3, 3),
            "plan_edges_per_s": round(pairs / el_plan, 1),
            "plan_form": "the sequence recorded as one HIP graph, tuned setting",
            "plan_gain_vs_baseline": round(el_base / el_plan - 1.0, 4),
            "plan_gain_vs_tuned_eager": round(el_eager / el_plan - 1.0, 4),
            "results_match": True, "checksum": want[0], "edges_after": want[1]}


def served_form(gv, I, T, dev, B, scale=24, edges=1 << 28, nreq=1500, loads=(0.3, 0.6, 0.9),
                seed_name="served"):
    """The served form: requests of log-uniform size in [1, 10^5] pairs, 40 %
    edge inserts (R-MAT pairs), 40 % edge deletes (80 % stored pairs), 15 %
    queries (half stored pairs), 5 % vertex batches (min(size, 10^4) ids,
    insert or delete alike), served by continuous batching (ticks of at most
    2^20 pairs; one mixed update list and one query batch per tick; vertex
    requests alone).  Saturated throughput: every request available at time
    0.  Then open-loop Poisson arrivals at `loads` x that throughput, a fresh
    request list each; latency = completion - scheduled arrival, p50 / p99
    by nearest rank.  Baseline: another request list of the same mix applied
    one request at a time with the single-batch calls, back to back."""
    import numpy as np
    import torch
    from paper_2306_08252_amd import served as S
    w = T.RmatWorkload(scale, edges, name=seed_name, device=dev)
    n = w.num_vertices

    def requests(tag):
        draws = I.splitmix64(I.stream_seed(seed_name, "requests", tag), 3 * nreq)
        base = 1_000_000 * (1 + ["warm", "baseline", "saturated",
                                 *(f"load{x}" for x in loads)].index(tag))
        reqs = []
        for j in range(nreq):
            u = float(draws[3 * j] >> np.uint64(11)) / float(1 << 53)
            size = max(1, int(round(np.exp(u * np.log(10**5)))))
            r = float(draws[3 * j + 1] >> np.uint64(11)) / float(1 << 53)
            if r < 0.40:
                reqs.append((S.INSERT,) + tuple(w.insert_batch(size, base + j)))
            elif r < 0.80:
                ne = int(round(0.8 * size))
                es, ed = T.pick(I.stream_seed(seed_name, "del", tag, j), ne, w.src, w.dst)
                us, ud = T.uniform_pairs(I.stream_seed(seed_name, "del-u", tag, j), size - ne, n,
                                         device=dev)
                reqs.append((S.DELETE, torch.cat([es, us]), torch.cat([ed, ud])))
            elif r < 0.95:
                qe = size // 2
                es, ed = T.pick(I.stream_seed(seed_name, "q", tag, j), qe, w.src, w.dst)
                us, ud = T.uniform_pairs(I.stream_seed(seed_name, "q-u", tag, j), size - qe, n,
                                         device=dev)
                reqs.append((S.QUERY, torch.cat([es, us]), torch.cat([ed, ud])))
            else:
                m = min(size, 10**4)
                ids = torch.from_numpy((I.splitmix64(I.stream_seed(seed_name, "v", tag, j), m)
                                        % np.uint64(n)).astype(np.uint32).view(np.int32)).to(dev)
                kind = S.VINSERT if draws[3 * j + 2] & np.uint64(1) else S.VDELETE
                reqs.append((kind, ids, None))
        return reqs

    def pairs_of(reqs):
        return sum(int(r[1].numel()) for r in reqs if r[0] in (S.INSERT, S.DELETE, S.QUERY))

    g = gv.Graph(n, w.src, w.dst, block_slots=B, device=dev)
    warm = requests("warm")
    S.serve(g, warm[:64])
    # one launch sequence per request, back to back (the baseline)
    base_reqs = requests("baseline")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for kind, a, b in base_reqs:
        if kind == S.INSERT:
            gv.gv_insert_edges(g.h, a, b, dev, stats=False)
        elif kind == S.DELETE:
            gv.gv_delete_edges(g.h, a, b, dev, stats=False)
        elif kind == S.QUERY:
            g.edge_exists(a, b)
        elif kind == S.VINSERT:
            g.insert_vertices(a)
        else:
            g.delete_vertices(a)
    torch.cuda.synchronize()
    el_base = time.perf_counter() - t0
    # served, saturated: every request available at time 0
    sat_reqs = requests("saturated")
    torch.cuda.synchronize()
    done, ticks, _ = S.serve(g, sat_reqs)
    sat = nreq / done[-1]
    out = {"workload": f"rmat{scale} {edges} edges, B={B}, {nreq} requests per run of "
                       "log-uniform size in [1, 1e5], 40/40/15/5 insert/delete/query/vertex",
           "one_launch_per_request": {"req_per_s": round(nreq / el_base, 1),
                                      "edges_per_s": round(pairs_of(base_reqs) / el_base, 1)},
           "saturated_req_per_s": round(sat, 1),
           "saturated_edges_per_s": round(pairs_of(sat_reqs) / done[-1], 1),
           "saturated_ticks": len(ticks), "runs": []}
    for load in loads:
        reqs = requests(f"load{load}")
        draws = I.splitmix64(I.stream_seed(seed_name, "arrivals", load), nreq)
        arr = S.poisson_arrivals(draws, load * sat)
        torch.cuda.synchronize()
        done, ticks, _ = S.serve(g, reqs, arr)
        lat = (done - arr) * 1e3
        out["runs"].append({"load": load, "offered_req_per_s": round(load * sat, 1),
                            "edges_per_s": round(pairs_of(reqs) / done[-1], 1),
                            "p50_ms": round(S.nearest_rank(lat, 0.5), 3),
                            "p99_ms": round(S.nearest_rank(lat, 0.99), 3),
                            "ticks": len(ticks), "span_s": round(float(done[-1]), 3)})
    rc = g.sync()
    g.close()
    if rc != 0:
        raise RuntimeError(f"served form: {gv.gv_strerror(rc)}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=10**6)
    ap.add_argument("--block-slots", type=int, default=16)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--edges", type=int, default=1 << 24)
    ap.add_argument("--queries", type=int, default=5, help="timed query batches")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-form workload (eager and recorded forms)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the block-size x batch-size sweep and the small-batch latencies")
    ap.add_argument("--no-cbt", action="store_true",
                    help="skip the paper-faithful ablation (complete binary tree, Alg. 1-3)")
    ap.add_argument("--no-config3", action="store_true",
                    help="skip R-MAT 2^24 / 2^28 and the 4096^2 lattice with 10^7-edge batches")
    ap.add_argument("--no-served", action="store_true",
                    help="skip the served-form workload (continuous batching, p50/p99)")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_DIR", "OUT_MD"),
                    help="write a kernel-trace summary (no GPU)")
    ap.add_argument("--summarize-traffic", nargs=5,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR", "OUT_MD"),
                    help="write the HBM traffic summary and its JSON (no GPU)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("PMC_DIR", "OUT_MD"),
                    help="write per-kernel averages of a rocprofv3 --pmc run (no GPU)")
    ap.add_argument("--title", default="Counters per dispatch")
    ap.add_argument("--command", action="append", default=[],
                    help="command line recorded in a summary")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()

    if args.summarize_trace:
        summarize_trace(*args.summarize_trace, "\n".join(args.command))
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, "\n".join(args.command), args.title)
        return
    if args.summarize_traffic:
        k = args.batch
        grid = {"sort_pass": (k + 4095) // 4096, "probe_insert": None, "probe_delete": None,
                "probe_query": None, "compact": None, "append": (k + 255) // 256,
                "sort_hist": None, "pack": min((k + 4095) // 4096, 256)}
        summarize_traffic(*args.summarize_traffic[:4], grid, args.summarize_traffic[4],
                          args.command)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        x = torch.ones(1 << 28, dtype=torch.int32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4,
                          "launches": 3}))
        return

    from paper_2306_08252_amd import graphvine as gv
    from paper_2306_08252_amd import inputs as I
    from paper_2306_08252_amd import inputs_torch as T

    dev = torch.device("cuda:0")
    k, B = args.batch, args.block_slots
    log(f"generating R-MAT 2^{args.scale} / {args.edges} edges on the GPU")
    w = T.RmatWorkload(args.scale, args.edges, device=dev)
    n = w.num_vertices
    # warm-up, pilot, timed steps, then as many steps again with events
    nsteps = args.warmup + 1 + 2 * args.steps
    ins = [w.insert_batch(k, j) for j in range(nsteps)]
    dels = [w.delete_batch(k, j) for j in range(nsteps)]
    qry = [w.query_batch(k, j) for j in range(args.queries + 1)]
    torch.cuda.synchronize()

    # ---- bulk build (init edges/s): one warm-up build, then the timed one
    g0 = gv.Graph(n, w.src, w.dst, block_slots=B, device=dev)
    g0.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = gv.Graph(n, w.src, w.dst, block_slots=B, device=dev)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t0
    log(f"init {init_s * 1e3:.2f} ms")

    # the step's tuning (probe shape, work-item size) stored by the tuner for
    # this workload, if any
    from paper_2306_08252_amd import tuner as Tu
    step_tuning = Tu.load(Tu.steps_key(args.scale, args.edges, k, B))
    if step_tuning:
        gv.gv_set_tuning(g.h, **step_tuning["setting"])
    step_setting = dict(gv.gv_get_tuning(g.h),
                        source="tuning.json" if step_tuning else "defaults")
    h = g.h
    for j in range(args.warmup):
        gv.gv_insert_edges(h, *ins[j], dev, stats=False)
        gv.gv_delete_edges(h, *dels[j], dev, stats=False)
    torch.cuda.synchronize()

    # the pilot step and the roofline's event run time each kernel alone: with
    # the sort overlap on, a pass would share the device with the other
    # stream's kernels and its events would also count its wait for a slot
    overlap = step_setting.get("overlap", 0)
    gv.gv_set_tuning(h, overlap=0)

    # ---- pilot step (untimed): every kernel timed, to find the dominant one
    gv.gv_profile_enable(h, True)
    gv.gv_profile_only(h, None)
    gv.gv_profile_reset(h)
    j = args.warmup
    gv.gv_insert_edges(h, *ins[j], dev, stats=False)
    gv.gv_delete_edges(h, *dels[j], dev, stats=False)
    torch.cuda.synchronize()
    names = gv.gv_kernel_names(h)
    pilot = {}
    for nm in names:
        cnt, ms = gv.gv_kernel_times(h, nm)
        if cnt:
            pilot[nm] = {"launches": cnt, "ms": round(ms, 4)}
    dominant = max(pilot, key=lambda x: pilot[x]["ms"])
    log("pilot step kernels:", json.dumps(pilot))

    # ---- timed region: steps of insert + delete, no events (an event record
    # between two kernels costs about 5 us of GPU time)
    gv.gv_profile_enable(h, False)
    gv.gv_set_tuning(h, overlap=overlap)
    c0 = g.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    first = args.warmup + 1
    for j in range(first, first + args.steps):
        gv.gv_insert_edges(h, *ins[j], dev, stats=False)
        gv.gv_delete_edges(h, *dels[j], dev, stats=False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    c1 = g.counters()
    # ---- the same number of steps again, with HIP events around every launch
    # of the dominant kernel on the stream it runs on (roofline entry), the
    # sort overlap off
    gv.gv_set_tuning(h, overlap=0)
    gv.gv_profile_enable(h, True)
    gv.gv_profile_only(h, dominant)
    gv.gv_profile_reset(h)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for j in range(first + args.steps, nsteps):
        gv.gv_insert_edges(h, *ins[j], dev, stats=False)
        gv.gv_delete_edges(h, *dels[j], dev, stats=False)
    torch.cuda.synchronize()
    elapsed_ev = time.perf_counter() - t1
    dom_launches, dom_ms = gv.gv_kernel_times(h, dominant)
    gv.gv_profile_enable(h, False)
    gv.gv_set_tuning(h, overlap=overlap)
    rc = g.sync()
    if rc != 0:
        raise RuntimeError(f"batch error during timed steps: {gv.gv_strerror(rc)}")
    K = args.steps
    value = 2 * k * K / elapsed

    d = counter_delta(c0, c1)
    ins_T, del_T = d["touched"][0], d["touched"][1]
    ins_S, del_S = d["scanned_slots"][0], d["scanned_slots"][1]
    m1 = m1_bytes(2 * K * k, d)
    pct_m1 = m1 / elapsed / (HBM_PEAK_GBS * 1e9)

    # per-launch quantities of the dominant kernel's batch type
    if dominant in ("probe_delete", "freed", "compact", "final_delete"):
        per = {"k": k, "T": del_T / K, "S": del_S / K, "NB": del_S / K / B,
               "W": 0, "M": d["moved_slots"] / K, "FREED": d["freed_blocks"] / K}
    else:
        per = {"k": k, "T": ins_T / K, "S": ins_S / K, "NB": ins_S / K / B,
               "W": d["written_slots"] / K, "M": 0, "FREED": 0}
    if dominant.startswith("sort_"):
        per["k"] = k
    per["passes"] = (2 * args.scale + 7) // 8  # 8-bit digits of (src << L) | dst
    bpl = bytes_model(dominant, per)
    ibpl = implementation_bytes(dominant, per)
    avg_s = dom_ms / 1e3 / dom_launches if dom_launches else None
    roof = None
    if bpl is not None and avg_s:
        ach = bpl / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": dominant, "achieved": round(ach, 2),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 5),
                "traffic": stored_traffic(dominant), "bytes_per_launch": int(bpl),
                "bytes_model": ("M1 share: 16 B per pair per batch, over %d radix passes" % per["passes"]
                                if dominant == "sort_pass" else
                                "M1 share: touched adjacency, 4 B per block-granular slot"
                                if dominant.startswith("probe") else
                                "the kernel's own algorithmic bytes (bytes_model in bench.py)"),
                "implementation_bytes_per_launch": None if ibpl is None else int(ibpl),
                "implementation_frac": None if ibpl is None else
                round(ibpl / avg_s / 1e9 / HBM_PEAK_GBS, 5),
                "avg_launch_us": round(avg_s * 1e6, 3), "launches": dom_launches,
                "step_m1_frac": round(pct_m1, 5),
                "timed_steps": "a second run of the same number of steps, right after the "
                               "timed region, with the sort overlap off (each kernel alone on "
                               "the device), one HIP event pair around each run of "
                               "consecutive launches of the kernel (%.4f ms per step with the "
                               "events)" % (elapsed_ev / K * 1e3)}

    # ---- queries, in their own loop
    gv.gv_edge_exists(h, *qry[0], dev)
    torch.cuda.synchronize()
    out = torch.empty(k, dtype=torch.uint8, device=dev)
    t0 = time.perf_counter()
    for j in range(1, args.queries + 1):
        gv.gv_edge_exists(h, *qry[j], dev, out=out)
    torch.cuda.synchronize()
    q_rate = k * args.queries / (time.perf_counter() - t0)

    # ---- adjacency of the largest hub, memory report
    deg = torch.bincount(w.src.to(torch.int64), minlength=n)
    hub = int(torch.argmax(deg))
    gv.gv_get_adjacency(h, hub, dev)
    t0 = time.perf_counter()
    adj = gv.gv_get_adjacency(h, hub, dev)
    adj_ms = (time.perf_counter() - t0) * 1e3
    mem = g.memory_used()

    # ---- vertex batches of 10^4: delete then re-insert the same ids, after
    # an untimed delete and re-insert of other ids (sizes the buffers)
    def vertex_ids(tag):
        return torch.from_numpy((I.splitmix64(I.stream_seed(tag), 10**4) % np.uint64(n))
                                .astype(np.uint32).view(np.int32)).to(dev)
    warm_ids = vertex_ids("bench-vertices-warm")
    g.delete_vertices(warm_ids)
    g.insert_vertices(warm_ids)
    vids = vertex_ids("bench-vertices")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vdel = g.delete_vertices(vids)
    vdel_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    vins = g.insert_vertices(vids)
    vins_ms = (time.perf_counter() - t0) * 1e3
    g.close()

    # ---- the paper's own layout on the same steps
    cbt = None
    if not args.no_cbt:
        cbt = cbt_form(gv, w, dev, B, ins, dels, first)
        cbt["directory_path_speedup"] = round(value / cbt["edges_per_s"], 2)
        log("paper-faithful ablation:", json.dumps(cbt))

    # ---- batched form on its own workload
    sweep = None if args.no_sweep else block_size_sweep(gv, w, dev)
    knobs = {f: step_setting[f] for f in gv.TUNING_FIELDS if f in step_setting}
    latency = None if args.no_sweep else batch_latency(gv, w, dev, knobs)
    if latency:
        log("batch latency:", json.dumps(latency))
    batched = None if args.no_batched else batched_form(gv, I, T, dev)
    served = None if args.no_served else served_form(gv, I, T, dev, B)
    config3 = None if args.no_config3 else config3_form(gv, I, T, dev)
    if config3:
        log("config3:", json.dumps(config3))

    # ---- CPU oracle baseline on a quarter of the sources
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import pyoracle as O
        src_np = w.src.cpu().numpy().view(np.uint32)
        dst_np = w.dst.cpu().numpy().view(np.uint32)
        keep_v = (I.mix64(np.arange(n, dtype=np.uint64)) & np.uint64(3)) == 0
        sel = keep_v[src_np]
        o = O.OracleGraph(n, src_np[sel], dst_np[sel], block_slots=B)
        # the restricted batches are copied to the host and selected before
        # the clock starts: only the oracle's own work is timed
        work, pairs = [], 0
        for j in range(min(CPU_STEPS, args.steps)):
            jj = args.warmup + 1 + j
            for batch, fn in ((ins[jj], o.insert_edges), (dels[jj], o.delete_edges)):
                bs = batch[0].cpu().numpy().view(np.uint32)
                bd = batch[1].cpu().numpy().view(np.uint32)
                m = keep_v[bs]
                work.append((fn, np.ascontiguousarray(bs[m]), np.ascontiguousarray(bd[m])))
                pairs += int(m.sum())
        t0 = time.perf_counter()
        for fn, bs, bd in work:
            fn(bs, bd)
        cpu_s = time.perf_counter() - t0
        o.close()
        cpu = {"value": round(pairs / cpu_s, 1), "unit": "edges/s", "cores": 1,
               "kind": "oracle", **host_cpu(), "threads": 1,
               "sample": f"{min(CPU_STEPS, args.steps)} insert + delete batch pairs whose source "
                         f"hashes to 0 mod 4 ({pairs} pairs) against the graph restricted "
                         f"to those sources ({int(sel.sum())} edges); host copies and "
                         f"selection outside the timed loop"}

    out = {
        "metric": "batch insert/delete edges/s + % HBM peak; init edges/s; served p50/p99 latency",
        "value": round(value, 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded R-MAT, drawn on the GPU)",
        "config": {"workload": f"rmat{args.scale} {args.edges} edges, B={B}, insert+delete "
                               f"batches of {k}", "vertices": n, "edges": args.edges,
                   "batch": k, "block_slots": B,
                   "tuning": step_setting},
        "pct_hbm_m1": round(pct_m1, 5),
        "m1_bytes_per_step": int(m1 / K),
        "init_edges_per_s": round(args.edges / init_s, 1),
        "init_ms": round(init_s * 1e3, 3),
        "query_edges_per_s": round(q_rate, 1),
        "adjacency_hub": {"vertex": hub, "degree": int(adj.numel()), "ms": round(adj_ms, 3)},
        "vertex_delete_1e4": {"ms": round(vdel_ms, 3), "stats": vdel},
        "vertex_insert_1e4": {"ms": round(vins_ms, 3), "stats": vins},
        "memory": {"live_bytes": mem["live_bytes"], "blocks_in_use": mem["blocks_in_use"],
                   "num_edges": mem["num_edges"]},
        "paper_cbt_ablation": cbt,
        "batched_form": batched,
        "config3": config3,
        "served_p50_p99": served,
        "block_size_sweep": sweep,
        "batch_latency_us": latency,
        "pilot_kernels_ms": pilot,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
