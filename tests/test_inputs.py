"""Seeded input generators: determinism and distribution checks (no GPU)."""
import math

import numpy as np

from paper_2306_08252_amd import inputs as I


def test_streams_are_deterministic():
    a = I.uniform_pairs(I.stream_seed("det"), 5000, 1000)
    b = I.uniform_pairs(I.stream_seed("det"), 5000, 1000)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    c = I.uniform_pairs(I.stream_seed("det2"), 5000, 1000)
    assert not np.array_equal(a[0], c[0])
    r1 = I.rmat_pairs(7, 3000, 14)
    r2 = I.rmat_pairs(7, 3000, 14)
    assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[1], r2[1])
    # a stream continues where a shorter draw stopped
    full = I.rmat_pairs_raw(9, 100, 12)
    tail = I.rmat_pairs_raw(9, 60, 12, start=40)
    assert np.array_equal(full[0][40:], tail[0]) and np.array_equal(full[1][40:], tail[1])


def test_uniform_pairs_range_and_no_self_loops():
    s, d = I.uniform_pairs(3, 20000, 777)
    assert s.max() < 777 and d.max() < 777
    assert not np.any(s == d)
    assert len(s) == 20000


def _binomial_ok(count, n, p, z=5.0):
    mu = n * p
    sd = math.sqrt(n * p * (1 - p))
    return abs(count - mu) <= z * sd


def test_rmat_quadrant_frequencies():
    n, scale = 200000, 16
    s, d = I.rmat_pairs_raw(I.stream_seed("rmat-freq"), n, scale)
    a, b, c = I.RMAT_ABC
    top_s = (s >> (scale - 1)) & 1
    top_d = (d >> (scale - 1)) & 1
    assert _binomial_ok(int(((top_s == 0) & (top_d == 0)).sum()), n, a)
    assert _binomial_ok(int(((top_s == 0) & (top_d == 1)).sum()), n, b)
    assert _binomial_ok(int(((top_s == 1) & (top_d == 0)).sum()), n, c)
    assert _binomial_ok(int(((top_s == 1) & (top_d == 1)).sum()), n, 1 - a - b - c)
    # every level draws the same distribution: check the lowest bit too
    lo_s, lo_d = s & 1, d & 1
    assert _binomial_ok(int(((lo_s == 1) & (lo_d == 1)).sum()), n, 1 - a - b - c)


def test_rmat_graph_is_distinct_without_self_loops():
    s, d = I.rmat_graph(I.stream_seed("rmat-graph"), 12, 20000)
    assert len(s) == 20000
    assert not np.any(s == d)
    assert len(np.unique(I.pair_keys(s, d))) == 20000
    # it is a prefix of the raw stream, in stream order
    rs, rd = I.rmat_pairs_raw(I.stream_seed("rmat-graph"), 40000, 12)
    keys = I.pair_keys(rs, rd)
    first = {}
    for i, k in enumerate(keys.tolist()):
        if rs[i] != rd[i] and k not in first:
            first[k] = i
    want = sorted(first.values())[:20000]
    assert np.array_equal(I.pair_keys(s, d), keys[want])


def test_lattice_exact_counts_and_symmetry():
    side = 64
    s, d = I.lattice_graph(I.stream_seed("lat"), side)
    e0 = 2 * side * (side - 1)
    kept = e0 - int(0.10 * e0)
    lr = int(0.01 * kept)
    assert len(s) == 2 * (kept + lr)
    keys = I.pair_keys(s, d)
    assert len(np.unique(keys)) == len(keys)
    assert np.array_equal(np.sort(keys), np.sort(I.pair_keys(d, s)))
    assert not np.any(s == d)


def test_tiny_workload_shape():
    w = I.tiny_workload()
    s, d = w["init"]
    assert len(s) == 8192 and s.max() < 1024 and not np.any(s == d)
    assert len(w["insert"]) == 4 and all(len(b[0]) == 1024 for b in w["insert"])
    assert len(w["delete"]) == 4 and all(len(b[0]) == 1024 for b in w["delete"])
    # half of each delete batch is absent from every known pair
    known = np.unique(I.pair_keys(np.concatenate([s] + [b[0] for b in w["insert"]]),
                                  np.concatenate([d] + [b[1] for b in w["insert"]])))
    for bs, bd in w["delete"]:
        hit = np.isin(I.pair_keys(bs, bd), known)
        assert int(hit.sum()) == 512
    assert len(w["query"][0]) == 1024


def test_torch_streams_match_numpy():
    import torch
    from paper_2306_08252_amd import inputs_torch as T
    seed = I.stream_seed("torch-eq")
    assert np.array_equal(T.splitmix64(seed, 1000, 17).numpy().view(np.uint64),
                          I.splitmix64(seed, 1000, 17))
    a = I.uniform_pairs(seed, 5000, 1000)
    b = T.uniform_pairs(seed, 5000, 1000)
    assert np.array_equal(a[0], b[0].numpy().view(np.uint32))
    assert np.array_equal(a[1], b[1].numpy().view(np.uint32))
    a = I.rmat_pairs(seed, 7000, 13)
    b = T.rmat_pairs(seed, 7000, 13)
    assert np.array_equal(a[0], b[0].numpy().view(np.uint32))
    assert np.array_equal(a[1], b[1].numpy().view(np.uint32))
    a = I.rmat_graph(seed, 11, 9000)
    b = T.rmat_graph(seed, 11, 9000)
    assert np.array_equal(a[0], b[0].numpy().view(np.uint32))
    assert np.array_equal(a[1], b[1].numpy().view(np.uint32))
    assert np.array_equal(I.permutation(seed, 3000), T.permutation(seed, 3000).numpy())
    wn = I.RmatWorkload(12, 20000, name="eq")
    wt = T.RmatWorkload(12, 20000, name="eq")
    for fn in ("insert_batch", "delete_batch", "query_batch"):
        for j in range(2):
            x = getattr(wn, fn)(3000, j)
            y = getattr(wt, fn)(3000, j)
            assert np.array_equal(x[0], y[0].numpy().view(np.uint32)), fn
            assert np.array_equal(x[1], y[1].numpy().view(np.uint32)), fn


def test_zero_length_draws():
    from paper_2306_08252_amd import inputs_torch as T
    for f in (lambda: I.uniform_pairs(1, 0, 10), lambda: I.rmat_pairs(1, 0, 10)):
        s, d = f()
        assert len(s) == 0 and s.dtype == np.uint32 and d.dtype == np.uint32
    for f in (lambda: T.uniform_pairs(1, 0, 10), lambda: T.rmat_pairs(1, 0, 10)):
        s, d = f()
        assert len(s) == 0 and str(s.dtype) == "torch.int32"
    w = I.RmatWorkload(10, 3000, name="z")
    s, d = w.delete_batch(1, 0)
    assert len(s) == 1
    s, d = T.RmatWorkload(10, 3000, name="z").delete_batch(1, 0)
    assert len(s) == 1 and str(s.dtype) == "torch.int32"
