"""Seeded operation sequences of the batched form, drawn on the GPU from the
streams of inputs.py (no method arithmetic: inputs for the library and for
the tests that check it)."""
import numpy as np
import torch

from . import inputs as I
from . import inputs_torch as T


def batched_ops(w, seed_name="batched", nbatch=256, device="cuda:0", lo=100, hi=10**6):
    """`nbatch` batches on R-MAT workload `w`, sizes log-uniform in [lo, hi]:
    45 % edge inserts (R-MAT pairs), 45 % edge deletes (80 % stored pairs,
    20 % uniform pairs), 10 % vertex batches of min(size, 10^4) uniform ids,
    inserts or deletes alike.  Returns ([(kind, a, b)], edge pairs, vertex
    ids) with kinds 0/1/2/3 = insert edges / delete edges / insert vertices /
    delete vertices and device int32 tensors."""
    n = w.num_vertices
    draws = I.splitmix64(I.stream_seed(seed_name, "ops"), 3 * nbatch)
    ops, pairs, vids = [], 0, 0
    span = np.log(hi / lo)
    for j in range(nbatch):
        u = float(draws[3 * j] >> np.uint64(11)) / float(1 << 53)
        size = int(round(lo * np.exp(u * span)))
        r = float(draws[3 * j + 1] >> np.uint64(11)) / float(1 << 53)
        if r < 0.45:
            s, d = w.insert_batch(size, j)
            ops.append((0, s, d))
            pairs += size
        elif r < 0.90:
            ne = int(round(0.8 * size))
            es, ed = T.pick(I.stream_seed(seed_name, "del-existing", j), ne, w.src, w.dst)
            us, ud = T.uniform_pairs(I.stream_seed(seed_name, "del-uniform", j), size - ne, n,
                                     device=device)
            ops.append((1, torch.cat([es, us]), torch.cat([ed, ud])))
            pairs += size
        else:
            m = min(size, 10**4)
            ids = torch.from_numpy((I.splitmix64(I.stream_seed(seed_name, "vertices", j), m)
                                    % np.uint64(n)).astype(np.uint32).view(np.int32)).to(device)
            ops.append((2 if draws[3 * j + 2] & np.uint64(1) else 3, ids, None))
            vids += m
    return ops, pairs, vids


def batched_warmup(ops):
    """A warm-up for a fresh graph before timing `ops`: an insert and a delete
    of the largest insert batch, a vertex delete and re-insert of one id of
    the first vertex-delete batch (sizes the scratch buffers)."""
    big = max((o for o in ops if o[0] == 0), key=lambda o: o[1].numel())
    one = ops[[o[0] for o in ops].index(3)][1][:1] if any(o[0] == 3 for o in ops) else None

    def warm(g):
        g.insert_edges(big[1], big[2], stats=False)
        g.delete_edges(big[1], big[2], stats=False)
        if one is not None:
            g.delete_vertices(one)
            g.insert_vertices(one)
        torch.cuda.synchronize()
    return warm
