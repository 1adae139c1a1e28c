"""The streams of `inputs` computed with torch, so large workloads can be
drawn directly on the GPU.  Every function returns exactly what its numpy
namesake in `inputs` returns (as int64/int32 tensors holding the same
unsigned values); the tests check this draw for draw.

Like `inputs`, this module holds none of the graph structure's arithmetic.
uint64 values live in int64 tensors: products wrap modulo 2^64 and right
shifts are made logical by masking.
"""
from __future__ import annotations

import torch

from . import inputs as _np_inputs

_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def _s64(x: int) -> int:
    """Unsigned 64-bit constant as the int64 with the same bits."""
    x &= (1 << 64) - 1
    return x - (1 << 64) if x >= 1 << 63 else x


def _lsr(z: torch.Tensor, k: int) -> torch.Tensor:
    return (z >> k) & ((1 << (64 - k)) - 1)


def mix64(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _lsr(z, 30)) * _s64(_M1)
    z = (z ^ _lsr(z, 27)) * _s64(_M2)
    return z ^ _lsr(z, 31)


def splitmix64(seed: int, n: int, start: int = 0, device="cpu") -> torch.Tensor:
    idx = torch.arange(start + 1, start + n + 1, dtype=torch.int64, device=device)
    return mix64(idx * _s64(_GAMMA) + _s64(seed))


def _below(r32: torch.Tensor, n: int) -> torch.Tensor:
    return _lsr((r32 & 0xFFFFFFFF) * n, 32)


def uniform_pairs(seed: int, n: int, num_vertices: int, self_loops: bool = False,
                  device="cpu"):
    out_s, out_d, have, start = [], [], 0, 0
    out_s.append(torch.zeros(0, dtype=torch.int64, device=device))
    out_d.append(torch.zeros(0, dtype=torch.int64, device=device))
    while have < n:
        want = (n - have) + (n - have) // 8 + 64
        r = splitmix64(seed, want, start, device)
        start += want
        s = _below(_lsr(r, 32), num_vertices)
        d = _below(r, num_vertices)
        if not self_loops:
            keep = s != d
            s, d = s[keep], d[keep]
        s, d = s[: n - have], d[: n - have]
        out_s.append(s)
        out_d.append(d)
        have += len(s)
    return torch.cat(out_s).to(torch.int32), torch.cat(out_d).to(torch.int32)


def rmat_pairs_raw(seed: int, n: int, scale: int, start: int = 0, abc=_np_inputs.RMAT_ABC,
                   device="cpu"):
    t1, t2, t3 = _np_inputs.rmat_thresholds(*abc)
    w = (scale + 1) // 2
    src = torch.empty(n, dtype=torch.int64, device=device)
    dst = torch.empty(n, dtype=torch.int64, device=device)
    weights = (1 << torch.arange(scale - 1, -1, -1, dtype=torch.int64, device=device))
    chunk = 1 << 22
    for c0 in range(0, n, chunk):
        m = min(chunk, n - c0)
        r = splitmix64(seed, m * w, (start + c0) * w, device).reshape(m, w)
        u = torch.empty((m, 2 * w), dtype=torch.int64, device=device)
        u[:, 0::2] = _lsr(r, 32)
        u[:, 1::2] = r & 0xFFFFFFFF
        u = u[:, :scale]
        q = (u >= t1).to(torch.int64) + (u >= t2).to(torch.int64) + (u >= t3).to(torch.int64)
        src[c0:c0 + m] = ((q >> 1) * weights).sum(dim=1)
        dst[c0:c0 + m] = ((q & 1) * weights).sum(dim=1)
    return src.to(torch.int32), dst.to(torch.int32)


def rmat_pairs(seed: int, n: int, scale: int, abc=_np_inputs.RMAT_ABC, device="cpu"):
    out_s, out_d, have, start = [], [], 0, 0
    out_s.append(torch.zeros(0, dtype=torch.int32, device=device))
    out_d.append(torch.zeros(0, dtype=torch.int32, device=device))
    while have < n:
        want = (n - have) + (n - have) // 16 + 64
        s, d = rmat_pairs_raw(seed, want, scale, start, abc, device)
        start += want
        keep = s != d
        s, d = s[keep][: n - have], d[keep][: n - have]
        out_s.append(s)
        out_d.append(d)
        have += len(s)
    return torch.cat(out_s), torch.cat(out_d)


def pair_keys(src: torch.Tensor, dst: torch.Tensor) -> torch.Tensor:
    return ((src.to(torch.int64) & 0xFFFFFFFF) << 32) | (dst.to(torch.int64) & 0xFFFFFFFF)


def rmat_graph(seed: int, scale: int, m: int, abc=_np_inputs.RMAT_ABC, device="cpu"):
    total = m + m // 4 + 1024
    while True:
        s, d = rmat_pairs_raw(seed, total, scale, 0, abc, device)
        ok = torch.nonzero(s != d).squeeze(1)
        keys = pair_keys(s[ok], d[ok])
        uniq, inv = torch.unique(keys, return_inverse=True)
        if len(uniq) >= m:
            first = torch.full((len(uniq),), len(keys), dtype=torch.int64, device=device)
            first = first.scatter_reduce(0, inv, torch.arange(len(keys), device=device),
                                         reduce="amin")
            pos = ok[torch.sort(first).values[:m]]
            return s[pos].contiguous(), d[pos].contiguous()
        total += total // 2


def permutation(seed: int, n: int, device="cpu") -> torch.Tensor:
    # same order as numpy's stable argsort of the uint64 draws: flip the sign
    # bit so that signed order equals unsigned order
    r = splitmix64(seed, n, 0, device) ^ _s64(1 << 63)
    return torch.sort(r, stable=True).indices


def shuffle_pairs(seed, src, dst):
    p = permutation(seed, len(src), src.device)
    return src[p], dst[p]


def pick(seed: int, n: int, src, dst):
    idx = _below(_lsr(splitmix64(seed, n, 0, src.device), 32), len(src))
    return src[idx], dst[idx]


class RmatWorkload:
    """Same workload as inputs.RmatWorkload, drawn with torch on `device`."""

    def __init__(self, scale: int = 20, m: int = 1 << 24, name: str = "rmat",
                 exist_frac: float = 0.8, device="cpu"):
        self.scale = scale
        self.num_vertices = 1 << scale
        self.m = m
        self.name = f"{name}{scale}-{m}"
        self.exist_frac = exist_frac
        self.device = torch.device(device)
        ss = _np_inputs.stream_seed
        self.src, self.dst = rmat_graph(ss(self.name, "graph"), scale, m, device=self.device)
        self._perm = None
        self._perm_pos = 0

    def insert_batch(self, k: int, j: int):
        return rmat_pairs(_np_inputs.stream_seed(self.name, "insert", k, j), k, self.scale,
                          device=self.device)

    def _take_existing(self, n: int):
        if self._perm is None:
            self._perm = permutation(_np_inputs.stream_seed(self.name, "delete-order"), self.m,
                                     self.device)
        idx = torch.arange(self._perm_pos, self._perm_pos + n, device=self.device) % self.m
        idx = self._perm[idx]
        self._perm_pos += n
        return self.src[idx], self.dst[idx]

    def delete_batch(self, k: int, j: int):
        ss = _np_inputs.stream_seed
        ne = int(round(self.exist_frac * k))
        es, ed = self._take_existing(ne)
        us, ud = uniform_pairs(ss(self.name, "delete-uniform", k, j), k - ne,
                               self.num_vertices, device=self.device)
        return shuffle_pairs(ss(self.name, "delete-mix", k, j), torch.cat([es, us]),
                             torch.cat([ed, ud]))

    def query_batch(self, q: int, j: int):
        ss = _np_inputs.stream_seed
        es, ed = pick(ss(self.name, "query-existing", q, j), q // 2, self.src, self.dst)
        us, ud = uniform_pairs(ss(self.name, "query-uniform", q, j), q - q // 2,
                               self.num_vertices, device=self.device)
        return shuffle_pairs(ss(self.name, "query-mix", q, j), torch.cat([es, us]),
                             torch.cat([ed, ud]))
