"""Shared helpers for the GPU parity tests: compare the GPU structure, read
through the C ABI, with the CPU oracle."""
import numpy as np
import pytest
import torch

from oracle import pyoracle as O


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_08252_amd import graphvine as gv
    gv.lib()  # raises loudly if the HIP library is missing
    return gv


def say(*a):
    print(*a, flush=True)


def u32(t):
    return t.detach().cpu().numpy().view(np.uint32)


def gpu_dump(g):
    offs, dst, ck, e = g.dump()
    return offs.cpu().numpy().astype(np.uint64), u32(dst), ck, e


def assert_same(g, o, label=""):
    """Canonical dump, checksum, edge count, block accounting and the
    structural audit all agree with the oracle."""
    offs, dst, ck, e = gpu_dump(g)
    ooffs, odst, ock = o.dump()
    assert e == o.num_edges, label
    assert g.info()["vertex_capacity"] == o.capacity, label
    np.testing.assert_array_equal(offs, ooffs, err_msg=label)
    np.testing.assert_array_equal(dst, odst, err_msg=label)
    assert ck == ock, label
    m = g.memory_used()
    assert m["blocks_in_use"] == o.blocks_in_use, label
    assert m["num_edges"] == o.num_edges, label
    assert g.audit() == 0, label


def same_answers(g, o, s, d, label=""):
    got = g.edge_exists(s, d).cpu().numpy()
    want = o.edge_exists(s, d)
    np.testing.assert_array_equal(got, want, err_msg=label)
