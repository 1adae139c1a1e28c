"""The paper-faithful ablation's block placement, pinned on the CPU (no GPU
compute): the library's bit string of a block against the paper's worked
example (tests/golden/cbt_bitstrings.txt) and against the complete binary tree
it must describe (following the string from the root reaches level-order node
k when left is 2i and right is 2i + 1)."""
import os

import pytest

from conftest import ROOT


@pytest.fixture(scope="module")
def gv():
    from paper_2306_08252_amd import graphvine as gv
    if not os.path.exists(gv.LIB_PATH):
        pytest.fail("libgraphvine.so is not built (run __graft_entry__.build())")
    return gv


def test_paper_example_ninth_block(gv):
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", "cbt_bitstrings.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, bits = line.split()
                rows.append((int(k), "" if bits == "-" else bits))
    assert rows == [(9, "001")]
    for k, bits in rows:
        assert gv.gv_cbt_bitstring(k) == bits


def test_strings_are_root_paths_of_a_complete_binary_tree(gv):
    seen = set()
    for k in range(1, 1 << 12):
        s = gv.gv_cbt_bitstring(k)
        node = 1
        for c in s:
            assert c in "01"
            node = 2 * node + (c == "1")
        assert node == k
        # the last bit says which child of the parent the block becomes
        if k > 1:
            assert s[-1] == ("1" if k % 2 else "0")
        assert s not in seen
        seen.add(s)
    assert gv.gv_cbt_bitstring(1) == ""


def test_bitstring_argument_checks(gv):
    import ctypes as C
    buf = C.create_string_buffer(2)
    L = gv.lib()
    assert L.gv_cbt_bitstring(0, buf, 2) == gv.GV_EINVAL
    assert L.gv_cbt_bitstring(9, buf, 2) == gv.GV_ERANGE  # needs 4 bytes
    assert L.gv_cbt_bitstring(2, buf, 2) == gv.GV_OK and buf.value == b"0"
