"""The paper's weak-scaling workloads (Sec. 3, Table 1) as generated inputs.

These inputs feed both the GPU path and the oracle; the pins here check the
generator against the paper's printed setup and against the element-level
definition of each structure.
"""
import os

import numpy as np
import pytest

from paper_2011_11762_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table1_rows():
    return [ln.split() for ln in open(os.path.join(GOLDEN, "table1_tflop.txt"))
            if ln.strip() and not ln.startswith("#")]


def test_growing_block_rule_reproduces_table1():
    """The doubling rule (nearest size) gives the printed growing-block sizes."""
    for n_s, _, blk_s, _ in _table1_rows()[:4]:
        assert W.paper_block_size(int(n_s)) == int(blk_s) == W.PAPER_TABLE1[int(n_s)][0]


def test_paper_element_flops_match_table1():
    """Element-level flops of A * A equal Table 1's Banded and Growing-block rows;
    the Random-blocks rows are nominal (the count depends on where the blocks
    fall; interior blocks add up to 2% more than the corner block)."""
    for n_s, band_s, _, gb_s in _table1_rows()[:3]:
        n = int(n_s)
        assert f"{W.paper_element_flops('banded', n) / 1e12:.4g}" == band_s
        assert f"{W.paper_element_flops('growing', n) / 1e12:.4g}" == gb_s
        rnd = W.paper_element_flops("random", n) / 1e12
        assert abs(rnd / float(gb_s) - 1) < 0.02


@pytest.mark.parametrize("kind", ["banded", "growing", "random"])
def test_paper_workload_element_structure(kind):
    """Nonzero elements are exactly the band |i - j| <= h united with the dense
    blocks; the leaves are exactly those holding such elements; the padding
    past n is zero; the element flop count follows the generated structure."""
    n, bs, h = 1000, 32, 70
    m = W.paper_workload(kind, n, bs, h, seed=7)
    dense = m.meta["dense_blocks"]
    assert (kind == "banded") == (len(dense) == 0)
    full = m.to_dense()
    assert not np.any(full[n:, :]) and not np.any(full[:, n:])
    nz = full[:n, :n] != 0
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    want = np.abs(i - j) <= h
    for p, sz in dense:
        want |= (i >= p) & (i < p + sz) & (j >= p) & (j < p + sz)
    assert np.array_equal(nz, want)
    # leaves = blocks holding at least one structure element, canonical order
    nb = -(-n // bs)
    held = np.zeros((nb, nb), dtype=bool)
    held[np.nonzero(want)[0] // bs, np.nonzero(want)[1] // bs] = True
    bi, bj = np.nonzero(held)
    assert np.array_equal(m.brow, bi) and np.array_equal(m.bcol, bj)
    # A * A element flops: 2 * sum_k (nonzeros in column k) * (nonzeros in row k)
    assert m.meta["element_flops"] == 2 * int((want.sum(0).astype(np.int64) * want.sum(1)).sum())
    assert np.all(np.abs(m.vals) <= 1.0)
