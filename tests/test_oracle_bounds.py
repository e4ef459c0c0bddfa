"""Entropy / Huffman bounds of the oracle pinned by closed forms and
textbook facts (CPU only)."""
import math

import numpy as np
import pytest

import oracle
from oracle import bounds


def test_entropy_closed_forms():
    assert bounds.entropy_bits([1] * 256) == 8.0
    assert bounds.entropy_bits([5]) == 0.0
    assert bounds.entropy_bits([1, 1]) == 1.0
    # dyadic PMF 1/2, 1/4, 1/8, 1/8 -> 1.75 bits
    assert bounds.entropy_bits([4, 2, 1, 1]) == 1.75


def test_huffman_closed_forms():
    assert bounds.huffman_lengths([4, 2, 1, 1]) == [1, 2, 3, 3]
    assert bounds.huffman_avg_bits([4, 2, 1, 1]) == 1.75        # dyadic: equals entropy
    assert bounds.huffman_avg_bits([1] * 256) == 8.0
    assert bounds.huffman_lengths([0, 7, 0]) == [0, 1, 0]
    # textbook example: weights 5,9,12,13,16,45 -> lengths 4,4,3,3,3,1
    assert bounds.huffman_lengths([5, 9, 12, 13, 16, 45]) == [4, 4, 3, 3, 3, 1]


@pytest.mark.parametrize("seed", range(5))
def test_bound_ordering(seed):
    """H <= L_huffman < H + 1 (Huffman is optimal, Background section) and
    L_huffman <= L_qlc for every QLC table; the searched table never
    exceeds 8 bits/symbol nor the printed schemes."""
    rng = np.random.default_rng(seed)
    h = (rng.pareto(rng.uniform(0.5, 2.5), 256) * 1000).astype(np.uint64) + (seed % 2)
    n = int(h.sum())
    H = bounds.entropy_bits(h)
    Lh = bounds.huffman_avg_bits(h)
    assert H <= Lh + 1e-12 < H + 1
    costs = {m: oracle.build_table(h, m).cost_bits / n for m in range(4)}
    for m, L in costs.items():
        assert Lh <= L + 1e-12
    assert costs[oracle.MODE_SEARCH_ANY] <= costs[oracle.MODE_SEARCH_QUAD]
    assert costs[oracle.MODE_SEARCH_QUAD] <= min(costs[oracle.MODE_PAPER_T1],
                                                 costs[oracle.MODE_PAPER_T2])
    assert costs[oracle.MODE_SEARCH_QUAD] <= 8.0
