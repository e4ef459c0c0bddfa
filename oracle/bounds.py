"""Compression bounds for the QLC oracle (float64).

TEST INFRASTRUCTURE ONLY: used by the tests and the benchmark report, never
by the GPU library.

* Shannon entropy of the byte PMF and the ideal compressibility (8 - H) / 8
  (Observations section and Adaptation section of arXiv 2602.17849).
* Huffman code lengths by the textbook two-smallest merge (Background
  section: Huffman codes are the optimal prefix codes the paper compares
  against).  Only lengths are needed: every optimal code has the same
  average length.
* Compressibility of an average code length L: (8 - L) / 8.
"""
from __future__ import annotations

import heapq
import math
from typing import Sequence


def entropy_bits(counts: Sequence[int]) -> float:
    """H = -sum p log2 p over symbols with non-zero count."""
    total = float(sum(int(c) for c in counts))
    if total == 0:
        return 0.0
    h = 0.0
    for c in counts:
        c = int(c)
        if c:
            p = c / total
            h -= p * math.log2(p)
    return h


def compressibility(avg_bits_per_symbol: float) -> float:
    """Fraction of the 8 bits per symbol saved: (8 - L) / 8."""
    return (8.0 - avg_bits_per_symbol) / 8.0


def huffman_lengths(counts: Sequence[int]) -> list[int]:
    """Code length of every symbol under a Huffman code of the non-zero
    counts (zero-count symbols get length 0).  A single used symbol gets
    length 1."""
    used = [(int(c), s) for s, c in enumerate(counts) if int(c) > 0]
    lengths = [0] * len(counts)
    if not used:
        return lengths
    if len(used) == 1:
        lengths[used[0][1]] = 1
        return lengths
    # heap entries: (weight, tie, list of symbols in the subtree)
    heap = [(c, i, [s]) for i, (c, s) in enumerate(used)]
    heapq.heapify(heap)
    tie = len(heap)
    while len(heap) > 1:
        w1, _, s1 = heapq.heappop(heap)
        w2, _, s2 = heapq.heappop(heap)
        for s in s1 + s2:  # every merge adds one bit to each member
            lengths[s] += 1
        heapq.heappush(heap, (w1 + w2, tie, s1 + s2))
        tie += 1
    return lengths


def huffman_avg_bits(counts: Sequence[int]) -> float:
    total = sum(int(c) for c in counts)
    if total == 0:
        return 0.0
    lengths = huffman_lengths(counts)
    return sum(int(c) * l for c, l in zip(counts, lengths)) / total


def kraft_sum(lengths: Sequence[int]) -> float:
    """Sum of 2^-len over all codewords (<= 1 for a prefix code)."""
    return float(sum(2.0 ** (-int(l)) for l in lengths))
