"""Oracle layout search pinned by brute force and closed forms (CPU only).

The paper's layouts were "obtained empirically" (Conclusion section) and it
suggests tuning the number of symbols per area and the number of distinct
lengths; the oracle reads that as an exhaustive search over non-decreasing
width tuples filled greedily in rank order (ties -> lexicographically
smallest tuple), optionally limited to four distinct lengths ("quad",
Quad Length Codes section).  The brute force below knows none of that: it
tries every assignment of symbols to areas, gives each area the fewest
suffix bits that distinguish its symbols, and keeps the cheapest code.
"""
import itertools
import math

import numpy as np
import pytest

import oracle


def brute_force_min_cost(h, M, A, prefix_bits, max_distinct, allow_empty):
    """Min over all maps symbol -> area of sum h[s] * (prefix + ceil(log2 n_area))."""
    h = np.asarray(h, dtype=np.int64)
    best = None
    total = A ** M
    step = 1 << 20
    digits_pow = A ** np.arange(M, dtype=np.int64)
    for lo in range(0, total, step):
        ids = np.arange(lo, min(total, lo + step), dtype=np.int64)
        maps = (ids[:, None] // digits_pow[None, :]) % A          # [k, M] area of each symbol
        n = np.stack([(maps == a).sum(1) for a in range(A)], 1)   # [k, A] symbols per area
        w = np.where(n > 0, np.ceil(np.log2(np.maximum(n, 1))).astype(np.int64), -1)
        ok = np.ones(len(ids), dtype=bool)
        if not allow_empty:
            ok &= (n > 0).all(1)
        # number of distinct widths among non-empty areas
        ws = np.sort(w, axis=1)
        distinct = ((ws[:, 1:] != ws[:, :-1]) & (ws[:, 1:] >= 0)).sum(1) + (ws[:, 0] >= 0)
        ok &= distinct <= max_distinct
        bits = prefix_bits + np.take_along_axis(w, maps, 1)        # [k, M]
        cost = (bits * h[None, :]).sum(1)
        cost = np.where(ok, cost, np.iinfo(np.int64).max)
        c = int(cost.min())
        best = c if best is None else min(best, c)
    return best


def admissible_count(M, A, max_distinct):
    """Count non-decreasing tuples with every area non-empty under greedy
    fill and full cover, written directly from that definition."""
    maxw = int(math.log2(M))
    n = 0
    order = []
    for w in itertools.combinations_with_replacement(range(maxw + 1), A):
        if len(set(w)) > max_distinct:
            continue
        if sum(2 ** b for b in w[:-1]) < M <= sum(2 ** b for b in w):
            n += 1
            order.append(w)
    return n, order


@pytest.mark.parametrize("max_distinct,expect", [(8, 3639), (4, 1308)])
def test_candidate_set_of_the_codec(max_distinct, expect):
    n, order = admissible_count(256, 8, max_distinct)
    assert n == expect
    got = oracle.enumerate_layouts(256, 8, max_distinct)
    assert len(got) == expect
    assert [tuple(r) for r in got] == order   # same tuples, lexicographic order


@pytest.mark.parametrize("M,A,p", [(8, 2, 1), (8, 3, 2), (8, 4, 2), (16, 2, 1)])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_search_matches_brute_force_small(M, A, p, seed):
    rng = np.random.default_rng(seed * 97 + M * 7 + A)
    # skewed, tie-free-ish counts, some zeros
    h = (rng.pareto(1.2, size=M) * 100).astype(np.int64)
    h[rng.integers(0, M)] = 0
    for max_distinct in sorted({1, 2, min(A, 4), A}):
        try:
            t = oracle.build_table_general(h, M, A, p, max_distinct)
        except ValueError:
            t = None  # no admissible tuple under this distinct limit
        bf = brute_force_min_cost(h, M, A, p, max_distinct, allow_empty=False)
        if t is None:
            assert bf == np.iinfo(np.int64).max or max_distinct < A
            continue
        assert t.cost_bits == bf, (max_distinct, t.width, bf)
        if max_distinct == A:
            assert brute_force_min_cost(h, M, A, p, A, allow_empty=True) == bf


@pytest.mark.parametrize("seed", [0])
def test_search_matches_brute_force_8_areas(seed):
    """The codec's shape at a small alphabet: 3 prefix bits, 8 areas."""
    rng = np.random.default_rng(1000 + seed)
    h = (rng.pareto(0.8, size=8) * 1000).astype(np.int64) + 1
    t = oracle.build_table_general(h, 8, 8, 3, 8)
    assert t.cost_bits == brute_force_min_cost(h, 8, 8, 3, 8, allow_empty=False)


def test_uniform_histogram_closed_form():
    """Uniform counts: 8 areas of 32 (5 suffix bits) give exactly 8 bits per
    symbol, and no other tuple reaches it (convexity of the width cost)."""
    h = np.full(256, 1000, dtype=np.uint64)
    for mode in (oracle.MODE_SEARCH_QUAD, oracle.MODE_SEARCH_ANY):
        t = oracle.build_table(h, mode)
        assert list(t.width) == [5] * 8
        assert t.cost_bits == 8 * 256 * 1000
    # the printed schemes on uniform data: 2456/256 and 2450/256 bits/symbol
    t1 = oracle.build_table(h, oracle.MODE_PAPER_T1)
    t2 = oracle.build_table(h, oracle.MODE_PAPER_T2)
    assert t1.cost_bits == 1000 * (40 * 6 + 16 * 7 + 32 * 8 + 168 * 11)
    assert t1.cost_bits / (256 * 1000) == 9.59375
    assert t2.cost_bits == 1000 * (2 * 4 + 32 * 6 + 64 * 8 + 158 * 11)
    assert t2.cost_bits / (256 * 1000) == 9.5703125


def test_single_symbol_closed_form():
    """One symbol only: a 0-bit first area gives 3 bits per symbol (the
    QLC ceiling of 62.5 %); the smallest such tuple is (0,...,0,8)."""
    h = np.zeros(256, dtype=np.uint64)
    h[77] = 12345
    t = oracle.build_table(h, oracle.MODE_SEARCH_QUAD)
    assert list(t.width) == [0, 0, 0, 0, 0, 0, 0, 8]
    assert t.cost_bits == 3 * 12345
    assert t.code_string(77) == "000"


def test_empty_histogram_is_valid():
    h = np.zeros(256, dtype=np.uint64)
    t = oracle.build_table(h, oracle.MODE_SEARCH_QUAD)
    assert t.cost_bits == 0
    assert list(t.width) == [0, 0, 0, 0, 0, 0, 0, 8]   # first tuple in the order
    assert list(t.rank_to_sym) == list(range(256))


def test_search_costs_against_every_candidate():
    """The chosen tuple costs no more than any candidate, and ties go to the
    first candidate in lexicographic order."""
    rng = np.random.default_rng(5)
    h = rng.integers(0, 50, size=256).astype(np.uint64)
    h[:4] = 0
    r2s, _ = oracle.rank(h)
    ranked = h[r2s]
    for max_distinct in range(1, 9):
        cands = oracle.enumerate_layouts(256, 8, max_distinct)
        costs = [sum(int(ranked[r]) * (3 + w[a]) for a, (f, c) in enumerate(zip(*oracle.fill(w)[1:]))
                     for r in range(f, f + c)) for w in cands]
        idx, w = oracle.search(ranked, max_distinct=max_distinct)
        assert costs[idx] == min(costs)
        assert idx == costs.index(min(costs))
        assert list(w) == list(cands[idx])


def test_quad_limits_distinct_lengths():
    rng = np.random.default_rng(11)
    for _ in range(20):
        h = (rng.pareto(rng.uniform(0.3, 3.0), size=256) * 1000).astype(np.uint64)
        t = oracle.build_table(h, oracle.MODE_SEARCH_QUAD)
        assert len(set(t.len.tolist())) <= 4
        ta = oracle.build_table(h, oracle.MODE_SEARCH_ANY)
        assert ta.cost_bits <= t.cost_bits
        for mode in (oracle.MODE_PAPER_T1, oracle.MODE_PAPER_T2):
            assert t.cost_bits <= oracle.build_table(h, mode).cost_bits


def test_distinct_caps_nest():
    """Capping the number of distinct code lengths at k = 1..8: the capped
    table honours the cap, its cost never rises with k, k = 4 is the quad
    search and k = 8 the unrestricted one."""
    rng = np.random.default_rng(13)
    for _ in range(10):
        h = (rng.pareto(rng.uniform(0.3, 3.0), size=256) * 1000).astype(np.uint64)
        costs = []
        for k in range(1, 9):
            t = oracle.build_table_general(h, 256, 8, 3, k)
            assert len(set(t.width.tolist())) <= k
            costs.append(t.cost_bits)
        assert all(a >= b for a, b in zip(costs, costs[1:]))
        for k, mode in ((4, oracle.MODE_SEARCH_QUAD), (8, oracle.MODE_SEARCH_ANY)):
            a, b = oracle.build_table_general(h, 256, 8, 3, k), oracle.build_table(h, mode)
            assert list(a.width) == list(b.width) and a.cost_bits == b.cost_bits
            assert list(a.code) == list(b.code) and list(a.len) == list(b.len)


def composition_brute_force_min_cost(h, M, A, prefix_bits):
    """Min over every split of the M symbols into A non-empty areas of any
    sizes (not only powers of two, not only greedy fills): for given area
    sizes n_a the cheapest assignment puts the most frequent symbols in the
    areas of fewest suffix bits (rearrangement inequality), so the search
    runs over all compositions n_0 + ... + n_{A-1} = M with n_a >= 1."""
    h = np.sort(np.asarray(h, dtype=np.int64))[::-1]          # most frequent first
    prefix = np.concatenate([[0], np.cumsum(h)])
    best = None
    # compositions of M into A positive parts = choices of A-1 cut points in 1..M-1
    cuts = np.array(list(itertools.combinations(range(1, M), A - 1)), dtype=np.int64)
    step = 1 << 16
    for lo in range(0, len(cuts), step):
        c = cuts[lo:lo + step]
        edges = np.concatenate([np.zeros((len(c), 1), np.int64), c,
                                np.full((len(c), 1), M, np.int64)], 1)
        sizes = np.diff(edges, axis=1)                          # [k, A] area sizes
        widths = np.ceil(np.log2(sizes)).astype(np.int64)
        # symbols sorted by frequency go to areas sorted by width
        order = np.argsort(widths, axis=1, kind="stable")
        sw = np.take_along_axis(widths, order, 1)
        ss = np.take_along_axis(sizes, order, 1)
        ends = np.cumsum(ss, axis=1)
        starts = ends - ss
        counts = prefix[ends] - prefix[starts]
        cost = (counts * (prefix_bits + sw)).sum(1)
        m = int(cost.min())
        best = m if best is None else min(best, m)
    return best


@pytest.mark.parametrize("M,A,p", [(16, 4, 2), (16, 8, 3), (32, 8, 3), (64, 4, 2), (8, 4, 2)])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_search_matches_composition_brute_force(M, A, p, seed):
    """The greedy fill over non-decreasing power-of-two width tuples loses
    nothing against areas of arbitrary sizes: 16 and 64 symbols with 4
    areas (the small-alphabet codecs), 8 areas of 16 and 32 symbols (the
    3-bit area code on a non-degenerate alphabet)."""
    rng = np.random.default_rng(seed * 31 + M + A)
    h = (rng.pareto(rng.uniform(0.5, 2.0), size=M) * 1000).astype(np.int64)
    h[rng.integers(0, M)] = 0
    t = oracle.build_table_general(h, M, A, p, A)
    assert t.cost_bits == composition_brute_force_min_cost(h, M, A, p)


def test_composition_brute_force_agrees_with_map_brute_force():
    """The composition search equals the search over every symbol -> area
    map where both are feasible."""
    rng = np.random.default_rng(77)
    for M, A, p in ((8, 2, 1), (8, 3, 2), (8, 4, 2)):
        h = (rng.pareto(1.0, size=M) * 100).astype(np.int64)
        assert composition_brute_force_min_cost(h, M, A, p) == \
            brute_force_min_cost(h, M, A, p, A, allow_empty=False)
