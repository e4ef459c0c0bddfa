"""Oracle histogram / rank / encode / decode pinned by library routines,
closed forms and properties (CPU only)."""
import numpy as np
import pytest

import oracle
from oracle import bounds


def _inputs():
    rng = np.random.default_rng(123)
    yield "random", rng.integers(0, 256, 5000).astype(np.uint8)
    yield "skewed", np.minimum(rng.geometric(0.2, 7001), 255).astype(np.uint8)
    yield "constant", np.full(3001, 42, np.uint8)
    yield "one", np.array([200], np.uint8)
    yield "two_symbols", rng.choice(np.array([3, 250], np.uint8), 4097)


def test_histogram_is_bincount():
    for _, x in _inputs():
        assert np.array_equal(oracle.histogram(x), np.bincount(x, minlength=256))
    assert oracle.histogram(np.zeros(0, np.uint8)).sum() == 0


def test_rank_is_sort_by_count_then_symbol():
    rng = np.random.default_rng(7)
    for trial in range(20):
        h = rng.integers(0, 5 if trial % 2 else 1000, 256).astype(np.uint64)
        r2s, s2r = oracle.rank(h)
        expect = sorted(range(256), key=lambda s: (-int(h[s]), s))
        assert list(r2s) == expect
        assert all(s2r[r2s[r]] == r for r in range(256))


def test_codes_are_prefix_free_and_cover():
    rng = np.random.default_rng(9)
    for mode in range(4):
        h = (rng.pareto(1.0, 256) * 100).astype(np.uint64)
        t = oracle.build_table(h, mode)
        assert t.count.sum() == 256 and (t.count > 0).all()
        codes = [t.code_string(s) for s in range(256)]
        assert len(set(codes)) == 256
        for a in codes:
            for b in codes:
                assert a == b or not b.startswith(a)
        # the first 3 bits name the area, whose width sets the length
        for s in range(256):
            area = int(codes[s][:3], 2)
            assert len(codes[s]) == 3 + t.width[area]
        assert bounds.kraft_sum(t.len) <= 1.0


@pytest.mark.parametrize("C", [256, 1024, 4096])
def test_round_trip_and_index(C):
    rng = np.random.default_rng(C)
    for name, x in _inputs():
        for mode in range(4):
            t = oracle.build_table(oracle.histogram(x), mode)
            st, bits, index, total = oracle.encode(x, t, C)
            assert st == oracle.OK
            assert total == t.cost_bits == int(sum(t.len[x]))
            assert bits.size == 4 * ((total + 31) // 32)
            assert index.size == (x.size + C - 1) // C
            # index[j] = sum of code lengths before symbol j*C
            csum = np.concatenate([[0], np.cumsum(t.len[x])])
            assert np.array_equal(index, csum[np.arange(index.size) * C])
            st, out = oracle.decode(bits, total, index, C, t, x.size)
            assert st == oracle.OK and np.array_equal(out, x), (name, mode)
        # padding bits are zero
        if total % 32:
            last = int.from_bytes(bits[-4:].tobytes(), "big")
            assert last & ((1 << (32 - total % 32)) - 1) == 0


def test_bitstream_matches_string_concatenation():
    """Encode equals the concatenation of the code strings, MSB first."""
    rng = np.random.default_rng(2)
    x = rng.integers(0, 256, 999).astype(np.uint8)
    t = oracle.build_table(oracle.histogram(x), oracle.MODE_PAPER_T2)
    st, bits, index, total = oracle.encode(x, t, 256)
    s = "".join(t.code_string(v) for v in x)
    s += "0" * (-len(s) % 32)
    expect = np.array([int(s[i:i + 8], 2) for i in range(0, len(s), 8)], np.uint8)
    assert np.array_equal(bits, expect)


def test_bitstream_does_not_depend_on_chunk_size():
    rng = np.random.default_rng(3)
    x = rng.integers(0, 256, 10000).astype(np.uint8)
    t = oracle.build_table(oracle.histogram(x), 0)
    b1 = oracle.encode(x, t, 256)[1]
    b2 = oracle.encode(x, t, 65536)[1]
    assert np.array_equal(b1, b2)


def test_empty_input():
    t = oracle.build_table(np.zeros(256, np.uint64), 0)
    st, bits, index, total = oracle.encode(np.zeros(0, np.uint8), t, 4096)
    assert st == oracle.OK and total == 0 and bits.size == 0 and index.size == 0
    st, out = oracle.decode(bits, 0, index, 4096, t, 0)
    assert st == oracle.OK and out.size == 0


def test_capacity_error():
    x = np.arange(256, dtype=np.uint8)
    t = oracle.build_table(oracle.histogram(x), oracle.MODE_PAPER_T1)
    total = int(sum(t.len[x]))
    need = 4 * ((total + 31) // 32)
    assert oracle.encode(x, t, 256, cap_bytes=need)[0] == oracle.OK
    assert oracle.encode(x, t, 256, cap_bytes=need - 4)[0] == oracle.ERR_CAPACITY


def test_corruption_is_detected():
    rng = np.random.default_rng(4)
    x = rng.integers(0, 256, 3000).astype(np.uint8)
    # Table 1 on near-uniform data: area 7 holds 168 of 256 suffixes, so
    # suffixes 0..87 there are invalid
    t = oracle.build_table(oracle.histogram(x), oracle.MODE_PAPER_T1)
    st, bits, index, total = oracle.encode(x, t, 256)
    # truncated stream: read past total_bits
    assert oracle.decode(bits, total - 5, index, 256, t, x.size)[0] == oracle.ERR_CORRUPT_STREAM
    # chunk index permuted: chunks no longer end where the next begins
    bad = index.copy()
    bad[[1, 2]] = bad[[2, 1]]
    assert oracle.decode(bits, total, bad, 256, t, x.size)[0] == oracle.ERR_CORRUPT_STREAM
    # wrong symbol count
    assert oracle.decode(bits, total, index, 256, t, x.size - 1)[0] == oracle.ERR_CORRUPT_STREAM
    # an invalid suffix in area 111: code 111 00000000 (rank 0 < first rank 88)
    one = np.zeros(4, np.uint8)
    one[0], one[1] = 0b11100000, 0b00000000
    assert oracle.decode(one, 11, np.zeros(1, np.uint64), 256, t, 1)[0] == oracle.ERR_CORRUPT_STREAM
    one[0], one[1] = 0b11101011, 0b00000000   # 111 01011000 = rank 88: valid
    assert oracle.decode(one, 11, np.zeros(1, np.uint64), 256, t, 1)[0] == oracle.OK
    # flipped bits: either detected or decoded to different bytes, never equal
    for k in rng.integers(0, total, 20):
        b2 = bits.copy()
        b2[k // 8] ^= 0x80 >> (k % 8)
        st, out = oracle.decode(b2, total, index, 256, t, x.size)
        assert st == oracle.ERR_CORRUPT_STREAM or not np.array_equal(out, x)


def test_table_from_layout_round_trip():
    rng = np.random.default_rng(6)
    h = (rng.pareto(1.0, 256) * 100).astype(np.uint64)
    t = oracle.build_table(h, 0)
    t2 = oracle.table_from_layout(t.width, t.rank_to_sym)
    assert np.array_equal(t.code, t2.code) and np.array_equal(t.len, t2.len)
    with pytest.raises(ValueError):
        oracle.table_from_layout([3, 3, 3, 3, 3, 3, 3, 3], t.rank_to_sym)   # no cover
    bad = t.rank_to_sym.copy()
    bad[0] = bad[1]
    with pytest.raises(ValueError):
        oracle.table_from_layout(t.width, bad)                                # not a permutation
