"""The multi-threaded oracle equals the single-threaded oracle byte for byte:
histogram, bitstream, chunk index, total bits, decoded bytes and statuses
(random, skewed, uniform, empty, N = 1 and ragged inputs; several thread
counts and chunk sizes; corrupted streams and a short capacity)."""
import numpy as np
import pytest

import oracle


def _inputs():
    rng = np.random.default_rng(11)
    yield "empty", np.zeros(0, np.uint8)
    yield "one", np.array([200], np.uint8)
    yield "uniform", rng.integers(0, 256, 100_003).astype(np.uint8)
    z = rng.integers(0, 256, 262_144 + 77).astype(np.uint8)
    z[rng.random(z.size) < 0.9] = 0
    yield "zeros90", z
    g = np.clip(np.round(rng.laplace(0, 6, 300_001)), -100, 100).astype(np.int64) % 256
    yield "laplace", g.astype(np.uint8)
    yield "constant", np.full(4097, 0x5A, np.uint8)


@pytest.mark.parametrize("threads", [1, 2, 3, 8])
def test_histogram_mt_equals_st(threads):
    for name, x in _inputs():
        assert np.array_equal(oracle.histogram_mt(x, threads), oracle.histogram(x)), name


@pytest.mark.parametrize("threads", [2, 5, 8])
@pytest.mark.parametrize("C", [1, 7, 256, 4096])
@pytest.mark.parametrize("mode", [oracle.MODE_SEARCH_QUAD, oracle.MODE_PAPER_T1])
def test_encode_decode_mt_equal_st(threads, C, mode):
    for name, x in _inputs():
        t = oracle.build_table(oracle.histogram(x), mode)
        st, bits, index, total = oracle.encode(x, t, C)
        mst, mbits, mindex, mtotal = oracle.encode_mt(x, t, C, threads=threads)
        assert (mst, mtotal) == (st, total), name
        assert np.array_equal(mbits, bits), name
        assert np.array_equal(mindex, index), name
        dst, out = oracle.decode(bits, total, index, C, t, x.size)
        mdst, mout = oracle.decode_mt(bits, total, index, C, t, x.size, threads=threads)
        assert dst == mdst == oracle.OK, name
        assert np.array_equal(mout, x) and np.array_equal(out, x), name


def test_small_alphabet_tables_mt_equal_st():
    """Tables of 16 symbols with a 2-bit area code (codes as short as 2 bits)."""
    rng = np.random.default_rng(12)
    x = np.minimum(rng.geometric(0.3, 50_001) - 1, 15).astype(np.uint8)
    h = oracle.histogram(x)[:16]
    t = oracle.build_table_general(h, 16, 4, 2, 4)
    for C in (1, 2, 3, 256):
        ref = oracle.encode(x, t, C)
        got = oracle.encode_mt(x, t, C, threads=4)
        assert got[0] == ref[0] and got[3] == ref[3]
        assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])
        assert oracle.decode_mt(ref[1], ref[3], ref[2], C, t, x.size, threads=4)[0] == oracle.OK


def test_capacity_and_corruption_statuses_match():
    rng = np.random.default_rng(13)
    x = rng.integers(0, 256, 50_000).astype(np.uint8)
    t = oracle.build_table(oracle.histogram(x), oracle.MODE_PAPER_T1)
    C = 256
    st, bits, index, total = oracle.encode(x, t, C)
    short = len(bits) - 4
    assert oracle.encode(x, t, C, cap_bytes=short)[0] == oracle.ERR_CAPACITY
    assert oracle.encode_mt(x, t, C, cap_bytes=short, threads=4)[0] == oracle.ERR_CAPACITY
    cases = []
    b = bits.copy()
    b[len(b) // 2] ^= 0xFF                       # flipped bits in the middle
    cases.append((b, total, index))
    idx = index.copy()
    idx[5], idx[6] = idx[6], idx[5]              # index entries out of order
    cases.append((bits, total, idx))
    cases.append((bits, total - 3, index))       # truncated stream
    idx0 = index.copy()
    idx0[0] = 1                                  # first chunk not at bit 0
    cases.append((bits, total, idx0))
    for b, tb, ix in cases:
        ref = oracle.decode(b, tb, ix, C, t, x.size)[0]
        assert ref == oracle.ERR_CORRUPT_STREAM
        for threads in (1, 3, 8):
            assert oracle.decode_mt(b, tb, ix, C, t, x.size, threads=threads)[0] == ref
    assert oracle.decode_mt(bits[:4], 5, np.zeros(0, np.uint64), C, t, 0, 4)[0] == \
        oracle.decode(bits[:4], 5, np.zeros(0, np.uint64), C, t, 0)[0]
