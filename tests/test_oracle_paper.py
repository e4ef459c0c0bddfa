"""Oracle pinned to what arXiv 2602.17849 prints (CPU only).

Each test names the table or passage of the paper that fixes the expected
values; the values themselves live in tests/golden/.
"""
import numpy as np
import pytest

import oracle
from conftest import read_golden
from helpers import paper_histogram


def _layout_rows(name):
    rows = []
    for area, code, n, b, length, lo, hi in read_golden(name):
        rows.append(dict(area=int(area) - 1, code=code, n=int(n), b=int(b), len=int(length),
                         lo=int(lo), hi=int(hi)))
    return rows


@pytest.mark.parametrize("name,mode", [("paper_table1.txt", oracle.MODE_PAPER_T1),
                                       ("paper_table2.txt", oracle.MODE_PAPER_T2)])
def test_fixed_layouts_reproduce_printed_tables(name, mode):
    """Tables 1 and 2: symbol counts, suffix bits, code lengths and rank
    ranges of every area come out of the oracle's greedy fill."""
    h, _ = paper_histogram()
    t = oracle.build_table(h, mode)
    for row in _layout_rows(name):
        a = row["area"]
        assert format(a, "03b") == row["code"]
        assert t.width[a] == row["b"]
        assert t.count[a] == row["n"]
        assert t.first[a] == row["lo"]
        assert t.first[a] + t.count[a] - 1 == row["hi"]
        assert t.prefix_bits + t.width[a] == row["len"]


def test_rank_order_reproduces_named_symbols():
    """Implementation section: 113, 241, 234, 106 are the most frequent and
    141, 137, 0, 128 the least frequent symbols."""
    h, _ = paper_histogram()
    r2s, s2r = oracle.rank(h)
    for r, s in read_golden("paper_ranking_order.txt"):
        assert r2s[int(r)] == int(s)
        assert s2r[int(s)] == int(r)


def test_encoder_lut_rows_of_table3():
    """Table 3: printed (input symbol, mapped-to rank, code) rows."""
    h, _ = paper_histogram()
    t = oracle.build_table(h, oracle.MODE_PAPER_T1)
    for sym, rank, code in read_golden("paper_table3_encoder_lut.txt"):
        sym, rank = int(sym), int(rank)
        assert t.sym_to_rank[sym] == rank
        assert t.code_string(sym) == code.replace("_", "")


def test_decoder_lut_rows_of_table4():
    """Table 4: printed (encoded symbol, output symbol) rows."""
    h, _ = paper_histogram()
    t = oracle.build_table(h, oracle.MODE_PAPER_T1)
    for rank, sym in read_golden("paper_table4_decoder_lut.txt"):
        assert t.rank_to_sym[int(rank)] == int(sym)


def test_decode_worked_example():
    """Implementation section: area 100 + suffix 010 -> 32 + 2 = 34; the
    oracle decoder maps that 6-bit code to the symbol at rank 34."""
    h, _ = paper_histogram()
    t = oracle.build_table(h, oracle.MODE_PAPER_T1)
    (area, suffix, off, rank), = read_golden("paper_decode_example.txt")
    a = int(area, 2)
    assert t.offset[a] == int(off)
    assert t.offset[a] + int(suffix, 2) == int(rank)
    # a one-symbol stream holding exactly that code
    bits = np.zeros(4, dtype=np.uint8)
    bits[0] = int(area + suffix + "00", 2)
    st, out = oracle.decode(bits, 6, np.zeros(1, np.uint64), 256, t, 1)
    assert st == oracle.OK
    assert out[0] == t.rank_to_sym[int(rank)]


@pytest.mark.parametrize("name", ["A", "B"])
def test_hand_worked_streams(name):
    """Streams worked by hand from the Table 3 codes (bit order reading:
    most significant bit first, zero padding to 32 bits)."""
    h, _ = paper_histogram()
    t = oracle.build_table(h, oracle.MODE_PAPER_T1)
    rows = {r[0]: r for r in read_golden("hand_streams.txt")}
    _, syms, total, hexbytes = rows[name]
    x = np.array([int(s) for s in syms.split(",")], dtype=np.uint8)
    st, bits, index, tb = oracle.encode(x, t, chunk_symbols=256)
    assert st == oracle.OK
    assert tb == int(total)
    assert [int(b, 16) for b in hexbytes.split(",")] == list(bits)
    assert list(index) == [0]
    st, out = oracle.decode(bits, tb, index, 256, t, x.size)
    assert st == oracle.OK and np.array_equal(out, x)


def test_code_lengths_of_the_two_schemes():
    """Quad Length Codes section: lengths 6, 7, 8, 11 (3+3, 3+4, 3+5, 3+8);
    Adaptation section: lengths 4, 6, 8, 11."""
    h, _ = paper_histogram()
    t1 = oracle.build_table(h, oracle.MODE_PAPER_T1)
    t2 = oracle.build_table(h, oracle.MODE_PAPER_T2)
    assert sorted(set(t1.len.tolist())) == [6, 7, 8, 11]
    assert sorted(set(t2.len.tolist())) == [4, 6, 8, 11]


def test_kraft_sums_of_printed_schemes():
    """Exact Kraft sums of the 256 codes of Tables 1 and 2 (closed forms
    from the printed counts and lengths): 40/64 + 16/128 + 32/256 + 168/2048
    and 2/16 + 32/64 + 64/256 + 158/2048."""
    h, _ = paper_histogram()
    for mode, expect in [(oracle.MODE_PAPER_T1, 40 / 64 + 16 / 128 + 32 / 256 + 168 / 2048),
                         (oracle.MODE_PAPER_T2, 2 / 16 + 32 / 64 + 64 / 256 + 158 / 2048)]:
        t = oracle.build_table(h, mode)
        assert sum(2.0 ** -int(l) for l in t.len) == expect
    assert 40 / 64 + 16 / 128 + 32 / 256 + 168 / 2048 == 0.95703125
    assert 2 / 16 + 32 / 64 + 64 / 256 + 158 / 2048 == 0.9521484375


def test_compressibility_arithmetic_of_the_paper():
    """Observations / Adaptation sections: (8 - 6.69)/8 is printed as about
    16.3 % and (8 - 6.11)/8 as 23.6 %; Table 2 gains 2.3 points over
    Table 1 (19.0 vs 16.7) and QLC is 2.0 points below Huffman (13.9 vs
    15.9)."""
    from oracle.bounds import compressibility
    assert abs(compressibility(6.69) - 0.16375) < 1e-12
    assert round(compressibility(6.11) * 100, 1) == 23.6
    assert round(19.0 - 16.7, 1) == 2.3
    assert round(15.9 - 13.9, 1) == 2.0
