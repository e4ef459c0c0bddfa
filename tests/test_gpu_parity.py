"""GPU parity: libqlc's HIP kernels against the CPU oracle, element by
element, on seeded synthetic inputs (histogram, table, bitstream, chunk
index, total bits, round trip, error codes).  Bit-exact throughout."""
import numpy as np
import pytest
import torch

import oracle
from helpers import paper_histogram
from paper_2602_17849_amd import datagen, qlc

pytestmark = pytest.mark.gpu

from gpu_util import (DEV, assert_table_equal, gpu_decode, gpu_encode, gpu_table,  # noqa: E402
                      table_from_oracle, to_dev)

SIZES = [0, 1, 15, 16, 17, 255, 4095, 4096, 4097, 3 * 4096 + 1234, 100003, 262144 + 77]


def _inputs(n, seed=0):
    yield "gaussian", datagen.gaussian(n, seed).numpy() if n % 32 == 0 else \
        np.resize(datagen.gaussian(((n + 31) // 32) * 32, seed).numpy(), n)
    rng = np.random.default_rng(seed + n)
    yield "uniform", rng.integers(0, 256, n).astype(np.uint8)
    z = rng.integers(0, 256, n).astype(np.uint8)
    z[rng.random(n) < 0.9] = 0
    yield "zeros90", z
    yield "constant", np.full(n, 0x5A, np.uint8)


@pytest.mark.parametrize("n", SIZES)
def test_histogram(n):
    for name, x in _inputs(n):
        h = torch.zeros(256, dtype=torch.int64, device=DEV)
        ws = qlc.new_workspace(n)
        qlc.qlc_histogram(to_dev(x), h, ws)
        assert np.array_equal(h.cpu().numpy().astype(np.uint64), oracle.histogram(x)), name


def test_histogram_accumulate_and_shared_table():
    """Histograms summed over several tensors on the device equal the
    oracle's histogram of their concatenation; the table built from the sum
    (one LUT for the tensor type) equals the oracle's, and encoding each
    tensor with it equals the oracle's encode with that table."""
    xs = [x for n in (0, 17, 4097, 100003, 262144 + 77) for _, x in _inputs(n, seed=3)]
    h = torch.zeros(256, dtype=torch.int64, device=DEV)
    h[:] = 5                                        # accumulation adds to what is there
    ws = qlc.new_workspace(max(x.size for x in xs))
    for x in xs:
        qlc.qlc_histogram_accumulate(to_dev(x), h, ws)
    torch.cuda.synchronize()
    ref = oracle.histogram(np.concatenate(xs)) + np.uint64(5)
    assert np.array_equal(h.cpu().numpy().astype(np.uint64), ref)
    for mode in (qlc.LAYOUT_SEARCH_QUAD, qlc.LAYOUT_PAPER_T1):
        t = qlc.shared_table([to_dev(x) for x in xs], mode)
        torch.cuda.synchronize()
        ot = oracle.build_table(oracle.histogram(np.concatenate(xs)), mode)
        assert_table_equal(t, ot)
        for x in xs[::3]:
            err, bits, nb, index, total = gpu_encode(to_dev(x), t, 4096)
            st, obits, oindex, ototal = oracle.encode(x, ot, 4096)
            assert err == 0 and total == ototal
            assert np.array_equal(bits[:nb], obits) and np.array_equal(index, oindex)


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [0, 1, 4097, 100003, 1 << 20])
def test_build_table(mode, n):
    for name, x in _inputs(n, seed=1):
        t = gpu_table(to_dev(x), mode)
        assert_table_equal(t, oracle.build_table(oracle.histogram(x), mode))


@pytest.mark.parametrize("k", range(1, 9))
def test_distinct_cap_modes(k):
    """SEARCH_DISTINCT_k (at most k distinct code lengths): the GPU table
    equals the oracle's capped search on skewed, uniform, tied and
    single-symbol histograms; a compress with it matches the oracle's
    encode and round-trips."""
    mode = qlc.LAYOUT_SEARCH_DISTINCT(k)
    rng = np.random.default_rng(40 + k)
    hists = [(rng.pareto(1.0, 256) * 1000).astype(np.uint64), np.ones(256, np.uint64),
             np.repeat(np.arange(8, dtype=np.uint64), 32) * 5]
    one = np.zeros(256, np.uint64)
    one[17] = 1000
    hists.append(one)
    for hh in hists:
        t = qlc.new_table()
        qlc.qlc_table_from_histogram(to_dev(hh.astype(np.int64)), mode, t)
        torch.cuda.synchronize()
        assert_table_equal(t, oracle.build_table_general(hh, 256, 8, 3, k))
    x = datagen.gaussian(200000, 50 + k).numpy()
    ot = oracle.build_table_general(oracle.histogram(x), 256, 8, 3, k)
    c = qlc.compress(to_dev(x), mode=mode, chunk_symbols=4096)
    torch.cuda.synchronize()
    assert_table_equal(c.table, ot)
    st, obits, oindex, ototal = oracle.encode(x, ot, 4096)
    assert c.total_bits() == ototal
    assert np.array_equal(c.bits[:c.nbytes()].cpu().numpy(), obits)
    out, err = qlc.decompress(c)
    torch.cuda.synchronize()
    assert int(err.item()) == 0 and np.array_equal(out.cpu().numpy(), x)


def _assert_areas4_table(t_dev, ot):
    """A 4-area GPU table against the oracle's general (256 symbols, 4
    areas, 2-bit area code) table."""
    t = qlc.parse_table(t_dev)
    assert list(t["width"][:4]) == list(ot.width) and list(t["width"][4:]) == [0xFF] * 4
    assert list(t["first"][:4]) == list(ot.first) and list(t["count"][:4]) == list(ot.count)
    assert list(t["count"][4:]) == [0] * 4
    assert list(t["offset"][:4]) == list(ot.offset)
    assert np.array_equal(t["rank_to_sym"], ot.rank_to_sym)
    assert np.array_equal(t["enc"] >> 11, ot.len) and np.array_equal(t["enc"] & 0x7FF, ot.code)
    assert t["cost_bits"] == ot.cost_bits


def test_areas4_tables():
    """SEARCH_AREAS4 (2-bit area code, 4 areas): the GPU table equals the
    oracle's general search on skewed, uniform, tied and single-symbol
    histograms, and the host deserializer rebuilds the same table."""
    rng = np.random.default_rng(77)
    hists = [(rng.pareto(1.0, 256) * 1000).astype(np.uint64), np.ones(256, np.uint64),
             np.repeat(np.arange(8, dtype=np.uint64), 32) * 5,
             (rng.pareto(0.4, 256) * 50).astype(np.uint64)]
    one = np.zeros(256, np.uint64)
    one[200] = 7
    hists.append(one)
    for hh in hists:
        t = qlc.new_table()
        qlc.qlc_table_from_histogram(to_dev(hh.astype(np.int64)), qlc.LAYOUT_SEARCH_AREAS4, t)
        torch.cuda.synchronize()
        ot = oracle.build_table_general(hh, 256, 4, 2, 8)
        _assert_areas4_table(t, ot)
        blob = bytes(list(ot.width.astype(np.uint8)) + [0xFF] * 4) + \
            bytes(ot.rank_to_sym.astype(np.uint8))
        h = qlc.parse_table(qlc.qlc_table_deserialize(blob))
        g = qlc.parse_table(t)
        for key in ("enc", "width", "first", "count", "offset", "rank_to_sym", "sym_to_rank"):
            assert np.array_equal(h[key], g[key]), key


@pytest.mark.parametrize("C", [256, 4096])
def test_areas4_encode_decode(C):
    """Compress with SEARCH_AREAS4 matches the oracle's encode with the
    oracle's 4-area table (stream, index, total), the GPU decode restores
    every byte, and a corrupted stream is reported as the oracle reports it."""
    for n in (0, 1, 4097, 100003, 262144 + 77):
        for name, x in _inputs(n, seed=9):
            ot = oracle.build_table_general(oracle.histogram(x), 256, 4, 2, 8)
            c = qlc.compress(to_dev(x), mode=qlc.LAYOUT_SEARCH_AREAS4, chunk_symbols=C)
            torch.cuda.synchronize()
            assert int(c.err.item()) == 0
            _assert_areas4_table(c.table, ot)
            st, obits, oindex, ototal = oracle.encode(x, ot, C)
            assert c.total_bits() == ototal, name
            assert np.array_equal(c.bits[:c.nbytes()].cpu().numpy(), obits), name
            k = qlc.qlc_chunk_count(n, C)
            assert np.array_equal(c.index[:k].cpu().numpy().astype(np.uint64),
                                  oindex.astype(np.uint64)), name
            out, err = qlc.decompress(c)
            torch.cuda.synchronize()
            assert int(err.item()) == 0 and np.array_equal(out.cpu().numpy(), x), name
    # corrupt: flip bits in the middle of a stream; both sides must agree
    x = datagen.gaussian(65536, 3).numpy()
    ot = oracle.build_table_general(oracle.histogram(x), 256, 4, 2, 8)
    c = qlc.compress(to_dev(x), mode=qlc.LAYOUT_SEARCH_AREAS4, chunk_symbols=C)
    torch.cuda.synchronize()
    bits = c.bits[:c.nbytes()].cpu().numpy().copy()
    bits[len(bits) // 2] ^= 0x5A
    index = c.index[:qlc.qlc_chunk_count(x.size, C)].cpu().numpy().astype(np.uint64)
    ost, _ = oracle.decode(bits, c.total_bits(), index, C, ot, x.size)
    err, _ = gpu_decode(bits, c.total_bits(), index, C, c.table, x.size)
    assert err == ost


def test_areas4_batched_matches_plain():
    """The batched form with SEARCH_AREAS4 equals the single-tensor entry
    points per job."""
    C = 2048
    sizes = [100000, 4096, 262145, 1, 70000]
    b = qlc.Batch(sizes, chunk_symbols=C, device=DEV)
    xs = []
    for i, n in enumerate(sizes):
        x = datagen.gaussian(max(32, (n + 31) // 32 * 32), 90 + i)[:n].contiguous()
        xs.append(x)
        b.input(i).copy_(x.to(DEV))
    ws = b.workspace()
    b.encode(ws, qlc.LAYOUT_SEARCH_AREAS4)
    b.decode(ws)
    torch.cuda.synchronize()
    assert not b.err.any().item()
    for i, x in enumerate(xs):
        ref = qlc.compress(x.to(DEV), mode=qlc.LAYOUT_SEARCH_AREAS4, chunk_symbols=C)
        torch.cuda.synchronize()
        assert int(b.total[i].item()) == ref.total_bits()
        nb = ref.nbytes()
        assert torch.equal(b.bitstream(i, nb), ref.bits[:nb])
        assert torch.equal(b.table(i), ref.table)
        assert torch.equal(b.output(i).cpu(), x)


def test_table_from_histogram_paper_rows():
    """Constructed histogram reproducing Tables 3/4 on the GPU, plus
    histograms with many ties and counts beyond 2^32."""
    h, _ = paper_histogram()
    cases = [h, np.ones(256, np.uint64), np.repeat(np.arange(8, dtype=np.uint64), 32) * 5,
             (np.arange(256, dtype=np.uint64) % 3) << np.uint64(34)]
    for hh in cases:
        for mode in range(4):
            t = qlc.new_table()
            qlc.qlc_table_from_histogram(to_dev(hh.astype(np.int64)), mode, t)
            torch.cuda.synchronize()
            assert_table_equal(t, oracle.build_table(hh, mode))


@pytest.mark.parametrize("C", [256, 4096, 65536])
@pytest.mark.parametrize("n", SIZES)
def test_encode_bit_exact(n, C):
    for name, x in _inputs(n, seed=2):
        for mode in (0, 2):
            ot = oracle.build_table(oracle.histogram(x), mode)
            t = table_from_oracle(ot)
            err, bits, nbytes, index, total = gpu_encode(to_dev(x), t, C)
            st, obits, oindex, ototal = oracle.encode(x, ot, C)
            assert err == 0 and st == 0
            assert total == ototal
            assert nbytes == obits.size
            assert np.array_equal(bits[:nbytes], obits), (name, mode)
            assert np.array_equal(index, oindex), (name, mode)


DECODERS = [qlc.DECODER_LANE, qlc.DECODER_SPLIT]


@pytest.mark.parametrize("decoder", DECODERS)
@pytest.mark.parametrize("C", [256, 1024, 4096, 65536])
@pytest.mark.parametrize("n", SIZES)
def test_decode_oracle_streams(n, C, decoder):
    """Decode streams written by the oracle (independent of the GPU encoder),
    with either decoder (the split one takes C <= 16384)."""
    if decoder == qlc.DECODER_SPLIT and C > qlc.SPLIT_MAX_CHUNK:
        pytest.skip("split decoder: C <= 16384")
    for name, x in _inputs(n, seed=3):
        for mode in (0, 1, 2, 3):
            ot = oracle.build_table(oracle.histogram(x), mode)
            st, obits, oindex, ototal = oracle.encode(x, ot, C)
            err, out = gpu_decode(obits, ototal, oindex, C, table_from_oracle(ot), n, decoder)
            assert err == 0, (name, mode)
            assert np.array_equal(out, x), (name, mode)


def test_round_trip_gpu_only():
    x = datagen.single_tensor_gaussian(seed=0, device=DEV)
    c = qlc.compress(x, chunk_symbols=4096)
    out, err = qlc.decompress(c)
    torch.cuda.synchronize()
    assert int(c.err.item()) == 0 and int(err.item()) == 0
    assert torch.equal(out, x)


@pytest.mark.parametrize("decoder", DECODERS)
def test_decode_error_codes_match_oracle(decoder):
    rng = np.random.default_rng(4)
    x = rng.integers(0, 256, 20000).astype(np.uint8)
    C = 256
    ot = oracle.build_table(oracle.histogram(x), oracle.MODE_PAPER_T1)
    t = table_from_oracle(ot)
    st, bits, index, total = oracle.encode(x, ot, C)
    cases = {"truncated": (bits, total - 5, index, x.size)}
    bad = index.copy(); bad[[3, 4]] = bad[[4, 3]]
    cases["permuted_index"] = (bits, total, bad, x.size)
    cases["short_n"] = (bits, total, index, x.size - 1)
    bad0 = index.copy(); bad0[0] = 11
    cases["index0"] = (bits, total, bad0, x.size)
    for k in rng.integers(0, total, 12):
        b2 = bits.copy(); b2[k // 8] ^= 0x80 >> (k % 8)
        cases["flip%d" % k] = (b2, total, index, x.size)
    for name, (b, tb, idx, n) in cases.items():
        ost, oout = oracle.decode(b, tb, idx, C, ot, n)
        err, out = gpu_decode(b, tb, idx, C, t, n, decoder)
        assert err == ost, name
        if ost == 0:
            assert np.array_equal(out, oout), name


def test_capacity_error():
    x = datagen.gaussian(100000, 5).numpy()
    ot = oracle.build_table(oracle.histogram(x), 0)
    t = table_from_oracle(ot)
    st, obits, oindex, ototal = oracle.encode(x, ot, 4096)
    cap = (obits.size // 2) & ~15
    err, bits, nbytes, index, total = gpu_encode(to_dev(x), t, 4096, cap=cap)
    assert err == qlc.QLC_ERR_CAPACITY
    assert total == ototal
    assert np.array_equal(bits[:cap], obits[:cap])
    assert not bits[cap:].any()          # nothing written past the capacity


@pytest.mark.parametrize("sym,length", [(0, 0), (131, 12), (255, 31)])
def test_bad_table_rejected(sym, length):
    """A given table with a code length outside 1..11 is rejected by every
    workgroup of the encode (device error word), plain and batched.  (One-bit
    codes are legal: a two-area table of 16 symbols has them.)"""
    n = 5_000_000
    x = datagen.gaussian(n, 13).numpy()
    t = table_from_oracle(oracle.build_table(oracle.histogram(x), 0))
    enc = t[:512].view(torch.int16)
    enc[sym] = (enc[sym] & 0x7FF) | (length << 11)
    err, bits, nbytes, index, total = gpu_encode(to_dev(x), t, 4096)
    assert err == qlc.QLC_ERR_INVALID_ARGUMENT
    b = qlc.Batch([n, 1000], chunk_symbols=4096, device=DEV, capacity="bound", build_table=False)
    b.input(0).copy_(to_dev(x))
    b.input(1).copy_(to_dev(x[:1000]))
    b.table(0).copy_(t)
    b.table(1).copy_(table_from_oracle(oracle.build_table(oracle.histogram(x[:1000]), 0)))
    ws = b.workspace()
    b.encode(ws)
    torch.cuda.synchronize()
    assert int(b.err[0]) == qlc.QLC_ERR_INVALID_ARGUMENT and int(b.err[1]) == 0


@pytest.mark.parametrize("case", ["one_count", "sum"])
def test_table_from_oversized_histogram_is_unusable(case):
    """Counts summing to 2^48 or more (or any count that large) give a table
    marked unusable (every code length 0, every width 0xFF), which the
    encoder rejects; a sum just below 2^48 still gives the oracle's table."""
    hh = np.ones(256, np.uint64)
    if case == "one_count":
        hh[3] = np.uint64(1) << np.uint64(50)
    else:
        hh[:] = np.uint64(1) << np.uint64(41)          # 256 * 2^41 = 2^49
    t = qlc.new_table()
    qlc.qlc_table_from_histogram(to_dev(hh.astype(np.int64)), qlc.LAYOUT_SEARCH_QUAD, t)
    torch.cuda.synchronize()
    raw = qlc.parse_table(t)
    assert all(v == 0 for v in raw["enc"]) and all(w == 0xFF for w in raw["width"])
    x = datagen.gaussian(100_000, 14).numpy()
    err = gpu_encode(to_dev(x), t, 4096)[0]
    assert err == qlc.QLC_ERR_INVALID_ARGUMENT
    # just below the limit: the exact table
    below = np.ones(256, np.uint64)
    below[7] = (np.uint64(1) << np.uint64(48)) - np.uint64(256)   # sum = 2^48 - 1
    qlc.qlc_table_from_histogram(to_dev(below.astype(np.int64)), qlc.LAYOUT_SEARCH_QUAD, t)
    torch.cuda.synchronize()
    assert_table_equal(t, oracle.build_table(below, qlc.LAYOUT_SEARCH_QUAD))


@pytest.mark.parametrize("fmt", [(1, 2), (2, 3)])        # e2m1 (16 codes), e3m2 (64 codes)
@pytest.mark.parametrize("mode", [qlc.LAYOUT_SEARCH_QUAD, qlc.LAYOUT_SEARCH_ANY,
                                  qlc.LAYOUT_SEARCH_AREAS4])
def test_small_alphabets_one_code_per_byte(fmt, mode):
    """Narrower float types (4-bit e2m1, 6-bit e3m2) stored one code per
    byte: the unused byte values have zero counts and rank last, so every
    layout mode applies unchanged; table, stream and index equal the
    oracle's and the decode restores every code."""
    mant, exp = fmt
    x = datagen.small_float_codes(200003, mant, exp, seed=21 + mant)
    assert int(x.max()) < (1 << (1 + exp + mant))
    h = oracle.histogram(x)
    if mode == qlc.LAYOUT_SEARCH_AREAS4:
        ot = oracle.build_table_general(h, 256, 4, 2, 8)
    else:
        ot = oracle.build_table(h, mode)
    c = qlc.compress(to_dev(x), mode=mode, chunk_symbols=1024)
    torch.cuda.synchronize()
    assert int(c.err.item()) == 0
    if mode == qlc.LAYOUT_SEARCH_AREAS4:
        _assert_areas4_table(c.table, ot)
    else:
        assert_table_equal(c.table, ot)
    st, obits, oindex, ototal = oracle.encode(x, ot, 1024)
    assert c.total_bits() == ototal
    assert np.array_equal(c.bits[:c.nbytes()].cpu().numpy(), obits)
    k = qlc.qlc_chunk_count(x.size, 1024)
    assert np.array_equal(c.index[:k].cpu().numpy().astype(np.uint64), oindex.astype(np.uint64))
    out, err = qlc.decompress(c)
    torch.cuda.synchronize()
    assert int(err.item()) == 0 and np.array_equal(out.cpu().numpy(), x)


def test_deterministic_repeat():
    x = to_dev(datagen.gaussian(1 << 20, 9).numpy())
    t = gpu_table(x, 0)
    a = gpu_encode(x, t, 1024)
    for _ in range(3):
        b = gpu_encode(x, t, 1024)
        assert a[0] == b[0] and a[4] == b[4]
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[3], b[3])


@pytest.mark.parametrize("n", [0, 1, 4097, 100003, 5_000_013])
@pytest.mark.parametrize("mode", [0, 3])
def test_compress_fused(n, mode):
    """Histogram + table + encode in one call (two kernels), against the
    oracle's table and stream; sizes span several segments of different
    lengths and a ragged tail."""
    rng = np.random.default_rng(n + mode)
    x = np.resize(datagen.gaussian(((n + 31) // 32) * 32 or 32, 7).numpy(), n)
    x[rng.random(n) < 0.05] = rng.integers(0, 256)
    xd = to_dev(x)
    C = 1024
    c = qlc.compress(xd, mode=mode, chunk_symbols=C)
    torch.cuda.synchronize()
    ot = oracle.build_table(oracle.histogram(x), mode)
    assert_table_equal(c.table, ot)
    st, obits, oindex, ototal = oracle.encode(x, ot, C)
    assert int(c.err.item()) == 0
    assert c.total_bits() == ototal
    assert np.array_equal(c.bits[:obits.size].cpu().numpy(), obits)
    assert np.array_equal(c.index[:oindex.size].cpu().numpy().astype(np.uint64), oindex)
    out, err = qlc.decompress(c)
    torch.cuda.synchronize()
    assert int(err.item()) == 0 and np.array_equal(out.cpu().numpy(), x)


def test_binding_refuses_strided_and_host_tensors():
    x = torch.zeros(4096, dtype=torch.uint8, device=DEV)
    h = torch.zeros(256, dtype=torch.int64, device=DEV)
    ws = qlc.new_workspace(4096)
    with pytest.raises(ValueError):
        qlc.qlc_histogram(x[::2], h, ws)
    with pytest.raises(ValueError):
        qlc.qlc_histogram(x.cpu(), h, ws)
