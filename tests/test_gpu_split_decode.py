"""The split-chunk decoder (qlc_decode_ex with QLC_DECODER_SPLIT: C / 64
lanes per chunk, code boundaries found by walking code lengths from guessed
starts and correcting them from the neighbouring lane's exit).  Streams
written by the oracle decode to the oracle's input, bit-exact, on data whose
guessed starts need no correction (every code one length), one round, or
long chains of rounds (all-zero and zero-heavy chunks, where a wrong start
stays wrong for the whole piece); ragged tails, several workgroups, every
supported chunk size; 4- and 6-bit alphabets; error codes equal the
oracle's; the same output as the one-lane-per-chunk decoder."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DEV, gpu_decode, table_from_oracle, to_dev
from paper_2602_17849_amd import datagen, qlc

pytestmark = pytest.mark.gpu

SPLIT = qlc.DECODER_SPLIT
LANE = qlc.DECODER_LANE


def _kinds(n, seed):
    """(name, bytes, layout mode) triples."""
    rng = np.random.default_rng(seed * 7919 + n)
    g = np.resize(datagen.gaussian(((n + 31) // 32) * 32, seed).numpy(), n)
    yield "gaussian", g, qlc.LAYOUT_SEARCH_QUAD
    yield "uniform", rng.integers(0, 256, n).astype(np.uint8), qlc.LAYOUT_SEARCH_QUAD
    z = rng.integers(0, 256, n).astype(np.uint8)
    z[rng.random(n) < 0.9] = 0
    yield "zeros90_t2", z, qlc.LAYOUT_PAPER_T2
    a = np.zeros(n, np.uint8)
    a[rng.random(n) < 0.001] = 7
    yield "almost_zero", a, qlc.LAYOUT_SEARCH_QUAD


@pytest.mark.parametrize("C", [256, 512, 2048, 4096, 16384])
@pytest.mark.parametrize("n", [1, 255, 257, 16384, 3 * 16384 + 777, 100003])
def test_split_decodes_oracle_streams(C, n):
    for name, x, mode in _kinds(n, 1):
        ot = oracle.build_table(oracle.histogram(x), mode)
        st, bits, index, total = oracle.encode(x, ot, C)
        assert st == 0
        err, out = gpu_decode(bits, total, index, C, table_from_oracle(ot), n, SPLIT)
        assert err == 0, name
        assert np.array_equal(out, x), name


@pytest.mark.parametrize("C", [2048, 16384])
def test_split_constant_chunks(C):
    """Chunks of one symbol: all codes one length under a table with other
    lengths, so every wrong guess stays wrong and the corrections take G
    rounds; and a table whose codes all have one length (no correction)."""
    n = 5 * C + 3
    x = np.zeros(n, np.uint8)
    x[:64] = np.arange(64)                     # the other symbols appear once
    h = oracle.histogram(x)
    tables = [oracle.build_table(h, qlc.LAYOUT_SEARCH_QUAD), oracle.build_table(h, qlc.LAYOUT_PAPER_T1),
              oracle.build_table_general(h, 256, 8, 3, 1)]   # at most one code length
    for mode, ot in enumerate(tables):
        st, bits, index, total = oracle.encode(x, ot, C)
        err, out = gpu_decode(bits, total, index, C, table_from_oracle(ot), n, SPLIT)
        assert err == 0, mode
        assert np.array_equal(out, x), mode


@pytest.mark.parametrize("C", [256, 2048, 16384])
def test_split_equals_lane_decoder(C):
    """16 Mi symbols of the Laplace recipe, compressed on the GPU: both
    decoders and the automatic choice return the input."""
    x = datagen.laplace_outlier_rows(2048, 8192, 11, device=DEV)
    obj = qlc.compress(x, chunk_symbols=C)
    outs = {}
    for dec in (LANE, SPLIT, qlc.DECODER_AUTO):
        out, err = qlc.decompress(obj, decoder=dec)
        torch.cuda.synchronize()
        assert int(err.item()) == 0, dec
        outs[dec] = out
    assert torch.equal(outs[SPLIT], x)
    assert torch.equal(outs[LANE], x)
    assert torch.equal(outs[qlc.DECODER_AUTO], x)


@pytest.mark.parametrize("bits,mode", [(4, qlc.LAYOUT_M16_AREAS2), (4, qlc.LAYOUT_M16_AREAS4),
                                       (6, qlc.LAYOUT_M64_AREAS4), (6, qlc.LAYOUT_M64_AREAS8)])
@pytest.mark.parametrize("n", [1, 7, 4097, 3 * 16384 + 5, 100003])
def test_split_small_alphabets(bits, mode, n):
    C = 512
    mant, exp = (1, 2) if bits == 4 else (2, 3)
    codes = datagen.small_float_codes(n, mant, exp, 5)
    p = datagen.pack_symbols(codes, bits)
    buf = torch.zeros(max(p.size, 16) + 16, dtype=torch.uint8)
    buf[:p.size] = torch.from_numpy(p)
    xd = buf.to(DEV)
    cap = qlc.qlc_encode_bound_bytes(n)
    table = qlc.new_table(DEV)
    bstream = torch.zeros(max(cap, 16), dtype=torch.uint8, device=DEV)
    index = torch.zeros(max(qlc.qlc_chunk_count(n, C), 1), dtype=torch.int64, device=DEV)
    total = torch.zeros(1, dtype=torch.int64, device=DEV)
    err = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    ws = qlc.new_workspace(n, C)
    qlc.qlc_compress_sym(xd, n, bits, mode, table, C, bstream[:cap], index, total, err, ws)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    for dec in (SPLIT, LANE):
        out = torch.full((p.size + 16,), 0xAA, dtype=torch.uint8, device=DEV)
        derr = torch.full((1,), -1, dtype=torch.int32, device=DEV)
        qlc.qlc_decode_ex(bstream, total, index, C, table, n, bits, dec, out, derr, ws)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        assert int(derr.item()) == 0, dec
        assert np.array_equal(o[:p.size], p), dec                 # pad bits zero
        assert (o[p.size:] == 0xAA).all(), dec                     # nothing past the end


@pytest.mark.parametrize("C", [256, 2048])
def test_split_error_codes_match_oracle(C):
    rng = np.random.default_rng(6)
    n = 3 * 16384 + 1001
    x = rng.integers(0, 256, n).astype(np.uint8)
    x[rng.random(n) < 0.5] = 0
    ot = oracle.build_table(oracle.histogram(x), oracle.MODE_PAPER_T1)
    t = table_from_oracle(ot)
    st, bits, index, total = oracle.encode(x, ot, C)
    k = index.size
    cases = {"truncated": (bits, total - 5, index, n), "long": (bits, total + 3, index, n)}
    bad = index.copy(); bad[[3, 4]] = bad[[4, 3]]
    cases["permuted_index"] = (bits, total, bad, n)
    cases["short_n"] = (bits, total, index, n - 1)
    bad0 = index.copy(); bad0[0] = 11
    cases["index0"] = (bits, total, bad0, n)
    gap = index.copy(); gap[k // 2] += 1
    cases["shifted_entry"] = (bits, total, gap, n)
    far = index.copy(); far[k - 1] = total + 100
    cases["entry_past_total"] = (bits, total, far, n)
    for kk in rng.integers(0, total, 12):
        b2 = bits.copy(); b2[kk // 8] ^= 0x80 >> (kk % 8)
        cases["flip%d" % kk] = (b2, total, index, n)
    for name, (b, tb, idx, nn) in cases.items():
        b = np.concatenate([b, np.zeros(16, np.uint8)])
        ost, oout = oracle.decode(b, tb, idx, C, ot, nn)
        err, out = gpu_decode(b, tb, idx, C, t, nn, SPLIT)
        assert err == ost, name
        if ost == 0:
            assert np.array_equal(out, oout), name


def test_split_rejects_large_chunks_and_unknown_decoders():
    n = 1000
    x = np.zeros(n, np.uint8)
    ot = oracle.build_table(oracle.histogram(x), 0)
    t = table_from_oracle(ot)
    for C in (32768, 65536):
        st, bits, index, total = oracle.encode(x, ot, C)
        with pytest.raises(qlc.QLCError):
            gpu_decode(bits, total, index, C, t, n, SPLIT)
        err, out = gpu_decode(bits, total, index, C, t, n, qlc.DECODER_AUTO)
        assert err == 0 and np.array_equal(out, x)
    st, bits, index, total = oracle.encode(x, ot, 256)
    with pytest.raises(qlc.QLCError):
        gpu_decode(bits, total, index, 256, t, n, 7)


def test_split_refuses_a_table_of_another_alphabet():
    """A byte stream decoded with a 16-symbol table (and the reverse) is
    refused: QLC_ERR_INVALID_ARGUMENT, nothing written."""
    n, C = 40000, 512
    x = np.resize(datagen.gaussian(40000, 9).numpy(), n)
    ot = oracle.build_table(oracle.histogram(x), qlc.LAYOUT_SEARCH_QUAD)
    st, bits, index, total = oracle.encode(x, ot, C)
    codes = datagen.small_float_codes(n, 1, 2, 9)
    t16 = table_from_oracle(oracle.build_table_general(oracle.histogram(codes)[:16], 16, 4, 2, 4))
    assert qlc.mode_symbol_bits(int(qlc.parse_table(t16)["mode"])) == 4
    for t, sb in ((t16, 8), (table_from_oracle(ot), 4)):
        err, out = gpu_decode(bits, total, index, C, t, n, SPLIT, symbol_bits=sb)
        assert err == qlc.QLC_ERR_INVALID_ARGUMENT, sb
        assert (out == 0xAA).all(), sb



def _random_case(rng):
    n = int(np.exp(rng.uniform(0, np.log(1 << 21))))
    C = int(2 ** rng.integers(8, 15))
    kind = rng.integers(0, 5)
    if kind == 0:
        x = np.resize(datagen.gaussian(((n + 31) // 32) * 32, int(rng.integers(1 << 30))).numpy(), n)
    elif kind == 1:
        x = rng.integers(0, 256, n).astype(np.uint8)
        x[rng.random(n) < rng.uniform(0.5, 0.999)] = 0
    elif kind == 2:                      # long runs of one byte with bursts of others
        x = np.full(n, rng.integers(0, 256), np.uint8)
        for _ in range(int(rng.integers(0, 20))):
            a = int(rng.integers(0, n)); b = min(n, a + int(rng.integers(1, 5000)))
            x[a:b] = rng.integers(0, 256, b - a)
    elif kind == 3:
        x = rng.integers(0, 256, n).astype(np.uint8)
    else:                                # a few symbols only
        x = rng.choice(rng.integers(0, 256, int(rng.integers(1, 6))), n).astype(np.uint8)
    mode = [0, 2, 3, 0, "d1", "d2", "d3", "a4"][int(rng.integers(0, 8))]
    return n, C, x, mode


def test_split_random_cases_match_oracle():
    """60 seeded random cases (sizes 1..2 Mi, C 256..16384, skewed, uniform,
    run-heavy and few-symbol data, several layouts): the split decoder
    returns the oracle stream's input."""
    rng = np.random.default_rng(2024)
    for case in range(60):
        n, C, x, mode = _random_case(rng)
        h = oracle.histogram(x)
        if mode == "a4":
            ot = oracle.build_table_general(h, 256, 4, 2, 4)
        elif isinstance(mode, str):
            ot = oracle.build_table_general(h, 256, 8, 3, int(mode[1]))
        else:
            ot = oracle.build_table(h, mode)
        st, bits, index, total = oracle.encode(x, ot, C)
        assert st == 0
        err, out = gpu_decode(bits, total, index, C, table_from_oracle(ot), n, SPLIT)
        assert err == 0, (case, n, C, mode)
        assert np.array_equal(out, x), (case, n, C, mode)
