"""Native small alphabets: 4-bit codes packed two per byte (16 symbols,
e.g. e2m1) and 6-bit codes packed four per three bytes (64 symbols, e.g.
e3m2), coded with their own tables of 2, 4 or 8 areas.  Histogram, table,
bitstream, chunk index and total bits against the oracle's general table
(build_table_general with M = 16 or 64) on the unpacked codes; the decode
restores the packed bytes (pad bits zero); plain and batched; a table of
another alphabet is refused."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2602_17849_amd import datagen, qlc

pytestmark = pytest.mark.gpu

DEV = "cuda"

# (mode, M, areas, area-code bits, symbol bits)
MODES = [(qlc.LAYOUT_M16_AREAS2, 16, 2, 1, 4), (qlc.LAYOUT_M16_AREAS4, 16, 4, 2, 4),
         (qlc.LAYOUT_M64_AREAS4, 64, 4, 2, 6), (qlc.LAYOUT_M64_AREAS8, 64, 8, 3, 6)]
MODE_IDS = ["M16A2", "M16A4", "M64A4", "M64A8"]
SIZES = [0, 1, 7, 15, 17, 255, 4097, 8192, 3 * 8192 + 1234, 100003, 262144 + 77]


def _codes(n, bits, kind, seed):
    rng = np.random.default_rng(seed * 101 + n)
    if kind == "float":
        mant, exp = (1, 2) if bits == 4 else (2, 3)
        return datagen.small_float_codes(n, mant, exp, seed)
    if kind == "uniform":
        return rng.integers(0, 1 << bits, n).astype(np.uint8)
    if kind == "skewed":
        x = rng.integers(0, 1 << bits, n).astype(np.uint8)
        x[rng.random(n) < 0.9] = 3
        return x
    return np.full(n, (1 << bits) - 2, np.uint8)           # constant


KINDS = ["float", "uniform", "skewed", "constant"]


def _packed_dev(codes, bits):
    p = datagen.pack_symbols(codes, bits)
    buf = torch.zeros(max(p.size, 16) + 16, dtype=torch.uint8)
    buf[:p.size] = torch.from_numpy(p)
    return buf.to(DEV), p


def _oracle_table(codes, M, A, p):
    h = oracle.histogram(codes)
    assert not h[M:].any()
    return oracle.build_table_general(h[:M], M, A, p, A)


def _assert_table(t_dev, ot, M, A):
    t = qlc.parse_table(t_dev)
    assert list(t["width"][:A]) == list(ot.width)
    assert all(w == 0xFF for w in t["width"][A:])
    assert list(t["first"][:A]) == list(ot.first)
    assert list(t["count"][:A]) == list(ot.count)
    assert list(t["offset"][:A]) == list(ot.offset)
    assert np.array_equal(t["rank_to_sym"][:M], ot.rank_to_sym)
    assert np.array_equal(t["sym_to_rank"][:M], ot.sym_to_rank)
    assert np.array_equal(t["enc"][:M] >> 11, ot.len)
    assert np.array_equal(t["enc"][:M] & 0x7FF, ot.code)
    assert not t["enc"][M:].any()
    assert t["cost_bits"] == ot.cost_bits


def _outputs(n, C):
    cap = qlc.qlc_encode_bound_bytes(n)
    return (qlc.new_table(DEV), torch.zeros(max(cap, 16), dtype=torch.uint8, device=DEV),
            torch.full((max(qlc.qlc_chunk_count(n, C), 1),), -1, dtype=torch.int64, device=DEV),
            torch.full((1,), -1, dtype=torch.int64, device=DEV),
            torch.full((1,), -1, dtype=torch.int32, device=DEV), cap)


@pytest.mark.parametrize("bits", [4, 6])
@pytest.mark.parametrize("n", SIZES)
def test_histogram_sym(bits, n):
    for kind in KINDS:
        codes = _codes(n, bits, kind, 1)
        xd, _ = _packed_dev(codes, bits)
        h = torch.zeros(256, dtype=torch.int64, device=DEV)
        ws = qlc.new_workspace(n)
        qlc.qlc_histogram_sym(xd, n, bits, h, ws)
        assert np.array_equal(h.cpu().numpy().astype(np.uint64), oracle.histogram(codes)), kind


@pytest.mark.parametrize("C", [256, 4096])
@pytest.mark.parametrize("mode,M,A,p,bits", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("n", SIZES)
def test_compress_decode_sym(n, mode, M, A, p, bits, C):
    for kind in KINDS:
        codes = _codes(n, bits, kind, 2)
        ot = _oracle_table(codes, M, A, p)
        xd, packed = _packed_dev(codes, bits)
        table, bstream, index, total, err, cap = _outputs(n, C)
        ws = qlc.new_workspace(n, C)
        qlc.qlc_compress_sym(xd, n, bits, mode, table, C, bstream[:cap], index, total, err, ws)
        torch.cuda.synchronize()
        assert int(err.item()) == 0, kind
        _assert_table(table, ot, M, A)
        st, obits, oindex, ototal = oracle.encode(codes, ot, C)
        tb = int(total.item())
        assert st == 0 and tb == ototal, kind
        assert np.array_equal(bstream[:obits.size].cpu().numpy(), obits), kind
        k = qlc.qlc_chunk_count(n, C)
        assert np.array_equal(index[:k].cpu().numpy().astype(np.uint64), oindex), kind
        # decode: the packed bytes come back, pad bits zero
        out = torch.full((max(packed.size, 16) + 16,), 0xAA, dtype=torch.uint8, device=DEV)
        derr = torch.full((1,), -1, dtype=torch.int32, device=DEV)
        qlc.qlc_decode_sym(bstream, total, index, C, table, n, bits, out, derr, ws)
        torch.cuda.synchronize()
        assert int(derr.item()) == 0, kind
        o = out.cpu().numpy()
        assert np.array_equal(o[:packed.size], packed), kind
        assert (o[packed.size:] == 0xAA).all(), kind               # nothing written past the end
        # the same table given back: identical stream
        b2 = torch.zeros_like(bstream)
        i2 = torch.full_like(index, -1)
        t2 = torch.full_like(total, -1)
        e2 = torch.full_like(err, -1)
        qlc.qlc_encode_sym(xd, n, bits, table, C, b2[:cap], i2, t2, e2, ws)
        torch.cuda.synchronize()
        assert int(e2.item()) == 0 and int(t2.item()) == tb
        assert torch.equal(b2, bstream) and torch.equal(i2[:k], index[:k])


@pytest.mark.parametrize("mode,M,A,p,bits", MODES, ids=MODE_IDS)
def test_decode_oracle_streams_sym(mode, M, A, p, bits):
    """Streams written by the oracle (from the oracle's table, handed over as
    the table the library built for the same histogram) decode to the codes."""
    n, C = 70001, 1024
    codes = _codes(n, bits, "float", 3)
    ot = _oracle_table(codes, M, A, p)
    st, obits, oindex, ototal = oracle.encode(codes, ot, C)
    xd, packed = _packed_dev(codes, bits)
    table = qlc.new_table(DEV)
    ws = qlc.new_workspace(n, C)
    qlc.qlc_build_table_sym(xd, n, bits, mode, table, ws)
    torch.cuda.synchronize()
    _assert_table(table, ot, M, A)
    b = torch.from_numpy(np.concatenate([obits, np.zeros(16, np.uint8)])).to(DEV)
    tot = torch.tensor([ototal], dtype=torch.int64, device=DEV)
    idx = torch.from_numpy(oindex.astype(np.int64)).to(DEV)
    out = torch.zeros(packed.size + 16, dtype=torch.uint8, device=DEV)
    err = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    qlc.qlc_decode_sym(b, tot, idx, C, table, n, bits, out, err, ws)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    assert np.array_equal(out[:packed.size].cpu().numpy(), packed)
    # a flipped bit is reported like the oracle reports it
    ob = obits.copy()
    ob[len(ob) // 3] ^= 0x10
    ost, _ = oracle.decode(ob, ototal, oindex, C, ot, n)
    b2 = torch.from_numpy(np.concatenate([ob, np.zeros(16, np.uint8)])).to(DEV)
    qlc.qlc_decode_sym(b2, tot, idx, C, table, n, bits, out, err, ws)
    torch.cuda.synchronize()
    assert int(err.item()) == ost


def test_table_of_another_alphabet_is_refused():
    n, C = 5000, 256
    codes = _codes(n, 4, "float", 4)
    xd, packed = _packed_dev(codes, 4)
    ws = qlc.new_workspace(n, C)
    t16 = qlc.new_table(DEV)
    qlc.qlc_build_table_sym(xd, n, 4, qlc.LAYOUT_M16_AREAS4, t16, ws)
    tb = qlc.new_table(DEV)
    qlc.qlc_build_table(xd[:packed.size], qlc.LAYOUT_SEARCH_QUAD, tb, ws)
    torch.cuda.synchronize()
    # encode: nibbles with a byte table, bytes with a nibble table
    for x, nn, bits, t in ((xd, n, 4, tb), (xd, packed.size, 8, t16)):
        _, bstream, index, total, err, cap = _outputs(nn, C)
        qlc.qlc_encode_sym(x, nn, bits, t, C, bstream[:cap], index, total, err, ws)
        torch.cuda.synchronize()
        assert int(err.item()) == qlc.QLC_ERR_INVALID_ARGUMENT
    # decode of a valid nibble stream with the byte table: refused
    table, bstream, index, total, err, cap = _outputs(n, C)
    qlc.qlc_compress_sym(xd, n, 4, qlc.LAYOUT_M16_AREAS4, table, C, bstream[:cap], index, total,
                         err, ws)
    out = torch.zeros(packed.size + 16, dtype=torch.uint8, device=DEV)
    derr = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    qlc.qlc_decode_sym(bstream, total, index, C, tb, n, 4, out, derr, ws)
    torch.cuda.synchronize()
    assert int(err.item()) == 0 and int(derr.item()) == qlc.QLC_ERR_INVALID_ARGUMENT
    # host-side checks: a mode of another alphabet, an unknown symbol width
    with pytest.raises(qlc.QLCError):
        qlc.qlc_compress_sym(xd, n, 4, qlc.LAYOUT_SEARCH_QUAD, table, C, bstream[:cap], index,
                             total, err, ws)
    with pytest.raises(qlc.QLCError):
        qlc.qlc_compress_sym(xd, n, 5, qlc.LAYOUT_M16_AREAS4, table, C, bstream[:cap], index,
                             total, err, ws)
    with pytest.raises(qlc.QLCError):
        qlc.qlc_compress(xd, qlc.LAYOUT_M64_AREAS4, table, C, bstream[:cap], index, total, err,
                         ws, n=n)


class _PackedBatch:
    """Device buffers and qlc_job records of packed small-symbol jobs."""

    def __init__(self, codes_list, bits, C):
        self.bits, self.C = bits, C
        self.codes = codes_list
        self.packed = [datagen.pack_symbols(c, bits) for c in codes_list]
        S = len(codes_list)
        self.inp = [torch.from_numpy(np.concatenate([p, np.zeros(32, np.uint8)])).to(DEV)
                    for p in self.packed]
        self.out = [torch.full((p.size + 32,), 0xAA, dtype=torch.uint8, device=DEV)
                    for p in self.packed]
        self.cap = [qlc.qlc_encode_bound_bytes(c.size) for c in codes_list]
        self.bstream = [torch.zeros(max(cp, 16), dtype=torch.uint8, device=DEV) for cp in self.cap]
        self.index = [torch.full((max(qlc.qlc_chunk_count(c.size, C), 1),), -1, dtype=torch.int64,
                                 device=DEV) for c in codes_list]
        self.tables = torch.zeros(S * qlc.TABLE_BYTES, dtype=torch.uint8, device=DEV)
        self.total = torch.full((S,), -1, dtype=torch.int64, device=DEV)
        self.err = torch.full((S,), -1, dtype=torch.int32, device=DEV)
        host = (qlc.Job * S)()
        for i, c in enumerate(codes_list):
            j = host[i]
            j.in_ = self.inp[i].data_ptr()
            j.out = self.out[i].data_ptr()
            j.n = c.size
            j.table = self.tables.data_ptr() + i * qlc.TABLE_BYTES
            j.bits = self.bstream[i].data_ptr()
            j.bits_capacity = self.cap[i]
            j.chunk_index = self.index[i].data_ptr()
            j.total_bits = self.total.data_ptr() + 8 * i
            j.err = self.err.data_ptr() + 4 * i
            j.build_table = 1
            j.reserved = 0
        self.jobs = torch.frombuffer(bytearray(host), dtype=torch.uint8).to(DEV)
        self.S = S

    def table(self, i):
        return self.tables[i * qlc.TABLE_BYTES:(i + 1) * qlc.TABLE_BYTES]


@pytest.mark.parametrize("tuning", [None, (13, 0, 0, 0), (14, 3, 5, 0),
                                    (0, 0, 0, qlc.DECODER_LANE), (0, 0, 0, qlc.DECODER_SPLIT)])
@pytest.mark.parametrize("mode,M,A,p,bits", MODES, ids=MODE_IDS)
def test_batched_sym(mode, M, A, p, bits, tuning):
    C = 1024
    sizes = [0, 1, 17, 8191, 8192, 65541, 300001, 4096, 1 << 20]
    codes = [_codes(n, bits, KINDS[i % 4], 5 + i) for i, n in enumerate(sizes)]
    b = _PackedBatch(codes, bits, C)
    ws = torch.zeros(max(qlc.qlc_batched_workspace_bytes(b.S, sum(sizes), C, tuning), 256),
                     dtype=torch.uint8, device=DEV)
    qlc.qlc_encode_batched_sym(b.jobs, b.S, bits, mode, C, ws, tuning)
    qlc.qlc_decode_batched_sym(b.jobs, b.S, bits, C, ws, tuning)
    torch.cuda.synchronize()
    for i, c in enumerate(codes):
        assert int(b.err[i].item()) == 0, i
        ot = _oracle_table(c, M, A, p)
        _assert_table(b.table(i), ot, M, A)
        st, obits, oindex, ototal = oracle.encode(c, ot, C)
        assert int(b.total[i].item()) == ototal, i
        assert np.array_equal(b.bstream[i][:obits.size].cpu().numpy(), obits), i
        k = qlc.qlc_chunk_count(c.size, C)
        assert np.array_equal(b.index[i][:k].cpu().numpy().astype(np.uint64), oindex), i
        o = b.out[i].cpu().numpy()
        assert np.array_equal(o[:b.packed[i].size], b.packed[i]), i
        assert (o[b.packed[i].size:] == 0xAA).all(), i
