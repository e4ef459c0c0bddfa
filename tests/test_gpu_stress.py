"""Stress at 4 GiB: three 4,294,967,296-byte buffers through the batched
form with C = 4096 — uniform random bytes (incompressible: must round-trip
and report its expansion), 90 % zeros (extreme skew), and OCP-style e4m3
whose NaN encodings never occur.  Full-size parity against the oracle:
histogram, table and total bits exactly; the bitstream and index on sampled
chunks, each re-encoded by the oracle on its own; the round trip on every
byte."""
import numpy as np
import pytest
import torch

import oracle
from paper_2602_17849_amd import datagen, qlc

pytestmark = pytest.mark.gpu

DEV = "cuda"
N = 1 << 32
C = 4096


def _stream_bits(b, i, start_bit, nbits):
    """Bits [start_bit, start_bit + nbits) of job i's stream, as 0/1."""
    lo = start_bit >> 3
    hi = (start_bit + nbits + 7) >> 3
    raw = b.bits[b.bits_off[i] + lo:b.bits_off[i] + hi].cpu().numpy()
    bits = np.unpackbits(raw)
    off = start_bit - 8 * lo
    return bits[off:off + nbits]


def _check_sampled_chunks(b, i, xh, ot, index, total):
    nchunks = (N + C - 1) // C
    rng = np.random.default_rng(7)
    for j in [0, 1, nchunks // 2, nchunks - 2, nchunks - 1] + list(rng.integers(0, nchunks, 6)):
        j = int(j)
        xc = xh[j * C:(j + 1) * C]
        st, obits, _, ototal = oracle.encode(xc, ot, C)
        assert st == 0
        end = int(index[j + 1]) if j + 1 < nchunks else total
        assert end - int(index[j]) == ototal, j
        got = _stream_bits(b, i, int(index[j]), ototal)
        assert np.array_equal(got, np.unpackbits(obits)[:ototal]), j


@pytest.mark.parametrize("kind", ["uniform", "zeros90", "ocp_gaussian"])
def test_stress_4gib(kind):
    x = datagen.stress_buffer(kind, N, device=DEV)
    b = qlc.Batch([N], chunk_symbols=C, device=DEV, inp=x)
    ws = b.workspace()
    b.encode(ws, qlc.LAYOUT_SEARCH_QUAD)
    b.decode(ws)
    torch.cuda.synchronize()
    assert int(b.err[0].item()) == 0
    assert torch.equal(b.output(0), x), "round trip"
    total = int(b.total[0].item())

    xh = x.cpu().numpy()
    h = oracle.histogram(xh)
    if kind == "ocp_gaussian":
        assert h[0x7F] == 0 and h[0xFF] == 0
    ot = oracle.build_table(h, oracle.MODE_SEARCH_QUAD)
    t = qlc.parse_table(b.table(0))
    assert list(t["width"]) == list(ot.width)
    assert np.array_equal(t["rank_to_sym"], ot.rank_to_sym)
    assert total == ot.cost_bits                       # stream length = sum h * len
    if kind == "uniform":
        assert list(ot.width) == [5] * 8 and total == 8 * N   # no expansion under SEARCH
    index = b.chunk_index(0).cpu().numpy()
    _check_sampled_chunks(b, 0, xh, ot, index, total)

    # the split decoder on the same stream: bit offsets past 2^32, 2^18
    # workgroups (under SEARCH_QUAD the uniform stream's codes all have one
    # length, so its guessed starts are exact; the others need corrections)
    b.out.zero_()
    derr = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    qlc.qlc_decode_ex(b.bitstream(0), b.total[0:1], b.chunk_index(0), C, b.table(0), N, 8,
                      qlc.DECODER_SPLIT, b.output(0), derr, qlc.new_workspace(0, C, DEV))
    torch.cuda.synchronize()
    assert int(derr.item()) == 0
    assert torch.equal(b.output(0), x), "split decoder round trip"

    if kind == "zeros90":
        # the single-tensor path on the same buffer: 4096 segments, more
        # encode workgroups than the device holds at once, so later ones
        # start as earlier ones finish; the stream equals the batched one
        o = qlc.compress(x, chunk_symbols=C)
        torch.cuda.synchronize()
        assert int(o.err.item()) == 0 and o.total_bits() == total
        nb = o.nbytes()
        assert torch.equal(o.bits[:nb], b.bits[b.bits_off[0]:b.bits_off[0] + nb])
        assert torch.equal(o.index[:(N + C - 1) // C], b.chunk_index(0))
        del o

    if kind == "uniform":
        # Table 1's layout expands incompressible data (8 -> ~9.59 bits)
        del b
        torch.cuda.empty_cache()
        b2 = qlc.Batch([N], chunk_symbols=C, device=DEV, capacity="bound", inp=x)
        ws2 = b2.workspace()
        b2.encode(ws2, qlc.LAYOUT_PAPER_T1)
        b2.decode(ws2)
        torch.cuda.synchronize()
        assert int(b2.err[0].item()) == 0
        assert torch.equal(b2.output(0), x)
        ot1 = oracle.build_table(h, oracle.MODE_PAPER_T1)
        total1 = int(b2.total[0].item())
        assert total1 == ot1.cost_bits
        assert 0.19 < total1 / (8.0 * N) - 1.0 < 0.21
        _check_sampled_chunks(b2, 0, xh, ot1, b2.chunk_index(0).cpu().numpy(), total1)
