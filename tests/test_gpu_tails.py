"""The ends of a tensor, where the kernels take paths of their own, against
the oracle bit for bit.

* Encoder: the input's ragged last tile.  A tile holds 8192 symbols and a
  thread two runs of 16 of them, one in each half of the tile; the last
  tile's symbols past the end are empty codes.  Tails around a run (16),
  the half (4096) and the whole tile, after 0, 1 and 3 whole tiles, given
  table (qlc_encode) and built table (qlc_compress).
* Lane decoder: the last wave of 64 chunks (lanes past the last chunk, a
  short last chunk, a last chunk of fewer than 8 symbols, the stream's
  first chunk with no whole group of 8), each decoder, and a flipped bit in
  such a wave's last chunk (the status equals the oracle's)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2602_17849_amd import datagen, qlc

pytestmark = pytest.mark.gpu

from gpu_util import (DEV, assert_table_equal, gpu_decode, gpu_encode,  # noqa: E402
                      table_from_oracle, to_dev)

TILE = 8192
TILE_TAILS = [1, 15, 16, 17, 4095, 4096, 4097, 4096 + 16, 8191]


def _x(n, seed):
    m = ((n + 31) // 32) * 32
    return datagen.gaussian(max(m, 32), seed).numpy()[:n].copy()


@pytest.mark.parametrize("tiles", [0, 1, 3])
@pytest.mark.parametrize("tail", TILE_TAILS)
def test_encode_ragged_last_tile(tiles, tail):
    n = tiles * TILE + tail
    x = _x(n, seed=tail + tiles)
    ot = oracle.build_table(oracle.histogram(x), qlc.LAYOUT_SEARCH_QUAD)
    t = table_from_oracle(ot)
    for C in (256, 4096):
        st, obits, oindex, ototal = oracle.encode(x, ot, C)
        assert st == 0
        err, bits, nb, index, total = gpu_encode(to_dev(x), t, C)
        assert err == 0 and total == ototal, (n, C)
        assert np.array_equal(bits[:nb], obits), (n, C)
        assert np.array_equal(index, oindex), (n, C)
    c = qlc.compress(to_dev(x), mode=qlc.LAYOUT_SEARCH_QUAD, chunk_symbols=4096)
    torch.cuda.synchronize()
    assert_table_equal(c.table, ot)
    st, obits, oindex, ototal = oracle.encode(x, ot, 4096)
    assert c.total_bits() == ototal
    assert np.array_equal(c.bits[:c.nbytes()].cpu().numpy(), obits)


# (chunks in the last wave, symbols of the last chunk; C = 256): one or 63
# chunks, a full, a short and a group-less last chunk
WAVE_CASES = [(1, 256), (1, 3), (63, 256), (63, 200), (63, 5), (64 + 1, 8), (64 + 63, 255)]


def _decode_case(n, C, seed):
    x = _x(n, seed)
    ot = oracle.build_table(oracle.histogram(x), qlc.LAYOUT_SEARCH_QUAD)
    st, obits, oindex, ototal = oracle.encode(x, ot, C)
    assert st == 0
    return x, ot, obits, oindex, ototal


@pytest.mark.parametrize("last_wave,last_chunk", WAVE_CASES)
def test_lane_decoder_last_wave(last_wave, last_chunk):
    C = 256
    n = (last_wave - 1) * C + last_chunk
    x, ot, obits, oindex, ototal = _decode_case(n, C, seed=last_wave * 7 + last_chunk)
    t = table_from_oracle(ot)
    for dec in (qlc.DECODER_LANE, qlc.DECODER_SPLIT, None):
        err, out = gpu_decode(obits, ototal, oindex, C, t, n, decoder=dec)
        assert err == 0 and np.array_equal(out, x), (n, dec)


@pytest.mark.parametrize("n", [1, 2, 7, 8, 9, 15])
def test_first_chunk_without_a_whole_group(n):
    """A stream whose only chunk starts at bit 0 and holds fewer than 16
    symbols (none or one whole group of 8), at two chunk sizes."""
    for C in (256, 2048):
        x, ot, obits, oindex, ototal = _decode_case(n, C, seed=n)
        t = table_from_oracle(ot)
        for dec in (qlc.DECODER_LANE, qlc.DECODER_SPLIT):
            err, out = gpu_decode(obits, ototal, oindex, C, t, n, decoder=dec)
            assert err == 0 and np.array_equal(out, x), (n, C, dec)


@pytest.mark.parametrize("last_wave,last_chunk", [(63, 200), (1, 3), (64 + 1, 8)])
def test_flipped_bit_in_the_last_wave(last_wave, last_chunk):
    """Bits flipped inside the last chunk of a partial wave: each decoder's
    status is the oracle's, and where the oracle decodes the stream, so do
    they, to the same bytes."""
    C = 256
    n = (last_wave - 1) * C + last_chunk
    x, ot, obits, oindex, ototal = _decode_case(n, C, seed=99 + last_chunk)
    t = table_from_oracle(ot)
    start = int(oindex[-1])
    rng = np.random.default_rng(last_wave + last_chunk)
    for bit in rng.integers(start, ototal, 6):
        b = obits.copy()
        b[bit >> 3] ^= np.uint8(0x80 >> (bit & 7))
        ost, oout = oracle.decode(b, ototal, oindex, C, ot, n)
        for dec in (qlc.DECODER_LANE, qlc.DECODER_SPLIT):
            err, out = gpu_decode(b, ototal, oindex, C, t, n, decoder=dec)
            assert err == ost, (n, int(bit), dec)
            if ost == 0:
                assert np.array_equal(out, oout), (n, int(bit), dec)
