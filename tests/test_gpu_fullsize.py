"""Parity at the benchmarks' full sizes and launch configurations: the 256 MiB
Laplace e4m3 tensor (8192 x 32768, seed 1), per-tensor SEARCH_QUAD table,
chunks of 2048 symbols, compressed by qlc_compress and decoded by qlc_decode
exactly as bench.py times them.  The oracle is too slow for the whole
stream, so it checks what it can at this size: the table (from the oracle's
own histogram of all 268 M bytes), total bits against the closed form
sum h * len, every index step against the chunk's summed code lengths, the
stream bits of sampled chunks (first, last and 62 random ones) against the
oracle's encoding of those chunks, and the full round trip.  Also the
batched form on the whole 1152-shard workload, with sampled shards against
the oracle."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DEV, assert_table_equal
from paper_2602_17849_amd import datagen, qlc

pytestmark = pytest.mark.gpu

C = 2048


def _bits(stream: np.ndarray, start: int, count: int) -> np.ndarray:
    """Bits [start, start + count) of an MSB-first byte stream."""
    b0, b1 = start // 8, (start + count + 7) // 8
    u = np.unpackbits(stream[b0:b1])
    return u[start - 8 * b0:start - 8 * b0 + count]


@pytest.fixture(scope="module")
def compressed():
    x = datagen.single_tensor_laplace(device=DEV)
    n = x.numel()
    obj = qlc.compress(x, mode=qlc.LAYOUT_SEARCH_QUAD, chunk_symbols=C)
    torch.cuda.synchronize()
    assert int(obj.err.item()) == 0
    return x, obj


def test_fullsize_table_and_totals(compressed):
    x, obj = compressed
    xh = x.cpu().numpy()
    h = oracle.histogram(xh)
    ot = oracle.build_table(h, qlc.LAYOUT_SEARCH_QUAD)
    assert_table_equal(obj.table, ot)
    total = obj.total_bits()
    assert total == int((h.astype(np.uint64) * ot.len.astype(np.uint64)).sum())
    # every index step is the sum of the chunk's code lengths
    k = qlc.qlc_chunk_count(x.numel(), C)
    index = obj.index[:k].cpu().numpy().astype(np.int64)
    lens = ot.len.astype(np.uint8)[xh]
    per_chunk = lens.reshape(-1, C).sum(axis=1, dtype=np.int64)
    assert index[0] == 0
    assert np.array_equal(np.diff(index), per_chunk[:-1])
    assert index[-1] + per_chunk[-1] == total


def test_fullsize_sampled_chunks_match_oracle(compressed):
    x, obj = compressed
    xh = x.cpu().numpy()
    ot = oracle.build_table(oracle.histogram(xh), qlc.LAYOUT_SEARCH_QUAD)
    k = qlc.qlc_chunk_count(x.numel(), C)
    index = obj.index[:k].cpu().numpy().astype(np.int64)
    total = obj.total_bits()
    stream = obj.bits[:obj.nbytes()].cpu().numpy()
    rng = np.random.default_rng(17)
    chunks = [0, k - 1] + sorted(rng.choice(np.arange(1, k - 1), 62, replace=False).tolist())
    for j in chunks:
        sym = xh[j * C:(j + 1) * C]
        st, obits, oindex, ototal = oracle.encode(sym, ot, C)
        assert st == 0
        end = index[j + 1] if j + 1 < k else total
        assert end - index[j] == ototal, j
        assert np.array_equal(_bits(stream, int(index[j]), ototal), _bits(obits, 0, ototal)), j
    # the stream's padding after the last code is zero
    tail = _bits(stream, total, 8 * obj.nbytes() - total)
    assert not tail.any()


@pytest.mark.parametrize("decoder", [qlc.DECODER_AUTO, qlc.DECODER_LANE, qlc.DECODER_SPLIT])
def test_fullsize_round_trip(compressed, decoder):
    x, obj = compressed
    out, err = qlc.decompress(obj, decoder=decoder)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    assert torch.equal(out, x)


def test_fullsize_batched_1152_shards():
    """The batched form on the full 1152-shard workload (10.25 GiB) at the
    benchmark's tuned setting: no job errors, every shard round-trips, and
    ten sampled shards (smallest, largest, eight random) have the oracle's
    table, total, bitstream and chunk index."""
    sizes = datagen.shard_sizes()
    b = qlc.Batch(sizes, chunk_symbols=C, device=DEV)
    for i, n in enumerate(sizes):
        b.input(i).copy_(datagen.shard(i, n, device=DEV))
    tuning = (19, 0, 0, 0)
    ws = b.workspace(tuning)
    b.encode(ws, qlc.LAYOUT_SEARCH_QUAD, tuning)
    b.decode(ws, tuning)
    torch.cuda.synchronize()
    assert not b.err.any().item()
    assert torch.equal(b.out, b.inp)
    rng = np.random.default_rng(23)
    picks = {int(np.argmin(sizes)), int(np.argmax(sizes))}
    picks |= set(rng.choice(len(sizes), 8, replace=False).tolist())
    for i in sorted(picks):
        xh = b.input(i).cpu().numpy()
        ot = oracle.build_table(oracle.histogram(xh), qlc.LAYOUT_SEARCH_QUAD)
        assert_table_equal(b.table(i), ot)
        st, obits, oindex, ototal = oracle.encode(xh, ot, C)
        total = int(b.total[i].item())
        assert st == 0 and total == ototal, i
        nb = 4 * ((total + 31) // 32)
        assert np.array_equal(b.bitstream(i, nb).cpu().numpy(), obits), i
        assert np.array_equal(b.chunk_index(i).cpu().numpy().astype(np.uint64),
                              oindex.astype(np.uint64)), i
    del b, ws
    torch.cuda.empty_cache()
