"""Helpers of the GPU parity tests: run libqlc through its binding and the
oracle on the same bytes (inputs from datagen; expected values from the
oracle only)."""
import numpy as np
import torch

import oracle
from paper_2602_17849_amd import qlc

DEV = "cuda"


def to_dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def gpu_table(x_dev, mode):
    ws = qlc.new_workspace(x_dev.numel())
    t = qlc.new_table()
    qlc.qlc_build_table(x_dev, mode, t, ws)
    torch.cuda.synchronize()
    return t


def table_from_oracle(ot) -> torch.Tensor:
    """Device table holding the oracle table's layout (width + rank order);
    a table of fewer areas or symbols is padded as the serialized form
    requires (widths 0xFF, ranks beyond M in symbol order)."""
    w = list(ot.width.astype(np.uint8)) + [0xFF] * (8 - len(ot.width))
    r = list(ot.rank_to_sym.astype(np.uint8)) + list(range(len(ot.rank_to_sym), 256))
    blob = bytes(w) + bytes(r)
    raw = qlc.qlc_table_deserialize(blob)
    return torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(DEV)


def assert_table_equal(t_dev, ot, check_cost=True):
    t = qlc.parse_table(t_dev)
    assert list(t["width"]) == list(ot.width)
    assert list(t["first"]) == list(ot.first)
    assert list(t["count"]) == list(ot.count)
    assert list(t["offset"]) == list(ot.offset)
    assert np.array_equal(t["rank_to_sym"], ot.rank_to_sym)
    assert np.array_equal(t["sym_to_rank"], ot.sym_to_rank)
    assert np.array_equal(t["enc"] >> 11, ot.len)
    assert np.array_equal(t["enc"] & 0x7FF, ot.code)
    if check_cost:
        assert t["cost_bits"] == ot.cost_bits


def gpu_encode(x_dev, t_dev, C, cap=None):
    n = x_dev.numel()
    ws = qlc.new_workspace(n, C)
    cap = qlc.qlc_encode_bound_bytes(n) if cap is None else cap
    bits = torch.zeros(max(cap, 16), dtype=torch.uint8, device=DEV)
    index = torch.full((max(qlc.qlc_chunk_count(n, C), 1),), -1, dtype=torch.int64, device=DEV)
    total = torch.full((1,), -1, dtype=torch.int64, device=DEV)
    err = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    qlc.qlc_encode(x_dev, t_dev, C, bits[:cap] if cap else bits[:0], index, total, err, ws)
    torch.cuda.synchronize()
    tb = int(total.item())
    nbytes = 4 * ((tb + 31) // 32)
    return (int(err.item()), bits.cpu().numpy(), nbytes,
            index[:qlc.qlc_chunk_count(n, C)].cpu().numpy().astype(np.uint64), tb)


def gpu_decode(bits_np, total, index_np, C, t_dev, n, decoder=None, symbol_bits=8):
    """Decode through qlc_decode (decoder None) or qlc_decode_ex with the
    given decoder; returns (err, output bytes)."""
    bits = to_dev(np.concatenate([bits_np, np.zeros(16, np.uint8)]))
    tot = torch.tensor([total], dtype=torch.int64, device=DEV)
    idx = to_dev(index_np.astype(np.int64)) if index_np.size else torch.zeros(1, dtype=torch.int64, device=DEV)
    nb = qlc.packed_bytes(n, symbol_bits)
    out = torch.full((max(nb, 16),), 0xAA, dtype=torch.uint8, device=DEV)
    err = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    ws = qlc.new_workspace(0, C)
    if decoder is None and symbol_bits == 8:
        qlc.qlc_decode(bits, tot, idx, C, t_dev, n, out, err, ws)
    else:
        qlc.qlc_decode_ex(bits, tot, idx, C, t_dev, n, symbol_bits,
                          qlc.DECODER_AUTO if decoder is None else decoder, out, err, ws)
    torch.cuda.synchronize()
    return int(err.item()), out[:nb].cpu().numpy()
