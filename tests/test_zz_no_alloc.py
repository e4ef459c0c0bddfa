"""The allocation-free compress (qlc_compress_noalloc), called through the C
ABI, against qlc_compress with a caller workspace: table, bitstream, chunk
index, total bits and status identical, on calls in a row whose second input
is smaller, and a size above the limit refused before any launch."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2602_17849_amd import datagen, qlc

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _outputs(n, C):
    cap = qlc.qlc_encode_bound_bytes(n)
    return (qlc.new_table(DEV), torch.full((max(cap, 16),), 0x77, dtype=torch.uint8, device=DEV),
            torch.full((max(qlc.qlc_chunk_count(n, C), 1),), -1, dtype=torch.int64, device=DEV),
            torch.full((1,), -1, dtype=torch.int64, device=DEV),
            torch.full((1,), -1, dtype=torch.int32, device=DEV), cap)


def _call_noalloc(x, mode, C):
    """qlc_compress_noalloc through ctypes (plain pointers and sizes)."""
    n = x.numel()
    table, bits, index, total, err, cap = _outputs(n, C)
    L = qlc.lib()
    st = L.qlc_compress_noalloc(ctypes.c_void_p(x.data_ptr()), n, mode,
                                ctypes.c_void_p(table.data_ptr()), C,
                                ctypes.c_void_p(bits.data_ptr()), cap,
                                ctypes.c_void_p(index.data_ptr()),
                                ctypes.c_void_p(total.data_ptr()),
                                ctypes.c_void_p(err.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == qlc.QLC_OK
    return table, bits, index, total, err


def _call_with_workspace(x, mode, C):
    n = x.numel()
    table, bits, index, total, err, cap = _outputs(n, C)
    ws = qlc.new_workspace(n, C, DEV)
    qlc.qlc_compress(x, mode, table, C, bits[:cap] if cap else bits[:0], index, total, err, ws)
    return table, bits, index, total, err


def _same(a, b):
    torch.cuda.synchronize()
    ta, bitsa, ia, tota, ea = a
    tb, bitsb, ib, totb, eb = b
    assert int(ea.item()) == 0 and int(eb.item()) == 0
    assert torch.equal(ta, tb)
    assert int(tota.item()) == int(totb.item())
    nb = 4 * ((int(tota.item()) + 31) // 32)
    assert torch.equal(bitsa[:nb], bitsb[:nb])
    assert torch.equal(ia, ib)


@pytest.mark.parametrize("mode,C", [(qlc.LAYOUT_SEARCH_QUAD, 2048), (qlc.LAYOUT_PAPER_T1, 256)])
def test_noalloc_matches_workspace_call_twice(mode, C):
    big = datagen.laplace_outlier_rows(1024, 8192, seed=61).reshape(-1).to(DEV)      # 8 Mi
    small = datagen.uniform_bytes(100_003, seed=62).to(DEV)
    for x in (big, small):
        _same(_call_noalloc(x, mode, C), _call_with_workspace(x, mode, C))
    # and once more after the smaller call, in the other order of sizes
    _same(_call_noalloc(big, mode, C), _call_with_workspace(big, mode, C))


def test_noalloc_refuses_sizes_above_the_limit():
    L = qlc.lib()
    p = ctypes.c_void_p(1 << 20)
    st = L.qlc_compress_noalloc(p, (1 << 30) + 1, 0, p, 4096, p, 1 << 40, p, p, p, None)
    assert st == qlc.QLC_ERR_INVALID_ARGUMENT
