"""Regression tests for two latent bugs of the codec paths, each run on the
fixed code and compared with the oracle bit for bit.

* Encode epoch wrap: the single-tensor encoder publishes each segment's bit
  count tagged with a 22-bit launch epoch.  Before the fix the words were
  never cleared, so a large encode running under the same epoch as an
  earlier large encode on the same workspace (2^22 launches later, or after
  the epoch is set back from the host as here) could take a stale count for
  a predecessor's and write a wrong stream with no error.
* Server reservation: a server built with the fixed widths of Table 1 or
  Table 2 reserved only n + 16 bytes of bitstream per compress request,
  although those layouts spend up to 9.6 bits per symbol on incompressible
  bytes; every such request failed with a capacity error.
"""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2602_17849_amd import datagen, qlc

pytestmark = pytest.mark.gpu

from gpu_util import DEV, assert_table_equal, table_from_oracle, to_dev  # noqa: E402

EPOCH_OFFSET = 12   # byte offset of the encoder's launch epoch in the workspace header
EPOCH_MASK = (1 << 22) - 1


def _epoch(ws):
    torch.cuda.synchronize()
    return int(ws[EPOCH_OFFSET:EPOCH_OFFSET + 4].view(torch.int32).item())


def _set_epoch(ws, v):
    ws[EPOCH_OFFSET:EPOCH_OFFSET + 4].copy_(
        torch.tensor([v], dtype=torch.int32, device=DEV).view(torch.uint8))
    torch.cuda.synchronize()


def _encode(x_dev, t_dev, C, ws):
    n = x_dev.numel()
    cap = qlc.qlc_encode_bound_bytes(n)
    bits = torch.zeros(cap, dtype=torch.uint8, device=DEV)
    index = torch.full((max(qlc.qlc_chunk_count(n, C), 1),), -1, dtype=torch.int64, device=DEV)
    total = torch.full((1,), -1, dtype=torch.int64, device=DEV)
    err = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    qlc.qlc_encode(x_dev, t_dev, C, bits, index, total, err, ws)
    torch.cuda.synchronize()
    tb = int(total.item())
    return (int(err.item()), tb, bits[:4 * ((tb + 31) // 32)].cpu().numpy(),
            index[:qlc.qlc_chunk_count(n, C)].cpu().numpy().astype(np.uint64))


@pytest.mark.parametrize("fused", [False, True])
def test_encode_after_epoch_wrap_matches_oracle(fused):
    """Large encode, then the epoch set so that one small encode brings it
    back to the large call's value, then a large encode of other data under
    that same epoch: bit-exact with the oracle."""
    n_large, n_small, C = 1 << 24, 10_000, 4096
    x1 = datagen.laplace_outlier_rows(512, n_large // 512, seed=41).reshape(-1).numpy()
    x2 = datagen.uniform_bytes(n_large, seed=42).numpy()
    xs = datagen.gaussian(n_small + 16, seed=43).numpy()[:n_small]
    ws = qlc.new_workspace(n_large, C)
    ot1 = oracle.build_table(oracle.histogram(x1), oracle.MODE_PAPER_T1)
    t1 = table_from_oracle(ot1)

    e0 = _epoch(ws)
    if fused:
        c = qlc.compress(to_dev(x1), qlc.LAYOUT_PAPER_T1, C, ws=ws)
        torch.cuda.synchronize()
        assert int(c.err.item()) == 0
    else:
        assert _encode(to_dev(x1), t1, C, ws)[0] == 0
    assert _epoch(ws) == (e0 + 1) & EPOCH_MASK
    # the small encode runs under epoch e0 - 1 and leaves e0 behind
    _set_epoch(ws, (e0 - 1) & EPOCH_MASK)
    assert _encode(to_dev(xs), t1, C, ws)[0] == 0
    assert _epoch(ws) == e0

    ot2 = oracle.build_table(oracle.histogram(x2), oracle.MODE_PAPER_T2)
    if fused:
        tdev = qlc.new_table(DEV)
        cap = qlc.qlc_encode_bound_bytes(n_large)
        bits = torch.zeros(cap, dtype=torch.uint8, device=DEV)
        index = torch.zeros(qlc.qlc_chunk_count(n_large, C), dtype=torch.int64, device=DEV)
        total = torch.zeros(1, dtype=torch.int64, device=DEV)
        err = torch.full((1,), -1, dtype=torch.int32, device=DEV)
        qlc.qlc_compress(to_dev(x2), qlc.LAYOUT_PAPER_T2, tdev, C, bits, index, total, err, ws)
        torch.cuda.synchronize()
        assert_table_equal(tdev, ot2)
        tb = int(total.item())
        got = (int(err.item()), tb, bits[:4 * ((tb + 31) // 32)].cpu().numpy(),
               index.cpu().numpy().astype(np.uint64))
    else:
        got = _encode(to_dev(x2), table_from_oracle(ot2), C, ws)
    st, obits, oindex, ototal = oracle.encode(x2, ot2, C)
    assert st == 0
    assert got[0] == 0 and got[1] == ototal
    assert np.array_equal(got[3], oindex)
    assert np.array_equal(got[2], obits)


@pytest.mark.parametrize("mode", [qlc.LAYOUT_PAPER_T1, qlc.LAYOUT_PAPER_T2])
def test_server_paper_mode_incompressible_bytes(mode):
    """A server with a fixed printed layout compresses uniform bytes (9.6
    bits per symbol under Table 1 or 2) and returns the oracle's stream."""
    C = 1024
    xs = [datagen.uniform_bytes(n, seed=50 + i).numpy() for i, n in
          enumerate([1 << 20, 100_003, 4096])]
    xd = [to_dev(x) for x in xs]        # inputs stay alive until their requests complete
    torch.cuda.synchronize()
    with qlc.Server(64 << 20, chunk_symbols=C, layout_mode=mode) as srv:
        ids = {srv.submit_compress(x): i for i, x in enumerate(xd)}
        got = {}
        t_end = time.time() + 60
        while len(got) < len(ids):
            assert time.time() < t_end, "serving loop did not finish"
            for r in srv.poll(16, 20000):
                i = ids[r.id]
                nb = 4 * ((r.total_bits + 31) // 32)
                k = qlc.qlc_chunk_count(r.n, C)
                got[i] = (r.status, r.total_bits, qlc.device_copy(r.bits, nb).cpu().numpy(),
                          qlc.device_copy(r.chunk_index, 8 * k).cpu().numpy().view(np.uint64),
                          qlc.device_copy(r.table, qlc.TABLE_BYTES))
                torch.cuda.synchronize()
                srv.release(r.id)
    for i, x in enumerate(xs):
        status, tb, bits, index, table = got[i]
        ot = oracle.build_table(oracle.histogram(x), mode)
        st, obits, oindex, ototal = oracle.encode(x, ot, C)
        assert st == 0 and ototal > 8 * x.size          # the layout expands these bytes
        assert status == 0 and tb == ototal
        assert_table_equal(table, ot)
        assert np.array_equal(index, oindex)
        assert np.array_equal(bits, obits)


_FALLBACK_CHILD = r"""
import sys
import numpy as np, torch
sys.path.insert(0, sys.argv[1])
import oracle
from paper_2602_17849_amd import datagen, qlc
C = 2048
for i, n in enumerate([9 * (1 << 20) + 77, (3 << 20) + 5, 262144, 100003]):
    x = datagen.laplace_outlier_rows(1, (n + 31) // 32 * 32, 40 + i)[:n].contiguous()
    o = qlc.compress(x.to("cuda"), chunk_symbols=C)
    torch.cuda.synchronize()
    xn = x.numpy()
    ot = oracle.build_table(oracle.histogram(xn), qlc.LAYOUT_SEARCH_QUAD)
    st, obits, oindex, ototal = oracle.encode(xn, ot, C)
    assert int(o.err.item()) == 0 and o.total_bits() == ototal, n
    assert np.array_equal(o.bits[:o.nbytes()].cpu().numpy(), obits), n
    assert np.array_equal(o.index[:qlc.qlc_chunk_count(n, C)].cpu().numpy().astype(np.uint64),
                          oindex), n
print("fallback ok")
"""


def test_encode_predecessor_counts_computed_when_not_yet_published():
    """With no polls allowed (QLC_ENCODE_SPIN_POLLS=0, read once per
    process, hence a child process), every predecessor bit count that is not
    yet published when a workgroup looks is computed by that workgroup from
    the predecessor's histogram: the streams and indexes still equal the
    oracle's."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, QLC_ENCODE_SPIN_POLLS="0")
    r = subprocess.run([sys.executable, "-c", _FALLBACK_CHILD, root], env=env, cwd=root,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0 and "fallback ok" in r.stdout, r.stdout + r.stderr
