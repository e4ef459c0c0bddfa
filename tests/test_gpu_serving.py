"""Serving form (qlc_server_*): admission against a device-memory budget and
continuous batching.  Each request's result must be the same alone and in a
mix (tolerance zero: the code is lossless), equal to the single-tensor entry
points, and the budget must hold at every moment."""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2602_17849_amd import datagen, qlc

pytestmark = pytest.mark.gpu

DEV = "cuda"
C = 1024
COMPRESS_SIZES = [0, 100, 4096, 65568, 300000, 1 << 20, 2_500_000, 8193]
DECOMPRESS_SIZES = [1, 5000, 262144, 1_000_003, 77777, 0]


def _bytes(n, seed):
    m = max(32, (n + 31) // 32 * 32)
    x = datagen.laplace_outlier_rows(1, m, seed) if seed % 2 else datagen.gaussian(m, seed)
    return x[:n].contiguous()


@pytest.fixture(scope="module")
def workload():
    comp = [_bytes(n, 100 + i).to(DEV) for i, n in enumerate(COMPRESS_SIZES)]
    dec_src = [_bytes(n, 200 + i) for i, n in enumerate(DECOMPRESS_SIZES)]
    objs = [qlc.compress(x.to(DEV), chunk_symbols=C) for x in dec_src]
    torch.cuda.synchronize()
    for o in objs:
        assert int(o.err.item()) == 0
    return comp, dec_src, objs


def _submit_all(srv, comp, objs, order):
    ids = {}
    for kind, i in order:
        if kind == "c":
            rid = srv.submit_compress(comp[i], user_tag=i)
        else:
            o = objs[i]
            rid = srv.submit_decompress(o.n, o.bits, o.index, o.total, o.table,
                                        user_tag=1000 + i)
        ids[rid] = (kind, i)
    return ids


def _collect(srv, ids, timeout_s=60.0):
    """Poll every submitted request; copy its outputs to the host; release.
    Returns {(kind, i): outputs} (the last one for a repeated request)."""
    got = {}
    seen = set()
    t_end = time.time() + timeout_s
    while len(seen) < len(ids):
        assert time.time() < t_end, "serving loop did not finish"
        for r in srv.poll(64, 20000):
            kind, i = ids[r.id]
            if kind == "c":
                nb = 4 * ((r.total_bits + 31) // 32)
                k = qlc.qlc_chunk_count(r.n, C)
                val = (r.status, r.total_bits, qlc.device_copy(r.bits, nb).cpu().numpy(),
                       qlc.device_copy(r.chunk_index, 8 * k).cpu().numpy(),
                       qlc.device_copy(r.table, qlc.TABLE_BYTES).cpu().numpy())
            else:
                val = (r.status, qlc.device_copy(r.out, r.n).cpu().numpy())
            torch.cuda.synchronize()
            got[(kind, i)] = val
            seen.add(r.id)
            assert r.submit_ns <= r.admit_ns <= r.complete_ns
            srv.release(r.id)
    return got


def _alone(comp, objs, order):
    out = {}
    with qlc.Server(64 << 20, chunk_symbols=C) as srv:
        for item in order:
            ids = _submit_all(srv, comp, objs, [item])
            out.update(_collect(srv, ids))
    return out


def _order():
    order = [("c", i) for i in range(len(COMPRESS_SIZES))] + \
            [("d", i) for i in range(len(DECOMPRESS_SIZES))]
    rng = np.random.default_rng(5)
    return [order[k] for k in rng.permutation(len(order))]


def test_alone_vs_mix_identical(workload):
    comp, dec_src, objs = workload
    order = _order()
    alone = _alone(comp, objs, order)
    # a budget that holds only a few requests at once, two ticks in flight,
    # at most three jobs per tick: requests queue and share ticks
    budget = 6 << 20
    with qlc.Server(budget, chunk_symbols=C, max_jobs_per_tick=3,
                    max_ticks_in_flight=2) as srv:
        ids = _submit_all(srv, comp, objs, order)
        mix = _collect(srv, ids)
        st = srv.stats()
        assert st.completed == len(order) and st.rejected == 0
        assert st.peak_bytes_in_use <= budget
        assert st.bytes_in_use == 0
        assert st.ticks >= 2
    assert alone.keys() == mix.keys()
    for k in alone:
        a, m = alone[k], mix[k]
        assert a[0] == 0 and m[0] == 0, k
        assert len(a) == len(m)
        for x, y in zip(a[1:], m[1:]):
            assert np.array_equal(np.asarray(x), np.asarray(y)), k
    # and both equal the single-tensor entry points / the original bytes
    for i, x in enumerate(comp):
        ref = qlc.compress(x, chunk_symbols=C)
        torch.cuda.synchronize()
        st, total, bits, index, table = mix[("c", i)]
        assert total == ref.total_bits()
        assert np.array_equal(bits, ref.bits[:ref.nbytes()].cpu().numpy())
        assert np.array_equal(index.view(np.int64),
                              ref.index[:qlc.qlc_chunk_count(x.numel(), C)].cpu().numpy())
        assert np.array_equal(table, ref.table.cpu().numpy())
    for i, x in enumerate(dec_src):
        assert np.array_equal(mix[("d", i)][1], x.numpy())


def test_many_requests_overlap(workload):
    """A burst of small requests shares ticks (continuous batching)."""
    comp, dec_src, objs = workload
    order = [("c", 3), ("d", 2)] * 40
    with qlc.Server(256 << 20, chunk_symbols=C, max_jobs_per_tick=16,
                    max_ticks_in_flight=4) as srv:
        ids = _submit_all(srv, comp, objs, order)
        got = _collect(srv, ids)
        st = srv.stats()
        assert st.completed == len(order)
        assert st.max_jobs_in_tick > 1
    assert all(v[0] == 0 for v in got.values())


@pytest.mark.parametrize("decoder", [qlc.DECODER_LANE, qlc.DECODER_SPLIT])
def test_decoders_of_the_decode_ticks(workload, decoder):
    """Decompress requests decoded by lane groups only or split units only
    return the original bytes."""
    comp, dec_src, objs = workload
    order = [("d", i) for i in range(len(dec_src))] * 2
    with qlc.Server(256 << 20, chunk_symbols=C, max_jobs_per_tick=8, decoder=decoder) as srv:
        ids = _submit_all(srv, comp, objs, order)
        got = _collect(srv, ids)
    for (kind, i), v in got.items():
        assert v[0] == 0 and np.array_equal(v[1], dec_src[i].numpy()), (kind, i)


def test_caller_table(workload):
    comp, _, _ = workload
    x = comp[5]
    xn = x.cpu().numpy()
    ot = oracle.build_table(oracle.histogram(xn), qlc.LAYOUT_PAPER_T1)
    blob = bytes(ot.width.astype(np.uint8)) + bytes(ot.rank_to_sym.astype(np.uint8))
    t = torch.frombuffer(bytearray(qlc.qlc_table_deserialize(blob)), dtype=torch.uint8).to(DEV)
    with qlc.Server(64 << 20, chunk_symbols=C) as srv:
        rid = srv.submit_compress(x, table=t)
        r = None
        while r is None:
            res = srv.poll(1, 100000)
            r = res[0] if res else None
        assert r.id == rid and r.status == 0 and r.table == t.data_ptr()
        st, obits, oindex, ototal = oracle.encode(xn, ot, C)
        assert r.total_bits == ototal
        assert np.array_equal(qlc.device_copy(r.bits, obits.size).cpu().numpy(), obits)
        srv.release(r.id)


def test_errors(workload):
    comp, dec_src, objs = workload
    with qlc.Server(2 << 20, chunk_symbols=C) as srv:
        with pytest.raises(qlc.QLCError) as e:       # reservation above the budget
            srv.submit_compress(comp[6])
        assert e.value.status == qlc.QLC_ERR_CAPACITY
        with pytest.raises(qlc.QLCError) as e:       # misaligned input
            srv.submit_compress(comp[4][1:], n=1000)
        assert e.value.status == qlc.QLC_ERR_INVALID_ARGUMENT
        assert srv.stats().rejected == 1
        # a corrupt stream fails its own request only
        o = objs[2]
        bad_index = o.index.clone()
        bad_index[1] += 1
        ids = {srv.submit_decompress(o.n, o.bits, bad_index, o.total, o.table): ("d", 0),
               srv.submit_decompress(o.n, o.bits, o.index, o.total, o.table): ("d", 1)}
        torch.cuda.synchronize()
        got = {}
        t_end = time.time() + 30
        while len(got) < 2:
            assert time.time() < t_end
            for r in srv.poll(8, 20000):
                got[ids[r.id][1]] = r.status
                srv.release(r.id)
        assert got == {0: qlc.QLC_ERR_CORRUPT_STREAM, 1: 0}
        with pytest.raises(qlc.QLCError):
            srv.release(12345)


def test_bad_config():
    with pytest.raises(qlc.QLCError):
        qlc.Server(0)
    with pytest.raises(qlc.QLCError):
        qlc.Server(1 << 20, chunk_symbols=1000)


def test_single_request_sizes_below_the_tick_limit():
    """A tick of one request runs the single-tensor entry points on a
    workspace sized when the server is created; the segment count is not
    monotone in n (2^22 - 32 symbols take 256 segments, 2^22 take 128), so
    that workspace must fit every size up to max_tick_symbols, not only the
    largest.  Each request alone must equal qlc_compress / the original."""
    limit = 1 << 22
    sizes = [limit - 32, limit, (1 << 20) - 96, 1025 * 8192 // 4 - 64]
    with qlc.Server(256 << 20, chunk_symbols=C, max_tick_symbols=limit) as srv:
        for j, n in enumerate(sizes):
            x = _bytes(n, 300 + j).to(DEV)
            ids = _submit_all(srv, [x], [], [("c", 0)])
            st, total, bits, index, table = _collect(srv, ids)[("c", 0)]
            ref = qlc.compress(x, chunk_symbols=C)
            torch.cuda.synchronize()
            assert st == 0, (n, st)
            assert total == ref.total_bits(), n
            assert np.array_equal(bits, ref.bits[:ref.nbytes()].cpu().numpy()), n
            o = qlc.compress(x, chunk_symbols=C)
            torch.cuda.synchronize()
            ids = _submit_all(srv, [], [o], [("d", 0)])
            st, out = _collect(srv, ids)[("d", 0)]
            assert st == 0 and np.array_equal(out, x.cpu().numpy()), n
