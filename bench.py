"""QLC codec benchmark on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--chunk C]

One step = the whole hot path on one synthetic tensor already resident in
HBM: histogram, rank, layout search and LUT emit (qlc_compress builds the
table), bit-packed encode, then chunk-parallel decode of the stream.  The
workload is the single 256 MiB e4m3 tensor (8192 x 32768, Laplace(0,1) with
1 % of the rows scaled x8, block-32 power-of-two scaling, seed 1).

Prints one JSON line.  `value` is uncompressed bytes per second of a whole
step (N / (t_compress + t_decode)); per-kernel rates, the roofline of the
dominant kernel and the CPU oracle baseline ride along.  The `batched`
object reports the batched form on 1152 uneven shards (one persistent
encode launch and one persistent decode launch, each replayed from a
hipGraph, work split from the autotuner) against plain per-shard launches
of the single-tensor entry points, with the outputs compared byte for byte.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "QLC encode/decode GB/s (uncompressed) + % HBM peak; batched vs plain at bit-exact"
WORKLOAD = ("single 256 MiB e4m3 tensor 8192x32768: FP32 Laplace(0,1), 1% rows x8, "
            "block-32 power-of-two scale, RNE e4m3; per-tensor SEARCH_QUAD table; seed 1")
KERNEL_SOURCES = ["paper_2602_17849_amd/csrc/qlc_kernels.hip",
                  "paper_2602_17849_amd/csrc/qlc_device.h",
                  "paper_2602_17849_amd/csrc/qlc_internal.h"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_profile(kernel: str) -> dict:
    """rocprofv3 figures of one kernel from profiles/traffic.json: HBM bytes
    per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) and the average
    kernel-trace duration, valid only while the kernel sources are
    unchanged (empty otherwise)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return {}
    if rec.get("source_hash") != kernel_source_hash():
        return {}
    for name, v in rec.get("kernels", {}).items():  # names carry template arguments
        if name.split("<")[0] == kernel:
            return v
    return {}


def _host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x_host, chunk, reps=5, st_sample=1 << 25):
    """The CPU oracle as it stands, timed on this host: the OpenMP oracle on
    every host core over the whole workload tensor, and the single-threaded
    oracle on one core over the tensor's first `st_sample` symbols (its
    full-tensor run would take about a minute per repetition).  Each op is
    timed on its own (build_table = histogram + rank + layout search + LUTs;
    encode; decode), median of `reps` after one warm-up; the multi-threaded
    outputs are checked against the single-threaded ones on the sample."""
    import numpy as np

    import oracle
    oracle.build()
    threads = oracle.mt_threads(0)

    def median_time(fn):
        fn()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    def ops(x, mt, table=None):
        if mt:
            hist = lambda: oracle.histogram_mt(x, threads)
            enc = lambda t: oracle.encode_mt(x, t, chunk, threads=threads)
            dec = lambda e, t: oracle.decode_mt(e[1], e[3], e[2], chunk, t, x.size, threads)
        else:
            hist = lambda: oracle.histogram(x)
            enc = lambda t: oracle.encode(x, t, chunk)
            dec = lambda e, t: oracle.decode(e[1], e[3], e[2], chunk, t, x.size)
        t_bt = median_time(lambda: oracle.build_table(hist(), oracle.MODE_SEARCH_QUAD))
        if table is None:
            table = oracle.build_table(hist(), oracle.MODE_SEARCH_QUAD)
        e = enc(table)
        t_enc = median_time(lambda: enc(table))
        d = dec(e, table)
        t_dec = median_time(lambda: dec(e, table))
        assert e[0] == 0 and d[0] == 0 and np.array_equal(d[1], x), "oracle round trip"
        n = x.size
        res = {"threads": threads if mt else 1, "symbols": int(n),
               "build_table_gbps": round(n / t_bt / 1e9, 4),
               "encode_gbps": round(n / t_enc / 1e9, 4),
               "decode_gbps": round(n / t_dec / 1e9, 4),
               "step_gbps": round(n / (t_bt + t_enc + t_dec) / 1e9, 4),
               "build_table_s": round(t_bt, 4), "encode_s": round(t_enc, 4),
               "decode_s": round(t_dec, 4)}
        return res, e, table

    mt, e_mt, table = ops(np.ascontiguousarray(x_host), True)
    print("cpu baseline, multi-threaded: %s" % mt, file=sys.stderr, flush=True)
    # the single-threaded encode and decode of the sample use the whole
    # tensor's table, so that its stream is the prefix of the whole stream
    xs = np.ascontiguousarray(x_host[:st_sample])
    st, e_st, _ = ops(xs, False, table)
    print("cpu baseline, single-threaded: %s" % st, file=sys.stderr, flush=True)
    # the multi-threaded stream starts with the single-threaded stream of
    # the prefix sample (whole bytes; the index entries of its chunks)
    nb = e_st[3] // 8
    k = (xs.size + chunk - 1) // chunk
    assert np.array_equal(e_mt[1][:nb], e_st[1][:nb]) and np.array_equal(e_mt[2][:k], e_st[2])
    return {"value": mt["step_gbps"], "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": "multi-threaded oracle (OpenMP, %d threads) on the whole %d-symbol "
                      "workload tensor: build_table + encode + decode, each the median of %d "
                      "runs after a warm-up; single-threaded oracle on 1 core over the first "
                      "%d symbols (encode and decode with the whole tensor's table)"
                      % (threads, x_host.size, reps, xs.size),
                      "multi_threaded": mt, "single_threaded": st,
                      "host_cpu": _host_cpu(), "host_cpus_visible": len(os.sched_getaffinity(0))}


BATCH_WORKLOAD = ("1152 shards (18 x 64), sizes log-uniform in 1-32 MiB, multiples of 32 B "
                  "(seed 2); shard i: N(0,1) activations, Student-t(3) gradients or N(0,0.02) "
                  "weights by i mod 3, block-32 e4m3; per-shard SEARCH_QUAD table")


def run_batched(dev, steps, plain_steps=2, fixed=None):
    """Batched form vs plain per-shard launches on the 1152-shard workload."""
    import torch

    from paper_2602_17849_amd import autotune, datagen, qlc

    mode = qlc.LAYOUT_SEARCH_QUAD
    sizes = datagen.shard_sizes()
    S, total = len(sizes), sum(sizes)
    cmin = min(autotune.CHUNKS)
    A = qlc.Batch(sizes, chunk_symbols=cmin, device=dev, min_chunk=cmin)
    for i, n in enumerate(sizes):
        A.input(i).copy_(datagen.shard(i, n, device=dev))
    torch.cuda.synchronize()
    print("batched: %d shards, %.2f GiB generated" % (S, total / 2**30), file=sys.stderr,
          flush=True)

    if fixed:  # (C, log2_segment, lag): the autotuner is skipped (profiling runs)
        ch = autotune.Choice(fixed[0], fixed[1], fixed[2], 0.0, 0.0)
    else:
        ch = autotune.tune_batched(A, mode)
    C = ch.chunk_symbols
    A.set_chunk(C)
    A.index.zero_()  # drop the entries other chunk sizes left while tuning
    tuning = ch.tuning()
    ws = A.workspace(tuning)
    stream = torch.cuda.current_stream()

    g_enc, g_dec = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_enc):
        A.encode(ws, mode, tuning)
    with torch.cuda.graph(g_dec):
        A.decode(ws, tuning)
    for _ in range(2):
        g_enc.replay()
        g_dec.replay()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for k in range(steps):
        evs[k][0].record(stream)
        g_enc.replay()
        evs[k][1].record(stream)
        g_dec.replay()
        evs[k][2].record(stream)
    torch.cuda.synchronize()
    t_enc = sum(e[0].elapsed_time(e[1]) for e in evs) / steps / 1e3
    t_dec = sum(e[1].elapsed_time(e[2]) for e in evs) / steps / 1e3
    assert not A.err.any().item(), "batched call reported an error"
    assert torch.equal(A.out, A.inp), "batched round trip mismatch"

    # plain per-shard launches of the single-tensor entry points, same C
    B = qlc.Batch(sizes, chunk_symbols=C, device=dev, min_chunk=cmin, inp=A.inp)
    wsp = torch.zeros(max(qlc.qlc_workspace_bytes(n, C) for n in sizes), dtype=torch.uint8,
                      device=dev)
    derr = torch.zeros(S, dtype=torch.int32, device=dev)
    args = [(B.input(i), B.table(i), B.bitstream(i), B.chunk_index(i, whole=True),
             B.total[i:i + 1], B.err[i:i + 1], B.output(i), derr[i:i + 1], n)
            for i, n in enumerate(sizes)]

    def plain_pass():
        for x, t, bits, idx, tot, err, out, de, n in args:
            qlc.qlc_compress(x, mode, t, C, bits, idx, tot, err, wsp)
            qlc.qlc_decode(bits, tot, idx, C, t, n, out, de, wsp)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3

    def plain_pass_lane():  # the same with the one-lane-per-chunk decoder forced
        for x, t, bits, idx, tot, err, out, de, n in args:
            qlc.qlc_compress(x, mode, t, C, bits, idx, tot, err, wsp)
            qlc.qlc_decode_ex(bits, tot, idx, C, t, n, 8, qlc.DECODER_LANE, out, de, wsp)

    t_plain_lane = timed(plain_pass_lane, plain_steps)
    assert not B.err.any().item() and not derr.any().item()
    assert torch.equal(B.out, A.inp), "plain round trip (lane decoder)"
    B.out.zero_()
    t_plain = timed(plain_pass, plain_steps)
    g_plain = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_plain):
        plain_pass()
    t_plain_graph = timed(g_plain.replay, plain_steps)
    assert not B.err.any().item() and not derr.any().item()
    same = {"bits": torch.equal(A.bits, B.bits), "index": torch.equal(A.index, B.index),
            "tables": torch.equal(A.tables, B.tables), "total": torch.equal(A.total, B.total),
            "plain_round_trip": torch.equal(B.out, A.inp)}
    exact = all(same.values())
    assert exact, "batched and plain outputs differ: %s" % same
    # The plain decoder runs one lane per chunk, so a shard of ~9 MiB at the
    # batched C leaves most of the device idle; the smallest chunk size (256
    # symbols, 8x the lanes at C = 2048) is the plain path's own best setting.
    # Another C changes the chunk index, so this pass is a throughput
    # baseline only (round trip checked, no byte comparison with the batch).
    C_small = qlc.MIN_CHUNK
    B2 = qlc.Batch(sizes, chunk_symbols=C_small, device=dev, inp=A.inp)
    derr2 = torch.zeros(S, dtype=torch.int32, device=dev)
    args2 = [(B2.input(i), B2.table(i), B2.bitstream(i), B2.chunk_index(i, whole=True),
              B2.total[i:i + 1], B2.err[i:i + 1], B2.output(i), derr2[i:i + 1], n)
             for i, n in enumerate(sizes)]

    def plain_pass_small():
        for x, t, bits, idx, tot, err, out, de, n in args2:
            qlc.qlc_compress(x, mode, t, C_small, bits, idx, tot, err, wsp)
            qlc.qlc_decode(bits, tot, idx, C_small, t, n, out, de, wsp)

    t_plain_small = timed(plain_pass_small, plain_steps)
    assert not B2.err.any().item() and not derr2.any().item()
    assert torch.equal(B2.out, A.inp), "plain round trip at the smallest chunk size"
    del B2
    t_b = t_enc + t_dec
    return {
        "workload": BATCH_WORKLOAD, "shards": S, "symbols": total, "chunk_symbols": C,
        "log2_segment": ch.log2_segment, "lag_segments": ch.lag_segments,
        "form": "qlc_encode_batched + qlc_decode_batched, each one hipGraph replay",
        "gbps": round(total / t_b / 1e9, 2),
        "encode_gbps": round(total / t_enc / 1e9, 2),
        "decode_gbps": round(total / t_dec / 1e9, 2),
        "plain_decoders": "qlc_decode picks per shard (QLC_DECODER_AUTO); 'lane' forces "
                          "one lane per chunk",
        "plain_decoder_split_shards": sum(
            qlc.qlc_decoder_choice(n, C) == qlc.DECODER_SPLIT for n in sizes),
        "plain_per_shard_gbps": round(total / t_plain / 1e9, 2),
        "plain_per_shard_lane_gbps": round(total / t_plain_lane / 1e9, 2),
        "plain_per_shard_graph_gbps": round(total / t_plain_graph / 1e9, 2),
        "speedup_vs_plain": round(t_plain / t_b, 3),
        "speedup_vs_plain_graph": round(t_plain_graph / t_b, 3),
        "plain_per_shard_c256_gbps": round(total / t_plain_small / 1e9, 2),
        "speedup_vs_plain_c256": round(t_plain_small / t_b, 3),
        "bit_exact_vs_plain": bool(exact),
        "stream_bytes": int(((A.total + 31) // 32 * 4).sum().item()),
    }


SMALL_WORKLOAD = ("single 1 Mi-symbol e4m3 tensor 1024x1024: FP32 N(0,1), block-32 "
                  "power-of-two scale, RNE e4m3; per-tensor SEARCH_QUAD table; seed 0")


def run_small(dev, reps=200):
    """Latency of one compress call and one decode call on the 1 Mi-symbol
    tensor (launch-bound: the data moves in well under a microsecond at
    HBM rates), eager launches timed one by one with HIP events, median."""
    import numpy as np
    import torch

    from paper_2602_17849_amd import datagen, qlc

    x = datagen.single_tensor_gaussian(seed=0, device=dev)
    n = x.numel()
    stream = torch.cuda.current_stream()
    out = {"workload": SMALL_WORKLOAD, "symbols": n, "timing": "median of %d calls, HIP "
           "events around each call on the launch stream" % reps}
    for C in (256, 2048):
        ws = qlc.new_workspace(n, C, dev)
        table = qlc.new_table(dev)
        bits = torch.empty(qlc.qlc_encode_bound_bytes(n), dtype=torch.uint8, device=dev)
        index = torch.empty(qlc.qlc_chunk_count(n, C), dtype=torch.int64, device=dev)
        total = torch.empty(1, dtype=torch.int64, device=dev)
        err = torch.zeros(1, dtype=torch.int32, device=dev)
        y = torch.empty_like(x)
        derr = torch.zeros(1, dtype=torch.int32, device=dev)
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
        for k in range(reps + 5):
            e = ev[k - 5] if k >= 5 else None
            if e:
                e[0].record(stream)
            qlc.qlc_compress(x, qlc.LAYOUT_SEARCH_QUAD, table, C, bits, index, total, err, ws)
            if e:
                e[1].record(stream)
            qlc.qlc_decode(bits, total, index, C, table, n, y, derr, ws)
            if e:
                e[2].record(stream)
        torch.cuda.synchronize()
        assert int(err.item()) == 0 and int(derr.item()) == 0 and torch.equal(x, y)
        tc = float(np.median([e[0].elapsed_time(e[1]) for e in ev])) * 1e3
        td = float(np.median([e[1].elapsed_time(e[2]) for e in ev])) * 1e3
        res = {"compress_us": round(tc, 2), "decode_us": round(td, 2),
               "compress_gbps": round(n / tc / 1e3, 2), "decode_gbps": round(n / td / 1e3, 2),
               "bits_per_symbol": round(int(total.item()) / n, 5),
               "decoder": "split" if qlc.qlc_decoder_choice(n, C) == qlc.DECODER_SPLIT
               else "lane"}
        for name, dec in (("lane", qlc.DECODER_LANE), ("split", qlc.DECODER_SPLIT)):
            evd = [[torch.cuda.Event(enable_timing=True) for _ in range(2)]
                   for _ in range(reps // 2)]
            for k in range(reps // 2 + 3):
                e = evd[k - 3] if k >= 3 else None
                if e:
                    e[0].record(stream)
                qlc.qlc_decode_ex(bits, total, index, C, table, n, 8, dec, y, derr, ws)
                if e:
                    e[1].record(stream)
            torch.cuda.synchronize()
            assert int(derr.item()) == 0 and torch.equal(x, y), name
            res["decode_%s_us" % name] = round(
                float(np.median([e[0].elapsed_time(e[1]) for e in evd])) * 1e3, 2)
        out["C%d" % C] = res
    return out


def run_calibrated(dev, x, C, reps=10):
    """Encode and decode of the workload tensor with a table fixed in
    advance: built on the device from a calibration tensor of the same
    recipe (seed 101), standing in for a per-tensor-type table obtained a
    priori.  No histogram pass over the workload tensor itself."""
    import torch

    from paper_2602_17849_amd import datagen, qlc

    n = x.numel()
    calib = datagen.single_tensor_laplace(seed=101, device=dev)
    table = qlc.new_table(dev)
    ws = qlc.new_workspace(n, C, dev)
    qlc.qlc_build_table(calib, qlc.LAYOUT_SEARCH_QUAD, table, ws)
    del calib
    bits = torch.empty(qlc.qlc_encode_bound_bytes(n), dtype=torch.uint8, device=dev)
    index = torch.empty(qlc.qlc_chunk_count(n, C), dtype=torch.int64, device=dev)
    total = torch.empty(1, dtype=torch.int64, device=dev)
    err = torch.zeros(1, dtype=torch.int32, device=dev)
    y = torch.empty_like(x)
    derr = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    # the cache-evicting read of the main step, before every encode + decode
    flush64 = torch.zeros(512 << 20, dtype=torch.uint8, device=dev).view(torch.int64)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
    for k in range(reps + 2):
        e = ev[k - 2] if k >= 2 else None
        flush64.sum()
        if e:
            e[0].record(stream)
        qlc.qlc_encode(x, table, C, bits, index, total, err, ws)
        if e:
            e[1].record(stream)
        qlc.qlc_decode(bits, total, index, C, table, n, y, derr, ws)
        if e:
            e[2].record(stream)
    torch.cuda.synchronize()
    assert int(err.item()) == 0 and int(derr.item()) == 0 and torch.equal(x, y)
    te = sum(e[0].elapsed_time(e[1]) for e in ev) / reps / 1e3
    td = sum(e[1].elapsed_time(e[2]) for e in ev) / reps / 1e3
    tb = int(total.item())
    enc_bytes = n + 4 * ((tb + 31) // 32) + 8 * qlc.qlc_chunk_count(n, C)
    return {"table": "SEARCH_QUAD table built from a calibration tensor of the same recipe "
                     "(seed 101), fixed before the workload tensor is seen",
            "bits_per_symbol": round(tb / n, 5),
            "encode_gbps": round(n / te / 1e9, 2), "decode_gbps": round(n / td / 1e9, 2),
            "encode_hbm_frac": round(enc_bytes / te / 1e9 / HBM_PEAK_GBS, 4)}


STRESS_WORKLOAD = ("three 4,294,967,296-byte buffers in one batched call, C = 4096: "
                   "(i) uniform random bytes (seed 4), (ii) N(0,1) block-32 e4m3 with 90% of "
                   "the bytes 0x00 (seed 5), (iii) OCP-style e4m3, N(0,1) block-32 with the "
                   "448 scale rule, 0x7F/0xFF never emitted (seed 6)")


def run_stress(dev, reps=3):
    """The three 4 GiB buffers through the batched form (one encode launch
    and one decode launch for all three jobs), under SEARCH_QUAD and under
    Table 1's fixed widths, with the expansion of each buffer."""
    import torch

    from paper_2602_17849_amd import datagen, qlc

    N, C = 1 << 32, 4096
    kinds = ("uniform", "zeros90", "ocp_gaussian")
    b = qlc.Batch([N] * 3, chunk_symbols=C, device=dev, capacity="bound")
    for i, k in enumerate(kinds):
        b.input(i).copy_(datagen.stress_buffer(k, N, device=dev))
    torch.cuda.synchronize()
    print("stress: 3 x 4 GiB generated", file=sys.stderr, flush=True)
    ws = b.workspace()
    stream = torch.cuda.current_stream()
    res = {"workload": STRESS_WORKLOAD, "symbols": 3 * N, "chunk_symbols": C}
    for name, mode in (("SEARCH_QUAD", qlc.LAYOUT_SEARCH_QUAD), ("PAPER_T1", qlc.LAYOUT_PAPER_T1)):
        b.encode(ws, mode)
        b.decode(ws)
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
        for e in ev:
            e[0].record(stream)
            b.encode(ws, mode)
            e[1].record(stream)
            b.decode(ws)
            e[2].record(stream)
        torch.cuda.synchronize()
        assert not b.err.any().item(), "stress batch reported an error"
        assert torch.equal(b.out, b.inp), "stress round trip"
        te = sum(e[0].elapsed_time(e[1]) for e in ev) / reps / 1e3
        td = sum(e[1].elapsed_time(e[2]) for e in ev) / reps / 1e3
        tot = [int(v) for v in b.total.tolist()]
        res[name] = {
            "encode_gbps": round(3 * N / te / 1e9, 2), "decode_gbps": round(3 * N / td / 1e9, 2),
            "bits_per_symbol": {k: round(t / N, 5) for k, t in zip(kinds, tot)},
            "expansion_pct": {k: round(100.0 * (t / (8.0 * N) - 1.0), 3)
                              for k, t in zip(kinds, tot)}}
    res["note"] = ("expansion = code bits / input bits - 1; the chunk index adds 8 bytes per "
                   "%d symbols (%.3f%%) and the table 264 bytes" % (C, 100.0 * 8 / C))
    del b, ws
    torch.cuda.empty_cache()
    return res


SERVE_WORKLOAD = ("Poisson arrivals, mean 2000 req/s for 10 s (seed 3), 50/50 compress / "
                  "decompress, sizes log-uniform 64 KiB-64 MiB (multiples of 32 B) of Laplace "
                  "block-32 e4m3; compress inputs are slices of a resident 1 GiB tensor, "
                  "decompress requests cycle over 256 objects pre-compressed at setup; "
                  "32 GiB device budget")


def _pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else None


def run_serving(dev, duration_s=10.0, chunk=512, log2_segment=0, budget=32 << 30,
                decoder=None):
    """The serving loop (qlc_server_*) under Poisson arrivals, then the same
    requests submitted at once (saturation)."""
    import torch

    from paper_2602_17849_amd import datagen, qlc

    reqs = datagen.serving_requests(duration_s=duration_s, rate=2000.0, seed=3)
    pool = datagen.laplace_outlier_rows(1024, 1 << 20, seed=30, device=dev)  # 1 GiB
    pool_n = pool.numel()
    dec_sizes = [n for _, k, n in reqs if k == "decompress"][:256]
    objs = []
    for j, n in enumerate(dec_sizes):
        off = (j * 1_048_573 * 256) % (pool_n - n) // 256 * 256
        objs.append(qlc.compress(pool[off:off + n], chunk_symbols=chunk))
    torch.cuda.synchronize()
    assert all(int(o.err.item()) == 0 for o in objs)
    print("serving: %d requests, %d objects resident" % (len(reqs), len(objs)), file=sys.stderr,
          flush=True)

    def submit(srv, i, kind, n):
        if kind == "compress":
            off = (i * 2_654_435 * 256) % (pool_n - n) // 256 * 256
            return srv.submit_compress(pool[off:off + n], n=n), n
        o = objs[i % len(objs)]
        return srv.submit_decompress(o.n, o.bits, o.index, o.total, o.table), o.n

    def drain(srv, pending, lat, done_bytes, last):
        for r in srv.poll(256, 0):
            t_arr, nbytes = pending.pop(r.id)
            if r.status != 0:
                raise RuntimeError("serving request failed with status %d" % r.status)
            lat.append((r.complete_ns - t_arr) / 1e3)
            done_bytes[0] += nbytes
            last[0] = max(last[0], r.complete_ns)
            srv.release(r.id)

    out = {}
    for mode in ("poisson", "saturation"):
        srv = qlc.Server(budget, chunk_symbols=chunk, max_jobs_per_tick=64,
                         max_ticks_in_flight=4, log2_segment=log2_segment,
                         decoder=qlc.DECODER_AUTO if decoder is None else decoder)
        lat, done_bytes, last, pending = [], [0], [0], {}
        t0 = time.perf_counter_ns()
        for i, (t_arr, kind, n) in enumerate(reqs):
            if mode == "poisson":
                due = t0 + int(t_arr * 1e9)
                while time.perf_counter_ns() < due:
                    drain(srv, pending, lat, done_bytes, last)
            else:
                due = t0
            rid, nbytes = submit(srv, i, kind, n)
            pending[rid] = (due, nbytes)
        while pending:
            drain(srv, pending, lat, done_bytes, last)
        st = srv.stats()
        srv.close()
        span = (last[0] - t0) / 1e9
        out[mode] = {
            "requests": len(reqs), "bytes": done_bytes[0],
            "gbps": round(done_bytes[0] / span / 1e9, 2),
            "p50_us": round(_pct(lat, 50), 1), "p99_us": round(_pct(lat, 99), 1),
            "p999_us": round(_pct(lat, 99.9), 1), "makespan_s": round(span, 4),
            "ticks": int(st.ticks), "max_jobs_in_tick": int(st.max_jobs_in_tick),
            "max_ticks_in_flight": int(st.max_ticks_in_flight),
            "peak_bytes_in_use": int(st.peak_bytes_in_use)}
        print("serving %s: %s" % (mode, out[mode]), file=sys.stderr, flush=True)
    return {"workload": SERVE_WORKLOAD, "chunk_symbols": chunk, "log2_segment": log2_segment,
            "decoder": ["auto", "lane", "split"][qlc.DECODER_AUTO if decoder is None else decoder],
            "budget_bytes": budget, "latency": "scheduled arrival to completion seen by the "
            "server thread", **out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--chunk", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 1 Mi-symbol latency, calibrated-table and 4 GiB legs")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--batched-tuning", default="",
                    help="C,LOG2_SEGMENT,LAG for the batched form instead of the autotuner")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(each tensor shard is compressed independently on its own GPU)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2602_17849_amd import datagen, qlc

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    x = datagen.single_tensor_laplace(device=dev)
    n = x.numel()
    C = args.chunk
    ws = qlc.new_workspace(n, C, dev)
    table = qlc.new_table(dev)
    cap = qlc.qlc_encode_bound_bytes(n)
    bits = torch.empty(cap, dtype=torch.uint8, device=dev)
    index = torch.empty(qlc.qlc_chunk_count(n, C), dtype=torch.int64, device=dev)
    total = torch.empty(1, dtype=torch.int64, device=dev)
    err = torch.zeros(1, dtype=torch.int32, device=dev)
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    derr = torch.zeros(1, dtype=torch.int32, device=dev)
    # read before every step: evicts the tensor from the 256 MB Infinity
    # Cache and leaves it holding clean lines (a write would leave dirty
    # lines whose write-back the next kernel pays for)
    flush = torch.zeros(512 << 20, dtype=torch.uint8, device=dev)
    flush64 = flush.view(torch.int64)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        qlc.qlc_compress(x, qlc.LAYOUT_SEARCH_QUAD, table, C, bits, index, total, err, ws)
        if ev is not None:
            ev[1].record(stream)
        qlc.qlc_decode(bits, total, index, C, table, n, out, derr, ws)
        if ev is not None:
            ev[2].record(stream)

    for k in range(args.warmup):
        flush64.sum()
        step()
    torch.cuda.synchronize()
    assert int(err.item()) == 0 and int(derr.item()) == 0
    assert torch.equal(out, x), "round trip mismatch"

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        flush64.sum()
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert int(err.item()) == 0 and int(derr.item()) == 0
    assert torch.equal(out, x), "round trip mismatch"
    t_comp = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps / 1e3
    t_dec = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps / 1e3
    ms_per_step = wall / args.steps * 1e3

    # per-kernel rates: encode with the table fixed, histogram+table alone;
    # each call after the same cache-evicting read as a step (mean of reps)
    def timed_cold(fn, reps=10):
        fn()
        evp = []
        for _ in range(reps):
            flush64.sum()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            evp.append((e0, e1))
        torch.cuda.synchronize()
        return sum(a.elapsed_time(b) for a, b in evp) / reps / 1e3

    # ... and back to back (each call also pays for the write-back of the
    # previous call's output lines)
    def timed(fn, reps=10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3

    t_enc = timed_cold(lambda: qlc.qlc_encode(x, table, C, bits, index, total, err, ws))
    t_enc_b2b = timed(lambda: qlc.qlc_encode(x, table, C, bits, index, total, err, ws))
    # bits per symbol of the tensor under every layout mode (tables built on
    # the device from its histogram; cost_bits = sum h * len)
    hist = torch.zeros(256, dtype=torch.int64, device=dev)
    qlc.qlc_histogram(x, hist, ws)
    layouts = {}
    lt = qlc.new_table(dev)
    named = [("SEARCH_QUAD", qlc.LAYOUT_SEARCH_QUAD), ("SEARCH_ANY", qlc.LAYOUT_SEARCH_ANY),
             ("PAPER_T1", qlc.LAYOUT_PAPER_T1), ("PAPER_T2", qlc.LAYOUT_PAPER_T2),
             ("SEARCH_AREAS4", qlc.LAYOUT_SEARCH_AREAS4)] + \
        [("SEARCH_DISTINCT_%d" % k, qlc.LAYOUT_SEARCH_DISTINCT(k)) for k in (1, 2, 3)]
    for name, mode in named:
        qlc.qlc_table_from_histogram(hist, mode, lt)
        torch.cuda.synchronize()
        layouts[name] = round(qlc.parse_table(lt)["cost_bits"] / n, 5)
    t_tab = timed_cold(lambda: qlc.qlc_build_table(x, qlc.LAYOUT_SEARCH_QUAD, table, ws))
    del flush, flush64
    qlc.qlc_compress(x, qlc.LAYOUT_SEARCH_QUAD, table, C, bits, index, total, err, ws)
    torch.cuda.synchronize()
    tb = int(total.item())
    L = tb / n
    stream_bytes = 4 * ((tb + 31) // 32)
    index_bytes = 8 * qlc.qlc_chunk_count(n, C)
    # algorithmic bytes of one decode launch: read stream + index, write symbols
    dec_bytes = stream_bytes + index_bytes + n
    achieved = dec_bytes / t_dec / 1e9
    prof = load_profile("k_decode")
    roof = {"kernel": "k_decode", "bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": prof.get("bytes_per_launch"),
            "algorithmic_bytes_per_launch": dec_bytes,
            "timing": "HIP events around the decode launch in each timed step (launch gap "
                      "included)"}
    if prof.get("avg_us"):
        a = dec_bytes / (prof["avg_us"] * 1e-6) / 1e9
        roof["rocprof_avg_us"] = round(prof["avg_us"], 2)
        roof["rocprof_achieved"] = round(a, 1)
        roof["rocprof_frac"] = round(a / HBM_PEAK_GBS, 4)

    res = {
        "metric": METRIC,
        "value": round(n / (t_comp + t_dec) / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "symbols": n, "chunk_symbols": C,
                   "layout_mode": "SEARCH_QUAD"},
        "cache": "a 512 MiB device read before every step (outside the event-timed region, "
                 "inside ms_per_step) evicts the input from the 256 MB Infinity Cache and "
                 "leaves it clean; within a step each kernel finds what the kernel before it "
                 "left there; the fixed-table encode, build_table and calibrated_table calls "
                 "are each timed after the same read (encode_fixed_table_back_to_back_gbps: "
                 "ten calls in a row, no read between)",
        "compress_gbps": round(n / t_comp / 1e9, 2),
        "decode_gbps": round(n / t_dec / 1e9, 2),
        "encode_fixed_table_gbps": round(n / t_enc / 1e9, 2),
        "encode_fixed_table_hbm_frac": round(
            (n + stream_bytes + index_bytes) / t_enc / 1e9 / HBM_PEAK_GBS, 4),
        "encode_fixed_table_back_to_back_gbps": round(n / t_enc_b2b / 1e9, 2),
        "build_table_gbps": round(n / t_tab / 1e9, 2),
        "bits_per_symbol": round(L, 5),
        "compressibility": round((8 - L) / 8, 5),
        "compressibility_with_index_and_table": round(
            1 - (stream_bytes + index_bytes + 264) / n, 5),
        "bits_per_symbol_by_layout": layouts,
        "roofline": roof,
    }
    x_host = None if args.no_cpu_baseline else x.cpu().numpy()
    if not args.no_extra:
        res["calibrated_table"] = run_calibrated(dev, x, C)
        print("calibrated_table: %s" % res["calibrated_table"], file=sys.stderr, flush=True)
    del x, out, bits, ws
    torch.cuda.empty_cache()
    if not args.no_extra:
        res["small_tensor"] = run_small(dev)
        print("small_tensor: %s" % res["small_tensor"], file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    if not args.no_batched:
        fixed = tuple(int(v) for v in args.batched_tuning.split(",")) if args.batched_tuning else None
        res["batched"] = run_batched(dev, max(3, min(args.steps, 10)), fixed=fixed)
        torch.cuda.empty_cache()
    if not args.no_serving:
        res["serving"] = run_serving(dev, args.serve_seconds)
        torch.cuda.empty_cache()
    if not args.no_extra:
        res["stress_4gib"] = run_stress(dev)
        print("stress_4gib: %s" % res["stress_4gib"], file=sys.stderr, flush=True)
    if x_host is not None:
        res["cpu_baseline"] = cpu_baseline(x_host, C)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
