"""Autotuner of the batched form: picks the chunk size C and the encode work
split (segment size, histogram lag) for a batch by timing candidates on the
device, and remembers the choice per device and batch shape.

The choice only moves work around: every candidate yields the same table
and bitstream for each tensor, and the same chunk index for a given C.
"""
from __future__ import annotations

import json
import os
from dataclasses import asdict, dataclass

import torch

from . import qlc

CHUNKS = (1024, 2048, 4096)
LOG2_SEGMENTS = (16, 17, 18, 19)
LAGS = (0, 1)         # 0: every histogram first; 1: raised to the largest job's segment count

_cache: dict | None = None


@dataclass
class Choice:
    chunk_symbols: int
    log2_segment: int
    lag_segments: int
    encode_ms: float
    decode_ms: float

    def tuning(self):
        return qlc.BatchTuning(self.log2_segment, self.lag_segments, 0, 0)


def _cache_path():
    return os.environ.get("QLC_AUTOTUNE_CACHE", "")


def _load():
    global _cache
    if _cache is None:
        _cache = {}
        p = _cache_path()
        if p and os.path.exists(p):
            with open(p) as f:
                _cache = json.load(f)
    return _cache


def _store():
    p = _cache_path()
    if p:
        with open(p, "w") as f:
            json.dump(_cache, f, indent=1)


def key(batch: "qlc.Batch", mode: int) -> str:
    name = torch.cuda.get_device_name(batch.device)
    mib = batch.total_symbols >> 20
    return "%s|jobs=%d|MiB=%d|mode=%d" % (name, batch.S, mib, mode)


def _time(fn, reps: int) -> float:
    fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_batched(batch: "qlc.Batch", mode: int = qlc.LAYOUT_SEARCH_QUAD, chunks=CHUNKS,
                 log2_segments=LOG2_SEGMENTS, lags=LAGS, reps: int = 3,
                 use_cache: bool = True) -> Choice:
    """Time batched encode for every (C, segment, lag) and batched decode
    for every C on `batch` (its inputs already on the device; its index
    slots sized for min(chunks)); return the fastest encode + decode."""
    k = key(batch, mode)
    cache = _load()
    if use_cache and k in cache:
        return Choice(**cache[k])
    assert min(chunks) >= batch.min_chunk
    c_prev = batch.C
    wsb = max(qlc.qlc_batched_workspace_bytes(batch.S, batch.total_symbols, min(chunks),
                                              (min(log2_segments), 0, 0, 0)), 256)
    ws = torch.zeros(wsb, dtype=torch.uint8, device=batch.device)
    best = None
    for C in chunks:
        batch.set_chunk(C)
        enc = {}
        for l2 in log2_segments:
            for lag in lags:
                t = qlc.BatchTuning(l2, lag, 0, 0)
                enc[(l2, lag)] = _time(lambda: batch.encode(ws, mode, t), reps)
        (l2, lag), te = min(enc.items(), key=lambda kv: kv[1])
        batch.encode(ws, mode, qlc.BatchTuning(l2, lag, 0, 0))
        td = _time(lambda: batch.decode(ws), reps)
        assert not batch.err.any().item(), "batched call reported an error while tuning"
        c = Choice(C, l2, lag, te, td)
        if best is None or c.encode_ms + c.decode_ms < best.encode_ms + best.decode_ms:
            best = c
    batch.set_chunk(c_prev)
    cache[k] = asdict(best)
    _store()
    return best
