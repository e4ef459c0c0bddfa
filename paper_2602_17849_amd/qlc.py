"""Python binding of libqlc (argument marshalling only).

Every function named ``qlc_*`` mirrors the C entry point of the same name in
include/qlc.h: torch tensors provide device memory (``data_ptr()``) and the
current torch stream provides the HIP stream; all work runs in the HIP
kernels of libqlc.so.  There is no fallback: if the library is missing the
calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqlc.so")

QLC_OK = 0
QLC_ERR_INVALID_ARGUMENT = 1
QLC_ERR_CAPACITY = 2
QLC_ERR_CORRUPT_STREAM = 3
QLC_ERR_UNSUPPORTED = 4
QLC_ERR_HIP = 5
QLC_ERR_BUSY = 6

LAYOUT_SEARCH_QUAD = 0
LAYOUT_SEARCH_ANY = 1
LAYOUT_PAPER_T1 = 2
LAYOUT_PAPER_T2 = 3


LAYOUT_SEARCH_AREAS4 = 32   # 2-bit area code, 4 areas
# small alphabets (the *_sym entry points): 16 symbols (4-bit) or 64 (6-bit)
LAYOUT_M16_AREAS2 = 48
LAYOUT_M16_AREAS4 = 49
LAYOUT_M64_AREAS4 = 50
LAYOUT_M64_AREAS8 = 51


# decoder choice of qlc_decode_ex
DECODER_AUTO = 0
DECODER_LANE = 1
DECODER_SPLIT = 2
SPLIT_MAX_CHUNK = 16384


def mode_symbol_bits(mode: int) -> int:
    """Bits per symbol of the alphabet a layout mode codes."""
    return 4 if mode in (48, 49) else 6 if mode in (50, 51) else 8


def packed_bytes(n: int, symbol_bits: int) -> int:
    """Bytes holding n packed symbols of symbol_bits bits."""
    return (n * symbol_bits + 7) // 8


def LAYOUT_SEARCH_DISTINCT(k: int) -> int:
    """Layout mode: cheapest tuple with at most k (1..8) distinct code lengths."""
    if not 1 <= k <= 8:
        raise ValueError("k must be in 1..8")
    return 16 + k

TABLE_BYTES = 1088
SERIALIZED_TABLE_BYTES = 264
MIN_CHUNK = 256
MAX_CHUNK = 65536


class QLCError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what, _status_string(status), status))


class _Table(ctypes.Structure):
    _fields_ = [
        ("enc", ctypes.c_uint16 * 256),
        ("rank_to_sym", ctypes.c_uint8 * 256),
        ("sym_to_rank", ctypes.c_uint8 * 256),
        ("width", ctypes.c_uint8 * 8),
        ("offset", ctypes.c_uint8 * 8),
        ("first", ctypes.c_uint16 * 8),
        ("count", ctypes.c_uint16 * 8),
        ("cost_bits", ctypes.c_uint64),
        ("mode", ctypes.c_uint32),
        ("version", ctypes.c_uint32),
    ]


assert ctypes.sizeof(_Table) == TABLE_BYTES


class Job(ctypes.Structure):
    """qlc_job: one tensor of a batched call (device pointers)."""
    _fields_ = [
        ("in_", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("n", ctypes.c_uint64),
        ("table", ctypes.c_void_p),
        ("bits", ctypes.c_void_p),
        ("bits_capacity", ctypes.c_uint64),
        ("chunk_index", ctypes.c_void_p),
        ("total_bits", ctypes.c_void_p),
        ("err", ctypes.c_void_p),
        ("build_table", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


JOB_BYTES = 80
assert ctypes.sizeof(Job) == JOB_BYTES


class BatchTuning(ctypes.Structure):
    """qlc_batch_tuning: work split of a batched call (0 = automatic)."""
    _fields_ = [
        ("log2_segment", ctypes.c_uint32),
        ("lag_segments", ctypes.c_uint32),
        ("workgroups", ctypes.c_uint32),
        ("decoder", ctypes.c_uint32),   # decode: DECODER_AUTO / _LANE / _SPLIT
    ]

_lib = None
_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_sz = ctypes.c_size_t

_SIGNATURES = {
    "qlc_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "qlc_chunk_count": ([_u64, _u32], _u64),
    "qlc_encode_bound_bytes": ([_u64], _u64),
    "qlc_workspace_bytes": ([_u64, _u32], _sz),
    "qlc_workspace_init": ([_vp, _sz, _vp], ctypes.c_int),
    "qlc_histogram": ([_vp, _u64, _vp, _vp, _sz, _vp], ctypes.c_int),
    "qlc_histogram_accumulate": ([_vp, _u64, _vp, _vp, _sz, _vp], ctypes.c_int),
    "qlc_table_from_histogram": ([_vp, ctypes.c_int, _vp, _vp], ctypes.c_int),
    "qlc_build_table": ([_vp, _u64, ctypes.c_int, _vp, _vp, _sz, _vp], ctypes.c_int),
    "qlc_encode": ([_vp, _u64, _vp, _u32, _vp, _u64, _vp, _vp, _vp, _vp, _sz, _vp], ctypes.c_int),
    "qlc_compress": ([_vp, _u64, ctypes.c_int, _vp, _u32, _vp, _u64, _vp, _vp, _vp, _vp, _sz, _vp],
                     ctypes.c_int),
    "qlc_compress_noalloc": ([_vp, _u64, ctypes.c_int, _vp, _u32, _vp, _u64, _vp, _vp, _vp, _vp],
                             ctypes.c_int),
    "qlc_decode": ([_vp, _vp, _vp, _u32, _vp, _u64, _vp, _vp, _vp, _sz, _vp], ctypes.c_int),
    "qlc_histogram_sym": ([_vp, _u64, _u32, _vp, _vp, _sz, _vp], ctypes.c_int),
    "qlc_histogram_accumulate_sym": ([_vp, _u64, _u32, _vp, _vp, _sz, _vp], ctypes.c_int),
    "qlc_build_table_sym": ([_vp, _u64, _u32, ctypes.c_int, _vp, _vp, _sz, _vp], ctypes.c_int),
    "qlc_compress_sym": ([_vp, _u64, _u32, ctypes.c_int, _vp, _u32, _vp, _u64, _vp, _vp, _vp,
                          _vp, _sz, _vp], ctypes.c_int),
    "qlc_encode_sym": ([_vp, _u64, _u32, _vp, _u32, _vp, _u64, _vp, _vp, _vp, _vp, _sz, _vp],
                       ctypes.c_int),
    "qlc_decode_sym": ([_vp, _vp, _vp, _u32, _vp, _u64, _u32, _vp, _vp, _vp, _sz, _vp],
                       ctypes.c_int),
    "qlc_decoder_choice": ([_u64, _u32], ctypes.c_int),
    "qlc_decode_ex": ([_vp, _vp, _vp, _u32, _vp, _u64, _u32, ctypes.c_int, _vp, _vp, _vp, _sz,
                       _vp], ctypes.c_int),
    "qlc_encode_batched_sym": ([_vp, _u32, _u32, ctypes.c_int, _u32, _vp, _vp, _sz, _vp],
                               ctypes.c_int),
    "qlc_decode_batched_sym": ([_vp, _u32, _u32, _u32, _vp, _vp, _sz, _vp], ctypes.c_int),
    "qlc_batched_workspace_bytes": ([_u32, _u64, _u32, _vp], _sz),
    "qlc_encode_batched": ([_vp, _u32, ctypes.c_int, _u32, _vp, _vp, _sz, _vp], ctypes.c_int),
    "qlc_decode_batched": ([_vp, _u32, _u32, _vp, _vp, _sz, _vp], ctypes.c_int),
    "qlc_table_serialize": ([_vp, _vp], ctypes.c_int),
    "qlc_table_deserialize": ([_vp, _vp], ctypes.c_int),
}


def lib():
    """Load libqlc.so (built in-tree by paper_2602_17849_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libqlc.so is not built; run `python -m paper_2602_17849_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _status_string(s: int) -> str:
    try:
        return lib().qlc_status_string(int(s)).decode()
    except Exception:  # the library could not be loaded
        return "status %d" % s


def _check(st: int, what: str):
    if st != QLC_OK:
        raise QLCError(st, what)


def _p(t) -> int:
    """Device address of a tensor argument (a plain int passes through).
    The library reads flat device buffers: strided views or host tensors
    are refused here rather than read wrongly."""
    if t is None:
        return 0
    if isinstance(t, int):
        return t
    if not t.is_contiguous():
        raise ValueError("libqlc arguments must be contiguous tensors")
    if t.device.type != "cuda" and t.numel() > 0:
        raise ValueError("libqlc arguments must be device (cuda) tensors")
    return t.data_ptr()


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _nbytes(t) -> int:
    return t.numel() * t.element_size()


# ------------------------------------------------------------ size queries
def qlc_chunk_count(n: int, chunk_symbols: int) -> int:
    return int(lib().qlc_chunk_count(n, chunk_symbols))


def qlc_encode_bound_bytes(n: int) -> int:
    return int(lib().qlc_encode_bound_bytes(n))


def qlc_workspace_bytes(n: int, chunk_symbols: int = 4096) -> int:
    return int(lib().qlc_workspace_bytes(n, chunk_symbols))


# ------------------------------------------------------------ entry points
def qlc_workspace_init(ws: torch.Tensor, stream=None):
    _check(lib().qlc_workspace_init(_p(ws), _nbytes(ws), _stream(stream)), "qlc_workspace_init")


def qlc_histogram(x: torch.Tensor, hist_out: torch.Tensor, ws: torch.Tensor, stream=None):
    _check(lib().qlc_histogram(_p(x), x.numel(), _p(hist_out), _p(ws), _nbytes(ws),
                               _stream(stream)), "qlc_histogram")


def qlc_histogram_accumulate(x: torch.Tensor, hist_inout: torch.Tensor, ws: torch.Tensor,
                             stream=None):
    _check(lib().qlc_histogram_accumulate(_p(x), x.numel(), _p(hist_inout), _p(ws), _nbytes(ws),
                                          _stream(stream)), "qlc_histogram_accumulate")


def shared_table(xs, mode: int = LAYOUT_SEARCH_QUAD, stream=None) -> torch.Tensor:
    """One table for all device tensors in `xs` (a tensor type's LUT built
    a priori): their histograms summed on the device, then steps 2-4."""
    xs = list(xs)
    dev = xs[0].device if xs else torch.device("cuda")
    hist = torch.zeros(256, dtype=torch.int64, device=dev)
    ws = torch.zeros(max([qlc_workspace_bytes(x.numel()) for x in xs] + [256]),
                     dtype=torch.uint8, device=dev)
    for x in xs:
        qlc_histogram_accumulate(x, hist, ws, stream)
    table = new_table(dev)
    qlc_table_from_histogram(hist, mode, table, stream)
    return table


def qlc_table_from_histogram(hist: torch.Tensor, mode: int, table_out: torch.Tensor, stream=None):
    _check(lib().qlc_table_from_histogram(_p(hist), mode, _p(table_out), _stream(stream)),
           "qlc_table_from_histogram")


def qlc_build_table(x: torch.Tensor, mode: int, table_out: torch.Tensor, ws: torch.Tensor,
                    stream=None):
    _check(lib().qlc_build_table(_p(x), x.numel(), mode, _p(table_out), _p(ws), _nbytes(ws),
                                 _stream(stream)), "qlc_build_table")


def qlc_encode(x: torch.Tensor, table: torch.Tensor, chunk_symbols: int, bits_out: torch.Tensor,
               index_out: torch.Tensor, total_out: torch.Tensor, err_out: torch.Tensor,
               ws: torch.Tensor, stream=None, n: int | None = None):
    n = x.numel() if n is None else n
    _check(lib().qlc_encode(_p(x), n, _p(table), chunk_symbols, _p(bits_out), _nbytes(bits_out),
                            _p(index_out), _p(total_out), _p(err_out), _p(ws), _nbytes(ws),
                            _stream(stream)), "qlc_encode")


def qlc_compress(x: torch.Tensor, mode: int, table_out: torch.Tensor, chunk_symbols: int,
                 bits_out: torch.Tensor, index_out: torch.Tensor, total_out: torch.Tensor,
                 err_out: torch.Tensor, ws: torch.Tensor, stream=None, n: int | None = None):
    n = x.numel() if n is None else n
    _check(lib().qlc_compress(_p(x), n, mode, _p(table_out), chunk_symbols, _p(bits_out),
                              _nbytes(bits_out), _p(index_out), _p(total_out), _p(err_out), _p(ws),
                              _nbytes(ws), _stream(stream)), "qlc_compress")


COMPRESS_NOALLOC_MAX_SYMBOLS = 1 << 30


def qlc_compress_noalloc(x: torch.Tensor, mode: int, table_out: torch.Tensor,
                         chunk_symbols: int, bits_out: torch.Tensor, index_out: torch.Tensor,
                         total_out: torch.Tensor, err_out: torch.Tensor, stream=None,
                         n: int | None = None):
    """qlc_compress without a workspace argument (the library's own device
    array serves as workspace; calls overlapping on one device race)."""
    n = x.numel() if n is None else n
    _check(lib().qlc_compress_noalloc(_p(x), n, mode, _p(table_out), chunk_symbols, _p(bits_out),
                                      _nbytes(bits_out), _p(index_out), _p(total_out),
                                      _p(err_out), _stream(stream)), "qlc_compress_noalloc")


def qlc_decode(bits: torch.Tensor, total: torch.Tensor, index: torch.Tensor, chunk_symbols: int,
               table: torch.Tensor, n: int, out: torch.Tensor, err_out: torch.Tensor,
               ws: torch.Tensor, stream=None):
    _check(lib().qlc_decode(_p(bits), _p(total), _p(index), chunk_symbols, _p(table), n, _p(out),
                            _p(err_out), _p(ws), _nbytes(ws), _stream(stream)), "qlc_decode")


# ------------------------------------------------------------ small alphabets
# n counts symbols; tensors hold the packed bytes (see include/qlc.h).
def qlc_histogram_sym(x: torch.Tensor, n: int, symbol_bits: int, hist_out: torch.Tensor,
                      ws: torch.Tensor, stream=None):
    _check(lib().qlc_histogram_sym(_p(x), n, symbol_bits, _p(hist_out), _p(ws), _nbytes(ws),
                                   _stream(stream)), "qlc_histogram_sym")


def qlc_histogram_accumulate_sym(x: torch.Tensor, n: int, symbol_bits: int,
                                 hist_inout: torch.Tensor, ws: torch.Tensor, stream=None):
    _check(lib().qlc_histogram_accumulate_sym(_p(x), n, symbol_bits, _p(hist_inout), _p(ws),
                                              _nbytes(ws), _stream(stream)),
           "qlc_histogram_accumulate_sym")


def qlc_build_table_sym(x: torch.Tensor, n: int, symbol_bits: int, mode: int,
                        table_out: torch.Tensor, ws: torch.Tensor, stream=None):
    _check(lib().qlc_build_table_sym(_p(x), n, symbol_bits, mode, _p(table_out), _p(ws),
                                     _nbytes(ws), _stream(stream)), "qlc_build_table_sym")


def qlc_compress_sym(x: torch.Tensor, n: int, symbol_bits: int, mode: int,
                     table_out: torch.Tensor, chunk_symbols: int, bits_out: torch.Tensor,
                     index_out: torch.Tensor, total_out: torch.Tensor, err_out: torch.Tensor,
                     ws: torch.Tensor, stream=None):
    _check(lib().qlc_compress_sym(_p(x), n, symbol_bits, mode, _p(table_out), chunk_symbols,
                                  _p(bits_out), _nbytes(bits_out), _p(index_out), _p(total_out),
                                  _p(err_out), _p(ws), _nbytes(ws), _stream(stream)),
           "qlc_compress_sym")


def qlc_encode_sym(x: torch.Tensor, n: int, symbol_bits: int, table: torch.Tensor,
                   chunk_symbols: int, bits_out: torch.Tensor, index_out: torch.Tensor,
                   total_out: torch.Tensor, err_out: torch.Tensor, ws: torch.Tensor, stream=None):
    _check(lib().qlc_encode_sym(_p(x), n, symbol_bits, _p(table), chunk_symbols, _p(bits_out),
                                _nbytes(bits_out), _p(index_out), _p(total_out), _p(err_out),
                                _p(ws), _nbytes(ws), _stream(stream)), "qlc_encode_sym")


def qlc_decode_sym(bits: torch.Tensor, total: torch.Tensor, index: torch.Tensor,
                   chunk_symbols: int, table: torch.Tensor, n: int, symbol_bits: int,
                   out: torch.Tensor, err_out: torch.Tensor, ws: torch.Tensor, stream=None):
    _check(lib().qlc_decode_sym(_p(bits), _p(total), _p(index), chunk_symbols, _p(table), n,
                                symbol_bits, _p(out), _p(err_out), _p(ws), _nbytes(ws),
                                _stream(stream)), "qlc_decode_sym")


def qlc_decoder_choice(n: int, chunk_symbols: int) -> int:
    """The decoder DECODER_AUTO takes for n symbols at chunk size C."""
    return int(lib().qlc_decoder_choice(n, chunk_symbols))


def qlc_decode_ex(bits: torch.Tensor, total: torch.Tensor, index: torch.Tensor,
                  chunk_symbols: int, table: torch.Tensor, n: int, symbol_bits: int, decoder: int,
                  out: torch.Tensor, err_out: torch.Tensor, ws: torch.Tensor, stream=None):
    _check(lib().qlc_decode_ex(_p(bits), _p(total), _p(index), chunk_symbols, _p(table), n,
                               symbol_bits, decoder, _p(out), _p(err_out), _p(ws), _nbytes(ws),
                               _stream(stream)), "qlc_decode_ex")


def qlc_encode_batched_sym(jobs: torch.Tensor, n_jobs: int, symbol_bits: int, mode: int,
                           chunk_symbols: int, ws: torch.Tensor, tuning=None, stream=None):
    keep, tp = _tuning_ptr(tuning)
    _check(lib().qlc_encode_batched_sym(_p(jobs), n_jobs, symbol_bits, mode, chunk_symbols, tp,
                                        _p(ws), _nbytes(ws), _stream(stream)),
           "qlc_encode_batched_sym")


def qlc_decode_batched_sym(jobs: torch.Tensor, n_jobs: int, symbol_bits: int,
                           chunk_symbols: int, ws: torch.Tensor, tuning=None, stream=None):
    keep, tp = _tuning_ptr(tuning)
    _check(lib().qlc_decode_batched_sym(_p(jobs), n_jobs, symbol_bits, chunk_symbols, tp,
                                        _p(ws), _nbytes(ws), _stream(stream)),
           "qlc_decode_batched_sym")


def _tuning_ptr(tuning):
    if tuning is None:
        return None, 0
    if not isinstance(tuning, BatchTuning):
        tuning = BatchTuning(*tuning)
    return tuning, ctypes.addressof(tuning)


def qlc_batched_workspace_bytes(n_jobs: int, total_symbols: int, chunk_symbols: int,
                                tuning=None) -> int:
    keep, tp = _tuning_ptr(tuning)
    return int(lib().qlc_batched_workspace_bytes(n_jobs, total_symbols, chunk_symbols, tp))


def qlc_encode_batched(jobs: torch.Tensor, n_jobs: int, mode: int, chunk_symbols: int,
                       ws: torch.Tensor, tuning=None, stream=None):
    """jobs: device tensor holding n_jobs qlc_job records."""
    keep, tp = _tuning_ptr(tuning)
    _check(lib().qlc_encode_batched(_p(jobs), n_jobs, mode, chunk_symbols, tp, _p(ws), _nbytes(ws),
                                    _stream(stream)), "qlc_encode_batched")


def qlc_decode_batched(jobs: torch.Tensor, n_jobs: int, chunk_symbols: int, ws: torch.Tensor,
                       tuning=None, stream=None):
    keep, tp = _tuning_ptr(tuning)
    _check(lib().qlc_decode_batched(_p(jobs), n_jobs, chunk_symbols, tp, _p(ws), _nbytes(ws),
                                    _stream(stream)), "qlc_decode_batched")


def qlc_table_serialize(table_host: bytes | np.ndarray) -> bytes:
    t = np.frombuffer(bytes(table_host), dtype=np.uint8).copy()
    out = np.zeros(SERIALIZED_TABLE_BYTES, dtype=np.uint8)
    _check(lib().qlc_table_serialize(t.ctypes.data, out.ctypes.data), "qlc_table_serialize")
    return out.tobytes()


def qlc_table_deserialize(blob: bytes) -> bytes:
    b = np.frombuffer(bytes(blob), dtype=np.uint8).copy()
    if b.size != SERIALIZED_TABLE_BYTES:
        raise QLCError(QLC_ERR_INVALID_ARGUMENT, "qlc_table_deserialize")
    out = np.zeros(TABLE_BYTES, dtype=np.uint8)
    _check(lib().qlc_table_deserialize(b.ctypes.data, out.ctypes.data), "qlc_table_deserialize")
    return out.tobytes()


# ------------------------------------------------------------ helpers
def parse_table(raw) -> dict:
    """Decode the 1088 table bytes (host bytes or a device tensor) into numpy arrays."""
    if isinstance(raw, torch.Tensor):
        raw = raw.detach().cpu().numpy().tobytes()
    t = _Table.from_buffer_copy(bytes(raw))
    return dict(
        enc=np.array(t.enc, dtype=np.int64), rank_to_sym=np.array(t.rank_to_sym, dtype=np.int64),
        sym_to_rank=np.array(t.sym_to_rank, dtype=np.int64), width=np.array(t.width, np.int64),
        offset=np.array(t.offset, np.int64), first=np.array(t.first, np.int64),
        count=np.array(t.count, np.int64), cost_bits=int(t.cost_bits), mode=int(t.mode),
        version=int(t.version))


def new_table(device="cuda") -> torch.Tensor:
    return torch.zeros(TABLE_BYTES, dtype=torch.uint8, device=device)


def new_workspace(n: int, chunk_symbols: int = 4096, device="cuda") -> torch.Tensor:
    """A zeroed workspace (torch allocations are 256-byte aligned)."""
    return torch.zeros(qlc_workspace_bytes(n, chunk_symbols), dtype=torch.uint8, device=device)


class Compressed:
    """Device-resident compressed object: table, bitstream, chunk index."""

    def __init__(self, n, chunk_symbols, table, bits, index, total, err):
        self.n, self.chunk_symbols = n, chunk_symbols
        self.table, self.bits, self.index, self.total, self.err = table, bits, index, total, err

    def total_bits(self) -> int:
        return int(self.total.item())

    def nbytes(self) -> int:
        return 4 * ((self.total_bits() + 31) // 32)


def compress(x: torch.Tensor, mode: int = LAYOUT_SEARCH_QUAD, chunk_symbols: int = 4096,
             table: torch.Tensor | None = None, ws: torch.Tensor | None = None,
             capacity: int | None = None) -> Compressed:
    """Histogram + table (unless `table` is given) + encode, on the current stream."""
    x = x.reshape(-1)
    n = x.numel()
    dev = x.device
    ws = new_workspace(n, chunk_symbols, dev) if ws is None else ws
    cap = qlc_encode_bound_bytes(n) if capacity is None else capacity
    bits = torch.empty(max(cap, 16), dtype=torch.uint8, device=dev)[:cap]
    index = torch.empty(max(qlc_chunk_count(n, chunk_symbols), 1), dtype=torch.int64, device=dev)
    total = torch.empty(1, dtype=torch.int64, device=dev)
    err = torch.empty(1, dtype=torch.int32, device=dev)
    if table is None:
        table = new_table(dev)
        qlc_compress(x, mode, table, chunk_symbols, bits, index, total, err, ws)
    else:
        qlc_encode(x, table, chunk_symbols, bits, index, total, err, ws)
    return Compressed(n, chunk_symbols, table, bits, index, total, err)


def decompress(c: Compressed, out: torch.Tensor | None = None, ws: torch.Tensor | None = None,
               decoder: int = DECODER_AUTO):
    dev = c.bits.device
    out = torch.empty(max(c.n, 16), dtype=torch.uint8, device=dev)[:c.n] if out is None else out
    err = torch.empty(1, dtype=torch.int32, device=dev)
    ws = new_workspace(0, c.chunk_symbols, dev) if ws is None else ws
    qlc_decode_ex(c.bits, c.total, c.index, c.chunk_symbols, c.table, c.n, 8, decoder, out, err,
                  ws)
    return out, err


# ------------------------------------------------------------ batches
def _align(x: int, a: int = 256) -> int:
    return (x + a - 1) // a * a


class Batch:
    """Device buffers of a batch of tensors, carved from a few pooled
    allocations (256-byte aligned slices), and the device array of qlc_job
    records that points into them.

    capacity: "search" (n + 16 bytes of bitstream per tensor: enough for any
    table a SEARCH mode builds from the tensor's own histogram, whose cost
    never exceeds 8 bits per symbol) or "bound" (qlc_encode_bound_bytes).
    """

    def __init__(self, sizes, chunk_symbols: int = 4096, device="cuda", capacity="search",
                 build_table: bool = True, min_chunk: int | None = None,
                 inp: torch.Tensor | None = None):
        self.sizes = [int(v) for v in sizes]
        self.S = len(self.sizes)
        self.C = chunk_symbols
        # chunk indexes are sized for min_chunk, so any C >= min_chunk fits
        self.min_chunk = chunk_symbols if min_chunk is None else min(min_chunk, chunk_symbols)
        self.device = torch.device(device)
        self.in_off, self.bits_off, self.idx_off, self.cap = [], [], [], []
        oi = ob = ox = 0
        for n in self.sizes:
            cap = _align(n + 16, 16) if capacity == "search" else qlc_encode_bound_bytes(n)
            self.in_off.append(oi)
            self.bits_off.append(ob)
            self.idx_off.append(ox)
            self.cap.append(cap)
            oi += _align(max(n, 1))
            ob += _align(max(cap, 16))
            ox += _align(max(qlc_chunk_count(n, self.min_chunk), 1), 32)
        dev = self.device
        if inp is not None:
            assert inp.dtype == torch.uint8 and inp.numel() >= oi and inp.data_ptr() % 256 == 0
            self.inp = inp
        else:
            self.inp = torch.zeros(max(oi, 256), dtype=torch.uint8, device=dev)
        self.out = torch.zeros(max(oi, 256), dtype=torch.uint8, device=dev)
        self.bits = torch.zeros(max(ob, 256), dtype=torch.uint8, device=dev)
        self.index = torch.zeros(max(ox, 32), dtype=torch.int64, device=dev)
        self.tables = torch.zeros(self.S * TABLE_BYTES, dtype=torch.uint8, device=dev)
        self.total = torch.zeros(self.S, dtype=torch.int64, device=dev)
        self.err = torch.zeros(self.S, dtype=torch.int32, device=dev)
        self.build_table = build_table
        self.jobs_host = (Job * self.S)()
        self._fill_jobs()
        self.jobs = torch.frombuffer(bytearray(self.jobs_host), dtype=torch.uint8).to(dev)

    def _fill_jobs(self):
        for i, n in enumerate(self.sizes):
            j = self.jobs_host[i]
            j.in_ = self.inp.data_ptr() + self.in_off[i]
            j.out = self.out.data_ptr() + self.in_off[i]
            j.n = n
            j.table = self.tables.data_ptr() + i * TABLE_BYTES
            j.bits = self.bits.data_ptr() + self.bits_off[i]
            j.bits_capacity = self.cap[i]
            j.chunk_index = self.index.data_ptr() + 8 * self.idx_off[i]
            j.total_bits = self.total.data_ptr() + 8 * i
            j.err = self.err.data_ptr() + 4 * i
            j.build_table = 1 if self.build_table else 0
            j.reserved = 0

    def upload_jobs(self):
        """Copy the (edited) host job records to the device array."""
        self.jobs.copy_(torch.frombuffer(bytearray(self.jobs_host), dtype=torch.uint8))

    @property
    def total_symbols(self) -> int:
        return sum(self.sizes)

    def workspace(self, tuning=None) -> torch.Tensor:
        b = qlc_batched_workspace_bytes(self.S, self.total_symbols, self.C, tuning)
        return torch.zeros(max(b, 256), dtype=torch.uint8, device=self.device)

    def input(self, i: int) -> torch.Tensor:
        return self.inp[self.in_off[i]:self.in_off[i] + self.sizes[i]]

    def output(self, i: int) -> torch.Tensor:
        return self.out[self.in_off[i]:self.in_off[i] + self.sizes[i]]

    def table(self, i: int) -> torch.Tensor:
        return self.tables[i * TABLE_BYTES:(i + 1) * TABLE_BYTES]

    def bitstream(self, i: int, nbytes: int | None = None) -> torch.Tensor:
        nb = self.cap[i] if nbytes is None else nbytes
        return self.bits[self.bits_off[i]:self.bits_off[i] + nb]

    def chunk_index(self, i: int, whole: bool = False) -> torch.Tensor:
        """Job i's index entries at the current C (whole: its whole slot)."""
        k = qlc_chunk_count(self.sizes[i], self.min_chunk if whole else self.C)
        return self.index[self.idx_off[i]:self.idx_off[i] + max(k, 1 if whole else 0)]

    def set_chunk(self, chunk_symbols: int):
        assert chunk_symbols >= self.min_chunk
        self.C = chunk_symbols

    def encode(self, ws: torch.Tensor, mode: int = LAYOUT_SEARCH_QUAD, tuning=None, stream=None):
        qlc_encode_batched(self.jobs, self.S, mode, self.C, ws, tuning, stream)

    def decode(self, ws: torch.Tensor, tuning=None, stream=None):
        qlc_decode_batched(self.jobs, self.S, self.C, ws, tuning, stream)


# ------------------------------------------------------------ serving
REQUEST_COMPRESS = 0
REQUEST_DECOMPRESS = 1


class ServerConfig(ctypes.Structure):
    _fields_ = [("memory_budget_bytes", ctypes.c_uint64), ("max_tick_symbols", ctypes.c_uint64),
                ("chunk_symbols", ctypes.c_uint32), ("layout_mode", ctypes.c_uint32),
                ("max_jobs_per_tick", ctypes.c_uint32), ("max_ticks_in_flight", ctypes.c_uint32),
                ("log2_segment", ctypes.c_uint32), ("decoder", ctypes.c_uint32)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("n", ctypes.c_uint64),
                ("in_", ctypes.c_void_p), ("table", ctypes.c_void_p), ("bits", ctypes.c_void_p),
                ("chunk_index", ctypes.c_void_p), ("total_bits", ctypes.c_void_p),
                ("user_tag", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("user_tag", ctypes.c_uint64), ("kind", ctypes.c_uint32),
                ("status", ctypes.c_uint32), ("n", ctypes.c_uint64),
                ("total_bits", ctypes.c_uint64), ("table", ctypes.c_void_p),
                ("bits", ctypes.c_void_p), ("chunk_index", ctypes.c_void_p),
                ("total_bits_dev", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("submit_ns", ctypes.c_uint64), ("admit_ns", ctypes.c_uint64),
                ("complete_ns", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("bytes_in_use", ctypes.c_uint64),
                ("peak_bytes_in_use", ctypes.c_uint64), ("submitted", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("ticks", ctypes.c_uint64), ("max_jobs_in_tick", ctypes.c_uint32),
                ("max_ticks_in_flight", ctypes.c_uint32), ("queued", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


assert ctypes.sizeof(ServerConfig) == 40 and ctypes.sizeof(Request) == 64
assert ctypes.sizeof(Result) == 104 and ctypes.sizeof(ServerStats) == 72

_SIGNATURES.update({
    "qlc_server_create": ([_vp, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "qlc_server_submit": ([_vp, _vp, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "qlc_server_poll": ([_vp, _vp, _u32, ctypes.c_int64], _u32),
    "qlc_server_release": ([_vp, _u64], ctypes.c_int),
    "qlc_server_get_stats": ([_vp, _vp], ctypes.c_int),
    "qlc_server_destroy": ([_vp], ctypes.c_int),
})


def device_copy(ptr: int, nbytes: int, device="cuda") -> torch.Tensor:
    """A new uint8 tensor holding `nbytes` of device memory at `ptr` (server
    results live in the server's pool); the copy runs on the current stream."""
    out = torch.empty(nbytes, dtype=torch.uint8, device=device)
    if nbytes:
        _hip_memcpy_d2d(out.data_ptr(), ptr, nbytes)
    return out


def _hip_memcpy_d2d(dst: int, src: int, nbytes: int):
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.argtypes = [_vp, _vp, _sz, ctypes.c_int, _vp]
        _hip.hipMemcpyAsync.restype = ctypes.c_int
    rc = _hip.hipMemcpyAsync(dst, src, nbytes, 3, _stream(None))  # device to device
    if rc != 0:
        raise QLCError(QLC_ERR_HIP, "hipMemcpyAsync")


_hip = None


class Server:
    """The serving loop of libqlc (qlc_server_*): submit compress /
    decompress requests, poll completions, release their outputs."""

    def __init__(self, memory_budget_bytes: int, chunk_symbols: int = 4096,
                 layout_mode: int = LAYOUT_SEARCH_QUAD, max_jobs_per_tick: int = 0,
                 max_ticks_in_flight: int = 0, log2_segment: int = 0, max_tick_symbols: int = 0,
                 decoder: int = DECODER_AUTO):
        lib()
        cfg = ServerConfig(memory_budget_bytes, max_tick_symbols, chunk_symbols, layout_mode,
                           max_jobs_per_tick, max_ticks_in_flight, log2_segment, decoder)
        h = ctypes.c_void_p()
        _check(_lib.qlc_server_create(ctypes.addressof(cfg), ctypes.byref(h)), "qlc_server_create")
        self._h = h
        self.chunk_symbols = chunk_symbols

    def submit_compress(self, x: torch.Tensor, table: torch.Tensor | None = None,
                        user_tag: int = 0, n: int | None = None) -> int:
        n = x.numel() if n is None else n
        r = Request(REQUEST_COMPRESS, 0, n, _p(x), _p(table), 0, 0, 0, user_tag)
        return self._submit(r)

    def submit_decompress(self, n: int, bits, index, total, table, user_tag: int = 0) -> int:
        r = Request(REQUEST_DECOMPRESS, 0, n, 0, _p(table), _p(bits), _p(index), _p(total),
                    user_tag)
        return self._submit(r)

    def _submit(self, r: Request) -> int:
        rid = ctypes.c_uint64()
        _check(_lib.qlc_server_submit(self._h, ctypes.addressof(r), ctypes.byref(rid)),
               "qlc_server_submit")
        return int(rid.value)

    def poll(self, max_results: int = 64, timeout_us: int = 0) -> list:
        buf = (Result * max_results)()
        k = _lib.qlc_server_poll(self._h, ctypes.addressof(buf), max_results, timeout_us)
        return [buf[i] for i in range(k)]

    def release(self, rid: int):
        _check(_lib.qlc_server_release(self._h, rid), "qlc_server_release")

    def stats(self) -> ServerStats:
        st = ServerStats()
        _check(_lib.qlc_server_get_stats(self._h, ctypes.addressof(st)), "qlc_server_get_stats")
        return st

    def close(self):
        if self._h:
            _check(_lib.qlc_server_destroy(self._h), "qlc_server_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
