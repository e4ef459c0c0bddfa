"""CPU oracle for Quad Length Codes (arXiv 2602.17849).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the GPU library never does,
and this package never imports the GPU library.  The arithmetic lives in
plain C (qlc_oracle.c, built with gcc into liboracle_qlc.so); this module
only marshals numpy arrays into it.  Bounds (entropy, Huffman) are in
bounds.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qlc_oracle.c")
_SRC_MT = os.path.join(_HERE, "qlc_oracle_mt.c")
_LIB_PATH = os.path.join(_HERE, "liboracle_qlc.so")

MODE_SEARCH_QUAD = 0
MODE_SEARCH_ANY = 1
MODE_PAPER_T1 = 2
MODE_PAPER_T2 = 3

OK = 0
ERR_INVALID_ARGUMENT = 1
ERR_CAPACITY = 2
ERR_CORRUPT_STREAM = 3

_MAX_AREAS = 16
_MAX_SYMBOLS = 256


class _Table(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_uint32),
        ("A", ctypes.c_uint32),
        ("prefix_bits", ctypes.c_uint32),
        ("symbol_bits", ctypes.c_uint32),
        ("width", ctypes.c_uint32 * _MAX_AREAS),
        ("first", ctypes.c_uint32 * _MAX_AREAS),
        ("count", ctypes.c_uint32 * _MAX_AREAS),
        ("offset", ctypes.c_uint32 * _MAX_AREAS),
        ("rank_to_sym", ctypes.c_uint32 * _MAX_SYMBOLS),
        ("sym_to_rank", ctypes.c_uint32 * _MAX_SYMBOLS),
        ("code", ctypes.c_uint32 * _MAX_SYMBOLS),
        ("len", ctypes.c_uint32 * _MAX_SYMBOLS),
        ("cost_bits", ctypes.c_uint64),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, -O2, no vectorisation tricks;
    OpenMP for the multi-threaded variants)."""
    srcs = [_SRC, _SRC_MT, os.path.join(_HERE, "qlc_oracle.h")]
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < max(os.path.getmtime(p) for p in srcs)):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-fopenmp",
             _SRC, _SRC_MT, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        tp = ctypes.POINTER(_Table)
        L.qref_histogram.argtypes = [u8p, ctypes.c_uint64, u64p]
        L.qref_histogram.restype = None
        L.qref_rank.argtypes = [u64p, ctypes.c_uint32, u32p, u32p]
        L.qref_rank.restype = None
        L.qref_fill.argtypes = [ctypes.c_uint32, ctypes.c_uint32, u32p, u32p, u32p]
        L.qref_fill.restype = ctypes.c_int
        L.qref_enumerate.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                     u32p, ctypes.c_int64]
        L.qref_enumerate.restype = ctypes.c_int64
        L.qref_cost.argtypes = [u64p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, u32p]
        L.qref_cost.restype = ctypes.c_uint64
        L.qref_search.argtypes = [u64p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_uint32, u32p]
        L.qref_search.restype = ctypes.c_int64
        L.qref_build_table_general.argtypes = [u64p, ctypes.c_uint32, ctypes.c_uint32,
                                               ctypes.c_uint32, ctypes.c_uint32, u32p, tp]
        L.qref_build_table_general.restype = ctypes.c_int
        L.qref_build_table.argtypes = [u64p, ctypes.c_int, tp]
        L.qref_build_table.restype = ctypes.c_int
        L.qref_table_from_layout.argtypes = [u32p, u32p, tp]
        L.qref_table_from_layout.restype = ctypes.c_int
        L.qref_encode.argtypes = [u8p, ctypes.c_uint64, tp, ctypes.c_uint32, u8p,
                                  ctypes.c_uint64, u64p, u64p]
        L.qref_encode.restype = ctypes.c_int
        L.qref_encoded_bits.argtypes = [u8p, ctypes.c_uint64, tp]
        L.qref_encoded_bits.restype = ctypes.c_uint64
        L.qref_decode.argtypes = [u8p, ctypes.c_uint64, u64p, ctypes.c_uint32, tp,
                                  ctypes.c_uint64, u8p]
        L.qref_decode.restype = ctypes.c_int
        L.qref_histogram_mt.argtypes = [u8p, ctypes.c_uint64, u64p, ctypes.c_int]
        L.qref_histogram_mt.restype = None
        L.qref_encode_mt.argtypes = [u8p, ctypes.c_uint64, tp, ctypes.c_uint32, u8p,
                                     ctypes.c_uint64, u64p, u64p, ctypes.c_int]
        L.qref_encode_mt.restype = ctypes.c_int
        L.qref_decode_mt.argtypes = [u8p, ctypes.c_uint64, u64p, ctypes.c_uint32, tp,
                                     ctypes.c_uint64, u8p, ctypes.c_int]
        L.qref_decode_mt.restype = ctypes.c_int
        L.qref_mt_threads.argtypes = [ctypes.c_int]
        L.qref_mt_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


@dataclass
class Table:
    """Oracle table as numpy arrays (one row per area / symbol)."""
    M: int
    A: int
    prefix_bits: int
    width: np.ndarray
    first: np.ndarray
    count: np.ndarray
    offset: np.ndarray
    rank_to_sym: np.ndarray
    sym_to_rank: np.ndarray
    code: np.ndarray
    len: np.ndarray
    cost_bits: int
    _raw: _Table

    @staticmethod
    def _from_raw(t: _Table) -> "Table":
        A, M = t.A, t.M
        return Table(
            M=M, A=A, prefix_bits=t.prefix_bits,
            width=np.array(t.width[:A], dtype=np.int64),
            first=np.array(t.first[:A], dtype=np.int64),
            count=np.array(t.count[:A], dtype=np.int64),
            offset=np.array(t.offset[:A], dtype=np.int64),
            rank_to_sym=np.array(t.rank_to_sym[:M], dtype=np.int64),
            sym_to_rank=np.array(t.sym_to_rank[:M], dtype=np.int64),
            code=np.array(t.code[:M], dtype=np.int64),
            len=np.array(t.len[:M], dtype=np.int64),
            cost_bits=int(t.cost_bits), _raw=t)

    def code_string(self, sym: int) -> str:
        """Code of an input symbol as a bit string, area code first."""
        l = int(self.len[sym])
        return format(int(self.code[sym]), "0%db" % l) if l else ""


def histogram(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.uint8).reshape(-1)
    h = np.zeros(256, dtype=np.uint64)
    lib().qref_histogram(_ptr(x, ctypes.c_uint8), x.size, _ptr(h, ctypes.c_uint64))
    return h


def rank(h, M: int = 256):
    h = np.ascontiguousarray(h, dtype=np.uint64)
    r2s = np.zeros(M, dtype=np.uint32)
    s2r = np.zeros(M, dtype=np.uint32)
    lib().qref_rank(_ptr(h, ctypes.c_uint64), M, _ptr(r2s, ctypes.c_uint32),
                    _ptr(s2r, ctypes.c_uint32))
    return r2s.astype(np.int64), s2r.astype(np.int64)


def fill(widths, M: int = 256):
    w = np.ascontiguousarray(widths, dtype=np.uint32)
    A = w.size
    first = np.zeros(A, dtype=np.uint32)
    count = np.zeros(A, dtype=np.uint32)
    ok = lib().qref_fill(M, A, _ptr(w, ctypes.c_uint32), _ptr(first, ctypes.c_uint32),
                         _ptr(count, ctypes.c_uint32))
    return bool(ok), first.astype(np.int64), count.astype(np.int64)


def enumerate_layouts(M: int = 256, A: int = 8, max_distinct: int = 8) -> np.ndarray:
    n = lib().qref_enumerate(M, A, max_distinct, None, 0)
    out = np.zeros((max(n, 1), A), dtype=np.uint32)
    lib().qref_enumerate(M, A, max_distinct, _ptr(out, ctypes.c_uint32), n)
    return out[:n].astype(np.int64)


def cost(ranked_counts, widths, M: int = 256, prefix_bits: int = 3) -> int:
    rc = np.ascontiguousarray(ranked_counts, dtype=np.uint64)
    w = np.ascontiguousarray(widths, dtype=np.uint32)
    return int(lib().qref_cost(_ptr(rc, ctypes.c_uint64), M, w.size, prefix_bits,
                               _ptr(w, ctypes.c_uint32)))


def search(ranked_counts, M: int = 256, A: int = 8, prefix_bits: int = 3,
           max_distinct: int = 4):
    rc = np.ascontiguousarray(ranked_counts, dtype=np.uint64)
    w = np.zeros(A, dtype=np.uint32)
    idx = lib().qref_search(_ptr(rc, ctypes.c_uint64), M, A, prefix_bits, max_distinct,
                            _ptr(w, ctypes.c_uint32))
    return int(idx), w.astype(np.int64)


def build_table(h, mode: int = MODE_SEARCH_QUAD) -> Table:
    h = np.ascontiguousarray(h, dtype=np.uint64)
    t = _Table()
    st = lib().qref_build_table(_ptr(h, ctypes.c_uint64), mode, ctypes.byref(t))
    if st != OK:
        raise ValueError("qref_build_table failed with status %d" % st)
    return Table._from_raw(t)


def build_table_general(h, M: int, A: int, prefix_bits: int, max_distinct: int,
                        widths=None) -> Table:
    h = np.ascontiguousarray(h, dtype=np.uint64)
    t = _Table()
    wp = None
    if widths is not None:
        w = np.ascontiguousarray(widths, dtype=np.uint32)
        wp = _ptr(w, ctypes.c_uint32)
    st = lib().qref_build_table_general(_ptr(h, ctypes.c_uint64), M, A, prefix_bits,
                                        max_distinct, wp, ctypes.byref(t))
    if st != OK:
        raise ValueError("qref_build_table_general failed with status %d" % st)
    return Table._from_raw(t)


def table_from_layout(widths, rank_to_sym) -> Table:
    w = np.ascontiguousarray(widths, dtype=np.uint32)
    r = np.ascontiguousarray(rank_to_sym, dtype=np.uint32)
    t = _Table()
    st = lib().qref_table_from_layout(_ptr(w, ctypes.c_uint32), _ptr(r, ctypes.c_uint32),
                                      ctypes.byref(t))
    if st != OK:
        raise ValueError("invalid layout (status %d)" % st)
    return Table._from_raw(t)


def chunk_count(n: int, C: int) -> int:
    return (n + C - 1) // C


def encoded_bits(x: np.ndarray, table: Table) -> int:
    x = np.ascontiguousarray(x, dtype=np.uint8).reshape(-1)
    return int(lib().qref_encoded_bits(_ptr(x, ctypes.c_uint8), x.size,
                                       ctypes.byref(table._raw)))


def encode(x: np.ndarray, table: Table, chunk_symbols: int = 4096, cap_bytes=None):
    """Returns (status, bits uint8[4*ceil(total/32)], index uint64[ceil(n/C)], total_bits)."""
    x = np.ascontiguousarray(x, dtype=np.uint8).reshape(-1)
    n = x.size
    total = encoded_bits(x, table)
    nbytes = 4 * ((total + 31) // 32)
    if cap_bytes is None:
        cap_bytes = nbytes
    bits = np.zeros(max(cap_bytes, 1), dtype=np.uint8)
    index = np.zeros(max(chunk_count(n, chunk_symbols), 1), dtype=np.uint64)
    tb = np.zeros(1, dtype=np.uint64)
    st = lib().qref_encode(_ptr(x, ctypes.c_uint8), n, ctypes.byref(table._raw),
                           chunk_symbols, _ptr(bits, ctypes.c_uint8), cap_bytes,
                           _ptr(index, ctypes.c_uint64), _ptr(tb, ctypes.c_uint64))
    return (int(st), bits[:nbytes] if st == OK else bits[:0],
            index[:chunk_count(n, chunk_symbols)], int(tb[0]))


def decode(bits: np.ndarray, total_bits: int, index: np.ndarray, chunk_symbols: int,
           table: Table, n: int):
    """Returns (status, out uint8[n])."""
    b = np.ascontiguousarray(bits, dtype=np.uint8).reshape(-1)
    if total_bits > 8 * b.size:
        raise ValueError("bitstream buffer shorter than total_bits")
    if b.size == 0:
        b = np.zeros(4, dtype=np.uint8)
    idx = np.ascontiguousarray(index, dtype=np.uint64).reshape(-1)
    if idx.size == 0:
        idx = np.zeros(1, dtype=np.uint64)
    out = np.zeros(max(n, 1), dtype=np.uint8)
    st = lib().qref_decode(_ptr(b, ctypes.c_uint8), total_bits, _ptr(idx, ctypes.c_uint64),
                           chunk_symbols, ctypes.byref(table._raw), n,
                           _ptr(out, ctypes.c_uint8))
    return int(st), out[:n]


# ------------------------------------------------------------------ threads
def mt_threads(threads: int = 0) -> int:
    """Threads the multi-threaded oracle runs with (0: OpenMP's default,
    i.e. every host core unless OMP_NUM_THREADS says otherwise)."""
    return int(lib().qref_mt_threads(threads))


def histogram_mt(x: np.ndarray, threads: int = 0) -> np.ndarray:
    """histogram() over contiguous slices in parallel (same counts)."""
    x = np.ascontiguousarray(x, dtype=np.uint8).reshape(-1)
    h = np.zeros(256, dtype=np.uint64)
    lib().qref_histogram_mt(_ptr(x, ctypes.c_uint8), x.size, _ptr(h, ctypes.c_uint64), threads)
    return h


def encode_mt(x: np.ndarray, table: Table, chunk_symbols: int = 4096, cap_bytes=None,
              threads: int = 0):
    """encode() over ranges of whole chunks in parallel (same bytes)."""
    x = np.ascontiguousarray(x, dtype=np.uint8).reshape(-1)
    n = x.size
    total = encoded_bits(x, table) if cap_bytes is None else 0
    nbytes = 4 * ((total + 31) // 32)
    if cap_bytes is None:
        cap_bytes = nbytes
    bits = np.empty(max(cap_bytes, 1), dtype=np.uint8)
    index = np.zeros(max(chunk_count(n, chunk_symbols), 1), dtype=np.uint64)
    tb = np.zeros(1, dtype=np.uint64)
    st = lib().qref_encode_mt(_ptr(x, ctypes.c_uint8), n, ctypes.byref(table._raw),
                              chunk_symbols, _ptr(bits, ctypes.c_uint8), cap_bytes,
                              _ptr(index, ctypes.c_uint64), _ptr(tb, ctypes.c_uint64), threads)
    nbytes = 4 * ((int(tb[0]) + 31) // 32)
    return (int(st), bits[:nbytes] if st == OK else bits[:0],
            index[:chunk_count(n, chunk_symbols)], int(tb[0]))


def decode_mt(bits: np.ndarray, total_bits: int, index: np.ndarray, chunk_symbols: int,
              table: Table, n: int, threads: int = 0):
    """decode() over ranges of whole chunks in parallel (same status and,
    on success, the same bytes)."""
    b = np.ascontiguousarray(bits, dtype=np.uint8).reshape(-1)
    if total_bits > 8 * b.size:
        raise ValueError("bitstream buffer shorter than total_bits")
    if b.size == 0:
        b = np.zeros(4, dtype=np.uint8)
    idx = np.ascontiguousarray(index, dtype=np.uint64).reshape(-1)
    if idx.size == 0:
        idx = np.zeros(1, dtype=np.uint64)
    out = np.zeros(max(n, 1), dtype=np.uint8)
    st = lib().qref_decode_mt(_ptr(b, ctypes.c_uint8), total_bits, _ptr(idx, ctypes.c_uint64),
                              chunk_symbols, ctypes.byref(table._raw), n,
                              _ptr(out, ctypes.c_uint8), threads)
    return int(st), out[:n]
