"""Seeded synthetic e4m3 workloads (inputs only: no QLC arithmetic here).

The paper measures block-32 quantised e4m3 tensors of Gemma-2B fine-tuning
(Experimental Setup section); those tensors are not available, so every
workload is synthetic with the shapes and value distributions below:

* ``gaussian``      FP32 ~ N(0, 1)
* ``laplace``       FP32 ~ Laplace(0, 1), 1 % of the rows scaled x8
                    (outlier channels), like FFN1 activations
* ``student_t``     FP32 ~ Student-t(nu = 3), like gradients
* ``weights``       FP32 ~ N(0, 0.02)

Each FP32 tensor is quantised in contiguous blocks of 32 values with a
power-of-two shared scale 2^ceil(log2(maxabs / 448)) (an all-zero block uses
scale 1) and rounded to nearest-even e4m3 (``torch.float8_e4m3fn``).  With
that scale no block value exceeds 448, so the NaN encodings 0x7F / 0xFF are
never produced: the "all 256 codes finite" eXmY e4m3 and the OCP e4m3
variants yield identical bytes.

Random numbers come from ``torch.Generator`` seeded per workload; the same
seed on the same device type gives the same bytes.  This module is shared
by the tests, the benchmark and the smoke check: it feeds identical bytes to
the GPU library and to the CPU oracle.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np
import torch

E4M3_MAX = 448.0
BLOCK = 32


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def quantize_e4m3_block32(x: torch.Tensor) -> torch.Tensor:
    """FP32 tensor (numel a multiple of 32) -> uint8 e4m3 codes, same device."""
    flat = x.reshape(-1, BLOCK).to(torch.float32)
    maxabs = flat.abs().amax(dim=1)
    # smallest k with maxabs <= 448 * 2^k, computed exactly via frexp
    v = maxabs.to(torch.float64) / E4M3_MAX
    mant, expo = torch.frexp(v)
    k = expo.to(torch.int32) - (mant == 0.5).to(torch.int32)
    k = torch.where(maxabs > 0, k, torch.zeros_like(k))
    y = torch.ldexp(flat, (-k).to(torch.float32).unsqueeze(1))
    return y.to(torch.float8_e4m3fn).view(torch.uint8).reshape(-1)


def _laplace(shape, g, device):
    e1 = torch.empty(shape, device=device, dtype=torch.float32).exponential_(1.0, generator=g)
    e2 = torch.empty(shape, device=device, dtype=torch.float32).exponential_(1.0, generator=g)
    return e1 - e2


def _student_t3(shape, g, device):
    z = torch.randn(shape, device=device, generator=g)
    chi = torch.zeros(shape, device=device)
    for _ in range(3):
        chi += torch.randn(shape, device=device, generator=g).square()
    return z / torch.sqrt(chi / 3.0)


def gaussian(numel: int, seed: int, device="cpu", std: float = 1.0) -> torch.Tensor:
    g = _gen(seed, device)
    return quantize_e4m3_block32(torch.randn(numel, device=device, generator=g) * std)


def laplace_outlier_rows(rows: int, cols: int, seed: int, device="cpu",
                         outlier_frac: float = 0.01, outlier_scale: float = 8.0) -> torch.Tensor:
    """Laplace(0,1) matrix with round(outlier_frac * rows) rows scaled."""
    g = _gen(seed, device)
    x = _laplace((rows, cols), g, device)
    n_out = int(round(outlier_frac * rows))
    if n_out:
        perm = torch.randperm(rows, generator=g, device=device)[:n_out]
        x[perm] *= outlier_scale
    return quantize_e4m3_block32(x)


def student_t(numel: int, seed: int, device="cpu") -> torch.Tensor:
    g = _gen(seed, device)
    return quantize_e4m3_block32(_student_t3((numel,), g, device))


def uniform_bytes(numel: int, seed: int, device="cpu") -> torch.Tensor:
    g = _gen(seed, device)
    return torch.randint(0, 256, (numel,), generator=g, device=device,
                         dtype=torch.int32).to(torch.uint8)


def zeros90_gaussian(numel: int, seed: int, device="cpu") -> torch.Tensor:
    """N(0,1) e4m3 with a Bernoulli(0.9) mask of bytes forced to 0x00."""
    g = _gen(seed, device)
    x = quantize_e4m3_block32(torch.randn(numel, device=device, generator=g))
    mask = torch.rand(numel, device=device, generator=g) < 0.9
    return x.masked_fill(mask, 0)


# ---------------------------------------------------------------- workloads
def single_tensor_gaussian(seed: int = 0, rows: int = 1024, cols: int = 1024,
                           device="cpu") -> torch.Tensor:
    """1024 x 1024 N(0,1) block-32 e4m3 (1,048,576 symbols)."""
    return gaussian(rows * cols, seed, device)


def single_tensor_laplace(seed: int = 1, rows: int = 8192, cols: int = 32768,
                          device="cpu") -> torch.Tensor:
    """8192 x 32768 Laplace with 1 % outlier rows (256 MiB of e4m3)."""
    return laplace_outlier_rows(rows, cols, seed, device)


SHARD_KINDS = ("gaussian", "student_t", "weights")


def shard_sizes(n_shards: int = 1152, seed: int = 2, lo: int = 1 << 20,
                hi: int = 32 << 20) -> list[int]:
    """Log-uniform sizes in [lo, hi], multiples of 32 bytes."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), size=n_shards)
    return [int(max(32, 32 * round(math.exp(v) / 32))) for v in u]


def shard(i: int, size: int, seed: int = 2, device="cpu") -> torch.Tensor:
    """Shard i: kind by i mod 3 (activations, gradients, weights)."""
    s = seed * 1_000_003 + i
    kind = SHARD_KINDS[i % 3]
    if kind == "gaussian":
        return gaussian(size, s, device)
    if kind == "student_t":
        return student_t(size, s, device)
    return gaussian(size, s, device, std=0.02)


def serving_requests(duration_s: float = 10.0, rate: float = 2000.0, seed: int = 3,
                     lo: int = 64 << 10, hi: int = 64 << 20):
    """Poisson arrivals: list of (arrival_s, kind, size) with kind in
    {'compress', 'decompress'} 50/50 and log-uniform sizes (multiples of 32)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s:
            break
        kind = "compress" if rng.random() < 0.5 else "decompress"
        size = int(max(32, 32 * round(math.exp(rng.uniform(math.log(lo), math.log(hi))) / 32)))
        out.append((t, kind, size))
    return out


STRESS_KINDS = {"uniform": 4, "zeros90": 5, "ocp_gaussian": 6}


def stress_buffer(kind: str, numel: int = 1 << 32, device="cpu",
                  piece: int = 1 << 28) -> torch.Tensor:
    """The 4 GiB stress buffers, generated in pieces of `piece` symbols
    (piece k of a buffer with seed s uses seed s * 1000 + k):
    ``uniform`` random bytes (seed 4), ``zeros90`` N(0,1) e4m3 with 90 % of
    the bytes forced to 0x00 (seed 5), ``ocp_gaussian`` N(0,1) block-32 e4m3
    under the 448 scale rule (seed 6), which never emits 0x7F / 0xFF."""
    seed = STRESS_KINDS[kind]
    out = torch.empty(numel, dtype=torch.uint8, device=device)
    for k, p0 in enumerate(range(0, numel, piece)):
        m = min(piece, numel - p0)
        m32 = (m + 31) // 32 * 32          # whole quantisation blocks
        s = seed * 1000 + k
        if kind == "uniform":
            out[p0:p0 + m] = uniform_bytes(m32, s, device)[:m]
        elif kind == "zeros90":
            out[p0:p0 + m] = zeros90_gaussian(m32, s, device)[:m]
        else:
            out[p0:p0 + m] = gaussian(m32, s, device)[:m]
    return out


def sha256(x: torch.Tensor) -> str:
    return hashlib.sha256(x.detach().cpu().contiguous().numpy().tobytes()).hexdigest()


# ------------------------------------------------------- packed small symbols
def pack_symbols(codes: np.ndarray, bits: int) -> np.ndarray:
    """Pack symbols of `bits` bits (4 or 6; 8 returns a copy) into bytes in
    little-endian bit order: symbol i occupies bits bits*i .. bits*i + bits - 1
    of the byte string read least significant bit first (for 4 bits: symbol
    2k is the low nibble of byte k).  Pad bits are zero."""
    codes = np.ascontiguousarray(codes, dtype=np.uint8).reshape(-1)
    if bits == 8:
        return codes.copy()
    assert int(codes.max(initial=0)) < (1 << bits)
    b = np.unpackbits(codes[:, None], axis=1, bitorder="little")[:, :bits].reshape(-1)
    return np.packbits(b, bitorder="little")


def unpack_symbols(packed: np.ndarray, n: int, bits: int) -> np.ndarray:
    """Inverse of pack_symbols: n symbols, one per byte."""
    packed = np.ascontiguousarray(packed, dtype=np.uint8).reshape(-1)
    if bits == 8:
        return packed[:n].copy()
    b = np.unpackbits(packed, bitorder="little")[:n * bits].reshape(n, bits)
    return np.packbits(b, axis=1, bitorder="little").reshape(-1)


def small_float_codes(n: int, mant_bits: int, exp_bits: int, seed: int) -> np.ndarray:
    """Codes of a small sign/exponent/mantissa float type (e2m1: 1, 2;
    e3m2: 2, 3) for Laplace(0, 1) samples, rounded to the nearest
    representable magnitude; one code per byte, below 2^(1 + exp + mant)."""
    rng = np.random.default_rng(seed)
    v = rng.laplace(0.0, 1.0, n)
    mags = []
    for e in range(1 << exp_bits):
        for m in range(1 << mant_bits):
            frac = m / (1 << mant_bits)
            mags.append(frac if e == 0 else (1 + frac) * 2.0 ** (e - 1))
    mags = np.array(mags)
    idx = np.abs(np.abs(v)[:, None] - mags[None, :]).argmin(1)
    half = len(mags)
    return (idx + half * (v < 0)).astype(np.uint8)
