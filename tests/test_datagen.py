"""Synthetic e4m3 workload generator (CPU only)."""
import numpy as np
import torch

from paper_2602_17849_amd import datagen


def e4m3_value(code):
    """Value of an e4m3 (fn) byte: 1 sign, 4 exponent (bias 7), 3 mantissa bits."""
    code = np.asarray(code, dtype=np.int64)
    s = np.where(code & 0x80, -1.0, 1.0)
    e = (code >> 3) & 0xF
    m = code & 7
    v = np.where(e == 0, m / 8.0 * 2.0 ** -6, (1 + m / 8.0) * 2.0 ** (e - 7))
    return s * v


def test_deterministic_and_seed_dependent():
    a = datagen.single_tensor_gaussian(seed=0, rows=64, cols=64)
    b = datagen.single_tensor_gaussian(seed=0, rows=64, cols=64)
    c = datagen.single_tensor_gaussian(seed=1, rows=64, cols=64)
    assert datagen.sha256(a) == datagen.sha256(b) != datagen.sha256(c)


def test_quantizer_block_scale_and_rounding():
    g = torch.Generator().manual_seed(5)
    x = torch.randn(32 * 400, generator=g) * torch.exp(torch.randn(32 * 400, generator=g) * 3)
    x[:32] = 0.0                                   # an all-zero block
    q = datagen.quantize_e4m3_block32(x).numpy()
    assert not np.isin(q, [0x7F, 0xFF]).any()      # NaN encodings never produced
    xb = x.numpy().astype(np.float64).reshape(-1, 32)
    vals = e4m3_value(q).reshape(-1, 32)
    grid = np.sort(np.unique(e4m3_value(np.array([c for c in range(256) if c & 0x7F != 0x7F]))))
    for blk in range(xb.shape[0]):
        m = np.abs(xb[blk]).max()
        k = 0 if m == 0 else int(np.ceil(np.log2(m / 448.0)))
        if m:
            assert m / 2.0 ** k <= 448.0 < m / 2.0 ** (k - 1)   # smallest power-of-two scale
        y = xb[blk] / 2.0 ** k
        for yi, vi in zip(y, vals[blk]):
            # nearest representable value (ties to even mantissa are allowed)
            d = np.abs(grid - yi)
            assert abs(vi - yi) <= d.min() + 1e-12


def test_workload_shapes():
    assert datagen.single_tensor_laplace(rows=16, cols=64).numel() == 1024
    sizes = datagen.shard_sizes()
    assert len(sizes) == 1152
    assert all(s % 32 == 0 and (1 << 20) - 32 <= s <= (32 << 20) + 32 for s in sizes)
    req = datagen.serving_requests(duration_s=0.5)
    assert all(k in ("compress", "decompress") for _, k, _ in req)
    z = datagen.zeros90_gaussian(1 << 16, seed=5)
    frac = (z == 0).float().mean().item()
    assert 0.88 < frac < 0.93


def test_stress_buffer_pieces():
    """The 4 GiB stress recipe, at a small size: deterministic, piecewise
    seeded, kind-specific structure."""
    for kind in datagen.STRESS_KINDS:
        a = datagen.stress_buffer(kind, numel=5000, piece=1024)
        b = datagen.stress_buffer(kind, numel=5000, piece=1024)
        assert a.numel() == 5000 and torch.equal(a, b)
        assert not torch.equal(a[:1024], a[1024:2048])     # pieces use their own seeds
    z = datagen.stress_buffer("zeros90", numel=1 << 16, piece=1 << 14)
    assert 0.88 < (z == 0).float().mean().item() < 0.93
    g = datagen.stress_buffer("ocp_gaussian", numel=1 << 16, piece=1 << 14)
    assert not ((g == 0x7F) | (g == 0xFF)).any()
