"""CPU model of the split-chunk decode's boundary search (the walks the GPU
kernel k_decode_split makes), run on streams the oracle writes: pieces of a
chunk's bits, walks of code lengths from guessed starts (a warm-up before
each piece, guesses on the grid of the gcd of the code lengths), correction
rounds against the previous piece's exit, the scan of the counts.  It checks
what the kernel's correctness rests on: the rounds end within G + 1, every
piece's start is a true code boundary, the counts sum to the chunk's
symbols and the decode of the pieces returns the input — including data
on which a wrong start never meets the true boundaries.  Independent of the
HIP code (a model of its algorithm, written from the same description)."""
import math

import numpy as np
import pytest

import oracle


def _lengths(t, sb):
    """Code length of the code starting at every bit of the stream sb."""
    p = t.prefix_bits
    w = [min(int(v), 8) for v in t.width]
    area = np.zeros(sb.size - 3, dtype=np.int64)
    for i in range(p):
        area = (area << 1) | sb[i:i + area.size]
    return p + np.array(w)[area]


def model_boundaries(bits, total, index, C, t, n, warm_bits):
    """Start bit and code count of every piece of every chunk, and the
    number of correction rounds each chunk took."""
    sb = np.concatenate([np.unpackbits(np.asarray(bits, dtype=np.uint8)),
                         np.zeros(512, np.uint8)])
    lens = _lengths(t, sb)
    d = 0
    for a in range(len(t.width)):
        if t.count[a]:
            d = math.gcd(d, t.prefix_bits + min(int(t.width[a]), 8))
    d = d or 1
    G = max(C // 64, 1)
    nch = (n + C - 1) // C
    out = []
    for j in range(nch):
        s = int(index[j])
        e = int(index[j + 1]) if j + 1 < nch else total
        L = e - s
        piece = (L + G - 1) // G
        lo = [s + min(g * piece, L) for g in range(G)]
        end = [s + min((g + 1) * piece, L) for g in range(G)]

        def walk(x, stop, count=True):
            c = 0
            while x < stop:
                x += int(lens[x])
                c += 1
            return x, c

        start, exitp, cnt = [], [], []
        for g in range(G):
            u = max(0, lo[g] - s - warm_bits) if g else 0
            u = s + (u + d - 1) // d * d
            st, _ = walk(u, lo[g])
            x, c = walk(st, end[g])
            start.append(st), exitp.append(x), cnt.append(c)
        rounds = 0
        while True:
            prev = [s] + exitp[:-1]
            changed = False
            for g in range(1, G):
                if prev[g] == start[g]:
                    continue
                a, b, ca, cb = prev[g], start[g], 0, 0
                met = False
                while True:
                    if a == b:
                        met = True
                        break
                    if a < b:
                        if a >= end[g]:
                            break
                        a += int(lens[a]); ca += 1
                    else:
                        if b >= end[g]:
                            break
                        b += int(lens[b]); cb += 1
                nx = exitp[g] if met else a
                cnt[g] = cnt[g] - cb + ca if met else ca
                changed |= nx != exitp[g]
                exitp[g], start[g] = nx, prev[g]
            rounds += 1
            if not changed:
                break
            assert rounds <= G + 1
        out.append((start, cnt, exitp, e, rounds))
    return out


def _check(x, t, C, warm_bits):
    st, bits, index, total = oracle.encode(x, t, C)
    assert st == 0
    n = x.size
    true_starts = set(np.concatenate([[0], np.cumsum(t.len[x])[:-1]]).tolist()) if n else set()
    rounds = []
    for j, (start, cnt, exitp, e, r) in enumerate(model_boundaries(bits, total, index, C, t, n,
                                                                   warm_bits)):
        nsym = min(C, n - j * C)
        assert sum(cnt) == nsym and exitp[-1] == e, j
        for g, (s0, c) in enumerate(zip(start, cnt)):
            if c:
                assert s0 in true_starts, (j, g)
        rounds.append(r)
    # the pieces decode to the input (the oracle's decode of the same stream)
    ost, out = oracle.decode(bits, total, index, C, t, n)
    assert ost == 0 and np.array_equal(out, x)
    return max(rounds) if rounds else 0


@pytest.mark.parametrize("C", [256, 2048])
@pytest.mark.parametrize("warm_bits", [0, 512])
def test_model_on_skewed_and_uniform_data(C, warm_bits):
    rng = np.random.default_rng(C + warm_bits)
    x = np.clip(np.round(rng.laplace(128, 6, 12289)), 0, 255).astype(np.uint8)
    for mode in (0, 2, 3):
        _check(x, oracle.build_table(oracle.histogram(x), mode), C, warm_bits)
    u = rng.integers(0, 256, 9001).astype(np.uint8)      # SEARCH: one code length
    assert _check(u, oracle.build_table(oracle.histogram(u), 0), C, warm_bits) == 1


def test_model_never_meeting_starts_take_g_rounds():
    """A chunk of one symbol under a table with several lengths: a wrong
    start never meets the true boundaries, lane g is exact after round g."""
    C = 2048
    x = np.zeros(3 * C, np.uint8)
    x[:40] = np.arange(40)
    t = oracle.build_table(oracle.histogram(x), 0)
    G = C // 64
    assert G - 1 <= _check(x, t, C, 0) <= G + 1     # one more exact lane per round
    assert _check(x, t, C, 512) <= G + 1


def test_model_small_alphabet_tables():
    rng = np.random.default_rng(3)
    for M, A, p in ((16, 2, 1), (16, 4, 2), (64, 8, 3)):
        x = np.minimum(rng.geometric(0.3, 7001) - 1, M - 1).astype(np.uint8)
        t = oracle.build_table_general(oracle.histogram(x)[:M], M, A, p, A)
        _check(x, t, 512, 512)
