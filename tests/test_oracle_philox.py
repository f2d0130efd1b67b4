"""Pins of the oracle's Philox4x32-10 (Salmon et al., SC'11).

The published known-answer vectors of the generator (tests/golden/
philox4x32_10_kat.txt: zero, all-ones and digits-of-pi inputs) must come out
word for word.  The second test inverts the generator from the published
definition: a round maps (c0, c1, c2, c3) to (hi(M1 c2) ^ c1 ^ k0,
lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)), both multipliers are odd so
lo(M c) determines c, and the key grows by the two Weyl constants between
rounds.  Running the ten inverse rounds on the oracle's output must give back
the counter, which fails for a wrong multiplier, Weyl constant, word
placement or round count.  Uniformity and bit balance are checked as well.
"""
import os

import numpy as np
from scipy import stats

import oracle

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def invert(out, key):
    inv0, inv1 = pow(M0, -1, 1 << 32), pow(M1, -1, 1 << 32)
    n0, n1, n2, n3 = (int(x) for x in out)
    for r in reversed(range(10)):
        k0 = (int(key[0]) + r * W0) & MASK
        k1 = (int(key[1]) + r * W1) & MASK
        c0 = (n3 * inv0) & MASK
        c2 = (n1 * inv1) & MASK
        hi0 = (M0 * c0) >> 32
        hi1 = (M1 * c2) >> 32
        c1 = n0 ^ hi1 ^ k0
        c3 = n2 ^ hi0 ^ k1
        n0, n1, n2, n3 = c0, c1, c2, c3
    return [n0, n1, n2, n3]


HERE = os.path.dirname(os.path.abspath(__file__))


def read_kat():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        assert len(w) == 10
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_published_known_answers():
    rows = read_kat()
    assert len(rows) == 3
    ctr = np.array([r[0] for r in rows], dtype=np.uint32)
    key = np.array([r[1] for r in rows], dtype=np.uint32)
    out = oracle.philox(ctr, key)
    for (c, k, want), got in zip(rows, out):
        assert [int(x) for x in got] == want, (c, k, [hex(int(x)) for x in got])


def test_philox_inverts_to_counter():
    rng = np.random.default_rng(11)
    ctr = rng.integers(0, 1 << 32, size=(200, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 1 << 32, size=(200, 2), dtype=np.uint64).astype(np.uint32)
    out = oracle.philox(ctr, key)
    for c, k, o in zip(ctr, key, out):
        assert invert(o, k) == [int(x) for x in c]


def test_philox_uniform_and_balanced():
    n = 1 << 15
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n) % 7
    ctr[:, 1] = np.arange(n)
    key = np.tile(np.array([0x12345678, 0x9ABCDEF0], dtype=np.uint32), (n, 1))
    out = oracle.philox(ctr, key).reshape(-1)
    counts = np.bincount(out >> 26, minlength=64)
    assert stats.chisquare(counts).pvalue > 1e-4
    bits = np.unpackbits(out.view(np.uint8)).reshape(-1, 32).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 0.01)


def test_philox_counter_avalanche():
    rng = np.random.default_rng(12)
    ctr = rng.integers(0, 1 << 32, size=(500, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 1 << 32, size=(500, 2), dtype=np.uint64).astype(np.uint32)
    flipped = ctr.copy()
    flipped[:, 1] ^= np.uint32(1)
    a = oracle.philox(ctr, key)
    b = oracle.philox(flipped, key)
    frac = np.unpackbits((a ^ b).view(np.uint8)).mean()
    assert abs(frac - 0.5) < 0.02
