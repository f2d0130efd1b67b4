"""Pins of the oracle's syndrome sampler.

 - The integer threshold is round(q * 2^32) clamped to 32 bits (checked with
   exact rational arithmetic).
 - Each detector fires with the closed-form probability
   (1 - prod_{m touching k} (1 - 2 q_m)) / 2 of independent mechanisms, and
   pairs of detectors (and detector/observable) fire together with the
   probability computed exactly from the DEM.
 - Drawing shots [a, b) directly equals drawing [0, b) and keeping [a, b):
   the draws depend only on the global shot index.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests.test_oracle_graphs import dem_pair_prob


def unpack(planes, n):
    """planes [..., W] uint64 -> bool [..., n]."""
    bits = np.unpackbits(planes.view(np.uint8), axis=-1, bitorder="little")
    return bits[..., :n].astype(bool)


def test_threshold_rule():
    rng = np.random.default_rng(51)
    q = np.concatenate([rng.uniform(0, 1, 2000), [0.0, 1.0, 0.5, 2.0 ** -33, 1 - 2.0 ** -40]])
    thr = oracle.threshold(q)
    for qi, ti in zip(q, thr):
        want = min(2 ** 32 - 1, int(Fraction(qi) * 2 ** 32 + Fraction(1, 2)))
        assert int(ti) == want


@pytest.mark.parametrize("kind,d,p,n", [("cc", 5, 0.15, 200_000), ("mz", 3, 0.01, 100_000)])
def test_firing_rates_closed_form(kind, d, p, n):
    dem = oracle.code_capacity(d, p) if kind == "cc" else oracle.memory_z(d, d, p)
    syn, obs = oracle.sample(dem, seed=0xC0FFEE + d, shot0=0, n=n)
    det = unpack(syn, n)
    rate = det.mean(axis=1)
    for k in range(dem.n_det):
        prod = 1.0
        for m in range(dem.n_mech):
            if k in dem.mech(m)[0]:
                prod *= 1 - 2 * dem.q[m]
        want = (1 - prod) / 2
        assert abs(rate[k] - want) < 5 * np.sqrt(want * (1 - want) / n), (k, rate[k], want)
    want_s = sum((1 - np.prod([1 - 2 * dem.q[m] for m in range(dem.n_mech) if k in dem.mech(m)[0]])) / 2
                 for k in range(dem.n_det))
    s = det.sum(axis=0)
    assert abs(s.mean() - want_s) < 5 * s.std() / np.sqrt(n)
    if kind == "mz":
        ob = unpack(obs[None, :], n)[0]
        for a in range(0, dem.n_det, 3):
            for b in [a + 1, -1]:
                if b == dem.n_det:
                    continue
                pr = dem_pair_prob(dem, a, b)
                both = (det[a] & (ob if b == -1 else det[b])).mean()
                assert abs(both - pr[3]) < 5 * np.sqrt(pr[3] * (1 - pr[3]) / n) + 1e-9


def test_shot_window_consistency_and_trailing_bits():
    dem = oracle.memory_z(3, 3, 0.02)
    syn, obs = oracle.sample(dem, seed=77, shot0=0, n=300)
    syn2, obs2 = oracle.sample(dem, seed=77, shot0=100, n=137)
    a = unpack(syn, 300)[:, 100:237]
    b = unpack(syn2, 137)
    assert np.array_equal(a, b)
    assert np.array_equal(unpack(obs[None], 300)[0, 100:237], unpack(obs2[None], 137)[0])
    # bits beyond n are zero
    assert np.all(unpack(syn2, 192)[:, 137:] == 0)
    other, _ = oracle.sample(dem, seed=78, shot0=0, n=300)
    assert not np.array_equal(other, syn)


@pytest.mark.parametrize("kind,d,p,n", [("cc", 5, 0.1, 5_003), ("mz", 3, 0.02, 4_001)])
def test_error_planes_explain_the_syndrome(kind, d, p, n):
    # the sampled error itself: the syndrome and the observable flip are the
    # XOR of the fired mechanisms' detectors and observable bits, and each
    # mechanism fires at its rate q_m (3.5 sigma on the total over mechanisms
    # of equal q)
    dem = oracle.code_capacity(d, p) if kind == "cc" else oracle.memory_z(d, d, p)
    syn, obs, err = oracle.sample(dem, seed=77 + d, shot0=1234, n=n, want_err=True)
    s2, o2 = oracle.sample(dem, seed=77 + d, shot0=1234, n=n)
    assert np.array_equal(syn, s2) and np.array_equal(obs, o2)
    E = unpack(err, n)                                         # [n_mech][n]
    H = np.zeros((dem.n_det, dem.n_mech), dtype=np.uint8)
    for m in range(dem.n_mech):
        H[dem.dets[dem.off[m]:dem.off[m + 1]], m] = 1
    want_syn = (H.astype(np.int64) @ E.astype(np.int64)) & 1
    assert np.array_equal(want_syn.astype(bool), unpack(syn, n))
    want_obs = (dem.obs.astype(np.int64) @ E.astype(np.int64)) & 1
    assert np.array_equal(want_obs.astype(bool), unpack(obs, n))
    for q in np.unique(dem.q):
        sel = dem.q == q
        k = int(E[sel].sum())
        tot = int(sel.sum()) * n
        assert abs(k - q * tot) <= 3.5 * np.sqrt(q * (1 - q) * tot) + 1, (q, k, tot)
