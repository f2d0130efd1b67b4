"""End-to-end pins of the oracle on the d = 3 rotated code, code capacity,
p = 0.05 (q = 2p/3 on the Z-error graph of 9 qubits and 4 X checks), T = 50.

 - All 16 syndromes are decoded; the exact logical error rate is the sum over
   all 2^9 error patterns of P(e) * [decoder fails on e].  Maximum-likelihood
   decoding (best logical class per syndrome) bounds it from below.
 - 10^4 sampled shots give a logical error rate within the binomial interval
   of the exact one, and every sampled shot decodes as its syndrome's entry
   in the exhaustive table.
 - Every correction reproduces its syndrome and its observable parity is
   the predicted flip (each defect is matched once, Sec. II.D).
"""
import numpy as np
import pytest

import oracle
from tests.inputs import WORKLOADS, seed_for
from tests.test_oracle_sampler import unpack

D, P, T = 3, 0.05, 50


def syndromes_as_planes(dem, syns):
    n = len(syns)
    W = (n + 63) // 64
    syn = np.zeros((dem.n_det, W), dtype=np.uint64)
    for b, sy in enumerate(syns):
        for k in range(dem.n_det):
            if (sy >> k) & 1:
                syn[k, b >> 6] |= np.uint64(1) << np.uint64(b & 63)
    return syn, np.zeros(W, dtype=np.uint64)


def exhaustive(dem, tab):
    syns = list(range(1 << dem.n_det))
    syn, obs = syndromes_as_planes(dem, syns)
    r = oracle.decode(dem, tab, syn, obs, len(syns), T, want_corr=True)
    return r


def test_c1_exact_ler_and_ml_bound():
    dem = oracle.code_capacity(D, P)
    tab = oracle.tables(dem)
    r = exhaustive(dem, tab)
    pred = r.pred.astype(int)
    q = dem.q[0]
    n = dem.n_mech
    ler = 0.0
    joint = np.zeros((1 << dem.n_det, 2))
    for e in range(1 << n):
        sy, ob, k = 0, 0, 0
        for m in range(n):
            if (e >> m) & 1:
                ds, o = dem.mech(m)
                for x in ds:
                    sy ^= 1 << x
                ob ^= o
                k += 1
        pe = q ** k * (1 - q) ** (n - k)
        joint[sy, ob] += pe
        ler += pe * (pred[sy] != ob)
    ml = joint.min(axis=1).sum()
    assert abs(joint.sum() - 1) < 1e-12
    assert ml <= ler + 1e-15
    # on this small graph BP4M decodes every syndrome like ML would
    assert ler < 2.5 * ml + 1e-12
    # sampled 10^4 shots
    kind, d, rounds, p, iters, nshots = WORKLOADS["cc_d3"]
    syn, obs = oracle.sample(dem, seed_for(0, d, p), 0, nshots)
    rs = oracle.decode(dem, tab, syn, obs, nshots, iters)
    sampled = rs.fail.mean()
    assert abs(sampled - ler) < 4 * np.sqrt(ler * (1 - ler) / nshots)
    det = unpack(syn, nshots)
    sy = (det.astype(np.int64) << np.arange(dem.n_det)[:, None]).sum(axis=0)
    assert np.array_equal(rs.pred, r.pred[sy])


@pytest.mark.parametrize("kind,d,p,n", [("cc", 3, 0.05, 16), ("cc", 7, 0.12, 400), ("mz", 5, 0.008, 300)])
def test_corrections_reproduce_syndrome(kind, d, p, n):
    dem = oracle.code_capacity(d, p) if kind == "cc" else oracle.memory_z(d, d, p)
    tab = oracle.tables(dem)
    if kind == "cc" and d == 3:
        syn, obs = syndromes_as_planes(dem, list(range(16)))
    else:
        syn, obs = oracle.sample(dem, 99, 0, n)
    r = oracle.decode(dem, tab, syn, obs, n, 25, want_corr=True, s_cap=dem.n_det)
    corr = unpack(r.corr, n)                # [n_mech, n]
    det = unpack(syn, n)
    for b in range(n):
        sy = np.zeros(dem.n_det, dtype=bool)
        ob = 0
        for m in np.nonzero(corr[:, b])[0]:
            ds, o = dem.mech(m)
            sy[list(ds)] ^= True
            ob ^= o
        assert np.array_equal(sy, det[:, b])
        assert ob == int(r.pred[b])
        s = r.s[b]
        part = r.partner[b, :s]
        assert all(part[part[i]] == i for i in range(s))


def test_edge_cases_zero_and_one_defect():
    dem = oracle.code_capacity(5, 0.05)
    tab = oracle.tables(dem)
    syns = [0, 1 << 3, 1 << 11]
    syn, obs = syndromes_as_planes(dem, syns)
    r = oracle.decode(dem, tab, syn, obs, 3, 10, s_cap=4)
    assert list(r.s) == [0, 1, 1]
    assert r.flags[0] == oracle.F_CONVERGED_ANY
    assert r.partner[1, 0] == 0
    assert r.pred[1] == bool(tab.par[3, 3]) and r.pred[2] == bool(tab.par[11, 11])
    # empty batch
    e = oracle.decode(dem, tab, syn[:, :0], obs[:0], 0, 10)
    assert e.flags.size == 0


def test_unrotated_d3_exact_ler_and_ml_bound():
    # unrotated d = 3, code capacity, p = 0.06, T = 25: 13 qubits, 6 X checks
    dem = oracle.code_capacity(3, 0.06, unrotated=True)
    tab = oracle.tables(dem)
    syns = list(range(1 << dem.n_det))
    syn, obs = syndromes_as_planes(dem, syns)
    r = oracle.decode(dem, tab, syn, obs, len(syns), 25, want_corr=True)
    pred = r.pred.astype(int)
    q, n = dem.q[0], dem.n_mech
    joint = np.zeros((1 << dem.n_det, 2))
    for e in range(1 << n):
        sy, ob, k = 0, 0, 0
        for m in range(n):
            if (e >> m) & 1:
                ds, o = dem.mech(m)
                for x in ds:
                    sy ^= 1 << x
                ob ^= o
                k += 1
        joint[sy, ob] += q ** k * (1 - q) ** (n - k)
    ler = float(sum(joint[s_, 1 - pred[s_]] for s_ in range(len(syns))))
    ml = joint.min(axis=1).sum()
    assert abs(joint.sum() - 1) < 1e-12
    assert ml <= ler + 1e-15 and ler < 2.5 * ml + 1e-12
    # corrections reproduce every syndrome
    corr = unpack(r.corr, len(syns))
    for b in range(len(syns)):
        sy = 0
        for m in np.nonzero(corr[:, b])[0]:
            for x in dem.mech(m)[0]:
                sy ^= 1 << x
        assert sy == syns[b]
