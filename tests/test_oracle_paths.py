"""Pins of the oracle's path tables and priors.

 - Path weights agree with scipy's Dijkstra on the same graph (boundary as a
   sink: edges lead into it but not out of it).
 - Every stored predecessor chain is a real path whose fixed-point weights
   sum exactly to the stored distance, whose length is the stored hop count
   and whose observable parity is the stored parity.
 - For code capacity all edges weigh the same, so distance = hops x weight:
   w_ij is the Pauli weight of the shortest matching error (Fig. 1 caption).
 - Prior LLRs equal ln(rho(1)/rho(0)) with rho(1) = exp(-D) computed at 50
   digits (prior equation, Sec. II.A; prior LLR, Sec. II.B).
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import dijkstra

import oracle

mpmath.mp.dps = 50


def edges_of(dem):
    N = dem.n_det
    out = []
    for m in range(dem.n_mech):
        ds, o = dem.mech(m)
        out.append((ds[0], ds[1] if len(ds) == 2 else N, o))
    return out


@pytest.mark.parametrize("kind,d,p", [("cc", 5, 0.1), ("cc", 7, 0.03), ("mz", 5, 0.006), ("mz", 3, 0.01)])
def test_tables_against_scipy_and_paths(kind, d, p):
    dem = oracle.code_capacity(d, p) if kind == "cc" else oracle.memory_z(d, d, p)
    tab = oracle.tables(dem)
    N = dem.n_det
    E = edges_of(dem)
    wfix = oracle.fixed_weight(dem.q)
    wf = wfix.astype(np.float64) / 2 ** 32
    # directed graph: boundary N has no outgoing edges
    best = {}
    for e, (a, b, _) in enumerate(E):
        for u, v in ((a, b), (b, a)):
            if u == N:
                continue
            best[(u, v)] = min(best.get((u, v), np.inf), wf[e])
    rows, cols = zip(*best.keys())
    G = csr_matrix((list(best.values()), (rows, cols)), shape=(N + 1, N + 1))
    ref = dijkstra(G, directed=True, indices=list(range(N)))
    got = tab.dist.astype(np.float64) / 2 ** 32
    for u in range(N):
        for v in range(N):
            want = ref[u, N] if u == v else ref[u, v]
            assert abs(got[u, v] - want) <= 1e-9 * max(1.0, want)
    # the stored predecessor chains are real shortest paths
    for u in range(N):
        for v in range(N):
            y = N if u == v else v
            w, h, par = 0, 0, 0
            while y != u:
                e = tab.pred[u, v] if (y == N) else tab.pred[u, y]
                a, b, o = E[e]
                assert y in (a, b)
                w += wfix[e]; h += 1; par ^= o
                y = a if b == y else b
                assert y != N
            assert w == tab.dist[u, v] and h == tab.hops[u, v] and par == tab.par[u, v]
    assert np.array_equal(tab.dist, tab.dist.T)


@pytest.mark.parametrize("d", [3, 5, 9])
def test_code_capacity_distance_is_pauli_weight(d):
    dem = oracle.code_capacity(d, 0.07)
    tab = oracle.tables(dem)
    w = oracle.fixed_weight(dem.q[:1])[0]
    assert np.array_equal(tab.dist, tab.hops.astype(np.int64) * w)
    # boundary distance of an X check: fewest qubits to a Z-type boundary
    assert tab.hops.diagonal().min() == 1


def test_fixed_weight_and_prior_llr():
    rng = np.random.default_rng(5)
    q = 10.0 ** rng.uniform(-7, math.log10(0.45), 300)
    w = oracle.fixed_weight(q)
    for qi, wi in zip(q, w):
        exact = mpmath.log((1 - mpmath.mpf(qi)) / mpmath.mpf(qi)) * 2 ** 32
        assert abs(wi - exact) <= 0.5 + 1e-6 * abs(exact) / 2 ** 32 * 2 ** 10
    D = rng.integers(1, 200 * 2 ** 32, 300)
    llr = oracle.prior_llr(D)
    for di, li in zip(D, llr):
        x = mpmath.mpf(int(di)) / 2 ** 32
        r1 = mpmath.exp(-x)
        exact = mpmath.log(r1 / (1 - r1))
        assert abs(li - float(exact)) <= 1e-14 * max(1.0, abs(float(exact)))
    # uniform weights: rho(1) = (q/(1-q))^w exactly as printed
    qq = 0.02
    wq = oracle.fixed_weight([qq])[0]
    for hops in (1, 2, 5):
        rho1 = (qq / (1 - qq)) ** hops
        assert abs(oracle.prior_llr([hops * wq])[0] - math.log(rho1 / (1 - rho1))) < 1e-8
