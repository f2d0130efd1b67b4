"""Pins of the oracle's B-BP4MF pieces (Sec. II.E, III.D), against what the code
and the mathematics fix rather than against the oracle itself:

 - Tanner graphs of both code-capacity layouts: X and Z checks commute, the
   observable's support commutes with every Z check, each qubit's X checks
   are its decoding-graph mechanism;
 - the joint depolarizing sampler: check firing rates and the joint rate of
   an X and a Z check sharing qubits, each from exact enumeration;
 - quaternary BP: exact marginals on tree-shaped Tanner graphs (brute force
   over all 4^n errors with the syndrome), and a converged hard decision
   reproduces both syndromes;
 - the fixed-order log, path prior and edge weight vs the C library;
 - re-weighted path tables vs a brute-force Bellman-Ford (boundary a sink);
 - the whole decoder: exhaustive d = 3 logical error rate >= the exact
   maximum-likelihood one, and B-BP4MF beats BP4MF on the same syndromes.
"""
import itertools
import math

import numpy as np
import pytest

import oracle


def dem_and_tanner(d, unrotated, p=0.1):
    dem = oracle.code_capacity(d, p, unrotated=unrotated)
    return dem, oracle.tanner(d, dem, unrotated=unrotated)


def qubit_checks(T):
    xs = [[c for c in T.qx[v] if c >= 0] for v in range(T.n_q)]
    zs = [[c for c in T.qz[v] if c >= 0] for v in range(T.n_q)]
    return xs, zs


@pytest.mark.parametrize("d,unrot", [(3, False), (5, False), (7, False), (2, True), (3, True), (5, True), (9, True)])
def test_tanner_structure(d, unrot):
    dem, T = dem_and_tanner(d, unrot)
    nq = d * d + (d - 1) ** 2 if unrot else d * d
    nc = d * (d - 1) if unrot else (d * d - 1) // 2
    assert T.n_q == nq and T.n_xc == nc and T.n_zc == nc
    xs, zs = qubit_checks(T)
    xsup = [set() for _ in range(T.n_xc)]
    zsup = [set() for _ in range(T.n_zc)]
    for v in range(nq):
        for c in xs[v]:
            xsup[c].add(v)
        for c in zs[v]:
            zsup[c].add(v)
    # the check lists agree with the qubit lists and are ascending
    for c in range(T.n_xc + T.n_zc):
        row = [v for v in T.cq[c] if v >= 0]
        assert row == sorted(xsup[c] if c < T.n_xc else zsup[c - T.n_xc])
        assert 2 <= len(row) <= 4
    # every X check commutes with every Z check (even overlap)
    for a in xsup:
        for b in zsup:
            assert len(a & b) % 2 == 0
    # the X logical's support (qubits whose Z error flips the observable)
    # commutes with every Z check and has weight d
    L = {v for v in range(nq) if T.qobs[v]}
    assert len(L) == d
    for b in zsup:
        assert len(L & b) % 2 == 0
    # each qubit's Z error is its mechanism: the same X checks and observable
    for v in range(nq):
        ds, o = dem.mech(int(T.qmech[v]))
        assert list(ds) == sorted(xs[v]) and o == int(T.qobs[v])
    assert sorted(T.qmech.tolist()) == list(range(nq))


def _rate(k, p):
    """P(odd number of anticommuting errors among k qubits), each 2p/3."""
    return (1 - (1 - 4 * p / 3) ** k) / 2


@pytest.mark.parametrize("d,unrot,p", [(3, False, 0.1), (5, True, 0.12)])
def test_depolarizing_sampler_statistics(d, unrot, p):
    dem, T = dem_and_tanner(d, unrot, p)
    n = 200_000
    sx, sz, ob = oracle.sample_depolarizing(T, p, 11, 0, n)
    bits = lambda planes: np.unpackbits(planes.view(np.uint8), axis=-1, bitorder="little")[..., :n].astype(bool)
    bx, bz, bo = bits(sx), bits(sz), bits(ob[None, :])[0]
    xs, zs = qubit_checks(T)
    for c in range(T.n_xc):
        k = sum(c in x for x in xs)
        e = _rate(k, p)
        assert abs(bx[c].mean() - e) < 5 * math.sqrt(e * (1 - e) / n)
    for c in range(T.n_zc):
        k = sum(c in z for z in zs)
        e = _rate(k, p)
        assert abs(bz[c].mean() - e) < 5 * math.sqrt(e * (1 - e) / n)
    e = _rate(d, p)
    assert abs(bo.mean() - e) < 5 * math.sqrt(e * (1 - e) / n)
    # joint firing of an X check and a Z check sharing two qubits, by
    # enumeration of the 4^k errors on their union (X=1, Y=2, Z=3)
    pairs = 0
    for cx in range(T.n_xc):
        for cz in range(T.n_zc):
            qa = {v for v in range(T.n_q) if cx in xs[v]}
            qb = {v for v in range(T.n_q) if cz in zs[v]}
            if len(qa & qb) != 2:
                continue
            qs = sorted(qa | qb)
            pr = 0.0
            for es in itertools.product(range(4), repeat=len(qs)):
                w = 1.0
                fx = fz = 0
                for v, E in zip(qs, es):
                    w *= (1 - p) if E == 0 else p / 3
                    if v in qa and E >= 2:
                        fx ^= 1
                    if v in qb and E in (1, 2):
                        fz ^= 1
                if fx and fz:
                    pr += w
            got = (bx[cx] & bz[cz]).mean()
            assert abs(got - pr) < 5 * math.sqrt(pr * (1 - pr) / n), (cx, cz, got, pr)
            pairs += 1
            if pairs >= 6:
                return
    assert pairs > 0


def tree_tanner(kind):
    """Tree-shaped Tanner graphs: a path X{0,1} Z{1,2} X{2,3}, and a star
    X{0,1,2} Z{2,3,4}."""
    if kind == "path":
        nq, xch, zch = 4, [[0, 1], [2, 3]], [[1, 2]]
    else:
        nq, xch, zch = 5, [[0, 1, 2]], [[2, 3, 4]]
    qx = -np.ones((nq, 2), np.int32)
    qz = -np.ones((nq, 2), np.int32)
    for c, qs in enumerate(xch):
        for v in qs:
            qx[v][list(qx[v]).index(-1)] = c
    for c, qs in enumerate(zch):
        for v in qs:
            qz[v][list(qz[v]).index(-1)] = c
    cq = -np.ones((len(xch) + len(zch), 4), np.int32)
    for c, qs in enumerate(xch + zch):
        cq[c, :len(qs)] = qs
    return oracle.Tanner(len(xch), len(zch), qx, qz, np.zeros(nq, np.uint8), np.arange(nq, dtype=np.int32), cq)


@pytest.mark.parametrize("kind", ["path", "star"])
def test_qbp_is_exact_on_trees(kind):
    T = tree_tanner(kind)
    p = 0.13
    xs, zs = qubit_checks(T)
    for zx in itertools.product([0, 1], repeat=T.n_xc):
        for zz in itertools.product([0, 1], repeat=T.n_zc):
            # exact marginals over all 4^n errors with this syndrome
            marg = np.zeros((T.n_q, 4))
            for es in itertools.product(range(4), repeat=T.n_q):
                sx = [0] * T.n_xc
                sz = [0] * T.n_zc
                w = 1.0
                for v, E in enumerate(es):
                    w *= (1 - p) if E == 0 else p / 3
                    for c in xs[v]:
                        sx[c] ^= E >= 2
                    for c in zs[v]:
                        sz[c] ^= E in (1, 2)
                if list(sx) == list(zx) and list(sz) == list(zz):
                    for v, E in enumerate(es):
                        marg[v, E] += w
            marg /= marg.sum(axis=1, keepdims=True)
            conv, it, hard, post = oracle.qbp(T, p, np.array(zx), np.array(zz), 12, stop=False)
            got = np.exp(post - post.max(axis=1, keepdims=True))
            got /= got.sum(axis=1, keepdims=True)
            assert np.abs(got - marg).max() < 1e-12, (zx, zz)
            assert it == 12


@pytest.mark.parametrize("d,unrot,p", [(5, True, 0.1), (7, False, 0.08)])
def test_converged_hard_decision_has_both_syndromes(d, unrot, p):
    dem, T = dem_and_tanner(d, unrot, p)
    n = 300
    sx, sz, _ = oracle.sample_depolarizing(T, p, 5, 0, n)
    xs, zs = qubit_checks(T)
    seen = 0
    for b in range(n):
        zx = ((sx[:, b >> 6] >> np.uint64(b & 63)) & np.uint64(1)).astype(np.uint8)
        zz = ((sz[:, b >> 6] >> np.uint64(b & 63)) & np.uint64(1)).astype(np.uint8)
        conv, it, hard, _ = oracle.qbp(T, p, zx, zz, 25)
        if not conv:
            continue
        seen += 1
        gx = np.zeros(T.n_xc, np.uint8)
        gz = np.zeros(T.n_zc, np.uint8)
        for v in range(T.n_q):
            for c in xs[v]:
                gx[c] ^= hard[v] >= 2
            for c in zs[v]:
                gz[c] ^= hard[v] in (1, 2)
        assert np.array_equal(gx, zx) and np.array_equal(gz, zz)
    assert seen > n // 4


def test_fixed_order_functions():
    rng = np.random.default_rng(3)
    for x in np.concatenate([10.0 ** rng.uniform(-300, 300, 500), rng.uniform(0.5, 2.0, 500)]):
        ref = math.log(x)
        # k ln2 + log1p(m - 1) with x = m 2^k: a few ulp of the larger term
        # (below 1 the two terms nearly cancel)
        k = math.frexp(x)[1] - 1
        assert abs(oracle.spec_log(x) - ref) <= 4 * np.spacing(max(abs(ref), abs(k) * math.log(2)))
        if x >= 1:
            assert abs(oracle.spec_log(x) - ref) <= 4 * np.spacing(abs(ref)) + 4 * np.spacing(k * math.log(2) + 1e-300)
    for D in [1, 2 ** 20, 2 ** 32, 3 * 2 ** 32, 2 ** 40, 2 ** 45]:
        Df = D / 2 ** 32
        ref = -Df - math.log1p(-math.exp(-Df))
        # 1 - exp(-D) loses relative accuracy ~ 2^-53 / D for small D
        assert abs(oracle.spec_prior(D) - ref) <= 1e-12 * abs(ref) + 4e-16 / Df
    for P in [1e-200, 1e-9, 0.01, 0.2, 0.4999]:
        want = math.floor(math.log((1 - P) / P) * 2 ** 32 + 0.5)
        got = oracle.qbp_weight(P)
        assert abs(got - min(max(want, 1), 2 ** 40)) <= 1
    assert oracle.qbp_weight(0.5) == 1 and oracle.qbp_weight(0.9) == 1
    assert oracle.qbp_weight(1e-300) == 2 ** 40
    L = np.log(np.array([0.7, 0.1, 0.05, 0.15]))
    assert abs(oracle.qbp_zprob(L) - 0.2) < 1e-15


def _bellman_ford(dem, w, src):
    """(weight, hops) labels from src; the boundary (node N) is a sink."""
    N = dem.n_det
    lab = [(math.inf, math.inf)] * (N + 1)
    lab[src] = (0, 0)
    edges = []
    for m in range(dem.n_mech):
        ds, _ = dem.mech(m)
        edges.append((ds[0], ds[1] if len(ds) == 2 else N, int(w[m])))
    for _ in range(N + 2):
        changed = False
        for a, b, ww in edges:
            for x, y in ((a, b), (b, a)):
                if x == N or lab[x][0] == math.inf:
                    continue
                cand = (lab[x][0] + ww, lab[x][1] + 1)
                if cand < lab[y]:
                    lab[y] = cand
                    changed = True
        if not changed:
            break
    return lab


@pytest.mark.parametrize("d,unrot", [(3, False), (5, True)])
def test_reweighted_tables(d, unrot):
    dem, T = dem_and_tanner(d, unrot)
    # with the graph's own weights the tables are the graph's
    w0 = oracle.fixed_weight(dem.q)
    a, b = oracle.tables_w(dem, w0), oracle.tables(dem)
    for f in ("dist", "hops", "par", "pred"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    # random weights: Bellman-Ford labels
    rng = np.random.default_rng(8)
    w = rng.integers(1, 2 ** 34, size=dem.n_mech, dtype=np.int64)
    t = oracle.tables_w(dem, w)
    N = dem.n_det
    for u in range(N):
        lab = _bellman_ford(dem, w, u)
        for v in range(N):
            tgt = N if v == u else v
            assert (t.dist[u, v], t.hops[u, v]) == lab[tgt]


def _syndrome_of(T, es):
    xs, zs = qubit_checks(T)
    sx = np.zeros(T.n_xc, np.uint8)
    sz = np.zeros(T.n_zc, np.uint8)
    ob = 0
    for v, E in enumerate(es):
        for c in xs[v]:
            sx[c] ^= E >= 2
        for c in zs[v]:
            sz[c] ^= E in (1, 2)
        if E >= 2 and T.qobs[v]:
            ob ^= 1
    return sx, sz, ob


@pytest.mark.slow
def test_exhaustive_d3_ler_bounded_by_ml():
    """Rotated d = 3 under depolarizing noise: the exact logical error rate of
    B-BP4MF over all 4^9 errors is at least that of maximum likelihood."""
    p = 0.1
    dem, T = dem_and_tanner(3, False, p)
    prob = {}
    for es in itertools.product(range(4), repeat=T.n_q):
        w = 1.0
        for E in es:
            w *= (1 - p) if E == 0 else p / 3
        sx, sz, ob = _syndrome_of(T, es)
        key = (tuple(sx), tuple(sz))
        prob.setdefault(key, [0.0, 0.0])[ob] += w
    keys = sorted(prob)
    n = len(keys)
    W = (n + 63) // 64
    sxp = np.zeros((T.n_xc, W), np.uint64)
    szp = np.zeros((T.n_zc, W), np.uint64)
    for b, (kx, kz) in enumerate(keys):
        for c, bit in enumerate(kx):
            if bit:
                sxp[c, b >> 6] |= np.uint64(1) << np.uint64(b & 63)
        for c, bit in enumerate(kz):
            if bit:
                szp[c, b >> 6] |= np.uint64(1) << np.uint64(b & 63)
    r = oracle.bbp4mf_decode(dem, T, p, sxp, szp, np.zeros(W, np.uint64), n, 25)
    ler = sum(prob[k][1 - int(pr)] for k, pr in zip(keys, r.pred))
    ml = sum(min(v) for v in prob.values())
    assert abs(sum(sum(v) for v in prob.values()) - 1) < 1e-12
    assert ler >= ml - 1e-15
    assert ler < 3 * ml                        # a sane decoder at this p


def test_bbp4mf_beats_bp4mf_on_the_same_syndromes():
    p = 0.1
    dem, T = dem_and_tanner(5, True, p)
    n = 2000
    sx, sz, ob = oracle.sample_depolarizing(T, p, 7, 0, n)
    r = oracle.bbp4mf_decode(dem, T, p, sx, sz, ob, n, 25)
    r2 = oracle.decode(dem, oracle.tables(dem), sx, ob, n, 25, variant=1)
    assert r.fail.mean() < 0.7 * r2.fail.mean()
    qb = (r.flags & oracle.F_QBP) != 0
    assert 0.3 < qb.mean() < 0.95
    # stage-3 matchings are involutions on the shot's defects
    for b in np.nonzero(~qb)[0][:200]:
        s = int(r.s[b])
        pt = r.partner[b][:s]
        assert all(0 <= pt[i] < s and pt[pt[i]] == i for i in range(s))
