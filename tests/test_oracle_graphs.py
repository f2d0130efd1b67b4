"""Pins of the oracle's detector error models (code capacity and memory-Z).

Checks are re-derived from the code's definition, not from the oracle:
 - detector and mechanism counts of the rotated surface code;
 - every stabilizer of the other type flips no detector and not the
   observable, and every logical string flips only the observable;
 - the graph distance (fewest mechanisms forming an undetectable logical
   error) equals d;
 - a direct Monte Carlo simulation of the memory-Z circuit (exclusive Pauli
   channels, written here from the circuit's description) reproduces the
   detector and observable statistics the DEM predicts.
"""
from collections import deque

import numpy as np
import pytest

import oracle


# ---------------------------------------------------------------- layout --

def plaquettes(d, want_x):
    out = []
    for r in range(-1, d):
        for c in range(-1, d):
            is_x = (r + c) % 2 == 0
            if is_x != want_x:
                continue
            rb, cb = r in (-1, d - 1), c in (-1, d - 1)
            if rb and cb:
                continue
            if rb and not want_x:
                continue
            if cb and want_x:
                continue
            out.append((r, c))
    return out


def corners(d, r, c):
    return [(a, b) for a, b in ((r, c), (r, c + 1), (r + 1, c), (r + 1, c + 1)) if 0 <= a < d and 0 <= b < d]


def symptom(dem, mechs):
    det = set()
    ob = 0
    for m in mechs:
        ds, o = dem.mech(m)
        det ^= set(ds)
        ob ^= o
    return det, ob


def graph_distance(dem):
    """Fewest mechanisms whose detectors cancel and whose observable is odd."""
    N = dem.n_det
    adj = [[] for _ in range(N + 1)]
    for m in range(dem.n_mech):
        ds, o = dem.mech(m)
        assert 1 <= len(ds) <= 2
        a, b = ds[0], ds[1] if len(ds) == 2 else N
        adj[a].append((b, o))
        adj[b].append((a, o))
    best = None
    for start in range(N + 1):
        dist = {(start, 0): 0}
        dq = deque([(start, 0)])
        while dq:
            v, par = dq.popleft()
            if best is not None and dist[(v, par)] >= best:
                break
            for w, o in adj[v]:
                st = (w, par ^ o)
                if st not in dist:
                    dist[st] = dist[(v, par)] + 1
                    dq.append(st)
        if (start, 1) in dist and (best is None or dist[(start, 1)] < best):
            best = dist[(start, 1)]
    return best


# --------------------------------------------------------- code capacity --

@pytest.mark.parametrize("d", [3, 5, 7, 9])
def test_code_capacity_structure(d):
    dem = oracle.code_capacity(d, 0.09)
    assert dem.n_det == (d * d - 1) // 2 == len(plaquettes(d, True))
    assert dem.n_mech == d * d
    assert np.allclose(dem.q, 2 * 0.09 / 3)
    sizes = np.diff(dem.off)
    assert (sizes == 1).sum() == 2 * d and (sizes == 2).sum() == d * d - 2 * d
    # Z stabilizers: products of Z errors that flip nothing
    for (r, c) in plaquettes(d, False):
        qs = [a * d + b for a, b in corners(d, r, c)]
        assert symptom(dem, qs) == (set(), 0)
    # each X check flips exactly on the qubits of its plaquette
    xs = plaquettes(d, True)
    for m in range(dem.n_mech):
        r, c = divmod(m, d)
        want = sorted(i for i, (pr, pc) in enumerate(xs) if (r, c) in corners(d, pr, pc))
        assert list(dem.mech(m)[0]) == want
    # a row of Z errors joins the two Z boundaries: undetectable and logical
    for r in range(d):
        assert symptom(dem, [r * d + c for c in range(d)]) == (set(), 1)


@pytest.mark.parametrize("d", [3, 5, 7])
def test_code_capacity_distance(d):
    assert graph_distance(oracle.code_capacity(d, 0.05)) == d


# ------------------------------------------------------------- memory-Z --

@pytest.mark.parametrize("d,rounds", [(3, 1), (3, 3), (5, 5), (7, 7), (9, 9), (13, 13)])
def test_memory_z_counts_and_determinism(d, rounds):
    dem = oracle.memory_z(d, rounds, 0.004)
    assert dem.n_det == (rounds + 1) * (d * d - 1) // 2
    assert dem.n_gauge_bad == 0        # every detector is deterministic
    assert dem.n_hyper == 0            # graphlike: 1 or 2 detectors each
    sizes = np.diff(dem.off)
    assert sizes.min() >= 1 and sizes.max() <= 2
    assert np.all((dem.q > 0) & (dem.q < 0.1))
    # canonical order: sorted by (detector tuple, observable), no duplicates
    keys = [dem.mech(m) for m in range(dem.n_mech)]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)


@pytest.mark.parametrize("d", [3, 5, 7])
def test_memory_z_distance(d):
    assert graph_distance(oracle.memory_z(d, d, 0.003)) == d


def rotated_layout(d):
    """(data qubits, X-check CNOT partners per layer, Z-check CNOT partners per
    layer, Z-check supports, observable data) of the rotated memory-Z round."""
    xs, zs = plaquettes(d, True), plaquettes(d, False)
    xo = [(0, 0), (0, 1), (1, 0), (1, 1)]
    zo = [(0, 0), (1, 0), (0, 1), (1, 1)]

    def at(r, c):
        return r * d + c if 0 <= r < d and 0 <= c < d else None
    xc = [[at(r + a, c + b) for a, b in xo] for r, c in xs]
    zc = [[at(r + a, c + b) for a, b in zo] for r, c in zs]
    zsup = [[a * d + b for a, b in corners(d, r, c)] for r, c in zs]
    return d * d, xc, zc, zsup, list(range(d))


def unrotated_layout(d):
    """The same for the unrotated code: data where r + c is even on the
    (2d-1)^2 grid, X checks at (odd, even), Z checks at (even, odd), layers
    N, W, E, S (X) and N, E, W, S (Z); the observable reads data column 0."""
    n = 2 * d - 1
    pos = [(r, c) for r in range(n) for c in range(n) if (r + c) % 2 == 0]
    index = {rc: i for i, rc in enumerate(pos)}
    xo = [(-1, 0), (0, -1), (0, 1), (1, 0)]
    zo = [(-1, 0), (0, 1), (0, -1), (1, 0)]
    xs = [(r, c) for r in range(1, n, 2) for c in range(0, n, 2)]
    zs = [(r, c) for r in range(0, n, 2) for c in range(1, n, 2)]
    xc = [[index.get((r + a, c + b)) for a, b in xo] for r, c in xs]
    zc = [[index.get((r + a, c + b)) for a, b in zo] for r, c in zs]
    zsup = [[q for q in row if q is not None] for row in zc]
    return len(pos), xc, zc, zsup, [index[(r, 0)] for r in range(0, n, 2)]


def simulate_memory_z(d, rounds, p, shots, rng, layout=None):
    """Direct frame simulation with exclusive depolarizing outcomes."""
    nd, xc, zc, zsup, obs_q = (layout or rotated_layout)(d)
    nx, nz = len(xc), len(zc)
    nq = nd + nx + nz
    X = np.zeros((nq, shots), dtype=bool)
    Z = np.zeros((nq, shots), dtype=bool)
    anc = list(range(nd, nq))
    xanc = list(range(nd, nd + nx))

    def dep1(q):
        r = rng.random(shots)
        k = np.minimum((r / (p / 3)).astype(np.int64), 3)     # 0 X, 1 Y, 2 Z, 3 none
        X[q] ^= (k == 0) | (k == 1)
        Z[q] ^= (k == 1) | (k == 2)

    def dep2(a, b):
        r = rng.random(shots)
        k = np.minimum((r / (p / 15)).astype(np.int64), 15) + 1   # 1..15 Pauli, 16 none
        k = np.where(k == 16, 0, k)
        X[a] ^= (k & 1) > 0
        Z[a] ^= (k & 2) > 0
        X[b] ^= (k & 4) > 0
        Z[b] ^= (k & 8) > 0

    def xerr(q):
        X[q] ^= rng.random(shots) < p

    for q in range(nq):
        xerr(q)
    meas = []
    for t in range(rounds):
        for q in range(nd):
            dep1(q)
        for q in xanc:
            X[q], Z[q] = Z[q].copy(), X[q].copy()
            dep1(q)
        for k in range(4):
            pairs = [(nd + i, row[k]) for i, row in enumerate(xc) if row[k] is not None]
            pairs += [(row[k], nd + nx + i) for i, row in enumerate(zc) if row[k] is not None]
            used = [q for pr in pairs for q in pr]
            assert len(used) == len(set(used))      # one gate per qubit and layer
            for c_, t_ in pairs:
                X[t_] ^= X[c_]
                Z[c_] ^= Z[t_]
            for c_, t_ in pairs:
                dep2(c_, t_)
        for q in xanc:
            X[q], Z[q] = Z[q].copy(), X[q].copy()
            dep1(q)
        for q in anc:
            xerr(q)
        meas.append(X[nd + nx:].copy())
        for q in anc:
            X[q] = False
            Z[q] = False
            xerr(q)
    for q in range(nd):
        xerr(q)
    final = X[:nd].copy()
    dets = [meas[0]] + [meas[t] ^ meas[t - 1] for t in range(1, rounds)]
    last = meas[-1].copy()
    for i, sup in enumerate(zsup):
        for q in sup:
            last[i] ^= final[q]
    dets.append(last)
    obs = np.logical_xor.reduce(final[obs_q], axis=0)
    return np.concatenate(dets, axis=0), obs


def dem_pair_prob(dem, a, b):
    """Exact P(detector a fires, detector b fires) (b = -1: observable)."""
    dist = np.array([1.0, 0.0, 0.0, 0.0])   # over bits (a, b)
    for m in range(dem.n_mech):
        ds, o = dem.mech(m)
        va = a in ds
        vb = (o == 1) if b == -1 else (b in ds)
        if not (va or vb):
            continue
        v = int(va) | (int(vb) << 1)
        q = dem.q[m]
        new = dist * (1 - q)
        for x in range(4):
            new[x ^ v] += dist[x] * q
        dist = new
    return dist


def _check_against_simulation(dem, det, obs, shots):
    N = dem.n_det
    for a in range(N):
        for b in list(range(a + 1, N)) + [-1]:
            pr = dem_pair_prob(dem, a, b)
            both = (det[a] & (obs if b == -1 else det[b])).mean()
            sd = np.sqrt(pr[3] * (1 - pr[3]) / shots) + 1e-9
            assert abs(both - pr[3]) < 5.5 * sd, (a, b, both, pr[3])
        pa = (det[a]).mean()
        pr = dem_pair_prob(dem, a, a)
        exp_a = pr[1] + pr[3]
        assert abs(pa - exp_a) < 5.5 * np.sqrt(exp_a * (1 - exp_a) / shots)
    po = obs.mean()
    eo = dem_pair_prob(dem, 0, -1)
    eo = eo[2] + eo[3]
    assert abs(po - eo) < 5.5 * np.sqrt(eo * (1 - eo) / shots)


@pytest.mark.slow
def test_memory_z_matches_direct_simulation():
    d, rounds, p, shots = 3, 3, 0.02, 200_000
    dem = oracle.memory_z(d, rounds, p)
    rng = np.random.default_rng(21)
    det, obs = simulate_memory_z(d, rounds, p, shots, rng)
    assert det.shape[0] == dem.n_det
    _check_against_simulation(dem, det, obs, shots)


# ------------------------------------------- unrotated code, code capacity --

def _mech_index(dem, dets, obs):
    dets = tuple(sorted(dets))
    for m in range(dem.n_mech):
        ds, o = dem.mech(m)
        if tuple(ds) == dets and o == obs:
            return m
    raise KeyError((dets, obs))


def _vertical(dem, d, a, j):
    """Z error on the data qubit between X-check rows a-1 and a of column j
    (rows -1 and d-1 are the boundary)."""
    ds = [x for x in ((a - 1) * d + j if a >= 1 else None, a * d + j if a <= d - 2 else None) if x is not None]
    return _mech_index(dem, ds, 1 if a == 0 else 0)


@pytest.mark.parametrize("d", [2, 3, 5, 7])
def test_unrotated_code_capacity_structure(d):
    dem = oracle.code_capacity(d, 0.09, unrotated=True)
    assert dem.n_det == d * (d - 1)
    assert dem.n_mech == d * d + (d - 1) ** 2
    assert np.allclose(dem.q, 2 * 0.09 / 3)
    sizes = np.diff(dem.off)
    assert (sizes == 1).sum() == 2 * d and (sizes == 2).sum() == dem.n_mech - 2 * d
    # only the top boundary edges (X checks of row 0) flip the observable
    for m in range(dem.n_mech):
        ds, o = dem.mech(m)
        if o:
            assert len(ds) == 1 and ds[0] < d
    assert int(dem.obs.sum()) == d
    # check degrees: 4 inside, 3 on the left and right columns
    deg = np.bincount(dem.dets, minlength=dem.n_det)
    for v in range(dem.n_det):
        assert deg[v] == (3 if v % d in (0, d - 1) else 4)
    # Z stabilizers (faces between columns j, j+1 and check rows a-1, a):
    # flip nothing and not the observable
    for a in range(d):
        for j in range(d - 1):
            qs = [_vertical(dem, d, a, j), _vertical(dem, d, a, j + 1)]
            if a >= 1:
                qs.append(_mech_index(dem, [(a - 1) * d + j, (a - 1) * d + j + 1], 0))
            if a <= d - 2:
                qs.append(_mech_index(dem, [a * d + j, a * d + j + 1], 0))
            assert symptom(dem, qs) == (set(), 0)
    # a column of Z errors joins top and bottom: undetectable and logical
    for j in range(d):
        assert symptom(dem, [_vertical(dem, d, a, j) for a in range(d)]) == (set(), 1)


@pytest.mark.parametrize("d", [2, 3, 5, 7])
def test_unrotated_code_capacity_distance(d):
    assert graph_distance(oracle.code_capacity(d, 0.05, unrotated=True)) == d


# ------------------------------------------------ unrotated code, memory-Z --

@pytest.mark.parametrize("d,rounds", [(2, 2), (3, 1), (3, 3), (5, 5), (7, 7), (9, 9)])
def test_unrotated_memory_z_counts_and_determinism(d, rounds):
    dem = oracle.memory_z(d, rounds, 0.004, unrotated=True)
    assert dem.n_det == (rounds + 1) * d * (d - 1)
    assert dem.n_gauge_bad == 0        # every detector is deterministic
    assert dem.n_hyper == 0            # graphlike: 1 or 2 detectors each
    sizes = np.diff(dem.off)
    assert sizes.min() >= 1 and sizes.max() <= 2
    keys = [dem.mech(m) for m in range(dem.n_mech)]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    # the test-side layout of the same round: one gate per qubit and layer
    nd, xc, zc, zsup, obs_q = unrotated_layout(d)
    assert nd == d * d + (d - 1) ** 2 and len(xc) == len(zc) == d * (d - 1) and len(obs_q) == d
    for k in range(4):
        used = [q for row in xc + zc for q in [row[k]] if q is not None]
        assert len(used) == len(set(used))


@pytest.mark.parametrize("d", [2, 3, 5])
def test_unrotated_memory_z_distance(d):
    assert graph_distance(oracle.memory_z(d, d, 0.003, unrotated=True)) == d


@pytest.mark.slow
def test_unrotated_memory_z_matches_direct_simulation():
    d, rounds, p, shots = 3, 2, 0.02, 200_000
    dem = oracle.memory_z(d, rounds, p, unrotated=True)
    rng = np.random.default_rng(22)
    det, obs = simulate_memory_z(d, rounds, p, shots, rng, layout=unrotated_layout)
    assert det.shape[0] == dem.n_det
    _check_against_simulation(dem, det, obs, shots)
