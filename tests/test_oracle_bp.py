"""Pins of the oracle's belief propagation, marginalization and forced
convergence (Sec. II.B-II.D, III.A-III.B).

 - The factor update equals the sum-product message of the exactly-one
   factor computed by brute force over all 2^s configurations.
 - First iteration: M[i][j] = -logsumexp_{k != j} l_ik (scipy).
 - s = 2 is a tree: after two iterations the posteriors are the exact
   closed forms and the messages are at a fixed point.
 - On tree-shaped instances (forbidden variables given prior -1000) BP's
   posteriors equal the exact marginals of P0, found by enumerating matchings.
 - Forced convergence reproduces the paper's Fig. 2 example and the global
   greedy choice on a conflict example; it equals marginalization whenever
   that converged (Sec. II.D); every output is a valid matching.
 - BP4MF's output weight never exceeds BP4M's (Sec. III.B).
"""
import itertools
import os

import mpmath
import numpy as np
import pytest
from scipy.special import logsumexp

import oracle
from tests.inputs import random_llr_instance

HERE = os.path.dirname(os.path.abspath(__file__))
BIG = -1000.0


def test_factor_update_equals_brute_force():
    rng = np.random.default_rng(31)
    for s in range(2, 10):
        for _ in range(3):
            x = rng.uniform(-30, 10, s)
            got = oracle.factor_update(x)
            for j in range(s):
                num = mpmath.mpf(0)
                den = mpmath.mpf(0)
                for cfg in itertools.product((0, 1), repeat=s):
                    if sum(cfg) != 1:
                        continue
                    w = mpmath.exp(sum(mpmath.mpf(x[k]) for k in range(s) if cfg[k]))
                    if cfg[j]:
                        num += 1   # the other variables are 0: weight e^0
                    else:
                        den += w
                want = mpmath.log(num / den)
                assert abs(got[j] - float(want)) <= 1e-13 * max(1.0, abs(float(want)))


def test_first_iteration_is_leave_one_out_lse():
    rng = np.random.default_rng(32)
    L, W = random_llr_instance(rng, 7)
    _, _, _, M, lam = oracle.bp4m_instance(L, W, max_iters=1)
    for i in range(7):
        for j in range(7):
            ref = -logsumexp(np.delete(L[i], j))
            assert abs(M[i, j] - ref) < 1e-12 * max(1, abs(ref))
    for i in range(7):
        for j in range(7):
            want = L[i, i] + M[i, i] if i == j else L[i, j] + M[i, j] + M[j, i]
            assert abs(lam[i, j] - want) < 1e-12 * max(1, abs(want))


def test_two_defects_closed_form_and_fixed_point():
    rng = np.random.default_rng(33)
    for _ in range(20):
        L, W = random_llr_instance(rng, 2)
        _, _, _, M2, lam2 = oracle.bp4m_instance(L, W, max_iters=2)
        _, _, _, M3, _ = oracle.bp4m_instance(L, W, max_iters=3)
        l11, l12, l22 = L[0, 0], L[0, 1], L[1, 1]
        assert abs(lam2[0, 1] - (l12 - l11 - l22)) < 1e-12
        assert abs(lam2[0, 0] - (l11 + l22 - l12)) < 1e-12
        assert abs(lam2[1, 1] - (l11 + l22 - l12)) < 1e-12
        assert np.array_equal(M2, M3)


def matchings(s, allowed):
    """All perfect matchings of s defects with boundary: partner lists."""
    def rec(part):
        if -1 not in part:
            yield list(part)
            return
        i = part.index(-1)
        if allowed[i][i]:
            part[i] = i
            yield from rec(part)
            part[i] = -1
        for j in range(i + 1, s):
            if part[j] == -1 and allowed[i][j]:
                part[i], part[j] = j, i
                yield from rec(part)
                part[i] = part[j] = -1
    yield from rec([-1] * s)


def exact_posteriors(L, allowed):
    s = L.shape[0]
    Z = mpmath.mpf(0)
    on = [[mpmath.mpf(0)] * s for _ in range(s)]
    for part in matchings(s, allowed):
        w = mpmath.exp(sum(mpmath.mpf(L[i, part[i]]) for i in range(s) if part[i] >= i))
        Z += w
        for i in range(s):
            if part[i] >= i:
                on[i][part[i]] += w
    post = np.zeros((s, s))
    for i in range(s):
        for j in range(i, s):
            post[i, j] = post[j, i] = float(mpmath.log(on[i][j] / (Z - on[i][j])))
    return post


@pytest.mark.parametrize("shape", ["chain", "tree"])
def test_bp_exact_on_tree_shaped_instances(shape):
    rng = np.random.default_rng(34 if shape == "chain" else 35)
    for s in (3, 4, 6, 7):
        allowed = np.eye(s, dtype=bool)
        if shape == "chain":
            for i in range(s - 1):
                allowed[i, i + 1] = allowed[i + 1, i] = True
        else:
            for i in range(1, s):
                j = int(rng.integers(0, i))
                allowed[i, j] = allowed[j, i] = True
        L = rng.uniform(-4, 1.5, (s, s))
        L = np.triu(L) + np.triu(L, 1).T
        L = np.where(allowed, L, BIG)
        W = np.ones((s, s), dtype=np.int64)
        _, _, _, _, lam = oracle.bp4m_instance(L, W, max_iters=4 * s)
        post = exact_posteriors(L, allowed)
        for i in range(s):
            for j in range(i, s):
                if allowed[i, j]:
                    assert abs(lam[i, j] - post[i, j]) < 1e-9, (s, i, j, lam[i, j], post[i, j])


def read_fig2():
    lam = np.zeros((4, 4))
    exp = {}
    for line in open(os.path.join(HERE, "golden", "fig2_forced_convergence.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        if parts[0].isdigit():
            i, j, pr = int(parts[0]) - 1, int(parts[1]) - 1, float(parts[2])
            lam[i, j] = lam[j, i] = np.log(pr / (1 - pr))
        else:
            exp[parts[0]] = parts[1:]
    return lam, exp


def pairs_of(partner):
    return sorted("%d-%d" % (i + 1, p + 1) for i, p in enumerate(partner) if p >= i)


def test_fig2_forced_convergence():
    lam, exp = read_fig2()
    conv, marg = oracle.marginal_decision(lam)
    assert conv == bool(int(exp["marginal_converged"][0]))
    assert sorted("%d-%d" % (i + 1, p + 1) for i, p in enumerate(marg) if p >= i) == sorted(exp["marginal_pairs"])
    fc = oracle.forced_convergence(lam)
    assert pairs_of(fc) == sorted(exp["fc_pairs"])


def test_forced_convergence_conflict_is_global_greedy():
    # block maxima (partition v_ij -> c_min(i,j)): c2 -> v23 (6), c1 -> v13 (5);
    # after matching c2-c3, c1's maximum conflicts; the greedy continues with
    # the best still-valid variables: v44 (0.2), then v11 (-3).
    v = {(1, 1): -3, (1, 2): 1, (1, 3): 5, (1, 4): -2, (2, 2): -4, (2, 3): 6,
         (2, 4): 0.5, (3, 3): -1, (3, 4): 2, (4, 4): 0.2}
    lam = np.zeros((4, 4))
    for (i, j), x in v.items():
        lam[i - 1, j - 1] = lam[j - 1, i - 1] = x
    assert pairs_of(oracle.forced_convergence(lam)) == ["1-1", "2-3", "4-4"]


def valid_matching(partner):
    s = len(partner)
    return all(0 <= partner[i] < s and partner[partner[i]] == i for i in range(s))


def test_forced_convergence_equals_marginal_when_converged():
    rng = np.random.default_rng(36)
    for _ in range(200):
        s = int(rng.integers(2, 12))
        perm = rng.permutation(s)
        partner = np.arange(s)
        k = int(rng.integers(0, s // 2 + 1))
        for a in range(k):
            i, j = perm[2 * a], perm[2 * a + 1]
            partner[i], partner[j] = j, i
        lam = -rng.uniform(0.01, 10, (s, s))
        lam = np.triu(lam) + np.triu(lam, 1).T
        for i in range(s):
            lam[i, partner[i]] = lam[partner[i], i] = rng.uniform(0.01, 10)
        conv, marg = oracle.marginal_decision(lam)
        assert conv and np.array_equal(marg, partner)
        assert np.array_equal(oracle.forced_convergence(lam), partner)


def test_forced_convergence_always_valid_with_ties():
    rng = np.random.default_rng(37)
    for _ in range(200):
        s = int(rng.integers(1, 15))
        lam = rng.integers(-3, 3, (s, s)).astype(float)   # many exact ties
        lam = np.triu(lam) + np.triu(lam, 1).T
        fc = oracle.forced_convergence(lam)
        assert valid_matching(fc)
        # greedy property: the first accepted variable is the maximum with
        # the smallest (i, j)
        iu = np.triu_indices(s)
        order = sorted(zip(-lam[iu], iu[0], iu[1]))
        _, i0, j0 = order[0]
        assert fc[i0] == j0


def test_bp4mf_weight_never_exceeds_bp4m():
    rng = np.random.default_rng(38)
    worse = 0
    for _ in range(60):
        s = int(rng.integers(2, 12))
        L, W = random_llr_instance(rng, s)
        f0, p0, w0, _, _ = oracle.bp4m_instance(L, W, max_iters=12, variant=0)
        f1, p1, w1, _, _ = oracle.bp4m_instance(L, W, max_iters=12, variant=1)
        assert valid_matching(p0) and valid_matching(p1)
        assert w1 <= w0
        worse += w1 < w0
    assert worse > 0     # the bound is not vacuous on these instances


def test_relabeling_permutes_messages():
    rng = np.random.default_rng(39)
    s = 9
    L, W = random_llr_instance(rng, s)
    perm = rng.permutation(s)
    _, _, _, M, lam = oracle.bp4m_instance(L, W, max_iters=7)
    _, _, _, Mp, lamp = oracle.bp4m_instance(L[np.ix_(perm, perm)], W[np.ix_(perm, perm)], max_iters=7)
    assert np.allclose(Mp, M[np.ix_(perm, perm)], rtol=1e-11, atol=1e-11)
    assert np.allclose(lamp, lam[np.ix_(perm, perm)], rtol=1e-11, atol=1e-11)


def test_memory_alpha_one_is_plain_bp_and_alpha_changes_messages():
    rng = np.random.default_rng(40)
    L, W = random_llr_instance(rng, 6)
    a = oracle.bp4m_instance(L, W, max_iters=5, alpha=1.0)
    b = oracle.bp4m_instance(L, W, max_iters=5)
    c = oracle.bp4m_instance(L, W, max_iters=5, alpha=0.85)
    assert np.array_equal(a[3], b[3])
    assert not np.allclose(a[3], c[3])
    # iteration 1 does not depend on alpha (all factor messages start at 0)
    a1 = oracle.bp4m_instance(L, W, max_iters=1, alpha=0.85)
    b1 = oracle.bp4m_instance(L, W, max_iters=1)
    assert np.array_equal(a1[3], b1[3])
