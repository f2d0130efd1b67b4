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
 - Memory factor (Sec. III.E, "BP Improvements"): the s = 2 closed form
   lambda_00 = l00 - l01 + l11 / alpha after two iterations, which
   multiplying by alpha, or scaling the prior too, would miss.
 - Candidate rules (Sec. III.A-B): the decoder equals its own message
   passing followed by the rules written out here from the text; the
   oracle's selector equals those rules on constructed posterior sequences
   whose candidates differ and tie, where keeping the last converged
   candidate, letting a later equal-weight candidate win, or letting forced
   convergence win a tie each give another output.
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


@pytest.mark.parametrize("alpha", [0.6, 0.85, 1.3, 2.0])
def test_memory_factor_two_defect_closed_form(alpha):
    # Sec. III.E ("BP Improvements"): a variable-to-factor message is the
    # prior plus 1/alpha times the other factor's message.  For s = 2 the
    # factor graph is a tree; by hand, iteration 1 gives M[0][1] = -l00,
    # M[1][0] = -l11, M[0][0] = -l01, M[1][1] = -l01, and iteration 2
    #   lambda_00 = l00 - l01 + l11 / alpha,  lambda_11 = l11 - l01 + l00 / alpha,
    #   lambda_01 = l01 - l00 - l11 (alpha-free),
    # after which the messages repeat.  Multiplying by alpha, or scaling the
    # prior as well, gives other values.
    rng = np.random.default_rng(41)
    for _ in range(10):
        L, W = random_llr_instance(rng, 2)
        l00, l01, l11 = L[0, 0], L[0, 1], L[1, 1]
        for T in (2, 3, 6):
            _, _, _, M, lam = oracle.bp4m_instance(L, W, max_iters=T, alpha=alpha)
            assert abs(lam[0, 0] - (l00 - l01 + l11 / alpha)) < 1e-12
            assert abs(lam[1, 1] - (l11 - l01 + l00 / alpha)) < 1e-12
            assert abs(lam[0, 1] - (l01 - l00 - l11)) < 1e-12
            assert abs(M[0, 0] - (-l01 + l11 / alpha)) < 1e-12
        # the pin is not vacuous: the plausible mistakes miss it
        wrong_mult = l00 - l01 + l11 * alpha
        wrong_prior = l00 - (l01 - l11) / alpha
        assert abs(lam[0, 0] - wrong_mult) > 1e-3 and abs(lam[0, 0] - wrong_prior) > 1e-3


# ---- candidate rules of BP4M and BP4MF, re-derived from the text ----------

def _weight(W, part):
    return int(sum(int(W[i, p]) for i, p in enumerate(part) if p >= i))


def rederived_rules(lam_seq, W, variant, keep="lowest", ties="earliest", fc_ties="converged"):
    """BP4M (Sec. III.A) / BP4MF (Sec. III.B) decisions over the posteriors
    lam_seq[t-1] of iterations t = 1..T, written from the text: marginalize
    at every iteration and keep the lowest-weight converged candidate; BP4MF
    offers the forced-convergence candidate of every iteration that did not
    converge; BP4M runs forced convergence once, after the last iteration,
    if that one did not converge, and outputs the lower-weight of the two.
    keep / ties / fc_ties name the reading (lowest / earliest / converged:
    equal weights keep the earlier candidate, and a converged candidate
    beats a forced one of the same weight); the other values are plausible
    misreadings (keep the last converged candidate; let a later candidate of
    equal weight replace an earlier one; let forced convergence win a tie)."""
    best, best_w, best_fc = None, None, False
    flags = 0

    def offer(part, fc):
        nonlocal best, best_w, best_fc
        w = _weight(W, part)
        if best is None:
            take = True
        elif keep == "last" and not fc:
            take = True
        elif w != best_w:
            take = w < best_w
        elif fc:
            take = fc_ties == "forced"
        else:
            take = ties == "later"
        if take:
            best, best_w, best_fc = part.copy(), w, fc

    conv = False
    for lam in lam_seq:
        conv, part = oracle.marginal_decision(lam)
        if conv:
            flags |= oracle.F_CONVERGED_ANY
            offer(part, False)
        elif variant == 1:
            flags |= oracle.F_FC_RAN
            offer(oracle.forced_convergence(lam), True)
    if variant == 0 and not conv:
        flags |= oracle.F_FC_RAN
        offer(oracle.forced_convergence(lam_seq[-1]), True)
    if best_fc:
        flags |= oracle.F_FC_CHOSEN
    return flags, best, best_w


def bp_posteriors(L, W, T, alpha=1.0):
    """lambda^(t), t = 1..T: the oracle's message passing run for t iterations."""
    return np.stack([oracle.bp4m_instance(L, W, max_iters=t, alpha=alpha)[4] for t in range(1, T + 1)])


@pytest.mark.parametrize("variant", [0, 1])
def test_decoder_equals_rules_applied_to_its_posteriors(variant):
    # the oracle's decoder is its message passing followed by the text's
    # candidate rules, on code-capacity shots where weights tie often
    dem = oracle.code_capacity(7, 0.12)
    tab = oracle.tables(dem)
    n, T = 120, 12
    syn, _ = oracle.sample(dem, 60 + variant, 0, n)
    bits = np.unpackbits(syn.view(np.uint8), axis=1, bitorder="little")[:, :n]
    fc_used = 0
    for b in range(n):
        dd = np.nonzero(bits[:, b])[0]
        if len(dd) < 2:
            continue
        L, W = tab.llr[np.ix_(dd, dd)], tab.dist[np.ix_(dd, dd)]
        fl, part, w, _, _ = oracle.bp4m_instance(L, W, max_iters=T, variant=variant)
        seq = bp_posteriors(L, W, T)
        rf, rp, rw = rederived_rules(seq, W, variant)
        assert fl == rf and w == rw and np.array_equal(part, rp), (b, fl, rf, part, rp)
        sf, sp, sw = oracle.select_sequence(seq, W, variant)
        assert sf == fl and sw == w and np.array_equal(sp, part)
        fc_used += bool(fl & oracle.F_FC_CHOSEN)
    assert fc_used > 0


def _lam_for(s, pairs, rng, pos=None):
    """Symmetric posteriors whose marginal decision picks exactly `pairs`
    (a perfect matching as partner list; None = no row has a positive
    variable, so marginalization does not converge); pos: extra values
    {(i, j): lambda} that shape the forced-convergence order."""
    lam = -rng.uniform(1.0, 3.0, (s, s))
    lam = np.triu(lam) + np.triu(lam, 1).T
    if pairs is not None:
        for i, p in enumerate(pairs):
            lam[i, p] = lam[p, i] = rng.uniform(1.0, 3.0)
    for (i, j), v in (pos or {}).items():
        lam[i, j] = lam[j, i] = v
    return lam


def test_candidate_rules_on_constructed_posteriors():
    # posterior sequences that make the candidates of different iterations
    # differ and tie, which BP itself rarely does (its marginal decisions
    # change little once they converge): the oracle's rules must equal the
    # text's reading, and each misreading must fail somewhere
    rng = np.random.default_rng(44)
    s = 4
    W = np.array([[3, 1, 2, 2], [1, 3, 2, 2], [2, 2, 3, 1], [2, 2, 1, 3]], dtype=np.int64)
    A = [1, 0, 3, 2]           # {01, 23}: weight 2
    B = [2, 3, 0, 1]           # {02, 13}: weight 4
    C = [3, 2, 1, 0]           # {03, 12}: weight 4
    D = [0, 1, 3, 2]           # {00, 11, 23}: weight 7
    # forced convergence on this picks v01 (5), then v23 (4): candidate A
    fcA = {(0, 1): -0.5, (2, 3): -0.6, (0, 0): -0.7}
    # forced convergence on this picks v02 then v13: candidate B
    fcB = {(0, 2): -0.5, (1, 3): -0.6}
    cases = {
        "lowest_not_last": [_lam_for(s, B, rng), _lam_for(s, A, rng), _lam_for(s, C, rng)],
        "tie_keeps_earliest": [_lam_for(s, B, rng), _lam_for(s, C, rng), _lam_for(s, D, rng)],
        "fc_tie_keeps_converged": [_lam_for(s, B, rng), _lam_for(s, None, rng, fcB)],
        "fc_lower_wins": [_lam_for(s, D, rng), _lam_for(s, None, rng, fcA)],
        "fc_only_if_last_failed": [_lam_for(s, None, rng, fcA), _lam_for(s, D, rng)],
        "bp4mf_fc_each_iteration": [_lam_for(s, None, rng, fcB), _lam_for(s, D, rng),
                                    _lam_for(s, None, rng, fcA), _lam_for(s, C, rng)],
    }
    caught = {"keep_last": 0, "ties_later": 0, "fc_wins_ties": 0}
    for name, seq in cases.items():
        seq = np.stack(seq)
        for variant in (0, 1):
            got = oracle.select_sequence(seq, W, variant)
            want = rederived_rules(seq, W, variant)
            assert got[0] == want[0] and np.array_equal(got[1], want[1]) and got[2] == want[2], (name, variant)
            for mis, kw in (("keep_last", {"keep": "last"}), ("ties_later", {"ties": "later"}),
                            ("fc_wins_ties", {"fc_ties": "forced"})):
                m = rederived_rules(seq, W, variant, **kw)
                caught[mis] += not (m[0] == got[0] and np.array_equal(m[1], got[1]))
    print("misreadings caught:", caught)
    assert all(v > 0 for v in caught.values()), caught
    # spot values, by hand from the text
    seq = np.stack(cases["lowest_not_last"])
    fl, part, w = oracle.select_sequence(seq, W, 0)
    assert list(part) == A and w == 2 and fl == oracle.F_CONVERGED_ANY
    seq = np.stack(cases["fc_tie_keeps_converged"])
    fl, part, w = oracle.select_sequence(seq, W, 0)
    assert list(part) == B and w == 4 and fl == oracle.F_CONVERGED_ANY | oracle.F_FC_RAN
    seq = np.stack(cases["fc_only_if_last_failed"])
    fl, part, w = oracle.select_sequence(seq, W, 0)
    assert list(part) == D and fl == oracle.F_CONVERGED_ANY           # BP4M: no forced convergence
    fl, part, w = oracle.select_sequence(seq, W, 1)
    assert list(part) == A and fl == oracle.F_CONVERGED_ANY | oracle.F_FC_RAN | oracle.F_FC_CHOSEN


# ---- diagnostic readings (not used by the library) -------------------------

def test_literal_schedule_repeats_each_flooding_iteration():
    # Sec. II.B's update indices taken literally form both message types of
    # iteration t+1 from those of iteration t; with m_vc = l and m_cv = 0 at
    # t = 0 every factor message then appears twice in a row: iterations
    # 2k-1 and 2k equal flooding iteration k, bit for bit (also with alpha)
    rng = np.random.default_rng(45)
    for s in (2, 3, 5, 8):
        L, W = random_llr_instance(rng, s)
        for alpha in (1.0, 0.85):
            for t in range(1, 9):
                a = oracle.bp4m_instance(L, W, max_iters=t, alpha=alpha, schedule=1)
                b = oracle.bp4m_instance(L, W, max_iters=(t + 1) // 2, alpha=alpha)
                assert np.array_equal(a[3], b[3]) and np.array_equal(a[4], b[4]), (s, alpha, t)
                # so the literal decoder with T iterations is the flooding one with ceil(T/2)
                for variant in (0, 1):
                    fa = oracle.bp4m_instance(L, W, max_iters=t, alpha=alpha, variant=variant, schedule=1)
                    fb = oracle.bp4m_instance(L, W, max_iters=(t + 1) // 2, alpha=alpha, variant=variant)
                    assert fa[0] == fb[0] and np.array_equal(fa[1], fb[1]) and fa[2] == fb[2]


def test_block_maxima_forced_convergence_reading():
    # the Sec. II.D block-maxima procedure over the partition v_ij -> c_min(i,j),
    # with a representative whose partner is taken matched to the boundary:
    # c2 -> v23 (6) and c1 -> v13 (5) lead; c2-c3 is matched, c1's representative
    # conflicts and c1 goes to the boundary, c4's block is {v44}.  The global
    # greedy instead continues with v14 (3).
    v = {(1, 1): -3, (1, 2): 1, (1, 3): 5, (1, 4): 3, (2, 2): -4, (2, 3): 6,
         (2, 4): 0.5, (3, 3): -1, (3, 4): 2, (4, 4): 0.2}
    lam = np.zeros((4, 4))
    for (i, j), x in v.items():
        lam[i - 1, j - 1] = lam[j - 1, i - 1] = x
    assert pairs_of(oracle.forced_convergence_blocks(lam)) == ["1-1", "2-3", "4-4"]
    assert pairs_of(oracle.forced_convergence(lam)) == ["1-4", "2-3"]
    # both readings give valid matchings, and agree when nothing conflicts
    rng = np.random.default_rng(46)
    for _ in range(200):
        s = int(rng.integers(1, 12))
        lam = rng.normal(0, 3, (s, s))
        lam = np.triu(lam) + np.triu(lam, 1).T
        assert valid_matching(oracle.forced_convergence_blocks(lam))
    lam = np.full((5, 5), -5.0)
    for i, j in ((0, 3), (1, 2)):
        lam[i, j] = lam[j, i] = 4.0
    lam[4, 4] = 1.0
    assert np.array_equal(oracle.forced_convergence_blocks(lam), oracle.forced_convergence(lam))


def test_xor_weight_reading_decodes_validly():
    # the XOR-of-paths candidate weight changes only which candidate is kept:
    # every output is still a matching of the shot's defects, whose
    # corrections reproduce the syndrome; on code capacity (paths rarely
    # overlap) it mostly agrees with the sum of path weights
    dem = oracle.code_capacity(7, 0.1, unrotated=True)
    tab = oracle.tables(dem)
    n = 600
    syn, obs = oracle.sample(dem, 47, 0, n)
    a = oracle.decode(dem, tab, syn, obs, n, 25, variant=1, s_cap=64, want_corr=True)
    b = oracle.decode(dem, tab, syn, obs, n, 25, variant=1, s_cap=64, want_corr=True, weight_rule=1)
    W = syn.shape[1]
    H = np.zeros((dem.n_det, dem.n_mech), dtype=np.int64)
    for m in range(dem.n_mech):
        H[dem.dets[dem.off[m]:dem.off[m + 1]], m] = 1
    cb = np.unpackbits(b.corr.view(np.uint8), axis=1, bitorder="little")[:, :n].astype(np.int64)
    sb = (H @ cb) & 1
    assert np.array_equal(sb.astype(bool), np.unpackbits(syn.view(np.uint8), axis=1, bitorder="little")[:, :n] == 1)
    same = (a.flags == b.flags).mean()
    assert same > 0.9, same
