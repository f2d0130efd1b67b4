"""Pins of the oracle's FP64 exp / log1p / max* against high-precision values.

The Jacobian logarithm max*(x, y) = max(x, y) + ln(1 + exp(-|x - y|)) is the
paper's pairwise soft maximum (Sec. II.B).  Its two transcendental parts are
the oracle's own; here they are checked against mpmath at 60 digits, so a
wrong coefficient, a wrong reduction constant or a wrong series fails.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle

mpmath.mp.dps = 60


def ulp_err(got, exact_mp):
    exact = float(exact_mp)
    if exact == 0.0:
        return 0.0 if got == 0.0 else float("inf")
    ulp = math.ulp(exact)
    return float(abs(mpmath.mpf(got) - exact_mp) / ulp)


def test_exp_accuracy():
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(-708, 0, 4000), rng.uniform(-1, 1, 2000),
                         rng.uniform(0, 700, 1000), np.array([0.0, -0.0, -1e-300, -708.0, 1.0])])
    ys = oracle.exp(xs)
    worst = max(ulp_err(y, mpmath.exp(mpmath.mpf(x))) for x, y in zip(xs, ys))
    assert worst <= 1.0, worst


def test_exp_cutoff_and_special_values():
    assert oracle.exp([-708.5])[0] == 0.0
    assert oracle.exp([0.0])[0] == 1.0
    assert math.isinf(oracle.exp([710.0])[0])


def test_log1p_accuracy():
    rng = np.random.default_rng(2)
    xs = np.concatenate([rng.uniform(0, 1, 4000), 10.0 ** rng.uniform(-300, 0, 2000),
                         np.array([0.0, 1.0, 5e-324, 1e-17, 0.5])])
    ys = oracle.log1p(xs)
    worst = max(ulp_err(y, mpmath.log1p(mpmath.mpf(x))) for x, y in zip(xs, ys))
    assert worst <= 3.0, worst


def test_maxstar_is_log_sum_exp():
    rng = np.random.default_rng(3)
    a = rng.uniform(-50, 50, 3000)
    b = a + rng.choice([-1, 1], 3000) * 10.0 ** rng.uniform(-12, 2.5, 3000)
    got = oracle.maxstar(a, b)
    for x, y, g in zip(a, b, got):
        ex = mpmath.log(mpmath.exp(mpmath.mpf(x)) + mpmath.exp(mpmath.mpf(y)))
        # the sum max + log1p(..) can cancel: bound the error by its operands
        scale = max(abs(x), abs(y), math.log(2.0))
        assert abs(mpmath.mpf(g) - ex) <= 4 * math.ulp(scale), (x, y, g, ex)


def test_maxstar_symmetric_bitwise():
    rng = np.random.default_rng(4)
    a = rng.normal(0, 20, 5000)
    b = rng.normal(0, 20, 5000)
    assert np.array_equal(oracle.maxstar(a, b), oracle.maxstar(b, a))
    assert oracle.maxstar([3.0], [3.0])[0] == 3.0 + math.log(2.0)
