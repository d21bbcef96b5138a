"""Pins for the oracle's correctly rounded exact sums."""

import math
from fractions import Fraction

import numpy as np
import pytest

from oracle.exact import exact_sum, exact_sum_fraction, rn_leq


def _wide(rng, n, signed):
    x = rng.random(n) * np.exp2(rng.integers(-200, 60, size=n))
    if signed:
        x *= rng.choice([-1.0, 1.0], size=n)
    return x


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("signed", [False, True])
def test_matches_math_fsum(seed, signed):
    rng = np.random.default_rng(seed)
    x = _wide(rng, 5000, signed)
    # ties, zeros and subnormals
    x[:50] = x[50:100]
    x[100:120] = 0.0
    x[120:130] = 5e-324 * rng.integers(1, 1000, size=10)
    assert exact_sum(x) == math.fsum(x.tolist())


@pytest.mark.parametrize("seed", range(4))
def test_matches_fraction_sum(seed):
    rng = np.random.default_rng(100 + seed)
    x = _wide(rng, 300, True)
    want = sum((Fraction(*v.as_integer_ratio()) for v in x.tolist()), Fraction(0))
    assert exact_sum_fraction(x) == want
    assert exact_sum(x) == float(want)


def test_round_half_even_closed_forms():
    u = 2.0 ** -53
    assert exact_sum([1.0, u]) == 1.0                          # tie -> even (1.0)
    assert exact_sum([1.0 + 2 * u, u]) == 1.0 + 4 * u           # tie -> even (up)
    assert exact_sum([1.0, u, 2.0 ** -105]) == 1.0 + 2 * u      # just above the tie
    assert exact_sum([1e300, -1e300, 1e-300]) == 1e-300         # cancellation
    assert exact_sum([0.1] * 10) == 1.0                         # fsum's classic case
    assert sum([0.1] * 10) != 1.0


def test_order_independent():
    rng = np.random.default_rng(7)
    x = _wide(rng, 20000, False)
    s = exact_sum(x)
    for _ in range(3):
        assert exact_sum(rng.permutation(x)) == s


def test_rn_leq():
    u = 2.0 ** -53
    assert rn_leq(Fraction(1) + Fraction(1, 2 ** 53), 1.0)       # rounds to 1.0
    assert not rn_leq(Fraction(1) + Fraction(1, 2 ** 53) + Fraction(1, 2 ** 200), 1.0)
    assert rn_leq(Fraction(0), 0.0)
    assert not rn_leq(Fraction(1, 2 ** 1074), 0.0)
    assert rn_leq(Fraction(1, 2 ** 1076), 0.0)  # below half the smallest subnormal
    assert u > 0
