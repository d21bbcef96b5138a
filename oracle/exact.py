"""Exact sums of FP64 terms and their correctly rounded FP64 value.

Test infrastructure (see the package header).  The global quantities of the
method -- the mass-weighted norm, the dropped energy S(v) below a candidate
threshold, the reconstruction error -- are defined as the round-to-nearest
value of the EXACT real sum of their FP64 terms, so they do not depend on any
summation order.

Method: every finite double is m * 2^x with an integer |m| < 2^53
(``numpy.frexp``).  Terms with equal exponent x are added as integers (split
into 26/27-bit halves so int64 never overflows), the per-exponent sums are
combined as Python integers, and the result is an exact ``Fraction``.
Python's int/int true division is correctly rounded, so ``float()`` of that
Fraction is the correctly rounded sum.  Pinned in the tests against
``math.fsum`` (Shewchuk's algorithm, correctly rounded) and against summing
``Fraction`` objects one by one.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np


def exact_sum_fraction(values) -> Fraction:
    """Exact sum of a 1-D array of finite float64 values, as a Fraction."""
    v = np.ascontiguousarray(values, dtype=np.float64).ravel()
    if v.size == 0:
        return Fraction(0)
    if not np.all(np.isfinite(v)):
        raise ValueError("exact_sum: non-finite input")
    f, e = np.frexp(v)                        # v = f * 2^e, 0.5 <= |f| < 1
    m = (f * 2.0 ** 53).astype(np.int64)      # exact integer significand
    x = e.astype(np.int64) - 53               # v = m * 2^x exactly
    nz = m != 0
    if not np.any(nz):
        return Fraction(0)
    m, x = m[nz], x[nz]
    xmin = int(x.min())
    span = int(x.max()) - xmin + 1
    idx = x - xmin
    total = 0
    for sign in (1, -1):
        sel = (m > 0) if sign == 1 else (m < 0)
        if not np.any(sel):
            continue
        a = np.abs(m[sel])
        hi = a >> 26
        lo = a & ((1 << 26) - 1)
        acc_hi = np.zeros(span, dtype=np.int64)
        acc_lo = np.zeros(span, dtype=np.int64)
        # each addend < 2^27, so up to 2^36 terms per exponent fit in int64
        if a.size >= (1 << 36):
            raise ValueError("exact_sum: too many terms")
        np.add.at(acc_hi, idx[sel], hi)
        np.add.at(acc_lo, idx[sel], lo)
        s = 0
        for k in np.flatnonzero((acc_hi != 0) | (acc_lo != 0)):
            s += ((int(acc_hi[k]) << 26) + int(acc_lo[k])) << int(k)
        total += sign * s
    if xmin >= 0:
        return Fraction(total << xmin)
    return Fraction(total, 1 << (-xmin))


def to_double(x: Fraction) -> float:
    """Correctly rounded FP64 value of an exact rational (+-inf on overflow)."""
    try:
        return float(x)
    except OverflowError:
        return float("inf") if x > 0 else float("-inf")


def exact_sum(values) -> float:
    """Correctly rounded (RNE) FP64 value of the exact sum."""
    return to_double(exact_sum_fraction(values))


def rn_leq(x: Fraction, bound: float) -> bool:
    """True iff RN(x) <= bound, for an exact rational x (the feasibility test
    of the threshold rule: the rounded dropped energy must not exceed B)."""
    return to_double(x) <= bound
