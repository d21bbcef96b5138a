"""Pins for the oracle's GLL / Legendre tables (textbook SEM quadrature)."""

import json
import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest
import scipy.special

from oracle.tables import gamma_exact, gll_nodes_weights_mp, gll_tables, legendre_mp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gll_closed_forms.json")
ORDERS = list(range(1, 16))


def _frac(x: float) -> Fraction:
    return Fraction(*float(x).as_integer_ratio())


def _mp_frac(x) -> Fraction:
    sign, man, exp, _ = x._mpf_
    f = Fraction(int(man)) * Fraction(2) ** int(exp)
    return -f if sign else f


@pytest.mark.parametrize("N", range(2, 16))
def test_interior_nodes_are_gauss_jacobi_roots(N):
    # interior GLL nodes = roots of P_N' = Gauss-Jacobi(alpha=beta=1) nodes of degree N-1
    ref, _ = scipy.special.roots_jacobi(N - 1, 1.0, 1.0)
    T = gll_tables(N)
    np.testing.assert_allclose(T.xi[1:-1], np.sort(ref), rtol=0, atol=4e-15)
    assert T.xi[0] == -1.0 and T.xi[-1] == 1.0


TINY = Fraction(1, 10 ** 80)


@pytest.mark.parametrize("N", ORDERS)
def test_quadrature_exact_to_degree_2N_minus_1(N):
    xs, ws = gll_nodes_weights_mp(N)
    X = [_mp_frac(x) for x in xs]
    Wt = [_mp_frac(w) for w in ws]
    for m in range(0, 2 * N):
        q = sum(w * x ** m for x, w in zip(X, Wt))
        exact = Fraction(0) if m % 2 else Fraction(2, m + 1)
        assert abs(q - exact) < TINY, (N, m)
    # and not exact at degree 2N (GLL, not Gauss): x^{2N} is under-integrated
    q = sum(w * x ** (2 * N) for x, w in zip(X, Wt))
    assert abs(q - Fraction(2, 2 * N + 1)) > Fraction(1, 10 ** 10)


def test_closed_forms_golden():
    rules = json.load(open(GOLDEN))["rules"]
    for key, rule in rules.items():
        N = int(key)
        xs, ws = gll_nodes_weights_mp(N)
        for got, (sgn, r) in zip(xs, rule["nodes"]):
            g = _mp_frac(got)
            assert (g > 0) - (g < 0) == sgn, (N, sgn, r)
            assert abs(g * g - Fraction(r)) < TINY, (N, r)
        for got, s in zip(ws, rule["weights"]):
            assert abs(_mp_frac(got) - Fraction(s)) < TINY, (N, s)


@pytest.mark.parametrize("N", ORDERS)
def test_legendre_matches_numpy_legval(N):
    x = np.linspace(-1, 1, 37)
    ctx = mpmath.mp.clone()
    ctx.dps = 40
    for xv in x:
        P = legendre_mp(ctx, N, ctx.mpf(float(xv)))
        for k in range(N + 1):
            ref = np.polynomial.legendre.legval(xv, [0] * k + [1])
            assert abs(float(P[k]) - ref) < 1e-13
    T = gll_tables(N)
    np.testing.assert_allclose(T.V[-1], np.ones(N + 1), rtol=0, atol=0)           # P_k(1) = 1
    np.testing.assert_allclose(T.V[0], (-1.0) ** np.arange(N + 1), rtol=0, atol=0)  # P_k(-1)


@pytest.mark.parametrize("N", ORDERS)
def test_discrete_orthogonality_and_inverse(N):
    xs, ws = gll_nodes_weights_mp(N)
    ctx = mpmath.mp.clone()
    ctx.dps = 100
    P = [[_mp_frac(v) for v in legendre_mp(ctx, N, x)] for x in xs]
    Wt = [_mp_frac(w) for w in ws]
    gam = gamma_exact(N)
    for a in range(N + 1):
        for b in range(N + 1):
            g = sum(Wt[i] * P[i][a] * P[i][b] for i in range(N + 1))
            want = gam[a] if a == b else Fraction(0)
            assert abs(g - want) < TINY, (N, a, b)
    # the textbook continuous norm 2/(2N+1) is NOT the discrete one at k = N
    assert gam[N] != Fraction(2, 2 * N + 1)
    T = gll_tables(N)
    np.testing.assert_allclose(T.A @ T.V, np.eye(N + 1), rtol=0, atol=2e-15)


def _is_rn(x: float, exact: Fraction) -> bool:
    """x is the round-to-nearest(-even) double of the exact value."""
    d = abs(_frac(x) - exact)
    for nb in (np.nextafter(x, -math.inf), np.nextafter(x, math.inf)):
        dn = abs(_frac(nb) - exact)
        if dn < d:
            return False
        if dn == d and (np.frombuffer(np.float64(x).tobytes(), np.uint64)[0] & 1):
            return False
    return True


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 9, 15])
def test_tables_are_correctly_rounded(N):
    T = gll_tables(N)
    xs, ws = gll_nodes_weights_mp(N)
    ctx = mpmath.mp.clone()
    ctx.dps = 100
    P = [legendre_mp(ctx, N, x) for x in xs]
    gam = gamma_exact(N)
    n = N + 1
    for i in range(n):
        assert _is_rn(T.xi[i], _mp_frac(xs[i]))
        assert _is_rn(T.w[i], _mp_frac(ws[i]))
        for k in range(n):
            assert _is_rn(T.V[i, k], _mp_frac(P[i][k]))
            a_exact = _mp_frac(P[i][k] * ws[i]) / gam[k]
            assert _is_rn(T.A[k, i], a_exact)
    rng = np.random.default_rng(0)
    for _ in range(40):
        a, b, c = rng.integers(0, n, size=3)
        assert _is_rn(T.g3[a, b, c], gam[a] * gam[b] * gam[c])
        assert _is_rn(T.w3[a, b, c], _mp_frac(ws[a]) * _mp_frac(ws[b]) * _mp_frac(ws[c]))
