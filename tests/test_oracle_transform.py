"""Pins for the oracle's per-element Legendre transforms."""

import numpy as np
import pytest
import scipy.special

import synth
from oracle.tables import gll_tables
from oracle.transform import forward, inverse


def _ref_nodes(N):
    inner, _ = scipy.special.roots_jacobi(N - 1, 1.0, 1.0) if N > 1 else (np.array([]), None)
    return np.concatenate(([-1.0], np.sort(inner), [1.0]))


def _legendre_at(N, x):
    """L[k, i] = P_k(x_i) from numpy's Legendre evaluator."""
    return np.stack([np.polynomial.legendre.legval(x, [0] * k + [1]) for k in range(N + 1)])


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 9])
def test_pure_legendre_field_gives_single_unit_coefficient(N):
    n = N + 1
    L = _legendre_at(N, _ref_nodes(N))
    T = gll_tables(N)
    rng = np.random.default_rng(N)
    picks = [(0, 0, 0), (N, N, N), (N, 0, 1 % n)] + [tuple(rng.integers(0, n, 3)) for _ in range(6)]
    for (r, q, p) in picks:
        u = np.einsum("k,j,i->kji", L[r], L[q], L[p])[None]
        c = forward(u, T.A)[0]
        want = np.zeros((n, n, n))
        want[r, q, p] = 1.0
        np.testing.assert_allclose(c, want, rtol=0, atol=2e-14)


@pytest.mark.parametrize("N", [2, 5, 7, 9])
def test_inverse_evaluates_the_legendre_series(N):
    n = N + 1
    L = _legendre_at(N, _ref_nodes(N))
    T = gll_tables(N)
    rng = np.random.default_rng(10 + N)
    c = rng.standard_normal((2, n, n, n))
    want = np.einsum("erqp,rk,qj,pi->ekji", c, L, L, L)
    np.testing.assert_allclose(inverse(c, T.V), want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("N", [1, 5, 7, 9, 15])
def test_keep_all_round_trip(N):
    u = synth.field(27, N, ncomp=1, seed=3)[0]
    T = gll_tables(N)
    back = inverse(forward(u, T.A), T.V)
    rel = np.sqrt(np.sum((back - u) ** 2) / np.sum(u ** 2))
    assert rel < 1e-14 * max(1, N / 4)


def test_linearity():
    N = 7
    T = gll_tables(N)
    rng = np.random.default_rng(5)
    a = rng.standard_normal((3, 8, 8, 8))
    b = rng.standard_normal((3, 8, 8, 8))
    lhs = forward(2.5 * a - 0.75 * b, T.A)
    rhs = 2.5 * forward(a, T.A) - 0.75 * forward(b, T.A)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-13)


def test_evaluation_order_is_sequential_without_fma():
    """Documents the fixed evaluation order on one element (not a pin: it
    restates the order with scalar Python floats)."""
    N = 2
    n = N + 1
    T = gll_tables(N)
    rng = np.random.default_rng(9)
    u = rng.standard_normal((1, n, n, n))
    A = T.A.tolist()
    x = u[0].tolist()
    t1 = [[[0.0] * n for _ in range(n)] for _ in range(n)]
    for k in range(n):
        for j in range(n):
            for p in range(n):
                acc = A[p][0] * x[k][j][0]
                for i in range(1, n):
                    acc = acc + A[p][i] * x[k][j][i]
                t1[k][j][p] = acc
    t2 = [[[0.0] * n for _ in range(n)] for _ in range(n)]
    for k in range(n):
        for q in range(n):
            for p in range(n):
                acc = A[q][0] * t1[k][0][p]
                for j in range(1, n):
                    acc = acc + A[q][j] * t1[k][j][p]
                t2[k][q][p] = acc
    c = np.zeros((n, n, n))
    for r in range(n):
        for q in range(n):
            for p in range(n):
                acc = A[r][0] * t2[0][q][p]
                for k in range(1, n):
                    acc = acc + A[r][k] * t2[k][q][p]
                c[r, q, p] = acc
    assert np.array_equal(forward(u, T.A)[0], c)
