"""GLL / Legendre tables in high precision, rounded once to FP64.

Test infrastructure (see the package header).  Textbook spectral-element
quantities (Deville, Fischer & Mund, the SEM reference the paper cites in
Sec. IV-A) for polynomial order N, n = N + 1 points per direction:

  xi_i     Gauss-Lobatto-Legendre nodes: -1, the N-1 roots of P_N', +1
  w_i      GLL weights  2 / (N (N+1) P_N(xi_i)^2)
  V[i,k]   Legendre Vandermonde  P_k(xi_i)  (standard P_k, P_k(1) = 1)
  gamma_k  discrete GLL norm of P_k: 2/(2k+1) for k < N and 2/N for k = N
           (GLL quadrature is inexact for P_N^2, hence the different top value)
  A[p,i]   V^{-1} = diag(1/gamma) V^T diag(w), i.e. P_p(xi_i) w_i / gamma_p
  w3       tensor mass weights  w_k w_j w_i    indexed [k, j, i]
  g3       tensor modal norms   gamma_r gamma_q gamma_p  indexed [r, q, p]

Every FP64 table entry is the correctly rounded (round-to-nearest-even) value
of the exact real quantity.  The exact quantities are evaluated with mpmath at
``DPS`` decimal digits (about 330 bits), then rounded through an exact binary
fraction (Python's int/int true division is correctly rounded; mpmath's own
float conversion truncates, so it is not used).
"""

from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction
from functools import lru_cache

import mpmath
import numpy as np

DPS = 100


def _mp():
    ctx = mpmath.mp.clone()
    ctx.dps = DPS
    return ctx


def mpf_to_double(x) -> float:
    """Correctly rounded FP64 value of an mpmath number (exact via Fraction)."""
    sign, man, exp, _ = x._mpf_  # exact binary value of the mpf (no re-rounding)
    if man == 0:
        return 0.0
    f = Fraction(int(man)) * (Fraction(2) ** int(exp))
    if sign:
        f = -f
    return float(f)


def legendre_mp(ctx, k_max, x):
    """[P_0(x), ..., P_k_max(x)] by the three-term recurrence
    (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}."""
    P = [ctx.mpf(1), x]
    for k in range(1, k_max):
        P.append(((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1))
    return P[: k_max + 1]


@lru_cache(maxsize=None)
def gll_nodes_weights_mp(N: int):
    """High-precision GLL nodes and weights for order N >= 1 (tuple of mpf)."""
    if N < 1:
        raise ValueError("order N must be >= 1")
    ctx = _mp()
    n = N + 1
    xs = [None] * n
    xs[0], xs[N] = ctx.mpf(-1), ctx.mpf(1)
    for i in range(1, N):
        # Newton on P_N'(x); start from the Chebyshev-Gauss-Lobatto point.
        x = -ctx.cos(ctx.pi * i / N)
        for _ in range(200):
            P = legendre_mp(ctx, N, x)
            dP = N * (P[N - 1] - x * P[N]) / (1 - x * x)          # P_N'
            d2P = (2 * x * dP - N * (N + 1) * P[N]) / (1 - x * x)  # Legendre ODE
            step = dP / d2P
            x = x - step
            if abs(step) < ctx.mpf(10) ** (-(DPS - 5)):
                break
        xs[i] = x
    # exact symmetry xi_{N-i} = -xi_i, xi = 0 at the centre for even N
    for i in range(n // 2):
        a = (xs[N - i] - xs[i]) / 2
        xs[i], xs[N - i] = -a, a
    if N % 2 == 0:
        xs[N // 2] = ctx.mpf(0)
    ws = []
    for x in xs:
        PN = legendre_mp(ctx, N, x)[N]
        ws.append(ctx.mpf(2) / (N * (N + 1) * PN * PN))
    return tuple(xs), tuple(ws)


def gamma_exact(N: int):
    """Discrete GLL norms of P_0..P_N as exact rationals."""
    return tuple(Fraction(2, 2 * k + 1) for k in range(N)) + (Fraction(2, N),)


@dataclass(frozen=True)
class Tables:
    N: int
    xi: np.ndarray     # [n]
    w: np.ndarray      # [n]
    V: np.ndarray      # [n, n]  V[i, k] = P_k(xi_i)
    A: np.ndarray      # [n, n]  A[p, i] = (V^-1)[p, i]
    gamma: np.ndarray  # [n]
    w3: np.ndarray     # [n, n, n] indexed [k, j, i]
    g3: np.ndarray     # [n, n, n] indexed [r, q, p]


@lru_cache(maxsize=None)
def gll_tables(N: int) -> Tables:
    """Canonical FP64 tables for order N (each entry correctly rounded)."""
    ctx = _mp()
    n = N + 1
    xs, ws = gll_nodes_weights_mp(N)
    gam = gamma_exact(N)
    P = [legendre_mp(ctx, N, x) for x in xs]  # P[i][k]
    V = np.array([[mpf_to_double(P[i][k]) for k in range(n)] for i in range(n)])
    A = np.array([[mpf_to_double(P[i][p] * ws[i] / ctx.mpf(gam[p].numerator) * gam[p].denominator)
                   for i in range(n)] for p in range(n)])
    w3 = np.empty((n, n, n))
    g3 = np.empty((n, n, n))
    for a in range(n):
        for b in range(n):
            for c in range(n):
                w3[a, b, c] = mpf_to_double(ws[a] * ws[b] * ws[c])
                g3[a, b, c] = float(gam[a] * gam[b] * gam[c])  # exact rational -> RN
    return Tables(
        N=N,
        xi=np.array([mpf_to_double(x) for x in xs]),
        w=np.array([mpf_to_double(x) for x in ws]),
        V=V,
        A=A,
        gamma=np.array([float(g) for g in gam]),
        w3=w3,
        g3=g3,
    )
