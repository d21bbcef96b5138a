"""Per-element tensor-product transforms, nodal <-> Legendre modal.

Test infrastructure (see the package header).

Field layout: u[e, k, j, i] -- element e, GLL node index k (z), j (y), i (x),
i fastest (element-local SEM storage; shared face nodes duplicated).
Coefficients: c[e, r, q, p] -- Legendre degree r (z), q (y), p (x), p fastest.

Forward (nodal -> modal), c = (A (x) A (x) A) u with A = V^{-1}, sum-factorised
into three one-direction contractions, in this order:

    t1[e,k,j,p] = sum_i A[p,i] u [e,k,j,i]
    t2[e,k,q,p] = sum_j A[q,j] t1[e,k,j,p]
    c [e,r,q,p] = sum_k A[r,k] t2[e,k,q,p]

Inverse (modal -> nodal), u~ = (V (x) V (x) V) c, contracting r first:

    s1[e,k,q,p] = sum_r V[k,r] c [e,r,q,p]
    s2[e,k,j,p] = sum_q V[j,q] s1[e,k,q,p]
    u~[e,k,j,i] = sum_p V[i,p] s2[e,k,j,p]

Evaluation order (it fixes every FP64 bit): each sum starts from its first
product and adds the remaining products in ascending summation index,
``acc = acc + a * b``, with the product and the sum rounded separately (no
fused multiply-add).  NumPy's element-wise ``*`` and ``+`` do exactly that.
"""

from __future__ import annotations

import numpy as np


def _contract_last(x: np.ndarray, M: np.ndarray) -> np.ndarray:
    """y[..., a] = sum_b M[a, b] x[..., b], b ascending, no FMA."""
    n = M.shape[0]
    y = np.empty(x.shape[:-1] + (n,), dtype=np.float64)
    for a in range(n):
        acc = M[a, 0] * x[..., 0]
        for b in range(1, n):
            acc = acc + M[a, b] * x[..., b]
        y[..., a] = acc
    return y


def _contract_axis(x: np.ndarray, M: np.ndarray, axis: int) -> np.ndarray:
    """Contract ``axis`` of x with M (same rule), result in the same position."""
    xm = np.moveaxis(x, axis, -1)
    return np.moveaxis(_contract_last(xm, M), -1, axis)


def forward(u: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Nodal [E, n, n, n] (k, j, i) -> Legendre coefficients [E, n, n, n] (r, q, p)."""
    u = np.asarray(u, dtype=np.float64)
    t1 = _contract_axis(u, A, 3)   # i -> p
    t2 = _contract_axis(t1, A, 2)  # j -> q
    return _contract_axis(t2, A, 1)  # k -> r


def inverse(c: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Legendre coefficients [E, n, n, n] (r, q, p) -> nodal [E, n, n, n] (k, j, i)."""
    c = np.asarray(c, dtype=np.float64)
    s1 = _contract_axis(c, V, 1)   # r -> k
    s2 = _contract_axis(s1, V, 2)  # q -> j
    return _contract_axis(s2, V, 3)  # p -> i
