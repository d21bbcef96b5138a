"""JPEG-like quantisation of the kept coefficients: a variant of the lossy step.

Test infrastructure (see the package header).

The paper calls its lossy step JPEG-inspired (Sec. IV-B); JPEG quantises the
transform coefficients it keeps.  Reading taken here: the kept Legendre
coefficients are quantised uniformly in the energy norm of the error, so the
error bound still holds.  Per component (unit Jacobians):

  budget   B = (tol * tol) * U2
  cut      the global value threshold of the plain method at the budget
           B_c = B * (1 - share): dropped energy S_c, K kept coefficients
  step     delta = (2 * sqrt((B - S_c) / K)) * (1 - 2^-20)   (0 when K = 0)
  code     q_m = rint((c_m * sqrt(g3_f)) / delta), round half to even; an
           integer of magnitude below 2^24, so an FP32 holds it exactly
  value    chat_m = (q_m * delta) / sqrt(g3_f)
  bound    g3_f (c_m - chat_m)^2 <= (delta / 2)^2 for every kept m (up to
           the rounding of these three operations), so by discrete Parseval
           err2 <= S_c + K (delta / 2)^2 < B
  check    err2 = RN(exact sum of w3 (u - u~)^2), u~ = inverse(chat masked),
           rel = sqrt(err2 / U2)
  repair   while rel > tol (only rounding can cause it), at most 4 times:
           delta <- (delta * (tol / rel)) * (1 - 2^-20), quantise again;
           then ETOL.

The step is one number per component and the codes are integers, which a
lossless coder packs better than FP32 values.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List

import numpy as np

from .compress import OK, ETOL, REPAIR_MAX, REPAIR_SHRINK, compress, norm_terms, unpack_bitmap
from .exact import exact_sum
from .tables import gll_tables
from .transform import inverse

CODE_LIMIT = 2 ** 24


def step(B: float, S: float, K: int) -> float:
    """The quantisation step left by a cut with dropped energy S and K kept
    coefficients under the budget B."""
    if K == 0:
        return 0.0
    return (2.0 * math.sqrt((B - S) / K)) * REPAIR_SHRINK


def quantise(c: np.ndarray, sq: np.ndarray, delta: float):
    """Codes and dequantised values of coefficients c with sqrt(g3) factors sq."""
    q = np.rint((c * sq) / delta)
    return q, (q * delta) / sq


@dataclass
class QuantComponent:
    U2: float
    B: float            # the full budget (tol*tol)*U2
    B_cut: float        # budget of the cut
    tau: float
    dropped: float      # S_c
    kept: int
    delta: float
    codes: np.ndarray   # float64 integers, kept coefficients in (element, f) order
    values: np.ndarray  # dequantised values, same order
    err2: float
    rel_err: float
    repair_iters: int
    status: int
    bitmap: np.ndarray


def compress_quantized(u: np.ndarray, order: int, tol: float, share: float = 0.5) -> List[QuantComponent]:
    """u[ncomp, E, n, n, n], unit Jacobians, tol >= 0, 0 <= share < 1."""
    if not (tol >= 0.0) or not (0.0 <= share < 1.0):
        raise ValueError("need tol >= 0 and 0 <= share < 1")
    u = np.asarray(u, dtype=np.float64)
    n = order + 1
    T = gll_tables(order)
    sq = np.sqrt(T.g3)  # correctly rounded FP64 square roots
    out = []
    for c in range(u.shape[0]):
        uc = u[c]
        U2 = exact_sum(norm_terms(uc, T.w3, None))
        B = (tol * tol) * U2
        cut = compress(uc[None], order, tol, keep_arrays=True, budget_scale=1.0 - share).comps[0]
        keep = unpack_bitmap(cut.bitmap, n)
        coef = cut.coef
        K = cut.kept
        delta = step(B, cut.dropped, K)
        sqb = np.broadcast_to(sq, coef.shape)
        it = 0
        while True:
            if K:
                q, chat = quantise(coef[keep], sqb[keep], delta)
            else:
                q, chat = np.zeros(0), np.zeros(0)
            if q.size and np.max(np.abs(q)) >= CODE_LIMIT:
                raise ValueError("quantisation step too fine for 24-bit codes")
            masked = np.zeros(coef.shape)
            masked[keep] = chat
            recon = inverse(masked, T.V)
            err2 = exact_sum(norm_terms(uc - recon, T.w3, None))
            rel = math.sqrt(err2 / U2) if U2 > 0 else 0.0
            if rel <= tol or it >= REPAIR_MAX:
                break
            delta = (delta * (tol / rel)) * REPAIR_SHRINK
            it += 1
        out.append(QuantComponent(U2=U2, B=B, B_cut=cut.B, tau=cut.tau, dropped=cut.dropped, kept=K, delta=delta,
                                  codes=q, values=chat, err2=err2, rel_err=rel, repair_iters=it,
                                  status=OK if rel <= tol else ETOL, bitmap=cut.bitmap))
    return out


def dequantise(bitmap: np.ndarray, codes: np.ndarray, delta: float, order: int) -> np.ndarray:
    """One component: bitmap [E, W] + codes + step -> nodal field [E, n, n, n]."""
    n = order + 1
    keep = unpack_bitmap(bitmap, n)
    sq = np.broadcast_to(np.sqrt(gll_tables(order).g3), keep.shape)
    c = np.zeros(keep.shape)
    c[keep] = (np.asarray(codes, dtype=np.float64) * delta) / sq[keep]
    return inverse(c, gll_tables(order).V)
