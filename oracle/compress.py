"""Error-bounded truncation of Legendre coefficients (the lossy reduction).

Test infrastructure (see the package header).

Follows arXiv 2407.20731 Sec. IV-B: the JPEG-inspired, physics-based lossy step
keeps only the data of the most energetic motions and drops the rest, subject
to a maximal allowed error; the paper's GPU version finds its cut with sorts.
The paper gives no formulas, so the steps below take the readings recorded in
the design notes (global value threshold per velocity component, GLL
mass-weighted relative L2 bound, discrete GLL norms).  Per component c:

  norm      U2 = RN( sum_e sum_kji (J_e * w3[k,j,i]) * (u*u) )      (exact sum)
  energy    e_m = (J_e * g3[r,q,p]) * (c_m * c_m)
  budget    B = (tol * tol) * U2
  threshold S(v) = RN( sum of the energies e_m < v )                 (exact sum)
            tau = max { v in {e_m} U {+inf} : S(v) <= B }
  kept      { m : e_m >= tau }   (all ties at tau are kept)
  check     err2 = RN( sum (J_e * w3) * (d*d) ),  d = u - inverse(c masked)
            rel = sqrt(err2 / U2)  (0 when U2 == 0)
  repair    while rel > tol (at most 4 times):
                B = (B * ((tol/rel) * (tol/rel))) * (1 - 2^-20); redo threshold..check
  tol < 0   keep every coefficient (tau = 0, B = 0), no threshold.

Dropping the smallest energies first keeps the fewest coefficients for a
given dropped energy (exchange argument), and by discrete Parseval under the
GLL mass matrix the squared nodal error equals the dropped energy, so the
threshold rule is the greedy-optimal cut the paper's sorts compute.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .exact import exact_sum, exact_sum_fraction, to_double
from .tables import gll_tables
from .transform import forward, inverse

REPAIR_MAX = 4
REPAIR_SHRINK = 1.0 - 2.0 ** -20

OK = 0
ETOL = -4


def norm_terms(u: np.ndarray, w3: np.ndarray, jac: Optional[np.ndarray]) -> np.ndarray:
    """(J_e * w3[k,j,i]) * (u*u) for u[E, n, n, n]."""
    if jac is None:
        jw = np.broadcast_to(w3, u.shape)
    else:
        jw = np.asarray(jac, dtype=np.float64)[:, None, None, None] * w3[None]
    return jw * (u * u)


def energies(c: np.ndarray, g3: np.ndarray, jac: Optional[np.ndarray]) -> np.ndarray:
    """(J_e * g3[r,q,p]) * (c*c) for c[E, n, n, n]."""
    return norm_terms(c, g3, jac)


def threshold(e: np.ndarray, B: float):
    """Exact global value threshold.

    Returns (tau, n_drop, S) with tau the largest value v among the energies
    (or +inf) whose dropped energy S(v) = RN(exact sum of energies < v) is
    <= B, n_drop the number of energies < tau and S = S(tau).
    """
    s = np.sort(np.asarray(e, dtype=np.float64).ravel())
    n = s.size
    if n == 0:
        return math.inf, 0, 0.0
    firsts = np.flatnonzero(np.concatenate(([True], s[1:] != s[:-1])))
    cuts = np.concatenate((firsts, [n]))  # a cut at n means tau = +inf

    def feasible(k: int) -> bool:
        return to_double(exact_sum_fraction(s[: cuts[k]])) <= B

    # Bracket the answer with ordinary prefix sums and a rigorous error bound
    # for recursive summation of non-negative terms, |err| <= (i-1) u P_i
    # (u = 2^-53, first order; a 2x margin covers the higher-order term),
    # then decide the remaining cuts exactly.
    approx = np.concatenate(([0.0], np.cumsum(s)))[cuts]
    bound = 2.0 * cuts.astype(np.float64) * 2.0 ** -53 * approx
    succ_B = np.nextafter(B, math.inf)
    sure_ok = approx + bound <= B
    sure_bad = approx - bound > succ_B
    lo = int(np.flatnonzero(sure_ok)[-1]) if np.any(sure_ok) else 0
    bad = np.flatnonzero(sure_bad)
    hi = int(bad[0]) if bad.size else cuts.size  # first index known infeasible
    # cut 0 has S = 0 <= B; feasibility is monotone (prefix sums only grow)
    if not feasible(lo):
        raise AssertionError("threshold bracket lost feasibility")
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if feasible(mid):
            lo = mid
        else:
            hi = mid
    n_drop = int(cuts[lo])
    tau = float(s[n_drop]) if n_drop < n else math.inf
    S = to_double(exact_sum_fraction(s[:n_drop]))
    return tau, n_drop, S


def pack_bitmap(keep: np.ndarray) -> np.ndarray:
    """keep[E, n, n, n] (r, q, p) -> uint64 words [E, ceil(n^3/64)], bit f of
    element e set iff flat coefficient f = p + n q + n^2 r is kept (LSB first)."""
    E = keep.shape[0]
    nf = int(np.prod(keep.shape[1:]))
    W = (nf + 63) // 64
    bits = np.zeros((E, W * 64), dtype=np.uint8)
    bits[:, :nf] = keep.reshape(E, nf)
    packed = np.packbits(bits, axis=1, bitorder="little")  # [E, 8W] bytes
    return packed.view("<u8").reshape(E, W)


def unpack_bitmap(words: np.ndarray, n: int) -> np.ndarray:
    E = words.shape[0]
    b = np.unpackbits(np.ascontiguousarray(words).view(np.uint8).reshape(E, -1),
                      axis=1, bitorder="little")
    return b[:, : n ** 3].astype(bool).reshape(E, n, n, n)


@dataclass
class OracleComponent:
    U2: float
    B: float
    tau: float
    dropped: float          # S(tau), correctly rounded dropped energy
    err2: float
    rel_err: float
    kept: int
    bitmap: np.ndarray      # uint64 [E, W]
    elem_ptr: np.ndarray    # uint64 [E + 1]
    values: np.ndarray      # float64 [kept], (element, flat index) order
    repair_iters: int
    status: int
    coef: np.ndarray = field(repr=False, default=None)      # [E, n, n, n]
    energy: np.ndarray = field(repr=False, default=None)    # [E, n, n, n]
    recon: np.ndarray = field(repr=False, default=None)     # [E, n, n, n]


@dataclass
class OracleResult:
    order: int
    tol: float
    comps: List[OracleComponent]

    @property
    def status(self) -> int:
        return ETOL if any(c.status == ETOL for c in self.comps) else OK


def repair_budget(B: float, tol: float, rel: float) -> float:
    """One rounding repair of the budget: B * (tol/rel)^2 * (1 - 2^-20), in
    the association (B * ((tol/rel) * (tol/rel))) * (1 - 2^-20).

    If the dropped energy were exactly the squared error, the ratio alone
    would bring the next cut onto the bound; the extra factor 1 - 2^-20 puts
    it strictly inside."""
    f = tol / rel
    return (B * (f * f)) * REPAIR_SHRINK


def repair_loop(cut_and_check, B: float, tol: float):
    """Cut at budget B and measure the relative error; while it exceeds tol
    (which only rounding can cause on the exact path), lower B with
    ``repair_budget`` and cut again, at most REPAIR_MAX times.

    ``cut_and_check(B) -> (rel, payload)``.  Returns
    ``(payload, B, iterations, status)`` with status ETOL when the last
    measured error still exceeds tol."""
    it = 0
    while True:
        rel, payload = cut_and_check(B)
        if rel <= tol or it >= REPAIR_MAX:
            break
        B = repair_budget(B, tol, rel)
        it += 1
    return payload, B, it, (OK if rel <= tol else ETOL)


def _compress_component(uc, T, tol, jac, keep_arrays, budget_scale=1.0):
    coef = forward(uc, T.A)
    e = energies(coef, T.g3, jac)
    U2 = exact_sum(norm_terms(uc, T.w3, jac))

    def cut_and_check(B):
        if tol < 0:
            tau, S = 0.0, 0.0
        else:
            tau, _, S = threshold(e, B)
        keep = e >= tau
        masked = np.where(keep, coef, 0.0)
        recon = inverse(masked, T.V)
        d = uc - recon
        err2 = exact_sum(norm_terms(d, T.w3, jac))
        rel = math.sqrt(err2 / U2) if U2 > 0 else 0.0
        return rel, (tau, S, keep, recon, err2, rel)

    if tol < 0:
        # keep every coefficient: no threshold, nothing to repair
        rel, payload = cut_and_check(0.0)
        B, it, status = 0.0, 0, OK
    else:
        B0 = (tol * tol) * U2
        if budget_scale != 1.0:
            B0 = B0 * budget_scale  # a share of the budget left to a later stage
        payload, B, it, status = repair_loop(cut_and_check, B0, tol)
    tau, S, keep, recon, err2, rel = payload
    counts = keep.reshape(keep.shape[0], -1).sum(axis=1).astype(np.uint64)
    elem_ptr = np.zeros(keep.shape[0] + 1, dtype=np.uint64)
    np.cumsum(counts, out=elem_ptr[1:])
    return OracleComponent(
        U2=U2, B=B, tau=tau, dropped=S, err2=err2, rel_err=rel,
        kept=int(elem_ptr[-1]), bitmap=pack_bitmap(keep), elem_ptr=elem_ptr,
        values=coef[keep], repair_iters=it, status=status,
        coef=coef if keep_arrays else None,
        energy=e if keep_arrays else None,
        recon=recon if keep_arrays else None,
    )


def compress(u: np.ndarray, order: int, tol: float, jac: Optional[np.ndarray] = None,
             keep_arrays: bool = False, budget_scale: float = 1.0) -> OracleResult:
    """Compress u[ncomp, E, n, n, n] (FP64, i fastest) at relative tolerance tol.
    budget_scale < 1 cuts at ((tol*tol)*U2)*budget_scale instead of the full
    budget (the quantised variant leaves the rest to its quantisation)."""
    u = np.asarray(u, dtype=np.float64)
    n = order + 1
    if u.ndim != 5 or u.shape[2:] != (n, n, n):
        raise ValueError(f"expected [ncomp, E, {n}, {n}, {n}], got {u.shape}")
    if not np.all(np.isfinite(u)):
        raise ValueError("non-finite field value")
    if math.isnan(tol):
        raise ValueError("tol is NaN")
    T = gll_tables(order)
    comps = [_compress_component(u[c], T, float(tol), jac, keep_arrays, budget_scale) for c in range(u.shape[0])]
    return OracleResult(order=order, tol=float(tol), comps=comps)


def decompress(bitmap: np.ndarray, values: np.ndarray, order: int) -> np.ndarray:
    """One component: bitmap [E, W] + kept values -> nodal field [E, n, n, n]."""
    n = order + 1
    keep = unpack_bitmap(bitmap, n)
    coef = np.zeros(keep.shape, dtype=np.float64)
    coef[keep] = np.asarray(values, dtype=np.float64)
    return inverse(coef, gll_tables(order).V)
