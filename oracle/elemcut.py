"""Per-element cut: a variant of the lossy step's selection.

Test infrastructure (see the package header).

The paper's profile names two sorting kernels as the lossy step's main cost
(Sec. IV-B, the timings of the hybrid approach), which fits a selection made
element by element.  Reading taken here: each element gets the share of the budget
that its own energy gives it, and the plain method's value rule (the
threshold of the global cut) is applied inside the element alone.  Per
component:

  element budget  U2_e = RN(exact sum of the element's norm terms),
                  B_e = ((tol * tol) * U2_e) * s, with s = 1 at first
  element cut     tau_e = the plain threshold of the element's energies at
                  B_e (largest energy v, or +inf, whose dropped energy
                  RN(exact sum of energies < v) is <= B_e); kept = e >= tau_e
  totals          U2 = RN(exact sum of all norm terms) (the plain method's),
                  B = (tol * tol) * U2 (reported), dropped = RN(exact sum of
                  every dropped energy)
  check           err2 = RN(exact sum of (J w3) (u - u~)^2) over the whole
                  component, rel = sqrt(err2 / U2)
  repair          while rel > tol (only rounding can cause it), at most 4
                  times: s <- repair_budget(s, tol, rel), the plain method's
                  budget update applied to the scale; then ETOL.

Every element then holds its own relative error below tol, up to rounding,
so the bound holds element by element as well as over the component; the
price is a larger kept set than the global cut needs.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from .compress import (ETOL, OK, REPAIR_MAX, energies, norm_terms, pack_bitmap, repair_budget, threshold)
from .exact import exact_sum
from .tables import gll_tables
from .transform import forward, inverse


@dataclass
class ElemCutComponent:
    U2: float
    B: float                # (tol * tol) * U2, the component's budget
    scale: float            # the final budget scale s
    dropped: float
    err2: float
    rel_err: float
    kept: int
    tau: np.ndarray         # [E] per-element thresholds (+inf: nothing kept)
    U2e: np.ndarray         # [E] per-element norms
    bitmap: np.ndarray      # uint64 [E, W]
    elem_ptr: np.ndarray    # uint64 [E + 1]
    values: np.ndarray      # float64 [kept]
    repair_iters: int
    status: int


def element_cut(en: np.ndarray, B: float):
    """The plain value threshold of one element's energies at budget B:
    (tau, dropped energy S(tau))."""
    tau, _, S = threshold(en, B)
    return tau, S


def compress_elemcut(u: np.ndarray, order: int, tol: float, jac: Optional[np.ndarray] = None,
                     elements: Optional[np.ndarray] = None) -> List[ElemCutComponent]:
    """u[ncomp, E, n, n, n], tol >= 0.  With `elements` given, only those
    elements' cuts are computed (tau, U2e, bitmap rows; no totals, no check):
    the cut of an element depends on that element alone."""
    if not (tol >= 0.0):
        raise ValueError("need tol >= 0")
    u = np.asarray(u, dtype=np.float64)
    n = order + 1
    T = gll_tables(order)
    E = u.shape[1]
    out = []
    for c in range(u.shape[0]):
        uc = u[c]
        ids = np.arange(E) if elements is None else np.asarray(elements)
        jsub = None if jac is None else np.asarray(jac, dtype=np.float64)[ids]
        coef = forward(uc[ids], T.A)
        en = energies(coef, T.g3, jsub)
        nt = norm_terms(uc[ids], T.w3, jsub)
        U2e = np.array([exact_sum(nt[k]) for k in range(ids.size)])
        if elements is not None:
            tau = np.array([element_cut(en[k], ((tol * tol) * U2e[k]) * 1.0)[0] for k in range(ids.size)])
            keep = en >= tau[:, None, None, None]
            out.append(ElemCutComponent(U2=math.nan, B=math.nan, scale=1.0, dropped=math.nan, err2=math.nan,
                                        rel_err=math.nan, kept=int(keep.sum()), tau=tau, U2e=U2e,
                                        bitmap=pack_bitmap(keep), elem_ptr=None, values=coef[keep],
                                        repair_iters=0, status=OK))
            continue
        U2 = exact_sum(norm_terms(uc, T.w3, jac))
        s = 1.0
        it = 0
        while True:
            tau = np.empty(E)
            for e in range(E):
                tau[e], _ = element_cut(en[e], ((tol * tol) * U2e[e]) * s)
            keep = en >= tau[:, None, None, None]
            dropped = exact_sum(en[~keep])
            recon = inverse(np.where(keep, coef, 0.0), T.V)
            err2 = exact_sum(norm_terms(uc - recon, T.w3, jac))
            rel = math.sqrt(err2 / U2) if U2 > 0 else 0.0
            if rel <= tol or it >= REPAIR_MAX:
                break
            s = repair_budget(s, tol, rel)
            it += 1
        counts = keep.reshape(E, -1).sum(axis=1).astype(np.uint64)
        elem_ptr = np.zeros(E + 1, dtype=np.uint64)
        np.cumsum(counts, out=elem_ptr[1:])
        out.append(ElemCutComponent(U2=U2, B=(tol * tol) * U2, scale=s, dropped=dropped, err2=err2, rel_err=rel,
                                    kept=int(elem_ptr[-1]), tau=tau, U2e=U2e, bitmap=pack_bitmap(keep),
                                    elem_ptr=elem_ptr, values=coef[keep], repair_iters=it,
                                    status=OK if rel <= tol else ETOL))
    return out
