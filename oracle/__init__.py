"""Plain, slow, CPU FP64 oracle for in-situ snapshot reduction.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
C ABI and the Python binding in ``paper_2407_20731_amd``) imports, links or
executes anything in this package.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code,
tables or constants with the GPU path: every table here is computed from the
mathematics with mpmath and exact rationals.

What it computes (arXiv 2407.20731, Sec. IV-B): the physics-based, JPEG-like
lossy reduction of a spectral-element (SEM) velocity snapshot -- keep the
Legendre coefficients of the most energetic motions, drop the rest, under a
relative L2 error bound -- as one data-parallel pass over the elements:

  * ``tables``    GLL nodes/weights, Legendre Vandermonde V, its inverse A,
                  discrete norms gamma, and the tensor tables w3, g3, each the
                  correctly rounded FP64 value of the exact quantity
                  (textbook SEM, Deville et al., the SEM reference of Sec. IV-A).
  * ``exact``     correctly rounded exact sums of FP64 terms (order free).
  * ``transform`` per-element sum-factorised forward (nodal -> modal) and
                  inverse transforms in a fixed evaluation order, no FMA.
  * ``compress``  mass-weighted norm, per-coefficient energies, the global
                  value threshold that enforces the bound, kept sets, the
                  compacted blob arrays, reconstruction, the error check and
                  the rounding repair.
  * ``quantize``  a variant of the lossy step: the cut at a share of the
                  budget, then JPEG-like uniform quantisation of the kept
                  coefficients in the energy norm with the rest of it.
  * ``elemcut``   a variant of the selection: every element cut alone by the
                  plain value rule at its own share of the budget.

Pins (what each function is checked against, in ``tests/test_oracle_*.py``):
closed-form GLL rules, scipy's Gauss-Jacobi roots, quadrature exactness,
numpy's Legendre evaluator, unit coefficients of pure Legendre fields, exact
keep-all round trip, discrete Parseval (with and without per-element
Jacobians), norms re-measured with independent weights and exact rationals,
math.fsum / Fraction sums, brute force over all subsets on tiny inputs,
hand-computed repair budgets and a repair run to its cap, bitmap words
written out by hand for known kept sets, and for the quantised variant its
step against hand values, the per-coefficient error bound on random data and
Parseval with independently summed coefficient-space errors; for the
per-element cut brute force over every subset of tiny elements, each
element equal to the plain method run on it alone, the bound per element and
the repair of the budget scale.  Every function has such a pin.
"""

from .tables import gll_tables, Tables  # noqa: F401
from .exact import exact_sum, exact_sum_fraction, rn_leq  # noqa: F401
from .transform import forward, inverse  # noqa: F401
from .compress import (  # noqa: F401
    OracleComponent,
    OracleResult,
    compress,
    repair_budget,
    repair_loop,
    decompress,
    energies,
    norm_terms,
    threshold,
)
