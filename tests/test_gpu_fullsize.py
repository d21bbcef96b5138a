"""GPU parity at the full single-snapshot size, in the launch configuration
that bench.py times: 65,536 elements, N = 7, 3 components, the bench's own
field (seed 2), a default context.

The oracle runs on component 0 in full (~7 s a component on one core) and
on all three components for the exact norm:
  * FP64 at tol 1e-3 and at tol 1e-5: U2, tau, kept count, bitmap, every
    kept value and the measured error of component 0 equal the oracle's bit
    for bit;
  * BF16 and FP32 at tol 1e-3: U2 of every component within 1e-12 of the
    oracle's exact sum, every component meets the bound, and component 0 passes every
    check of tests/mixed_checks.py (budget, threshold, its own cut, the
    oracle's cut at the same budget and at its own, coefficient bound, and
    the decompressed output's exact error <= tol and equal to the reported
    one).
"""

import numpy as np
import pytest

import oracle
import synth
from mixed_checks import verify_mixed
from oracle.compress import norm_terms
from oracle.exact import exact_sum
from oracle.tables import gll_tables

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

E, N, TOL, SEED = 65536, 7, 1e-3, 2


@pytest.fixture(scope="module")
def field():
    u_np = synth.field(E, N, seed=SEED)
    return u_np, torch.from_numpy(u_np).cuda(), {}


def oracle0(field, tol):
    """The oracle's component 0 at tol (computed once per tol)."""
    u_np, _, cache = field
    if tol not in cache:
        cache[tol] = oracle.compress(u_np[:1], N, tol, keep_arrays=True).comps[0]
    return cache[tol]


@pytest.mark.parametrize("tol", [1e-3, 1e-5])
def test_fp64_full_size_bit_exact(field, tol):
    from paper_2407_20731_amd import isr
    u_np, u, _ = field
    print(f"[case] fp64 E={E} N={N} tol={tol}", flush=True)
    rc = oracle0(field, tol)
    with isr.Context() as ctx:
        blob = ctx.compress(u, N, tol, "fp64")
        arr = blob.arrays()
        h = arr.comps[0]
        assert h["U2"] == rc.U2 and h["tau"] == rc.tau and h["kept"] == rc.kept
        assert np.array_equal(arr.bitmap[0], rc.bitmap)
        assert np.array_equal(arr.values[0].view(np.uint64), rc.values.view(np.uint64))
        assert h["rel_err"] == rc.rel_err and rc.rel_err <= tol
        assert blob.status == 0
        blob.free()


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_mixed_full_size(field, prec):
    from paper_2407_20731_amd import isr
    u_np, u, _ = field
    print(f"[case] {prec} E={E} N={N}", flush=True)
    rc = oracle0(field, TOL)
    w3 = gll_tables(N).w3
    with isr.Context() as ctx:
        blob = ctx.compress(u, N, TOL, prec)
        assert blob.status == 0
        arr = blob.arrays()
        for c in range(3):
            U2x = exact_sum(norm_terms(u_np[c], w3, None))
            assert abs(arr.comps[c]["U2"] - U2x) <= 1e-12 * U2x, c
            assert arr.comps[c]["rel_err"] <= TOL, c
        coef = ctx.forward(u[:1], N, prec)[0].cpu().numpy().astype(np.float64)[None]
        out = ctx.decompress(blob)[0].cpu().numpy()[None]
        torch.cuda.synchronize()
        report = verify_mixed(arr, blob.status, blob.stats["repair_iters"], u_np[:1], N, TOL, prec, coef, [rc],
                              out=out, comps=[0])
        print(f"[fullsize] {prec} comp0: {report}", flush=True)
        blob.free()
