"""GPU parity at the full single-snapshot size, in the launch configuration
that bench.py times: 65,536 elements, N = 7, 3 components, tol 1e-3, the
bench's own field (seed 2), a default context.

The oracle runs on component 0 in full (~20 s on one core) and on all three
components for the exact norm:
  * FP64: U2, tau, kept count, bitmap, every kept value and the measured
    error of component 0 equal the oracle's bit for bit;
  * BF16: U2 of every component equals the oracle's exact sum; every
    component meets the bound; component 0's kept set differs from the
    oracle's only inside the threshold band derived from the coefficient
    bound, and decompress() equals the oracle's FP64 inverse of the blob's
    kept values bit for bit.
"""

import math

import numpy as np
import pytest

import oracle
import synth
from oracle.compress import norm_terms, unpack_bitmap
from oracle.exact import exact_sum
from oracle.tables import gll_tables
from test_gpu_mixed import coef_bound

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

E, N, TOL, SEED = 65536, 7, 1e-3, 2


@pytest.fixture(scope="module")
def field():
    u_np = synth.field(E, N, seed=SEED)
    ref0 = oracle.compress(u_np[:1], N, TOL, keep_arrays=True).comps[0]
    return u_np, torch.from_numpy(u_np).cuda(), ref0


def test_fp64_full_size_bit_exact(field):
    from paper_2407_20731_amd import isr
    u_np, u, rc = field
    print(f"[case] fp64 E={E} N={N}", flush=True)
    with isr.Context() as ctx:
        blob = ctx.compress(u, N, TOL, "fp64")
        arr = blob.arrays()
        h = arr.comps[0]
        assert h["U2"] == rc.U2 and h["tau"] == rc.tau and h["kept"] == rc.kept
        assert np.array_equal(arr.bitmap[0], rc.bitmap)
        assert np.array_equal(arr.values[0].view(np.uint64), rc.values.view(np.uint64))
        assert h["rel_err"] == rc.rel_err and rc.rel_err <= TOL
        blob.free()


def test_bf16_full_size(field):
    from paper_2407_20731_amd import isr
    u_np, u, rc = field
    print(f"[case] bf16 E={E} N={N}", flush=True)
    w3 = gll_tables(N).w3
    with isr.Context() as ctx:
        blob = ctx.compress(u, N, TOL, "bf16")
        assert blob.status == 0
        arr = blob.arrays()
        for c in range(3):
            assert arr.comps[c]["U2"] == exact_sum(norm_terms(u_np[c], w3, None)), c
            assert arr.comps[c]["rel_err"] <= TOL, c
        # component 0: kept set against the oracle's, inside the band only
        keep_g = unpack_bitmap(arr.bitmap[0], N + 1)
        keep_o = rc.energy >= rc.tau
        diff = keep_g != keep_o
        bound = coef_bound("bf16", N, np.abs(u_np[0]).reshape(E, -1).max(axis=1))[:, None, None, None]
        g3 = np.broadcast_to(gll_tables(N).g3, rc.coef.shape)
        cabs = np.sqrt(rc.tau / g3)
        beta = 2 * bound / cabs + (bound / cabs) ** 2
        band = np.abs(rc.energy - rc.tau) <= 2 * beta * rc.tau
        assert np.all(band[diff]), (int(diff.sum()), int((~band & diff).sum()))
        # decompress = the oracle's FP64 inverse of the blob's own kept values
        out = ctx.decompress(blob)[0].cpu().numpy()
        mine = oracle.decompress(arr.bitmap[0], arr.values[0].astype(np.float64), N)
        assert np.array_equal(out.view(np.uint64), mine.view(np.uint64))
        # and its error, recomputed exactly, is within the bound up to the
        # FP32 rounding of the stored values and the reduced-precision inverse
        err2 = exact_sum(norm_terms(u_np[0] - mine, w3, None))
        assert math.sqrt(err2 / rc.U2) <= TOL * 1.01
        print(f"[fullsize] bf16 comp0: kept {arr.comps[0]['kept']} vs oracle {rc.kept}, "
              f"{int(diff.sum())} in the band, rel {arr.comps[0]['rel_err']:.7g}", flush=True)
        blob.free()
