"""Pins of the oracle's quantised variant (oracle/quantize.py), CPU only.

What fixes it independently of its own code: the step formula against hand
values; the per-coefficient error bound g3 (c - chat)^2 <= (delta/2)^2 on
random data; discrete Parseval (the nodal error of the dequantised field
equals the dropped energy plus the coefficient-space quantisation error,
summed independently); the error bound on seeded fields at several
tolerances and budget shares; integer codes below 2^24; the cut equal to the
plain method's cut at the scaled budget; dequantise() reproducing the checked
reconstruction; and planted mistakes that must fail these pins.
"""

import math

import numpy as np
import pytest

import oracle
import synth
from oracle import quantize as Q
from oracle.compress import norm_terms, unpack_bitmap
from oracle.exact import exact_sum
from oracle.tables import gll_tables


def test_step_hand_values():
    assert Q.step(1.0, 0.5, 2) == 1.0 * (1.0 - 2.0 ** -20)      # 2 sqrt(0.25)
    assert Q.step(8.0, 0.0, 8) == 2.0 * (1.0 - 2.0 ** -20)      # 2 sqrt(1)
    assert Q.step(1.0, 0.25, 0) == 0.0


def test_per_coefficient_bound_random():
    rng = np.random.default_rng(1)
    c = rng.normal(size=100000) * 10.0 ** rng.uniform(-6, 2, size=100000)
    g3 = rng.uniform(0.01, 8.0, size=c.size)
    sq = np.sqrt(g3)
    for delta in (1e-7, 3e-4, 0.5):
        q, chat = Q.quantise(c, sq, delta)
        assert np.array_equal(q, np.round(q))
        err = g3 * (c - chat) ** 2
        assert np.all(err <= (delta / 2) ** 2 * (1 + 2.0 ** -40)), float(np.max(err / (delta / 2) ** 2))


@pytest.mark.parametrize("order,E,tol,share", [(7, 40, 1e-3, 0.5), (5, 60, 1e-2, 0.25), (3, 50, 1e-4, 0.75),
                                               (7, 30, 1e-3, 0.0)])
def test_bound_parseval_codes_and_cut(order, E, tol, share):
    u = synth.field(E, order, seed=500 + order)
    T = gll_tables(order)
    res = Q.compress_quantized(u, order, tol, share)
    plain = oracle.compress(u, order, tol, keep_arrays=True, budget_scale=1.0 - share)
    n = order + 1
    for c, (r, p) in enumerate(zip(res, plain.comps)):
        # the cut is the plain method's at the scaled budget
        assert r.tau == p.tau and r.kept == p.kept and np.array_equal(r.bitmap, p.bitmap)
        assert r.B == (tol * tol) * r.U2 and r.dropped == p.dropped
        # codes are integers below 2^24
        assert np.array_equal(r.codes, np.round(r.codes)) and np.max(np.abs(r.codes)) < 2 ** 24
        # bound
        assert r.status == 0 and r.rel_err <= tol and r.err2 <= r.B
        # Parseval: nodal error = dropped energy + coefficient-space quantisation error
        keep = unpack_bitmap(r.bitmap, n)
        g3k = np.broadcast_to(T.g3, keep.shape)[keep]
        qerr = g3k * (p.values - r.values) ** 2
        assert np.all(qerr <= (r.delta / 2) ** 2 * (1 + 2.0 ** -40))
        coef_space = exact_sum(np.concatenate([p.energy[~keep], qerr]))
        assert abs(r.err2 - coef_space) <= 1e-12 * r.err2
        # the codes dequantise to the checked reconstruction
        rec = Q.dequantise(r.bitmap, r.codes, r.delta, order)
        err2 = exact_sum(norm_terms(u[c] - rec, T.w3, None))
        assert err2 == r.err2


def test_planted_mistakes_fail_the_pins():
    rng = np.random.default_rng(2)
    c = rng.normal(size=10000)
    g3 = rng.uniform(0.01, 8.0, size=c.size)
    delta = 1e-3
    # g3 instead of its square root: the bound fails
    q = np.rint((c * g3) / delta)
    chat = (q * delta) / g3
    assert not np.all(g3 * (c - chat) ** 2 <= (delta / 2) ** 2 * (1 + 2.0 ** -40))
    # multiplying by the factor on the way back: the bound fails
    sq = np.sqrt(g3)
    q = np.rint((c * sq) / delta)
    chat = (q * delta) * sq
    assert not np.all(g3 * (c - chat) ** 2 <= (delta / 2) ** 2 * (1 + 2.0 ** -40))
    # a step without the factor 2 keeps the bound but wastes budget; with a
    # factor 4 the budget itself is exceeded on a seeded field
    u = synth.field(40, 7, seed=9)
    T = gll_tables(7)
    plain = oracle.compress(u, 7, 1e-3, keep_arrays=True, budget_scale=0.5).comps[0]
    keep = unpack_bitmap(plain.bitmap, 8)
    B = (1e-3 * 1e-3) * plain.U2
    bad = 4.0 * math.sqrt((B - plain.dropped) / plain.kept)
    _, chat = Q.quantise(plain.values, np.broadcast_to(np.sqrt(T.g3), keep.shape)[keep], bad)
    masked = np.zeros(keep.shape)
    masked[keep] = chat
    err2 = exact_sum(norm_terms(u[0] - oracle.inverse(masked, T.V), T.w3, None))
    assert err2 > B
