"""Pins of the oracle's per-element cut (oracle/elemcut.py), CPU only.

What fixes it independently of its own code: brute force over every subset
of each element on tiny inputs (the smallest kept set whose dropped energy,
summed in exact rationals, fits the element's budget); each element's cut
equal to the plain method run on that element alone; the bound element by
element and over the component; Parseval between the error and the dropped
energy; invariants (a permutation of the elements permutes the bitmap rows,
scaling the field by 2^s leaves it unchanged, the kept set is at least the
global cut's); the repair acting on the scale; and planted mistakes that
must fail these pins.
"""

import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import elemcut as P
from oracle.compress import energies, norm_terms, unpack_bitmap
from oracle.exact import exact_sum
from oracle.tables import gll_tables
from oracle.transform import forward, inverse


def _brute_min_kept(en, B):
    """Smallest number of kept energies whose dropped rest sums to <= B
    exactly (in rationals), over all subsets."""
    vals = [Fraction(float(x)) for x in en]
    n = len(vals)
    Bq = Fraction(B)
    for k in range(n + 1):  # kept count
        for kept in itertools.combinations(range(n), k):
            ks = set(kept)
            if sum(v for i, v in enumerate(vals) if i not in ks) <= Bq:
                return k
    return n


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_tiny(seed):
    u = synth.field(3, 1, seed=900 + seed, ncomp=1)
    tol = [0.3, 0.1, 0.5][seed % 3]
    res = P.compress_elemcut(u, 1, tol)[0]
    T = gll_tables(1)
    en = energies(forward(u[0], T.A), T.g3, None)
    keep = unpack_bitmap(res.bitmap, 2)
    for e in range(3):
        Be = (tol * tol) * res.U2e[e] * res.scale
        # no ties in random data: the exact minimum is the oracle's count
        assert keep[e].sum() == _brute_min_kept(en[e].ravel(), Be)
        assert Fraction(float(exact_sum(en[e][~keep[e]]))) <= Fraction(Be)


@pytest.mark.parametrize("order,E,tol", [(3, 30, 1e-2), (5, 20, 1e-3), (7, 12, 1e-3)])
def test_each_element_is_the_plain_method_alone(order, E, tol):
    u = synth.field(E, order, seed=910 + order)
    res = P.compress_elemcut(u, order, tol)
    for c, r in enumerate(res):
        assert r.scale == 1.0 and r.repair_iters == 0
        for e in range(E):
            alone = oracle.compress(u[c:c + 1, e:e + 1], order, tol).comps[0]
            assert alone.U2 == r.U2e[e] and alone.tau == r.tau[e]
            assert np.array_equal(alone.bitmap[0], r.bitmap[e])


@pytest.mark.parametrize("order,E,tol,jac", [(5, 40, 1e-3, False), (7, 25, 1e-2, True), (3, 60, 1e-4, False)])
def test_bounds_parseval_and_global_cut(order, E, tol, jac):
    u = synth.field(E, order, seed=920 + order)
    J = np.random.default_rng(3).uniform(0.5, 2.0, size=E) if jac else None
    T = gll_tables(order)
    res = P.compress_elemcut(u, order, tol, jac=J)
    glob = oracle.compress(u, order, tol, jac=J)
    n = order + 1
    for c, (r, g) in enumerate(zip(res, glob.comps)):
        assert r.status == 0 and r.rel_err <= tol and r.U2 == g.U2 and r.B == g.B
        assert r.kept >= g.kept  # the global cut is the smallest for the global budget
        keep = unpack_bitmap(r.bitmap, n)
        coef = forward(u[c], T.A)
        en = energies(coef, T.g3, J)
        recon = inverse(np.where(keep, coef, 0.0), T.V)
        nt_err = norm_terms(u[c] - recon, T.w3, J)
        for e in range(E):
            # element by element: the dropped energy fits the element's budget
            assert exact_sum(en[e][~keep[e]]) <= ((tol * tol) * r.U2e[e]) * r.scale
            # and the element's own error stays within tol up to rounding
            if r.U2e[e] > 0:
                assert math.sqrt(exact_sum(nt_err[e]) / r.U2e[e]) <= tol * (1 + 1e-9)
        assert r.dropped == exact_sum(en[~keep])
        assert abs(r.err2 - r.dropped) <= 1e-12 * r.err2 + 1e-300
        assert np.array_equal(r.elem_ptr[1:] - r.elem_ptr[:-1], keep.reshape(E, -1).sum(axis=1))
        assert np.array_equal(r.values, coef[keep])


def test_permutation_scaling_zero_and_keep_all():
    u = synth.field(30, 5, seed=930)
    base = P.compress_elemcut(u, 5, 1e-3)
    perm = np.random.default_rng(4).permutation(30)
    pr = P.compress_elemcut(u[:, perm], 5, 1e-3)
    sc = P.compress_elemcut(u * 2.0 ** 7, 5, 1e-3)
    for a, b, s in zip(base, pr, sc):
        assert np.array_equal(a.bitmap[perm], b.bitmap)
        assert np.array_equal(a.bitmap, s.bitmap)
    z = np.zeros((1, 4, 6, 6, 6))
    z[0, 1] = synth.field(1, 5, seed=931, ncomp=1)[0, 0]
    r = P.compress_elemcut(z, 5, 1e-3)[0]
    assert np.all(np.isinf(r.tau[[0, 2, 3]])) and r.elem_ptr[1] == 0 and r.elem_ptr[4] - r.elem_ptr[2] == 0
    # tol 0 drops only exact zeros; the transform round trip's rounding then
    # leaves rel > 0, so the plain method's outcome follows: ETOL after repairs
    k = P.compress_elemcut(u[:1], 5, 0.0)[0]
    plain = oracle.compress(u[:1], 5, 0.0).comps[0]
    assert k.kept == np.count_nonzero(forward(u[0], gll_tables(5).A)) == plain.kept
    assert k.status == plain.status == oracle.compress.__globals__["ETOL"] and k.err2 == plain.err2


def test_sampled_elements_match_the_whole_run():
    u = synth.field(50, 7, seed=932)
    whole = P.compress_elemcut(u, 7, 1e-3)
    ids = np.array([0, 7, 23, 49])
    part = P.compress_elemcut(u, 7, 1e-3, elements=ids)
    for w, p in zip(whole, part):
        assert np.array_equal(w.tau[ids], p.tau) and np.array_equal(w.bitmap[ids], p.bitmap)


def test_repair_scales_every_element_budget(monkeypatch):
    """Force one repair by reporting a relative error above tol once: the
    scale must follow the plain update and every element's cut must then be
    the plain cut at the scaled budget."""
    import oracle.elemcut as mod
    u = synth.field(20, 5, seed=933, ncomp=1)
    real_sqrt = math.sqrt
    calls = {"n": 0}

    class FakeMath:
        inf = math.inf
        nan = math.nan

        @staticmethod
        def sqrt(x):
            calls["n"] += 1
            v = real_sqrt(x)
            return 2e-3 if calls["n"] == 1 else v

    monkeypatch.setattr(mod, "math", FakeMath)
    r = mod.compress_elemcut(u, 5, 1e-3)[0]
    assert r.repair_iters == 1
    assert r.scale == (1.0 * ((1e-3 / 2e-3) * (1e-3 / 2e-3))) * (1.0 - 2.0 ** -20)
    for e in range(20):
        alone = oracle.compress(u[:, e:e + 1], 5, 1e-3, budget_scale=r.scale).comps[0]
        assert alone.tau == r.tau[e]


def test_planted_mistakes_fail_the_pins():
    u = synth.field(12, 5, seed=934)
    T = gll_tables(5)
    res = P.compress_elemcut(u, 5, 1e-3)[0]
    coef = forward(u[0], T.A)
    en = energies(coef, T.g3, None)
    # the component's U2 in place of the element's: not the plain method alone
    wrong = [oracle.elemcut.element_cut(en[e], (1e-3 * 1e-3) * res.U2)[0] for e in range(12)]
    assert any(w != t for w, t in zip(wrong, res.tau))
    # tol instead of tol^2 in the element budget: the element bound fails
    loose = [oracle.elemcut.element_cut(en[e], 1e-3 * res.U2e[e])[0] for e in range(12)]
    assert any(exact_sum(en[e][en[e] < loose[e]]) > (1e-3 * 1e-3) * res.U2e[e] for e in range(12))
