"""Pins for three oracle parts: the per-element Jacobian weighting, the
rounding repair of the budget, and the bit order of the kept-set bitmaps.

The Jacobian J_e of an affine hexahedron multiplies every GLL mass weight of
its element, so it enters the norm terms, the coefficient energies and the
error terms to the first power (Sec. IV-B's error-bounded reduction under the
mass-weighted L2 norm; the norm is the textbook SEM one).  Independent
references here: scipy's Gauss-Jacobi nodes with weights from numpy's Legendre
evaluator, exact rationals, closed-form discrete Legendre norms, and
hand-computed budgets and bitmap words.  Each part also gets a planted
mistake that one of its pins must catch.
"""

import importlib
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.special

import oracle
import synth
from oracle.compress import (ETOL, OK, REPAIR_MAX, energies, norm_terms, pack_bitmap, repair_budget,
                             repair_loop, unpack_bitmap)
from oracle.exact import exact_sum, exact_sum_fraction
from oracle.tables import gll_tables
from oracle.transform import forward, inverse

# the module itself (the package re-exports a function of the same name)
oc = importlib.import_module("oracle.compress")


def _ref_nodes_weights(N):
    inner, _ = scipy.special.roots_jacobi(N - 1, 1.0, 1.0)
    x = np.concatenate(([-1.0], np.sort(inner), [1.0]))
    PN = np.polynomial.legendre.legval(x, [0] * N + [1])
    return x, 2.0 / (N * (N + 1) * PN * PN)


def _legendre_at(N, x):
    return np.stack([np.polynomial.legendre.legval(x, [0] * k + [1]) for k in range(N + 1)])


def _jacobians(E, seed):
    """Positive, strongly non-uniform Jacobians (2^-8 .. 2^8, not powers of two)."""
    rng = np.random.default_rng(seed)
    return np.exp2(rng.uniform(-8.0, 8.0, size=E))


def _ref_weighted_norm2(u, N, jac):
    """sum_e J_e sum_kji w_k w_j w_i u^2 with scipy-derived weights, exact rationals."""
    _, w = _ref_nodes_weights(N)
    w3 = np.einsum("k,j,i->kji", w, w, w)
    total = Fraction(0)
    for e in range(u.shape[0]):
        total += Fraction(float(jac[e])) * exact_sum_fraction((w3 * (u[e] * u[e])).ravel())
    return total


# ------------------------------------------------------------- Jacobians


@pytest.mark.parametrize("N", [2, 5, 7])
def test_parseval_with_jacobians(N):
    # sum J w3 u^2 == sum J g3 c^2 for any positive J (Parseval holds per element)
    u = synth.field(24, N, ncomp=1, seed=31)[0]
    J = _jacobians(24, N)
    T = gll_tables(N)
    U2 = exact_sum(norm_terms(u, T.w3, J))
    E2 = exact_sum(energies(forward(u, T.A), T.g3, J))
    assert abs(U2 - E2) <= 1e-13 * U2


@pytest.mark.parametrize("N", [3, 7])
def test_weighted_norm_matches_independent_weights(N):
    u = synth.field(12, N, ncomp=1, seed=32)[0]
    J = _jacobians(12, 100 + N)
    U2 = exact_sum(norm_terms(u, gll_tables(N).w3, J))
    ref = float(_ref_weighted_norm2(u, N, J))
    assert abs(U2 - ref) <= 1e-14 * ref


def test_energy_of_a_pure_mode_with_jacobian():
    # N = 3: gamma = (2, 2/3, 2/5, 2/3) (the top mode's discrete norm is 2/N).
    # Mode (r, q, p) = (1, 2, 3) with amplitude 1/2 in an element of J = 3:
    # e = 3 * (2/3)(2/5)(2/3) * (1/2)^2 = 2/15.
    N = 3
    x, _ = _ref_nodes_weights(N)
    L = _legendre_at(N, x)
    u = 0.5 * np.einsum("k,j,i->kji", L[1], L[2], L[3])[None]
    e = energies(forward(u, gll_tables(N).A), gll_tables(N).g3, np.array([3.0]))[0]
    assert abs(e[1, 2, 3] - 2.0 / 15.0) <= 1e-14
    others = e.copy()
    others[1, 2, 3] = 0.0
    assert others.max() <= 1e-28


def test_power_of_two_jacobian_scales_norm_and_keeps_bitmap():
    N = 7
    u = synth.field(30, N, ncomp=1, seed=33)
    a = oracle.compress(u, N, 1e-3).comps[0]
    for s in (-5, 3):
        b = oracle.compress(u, N, 1e-3, jac=np.full(30, 2.0 ** s)).comps[0]
        assert b.U2 == a.U2 * 2.0 ** s and b.tau == a.tau * 2.0 ** s
        assert np.array_equal(b.bitmap, a.bitmap) and np.array_equal(b.values, a.values)
        assert b.rel_err == a.rel_err


def test_permuting_jacobians_with_elements_permutes_bitmaps():
    N = 5
    u = synth.field(40, N, ncomp=1, seed=34)
    J = _jacobians(40, 35)
    perm = np.random.default_rng(1).permutation(40)
    a = oracle.compress(u, N, 1e-3, jac=J).comps[0]
    b = oracle.compress(u[:, perm], N, 1e-3, jac=J[perm]).comps[0]
    assert a.tau == b.tau and a.U2 == b.U2 and a.kept == b.kept
    assert np.array_equal(a.bitmap[perm], b.bitmap)
    # and the Jacobians change the cut: without them another set is kept
    c = oracle.compress(u, N, 1e-3).comps[0]
    assert not np.array_equal(a.bitmap, c.bitmap)


@pytest.mark.parametrize("tol", [1e-2, 1e-3])
def test_error_with_jacobians_equals_dropped_energy(tol):
    N = 5
    u = synth.field(40, N, ncomp=1, seed=36)
    J = _jacobians(40, 37)
    comp = oracle.compress(u, N, tol, jac=J, keep_arrays=True).comps[0]
    assert comp.status == OK and comp.rel_err <= tol
    assert abs(comp.err2 - comp.dropped) <= 1e-11 * comp.err2
    # re-measure the reconstruction error with independent weights and J
    x, _ = _ref_nodes_weights(N)
    L = _legendre_at(N, x)
    keep = unpack_bitmap(comp.bitmap, N + 1)
    recon = np.einsum("erqp,rk,qj,pi->ekji", np.where(keep, comp.coef, 0.0), L, L, L)
    rel = math.sqrt(float(_ref_weighted_norm2(u[0] - recon, N, J) / _ref_weighted_norm2(u[0], N, J)))
    assert abs(rel - comp.rel_err) <= 1e-8 * tol


def test_pins_catch_squared_jacobian_in_energy():
    N = 5
    u = synth.field(24, N, ncomp=1, seed=31)[0]
    J = _jacobians(24, N)
    T = gll_tables(N)
    U2 = exact_sum(norm_terms(u, T.w3, J))
    wrong = exact_sum(energies(forward(u, T.A), T.g3, J * J))
    assert abs(U2 - wrong) > 1e-2 * U2
    # the pure-mode pin catches it too: J^2 gives 9 * 8/45 / 4 = 2/5
    x, _ = _ref_nodes_weights(3)
    L = _legendre_at(3, x)
    v = 0.5 * np.einsum("k,j,i->kji", L[1], L[2], L[3])[None]
    e = energies(forward(v, gll_tables(3).A), gll_tables(3).g3, np.array([9.0]))[0]
    assert abs(e[1, 2, 3] - 2.0 / 15.0) > 0.1


def test_pins_catch_jacobian_dropped_from_error():
    N = 5
    u = synth.field(40, N, ncomp=1, seed=36)
    J = _jacobians(40, 37)
    comp = oracle.compress(u, N, 1e-3, jac=J, keep_arrays=True).comps[0]
    wrong = exact_sum(norm_terms(u[0] - comp.recon, gll_tables(N).w3, None))
    assert abs(wrong - comp.dropped) > 1e-2 * comp.dropped


# ----------------------------------------------------------------- repair


def test_repair_budget_hand_values():
    # tol/rel = 1e-3/2e-3 = 1/2 exactly (2e-3 is twice the double 1e-3), so
    # B = 1 -> 1 * 1/4 * (1 - 2^-20) = 2^-2 - 2^-22, exactly representable
    assert repair_budget(1.0, 1e-3, 2e-3) == 0.25 - 2.0 ** -22
    # ratio 1/4: B = 3 -> 3/16 (1 - 2^-20) = 3 * 2^-4 - 3 * 2^-24
    assert repair_budget(3.0, 0.25, 1.0) == 3 * 2.0 ** -4 - 3 * 2.0 ** -24
    # rel == tol leaves only the shrink factor
    assert repair_budget(5.0, 0.1, 0.1) == 5.0 * (1.0 - 2.0 ** -20)


def test_repair_loop_runs_to_its_cap():
    # a check that always measures twice the bound: four repairs, then ETOL.
    # B_k = (1/4)^k (1 - 2^-20)^k, rounded after each step:
    #   B1 = 2^-2 (1 - 2^-20)
    #   B2 = 2^-4 (1 - 2^-19 + 2^-40)                       (41 bits: exact)
    #   B3 = 2^-6 RN(1 - 3*2^-20 + 3*2^-40 - 2^-60)  = 2^-6 (1 - 3*2^-20 + 3*2^-40)
    #   B4 = 2^-8 RN(1 - 4*2^-20 + 6*2^-40 - 3*2^-60) = 2^-8 (1 - 4*2^-20 + 6*2^-40)
    # (the dropped 2^-60 terms are below half an ulp, 2^-54, of a number in [1/2, 1))
    seen = []

    def check(B):
        seen.append(B)
        return 2e-3, len(seen)

    payload, B, it, status = repair_loop(check, 1.0, 1e-3)
    want = [1.0,
            2.0 ** -2 * (1 - 2.0 ** -20),
            2.0 ** -4 * (1 - 2.0 ** -19 + 2.0 ** -40),
            2.0 ** -6 * (1 - 3 * 2.0 ** -20 + 3 * 2.0 ** -40),
            2.0 ** -8 * (1 - 4 * 2.0 ** -20 + 6 * 2.0 ** -40)]
    assert seen == want
    assert it == REPAIR_MAX == 4 and status == ETOL and payload == 5 and B == want[-1]


def test_repair_loop_stops_once_within_bound():
    rels = iter([3e-3, 1e-3])  # the second cut meets the bound exactly (rel == tol is fine)

    def check(B):
        return next(rels), B

    payload, B, it, status = repair_loop(check, 2.0, 1e-3)
    # tol/rel = 1e-3/3e-3 rounds to 0.333...; the budget follows the same association
    assert it == 1 and status == OK and B == payload == (2.0 * ((1e-3 / 3e-3) * (1e-3 / 3e-3))) * (1 - 2.0 ** -20)
    assert abs(B - 2.0 / 9.0) <= 1e-6


def test_repair_end_to_end_with_injected_reconstruction_error(monkeypatch):
    # Inflate every reconstruction by (1 + tol/2): the error then carries an
    # extra ~(tol/2)^2 U2 that no cut removes, so the loop repairs four times
    # and returns ETOL with the last cut's arrays.
    N, tol = 5, 1e-3
    u = synth.field(30, N, ncomp=1, seed=38)
    clean = oracle.compress(u, N, tol).comps[0]
    assert clean.repair_iters == 0
    budgets = []
    real_repair = oc.repair_budget

    def recording_repair(B, t, rel):
        assert rel > t
        budgets.append((B, rel))
        return real_repair(B, t, rel)

    monkeypatch.setattr(oc, "inverse", lambda c, V: inverse(c, V) * (1.0 + tol / 2))
    monkeypatch.setattr(oc, "repair_budget", recording_repair)
    comp = oracle.compress(u, N, tol).comps[0]
    assert comp.repair_iters == 4 and comp.status == ETOL and comp.rel_err > tol
    assert budgets[0][0] == (tol * tol) * clean.U2
    for (b0, r0), (b1, _) in zip(budgets, budgets[1:]):
        assert b1 == real_repair(b0, tol, r0) and b1 < b0
    assert comp.B == real_repair(*budgets[-1][:1], tol, budgets[-1][1])
    # the payload is the last cut: its dropped energy fits the last budget
    assert comp.dropped <= comp.B and comp.kept > clean.kept


def test_repair_end_to_end_one_step(monkeypatch):
    # Only the first reconstruction is off; one repair at the measured ratio
    # brings the next cut inside the bound.
    N, tol = 5, 1e-3
    u = synth.field(30, N, ncomp=1, seed=38)
    calls = []

    def first_off(c, V):
        calls.append(1)
        r = inverse(c, V)
        return r * (1.0 + tol) if len(calls) == 1 else r

    monkeypatch.setattr(oc, "inverse", first_off)
    comp = oracle.compress(u, N, tol).comps[0]
    B0 = (tol * tol) * comp.U2
    assert comp.repair_iters == 1 and comp.status == OK and comp.rel_err <= tol
    assert B0 * 0.2 < comp.B < B0


def test_pins_catch_unsquared_repair_ratio():
    def unsquared(B, tol, rel):
        return (B * (tol / rel)) * (1.0 - 2.0 ** -20)

    assert unsquared(1.0, 1e-3, 2e-3) != 0.25 - 2.0 ** -22

    def wrong_shrink(B, tol, rel):
        f = tol / rel
        return (B * (f * f)) * (1.0 - 2.0 ** -10)

    assert wrong_shrink(1.0, 1e-3, 2e-3) != 0.25 - 2.0 ** -22


# ------------------------------------------------------------- bitmaps


def _field_from_coefficients(c, N):
    x, _ = _ref_nodes_weights(N)
    L = _legendre_at(N, x)
    return np.einsum("erqp,rk,qj,pi->ekji", c, L, L, L)[None]


def test_bitmap_words_n3_hand():
    # N = 2 (n = 3): modes (r,q,p) = (0,0,0) and (1,0,0) kept -> flat f = 0 and
    # f = p + 3q + 9r = 9 -> word 0 = 2^0 + 2^9 = 513
    c = np.zeros((1, 3, 3, 3))
    c[0, 0, 0, 0] = 1.0
    c[0, 1, 0, 0] = 0.1
    c[0, 0, 2, 0] = 0.01
    comp = oracle.compress(_field_from_coefficients(c, 2), 2, 0.01).comps[0]
    assert comp.bitmap.shape == (1, 1) and int(comp.bitmap[0, 0]) == 513


def test_bitmap_words_n7_hand():
    # N = 7 (n = 8, 512 bits = 8 words): kept modes (0,0,0) -> f 0 (word 0 bit 0),
    # (r,q,p) = (1,2,3) -> f = 3 + 16 + 64 = 83 (word 1 bit 19), (7,7,7) -> f 511
    # (word 7 bit 63)
    c = np.zeros((1, 8, 8, 8))
    c[0, 0, 0, 0], c[0, 1, 2, 3], c[0, 7, 7, 7] = 1.0, 0.5, -0.25
    comp = oracle.compress(_field_from_coefficients(c, 7), 7, 1e-3).comps[0]
    want = [1, 1 << 19, 0, 0, 0, 0, 0, 1 << 63]
    assert [int(w) for w in comp.bitmap[0]] == want
    assert np.array_equal(comp.elem_ptr, np.array([0, 3], dtype=np.uint64))
    assert np.array_equal(comp.values, np.array([1.0, 0.5, -0.25])) or \
        np.allclose(comp.values, [1.0, 0.5, -0.25], rtol=1e-14)


def test_bitmap_words_n5_pad_bits_zero():
    # N = 5 (n = 6, 216 bits in 4 words, 40 pad bits): (5,5,5) -> f 215 = word 3 bit 23
    keep = np.zeros((2, 6, 6, 6), bool)
    keep[1, 5, 5, 5] = True
    keep[0, 0, 1, 0] = True  # f = 6
    words = pack_bitmap(keep)
    assert [int(w) for w in words[0]] == [1 << 6, 0, 0, 0]
    assert [int(w) for w in words[1]] == [0, 0, 0, 1 << 23]
    assert np.array_equal(unpack_bitmap(words, 6), keep)


def test_pins_catch_msb_first_bitmap():
    def msb_first(keep):
        E = keep.shape[0]
        nf = int(np.prod(keep.shape[1:]))
        W = (nf + 63) // 64
        bits = np.zeros((E, W * 64), dtype=np.uint8)
        bits[:, :nf] = keep.reshape(E, nf)
        return np.packbits(bits, axis=1, bitorder="big").view("<u8").reshape(E, W)

    keep = np.zeros((1, 3, 3, 3), bool)
    keep[0, 0, 0, 0] = keep[0, 1, 0, 0] = True
    assert int(msb_first(keep)[0, 0]) != 513
    assert int(pack_bitmap(keep)[0, 0]) == 513
