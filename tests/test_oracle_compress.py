"""Pins for the oracle's norm, energies, threshold, kept sets and error check.

Independent references used here: numpy's Legendre evaluator and scipy's
Gauss-Jacobi nodes (to synthesise and re-measure fields without the oracle's
own transforms), Fraction arithmetic, brute force over every subset on tiny
inputs, hand-worked cases, and invariants of the exact definition.  The last
section plants mistakes in copies of oracle pieces and shows the pins catch
them.
"""

import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.special

import oracle
import synth
from oracle.compress import ETOL, OK, energies, norm_terms, pack_bitmap, threshold, unpack_bitmap
from oracle.exact import exact_sum, exact_sum_fraction
from oracle.tables import gll_tables
from oracle.transform import forward, inverse


def _ref_nodes_weights(N):
    if N == 1:
        return np.array([-1.0, 1.0]), np.array([1.0, 1.0])
    inner, _ = scipy.special.roots_jacobi(N - 1, 1.0, 1.0)
    x = np.concatenate(([-1.0], np.sort(inner), [1.0]))
    PN = np.polynomial.legendre.legval(x, [0] * N + [1])
    return x, 2.0 / (N * (N + 1) * PN * PN)


def _legendre_at(N, x):
    return np.stack([np.polynomial.legendre.legval(x, [0] * k + [1]) for k in range(N + 1)])


def _synthesise(c, N):
    """Nodal values of a Legendre series (numpy evaluator, not the oracle)."""
    x, _ = _ref_nodes_weights(N)
    L = _legendre_at(N, x)
    return np.einsum("erqp,rk,qj,pi->ekji", c, L, L, L)


def _ref_mass_norm2(u, N):
    """Mass-weighted squared norm with scipy-derived GLL weights, as a Fraction."""
    _, w = _ref_nodes_weights(N)
    w3 = np.einsum("k,j,i->kji", w, w, w)
    return exact_sum_fraction((w3[None] * (u * u)).ravel())


# ---------------------------------------------------------------- Parseval


def _parseval_gap(u, N, g3=None):
    T = gll_tables(N)
    U2 = exact_sum(norm_terms(u, T.w3, None))
    c = forward(u, T.A)
    E = exact_sum(energies(c, T.g3 if g3 is None else g3, None))
    return abs(U2 - E) / U2


@pytest.mark.parametrize("N", [1, 3, 5, 7, 9])
def test_discrete_parseval(N):
    u = synth.field(64, N, ncomp=1, seed=11)[0]
    assert _parseval_gap(u, N) < 1e-13
    white = np.random.default_rng(N).standard_normal((16, N + 1, N + 1, N + 1))
    assert _parseval_gap(white, N) < 1e-13


def test_norm_matches_independent_weights():
    N = 7
    u = synth.field(32, N, ncomp=1, seed=2)[0]
    T = gll_tables(N)
    U2 = exact_sum(norm_terms(u, T.w3, None))
    ref = float(_ref_mass_norm2(u, N))
    assert abs(U2 - ref) <= 1e-14 * ref


# ------------------------------------------------------- brute-force cuts


def _brute_min_kept(e_flat, B):
    """Fewest kept coefficients over ALL subsets whose dropped energy has
    RN(exact sum) <= B (2^m subsets, exact rationals)."""
    m = e_flat.size
    ef = [Fraction(*float(v).as_integer_ratio()) for v in e_flat]
    sums = [Fraction(0)] * (1 << m)
    best = m
    for mask in range(1, 1 << m):
        low = mask & -mask
        sums[mask] = sums[mask ^ low] + ef[low.bit_length() - 1]
    for mask in range(1 << m):
        if float(sums[mask]) <= B:
            best = min(best, m - bin(mask).count("1"))
    return best


def _check_cut_is_minimal(threshold_fn, e_flat, B):
    tau, n_drop, S = threshold_fn(e_flat, B)
    kept = int(np.sum(e_flat >= tau))
    dropped = e_flat[e_flat < tau]
    ok_feasible = float(exact_sum_fraction(dropped)) <= B and S == exact_sum(dropped)
    return ok_feasible and kept == _brute_min_kept(e_flat, B) and n_drop == dropped.size


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("tol", [0.02, 0.1, 0.3, 0.7])
def test_threshold_is_minimum_cardinality_cut(seed, tol):
    # two N = 1 elements: 16 coefficients, 65536 subsets
    N = 1
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((2, 2, 2, 2)) * np.exp2(rng.integers(-6, 6, size=(2, 2, 2, 2)))
    T = gll_tables(N)
    e = energies(forward(u, T.A), T.g3, None).ravel()
    assert np.unique(e).size == e.size  # no ties: the minimum is unique in size
    U2 = exact_sum(norm_terms(u, T.w3, None))
    B = (tol * tol) * U2
    assert _check_cut_is_minimal(threshold, e, B)


def test_threshold_hand_cases_with_ties():
    e = np.array([1.0, 1.0, 1.0, 4.0])
    # B = 2: S(4) = 3 > 2, so tau = 1 and the whole tie group is kept
    assert threshold(e, 2.0)[:2] == (1.0, 0)
    # B = 3: S(4) = 3 <= 3 -> drop the three ties, keep 4
    assert threshold(e, 3.0)[:2] == (4.0, 3)
    # B = 7: S(inf) = 7 -> drop everything
    tau, n_drop, S = threshold(e, 7.0)
    assert tau == math.inf and n_drop == 4 and S == 7.0
    # zeros are always droppable, even at B = 0
    z = np.array([0.0, 0.0, 2.0 ** -1074, 3.0])
    assert threshold(z, 0.0)[:2] == (2.0 ** -1074, 2)
    # RN of the dropped sum is what is compared with B: 1 + 2^-53 rounds to 1
    r = np.array([2.0 ** -53, 1.0, 5.0])
    assert threshold(r, 1.0)[:2] == (5.0, 2)


def test_threshold_matches_brute_force_with_ties():
    rng = np.random.default_rng(1)
    for _ in range(20):
        e = rng.choice([0.0, 0.5, 1.0, 1.5, 3.0, 7.25], size=12)
        B = float(rng.choice([0.0, 0.5, 1.0, 2.5, 6.0, 40.0]))
        tau, n_drop, S = threshold(e, B)
        # brute force over value cuts: every v in the value set plus +inf
        best = None
        for v in sorted(set(e.tolist())) + [math.inf]:
            below = [Fraction(x) for x in e.tolist() if x < v]
            if float(sum(below, Fraction(0))) <= B:
                best = v
        assert tau == best


def test_hand_built_coefficients():
    # N = 2, one element: gamma = (2, 2/3, 1); energies g3 * c^2 are known
    N, n = 2, 3
    c = np.zeros((1, n, n, n))
    c[0, 0, 0, 0] = 1.0     # e = 8
    c[0, 1, 0, 0] = 0.1     # e = (2/3)*2*2 * 0.01  ~ 2.67e-2
    c[0, 0, 2, 0] = 0.01    # e = 2*1*2 * 1e-4      = 4e-4
    c[0, 2, 2, 2] = 0.001   # e = 1 * 1e-6
    u = _synthesise(c, N)[None]  # [ncomp=1, E=1, 3, 3, 3]
    r = oracle.compress(u, N, 0.01)
    comp = r.comps[0]
    keep = unpack_bitmap(comp.bitmap, n)[0]
    want = np.zeros((n, n, n), bool)
    want[0, 0, 0] = want[1, 0, 0] = True
    assert np.array_equal(keep, want)
    assert comp.kept == 2
    np.testing.assert_allclose(comp.values, [1.0, 0.1], rtol=1e-14)
    assert comp.rel_err <= 0.01
    # tighter bound keeps the 4e-4 mode too
    comp = oracle.compress(u, N, 0.005).comps[0]
    assert unpack_bitmap(comp.bitmap, n)[0][0, 2, 0] and comp.kept == 3


# --------------------------------------------------------- error check


@pytest.mark.parametrize("N", [5, 7, 9])
@pytest.mark.parametrize("tol", [1e-2, 1e-3, 1e-5])
def test_error_equals_dropped_energy_and_meets_tol(N, tol):
    u = synth.field(64, N, ncomp=1, seed=21)
    comp = oracle.compress(u, N, tol).comps[0]
    assert comp.status == OK and comp.rel_err <= tol
    assert abs(comp.err2 - comp.dropped) <= 1e-11 * comp.err2
    # re-measure the reconstruction error with independent weights and synthesis
    T = gll_tables(N)
    keep = unpack_bitmap(comp.bitmap, N + 1)
    cfull = forward(u[0], T.A)
    recon = _synthesise(np.where(keep, cfull, 0.0), N)
    rel = math.sqrt(float(_ref_mass_norm2(u[0] - recon, N) / _ref_mass_norm2(u[0], N)))
    assert abs(rel - comp.rel_err) <= 1e-9 * tol


def test_blob_arrays_consistent():
    N, n = 7, 8
    u = synth.field(40, N, ncomp=2, seed=5)
    r = oracle.compress(u, N, 1e-3, keep_arrays=True)
    for comp in r.comps:
        keep = unpack_bitmap(comp.bitmap, n)
        assert np.array_equal(pack_bitmap(keep), comp.bitmap)
        counts = keep.reshape(40, -1).sum(1)
        assert np.array_equal(np.diff(comp.elem_ptr.astype(np.int64)), counts)
        assert np.array_equal(comp.values, comp.coef[keep])
        assert np.array_equal(keep, comp.energy >= comp.tau)
        back = oracle.decompress(comp.bitmap, comp.values, N)
        assert np.array_equal(back, comp.recon)


# ------------------------------------------------------------ invariants


def test_kept_count_monotone_in_tol():
    u = synth.field(64, 7, ncomp=1, seed=8)
    kept = [oracle.compress(u, 7, t).comps[0].kept for t in (1e-6, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1, 0.5)]
    assert all(a >= b for a, b in zip(kept, kept[1:]))
    assert kept[0] > kept[-1]


def test_element_permutation_permutes_bitmaps():
    u = synth.field(50, 5, ncomp=1, seed=9)
    perm = np.random.default_rng(0).permutation(50)
    a = oracle.compress(u, 5, 1e-3).comps[0]
    b = oracle.compress(u[:, perm], 5, 1e-3).comps[0]
    assert a.tau == b.tau and a.U2 == b.U2 and a.kept == b.kept
    assert np.array_equal(a.bitmap[perm], b.bitmap)


@pytest.mark.parametrize("s", [-40, -3, 5, 60])
def test_power_of_two_scaling(s):
    u = synth.field(30, 7, ncomp=1, seed=12)
    a = oracle.compress(u, 7, 1e-3).comps[0]
    b = oracle.compress(u * 2.0 ** s, 7, 1e-3).comps[0]
    assert np.array_equal(a.bitmap, b.bitmap)
    assert b.U2 == a.U2 * 2.0 ** (2 * s) and b.tau == a.tau * 2.0 ** (2 * s)
    assert np.array_equal(b.values, a.values * 2.0 ** s)
    assert b.rel_err == a.rel_err


def test_components_are_independent():
    u = synth.field(30, 5, ncomp=3, seed=13)
    r = oracle.compress(u, 5, 1e-3)
    for c in range(3):
        one = oracle.compress(u[c:c + 1], 5, 1e-3).comps[0]
        assert np.array_equal(one.bitmap, r.comps[c].bitmap) and one.tau == r.comps[c].tau


# ------------------------------------------------------------ degenerate


def test_zero_field():
    u = np.zeros((1, 4, 6, 6, 6))
    comp = oracle.compress(u, 5, 1e-3).comps[0]
    assert comp.kept == 0 and comp.U2 == 0.0 and comp.rel_err == 0.0 and comp.tau == math.inf


def test_keep_all_and_drop_all():
    u = synth.field(8, 5, ncomp=1, seed=14)
    keep_all = oracle.compress(u, 5, -1.0).comps[0]
    assert keep_all.kept == 8 * 216 and keep_all.rel_err < 1e-14
    drop_all = oracle.compress(u, 5, 2.0).comps[0]
    assert drop_all.kept == 0 and drop_all.tau == math.inf and abs(drop_all.rel_err - 1.0) < 1e-14


def test_tol_zero_drops_only_exact_zeros():
    c = np.zeros((1, 3, 3, 3))
    c[0, 0, 0, 0] = 1.0
    u = _synthesise(c, 2)[None] * 0 + 1.0   # constant field: exact zeros?
    comp = oracle.compress(u, 2, 0.0, keep_arrays=True).comps[0]
    # every coefficient with nonzero energy is kept; exact zeros are dropped
    assert comp.kept == int(np.count_nonzero(comp.energy))
    assert comp.status in (OK, ETOL)


def test_rejects_nonfinite():
    u = np.zeros((1, 1, 3, 3, 3))
    u[0, 0, 1, 1, 1] = np.nan
    with pytest.raises(ValueError):
        oracle.compress(u, 2, 1e-3)


# ------------------------------------------------ planted mistakes (CPU)


def test_pins_catch_wrong_top_mode_norm():
    # the continuous norm 2/(2N+1) at k = N instead of the discrete 2/N
    N = 7
    n = N + 1
    gam = np.array([2.0 / (2 * k + 1) for k in range(n)])
    g3_wrong = np.einsum("a,b,c->abc", gam, gam, gam)
    white = np.random.default_rng(3).standard_normal((16, n, n, n))
    assert _parseval_gap(white, N, g3=g3_wrong) > 1e-3


def test_pins_catch_transposed_matrix():
    N = 5
    n = N + 1
    T = gll_tables(N)
    L = _legendre_at(N, _ref_nodes_weights(N)[0])
    u = np.einsum("k,j,i->kji", L[2], L[0], L[1])[None]
    c = forward(u, T.A.T.copy())[0]
    want = np.zeros((n, n, n))
    want[2, 0, 1] = 1.0
    assert np.abs(c - want).max() > 1e-3


def test_pins_catch_off_by_one_threshold():
    def keeps_one_less(e, B):
        tau, n_drop, S = threshold(e, B)
        s = np.sort(e)
        if n_drop < s.size:
            n_drop += 1
            tau = float(s[n_drop]) if n_drop < s.size else math.inf
        return tau, n_drop, exact_sum(s[:n_drop])

    def ties_dropped(e, B):  # "<= v" instead of "< v"
        tau, n_drop, S = threshold(e, B)
        return np.nextafter(tau, math.inf), int(np.sum(e <= tau)), S

    rng = np.random.default_rng(4)
    u = rng.standard_normal((2, 2, 2, 2))
    T = gll_tables(1)
    e = energies(forward(u, T.A), T.g3, None).ravel()
    B = (0.3 * 0.3) * exact_sum(norm_terms(u, T.w3, None))
    assert _check_cut_is_minimal(threshold, e, B)
    assert not _check_cut_is_minimal(keeps_one_less, e, B)
    assert not _check_cut_is_minimal(ties_dropped, e, B)
