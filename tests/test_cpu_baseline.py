"""The fast FP64 CPU baseline (cpubase/, C + OpenMP) against the oracle.

It uses the canonical transform order, so its coefficients and kept values
must equal the oracle's bit for bit; its sums are compensated FP64 sums, not
exact ones, so U2, S and err2 must agree within 1e-12 relative, and the
threshold and kept set exactly (the cases below have no energy group within
1e-12 of the cut)."""

import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle.tables import gll_tables

cpubase = pytest.importorskip("cpubase")
pytestmark = pytest.mark.skipif(not os.path.exists(cpubase.LIB), reason="libisr_cpu.so not built")


@pytest.mark.parametrize("order,E,tol,threads", [(7, 64, 1e-3, 1), (7, 200, 1e-3, 4), (5, 150, 1e-2, 3),
                                                 (9, 20, 1e-5, 2), (3, 77, 0.0, 2), (2, 30, -1.0, 2),
                                                 (1, 9, 0.5, 1), (7, 50, 2.0, 2)])
def test_cpu_baseline_matches_oracle(order, E, tol, threads):
    u = synth.field(E, order, seed=600 + order)
    jac = None
    if order == 5:
        jac = np.random.default_rng(5).uniform(0.5, 3.0, size=E)
    T = gll_tables(order)
    got = cpubase.compress(u, order, tol, T.A, T.V, T.w3, T.g3, jac=jac, threads=threads)
    ref = oracle.compress(u, order, tol, jac=jac)
    assert got.status == ref.status
    for c, rc in enumerate(ref.comps):
        s = got.stats[c]
        assert abs(s["U2"] - rc.U2) <= 1e-12 * rc.U2
        assert s["tau"] == rc.tau and s["kept"] == rc.kept, (c, s["tau"], rc.tau, s["kept"], rc.kept)
        assert np.array_equal(got.bitmap[c], rc.bitmap)
        assert np.array_equal(got.elem_ptr[c], rc.elem_ptr)
        assert np.array_equal(got.values[c].view(np.uint64), rc.values.view(np.uint64))
        assert abs(s["err2"] - rc.err2) <= 1e-12 * max(rc.err2, 1e-300) + 1e-300
        assert s["repair_iters"] == rc.repair_iters
        if tol >= 0:
            assert math.isclose(s["dropped"], rc.dropped, rel_tol=1e-12, abs_tol=1e-300)


def test_cpu_baseline_thread_count_does_not_change_the_cut():
    u = synth.field(300, 7, seed=650)
    T = gll_tables(7)
    a = cpubase.compress(u, 7, 1e-3, T.A, T.V, T.w3, T.g3, threads=1)
    b = cpubase.compress(u, 7, 1e-3, T.A, T.V, T.w3, T.g3, threads=7)
    for c in range(3):
        assert a.stats[c]["tau"] == b.stats[c]["tau"]
        assert np.array_equal(a.bitmap[c], b.bitmap[c])
