"""The per-element cut (isr_compress_elemcut) on the GPU against the oracle's
(oracle/elemcut.py), through the C ABI.

Small and ragged cases, every order class and Jacobians: U2, B, the dropped
energy, err2, rel, kept counts, bitmaps, element offsets and every kept value
equal the oracle's bit for bit, and the decompressed field equals the
oracle's reconstruction.  At the full bench size (65,536 elements, N = 7,
3 components) the oracle's cut of sampled elements (an element's cut depends
on that element alone), the exact U2 of every component, and, for
component 0, the dropped energy and err2 re-measured by the oracle from the
GPU's kept set; every element's kept set is a threshold set within its
budget.
"""

import math

import numpy as np
import pytest

import oracle
import synth
from oracle import elemcut as P
from oracle.compress import energies, norm_terms, unpack_bitmap
from oracle.exact import exact_sum
from oracle.tables import gll_tables
from oracle.transform import forward, inverse

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _check_equal(blob, ref, order, out=None):
    arr = blob.arrays()
    for c, r in enumerate(ref):
        h = arr.comps[c]
        assert h["U2"] == r.U2 and h["B"] == r.B and math.isnan(h["tau"])
        assert h["dropped"] == r.dropped and h["err2"] == r.err2 and h["rel_err"] == r.rel_err
        assert h["kept"] == r.kept
        assert np.array_equal(arr.bitmap[c], r.bitmap)
        assert np.array_equal(arr.elem_ptr[c], r.elem_ptr)
        assert np.array_equal(arr.values[c].view(np.uint64), r.values.view(np.uint64))
        if out is not None:
            rec = oracle.decompress(r.bitmap, r.values, order)
            assert np.array_equal(out[c].view(np.uint64), rec.view(np.uint64))


@pytest.mark.parametrize("order,E,tol,ncomp,jac", [
    (7, 300, 1e-3, 3, False), (5, 257, 1e-2, 3, False), (9, 40, 1e-4, 1, False), (1, 101, 1e-1, 2, False),
    (3, 77, 1e-5, 3, True), (12, 6, 1e-3, 1, False), (15, 3, 1e-3, 1, False), (7, 1, 1e-3, 1, False)])
def test_elemcut_equals_oracle(isr_ctx, order, E, tol, ncomp, jac):
    print(f"[case] elemcut N={order} E={E} tol={tol} ncomp={ncomp} jac={jac}", flush=True)
    u_np = synth.field(E, order, ncomp=ncomp, seed=800 + order)
    J = np.random.default_rng(order).uniform(0.25, 4.0, size=E) if jac else None
    u = torch.from_numpy(u_np).cuda()
    blob = isr_ctx.compress_elemcut(u, order, tol, jac=None if J is None else torch.from_numpy(J).cuda())
    assert blob.status == 0
    ref = P.compress_elemcut(u_np, order, tol, jac=J)
    out = isr_ctx.decompress(blob).cpu().numpy()
    _check_equal(blob, ref, order, out)
    # more coefficients than the global cut at the same tol
    plain = oracle.compress(u_np, order, tol, jac=J)
    for c in range(ncomp):
        assert ref[c].kept >= plain.comps[c].kept


def test_elemcut_zero_elements_and_serialisation(isr_ctx):
    u_np = synth.field(64, 5, ncomp=2, seed=811)
    u_np[0, 3] = 0.0
    u_np[1, 10:20] = 0.0
    u = torch.from_numpy(u_np).cuda()
    blob = isr_ctx.compress_elemcut(u, 5, 1e-3)
    ref = P.compress_elemcut(u_np, 5, 1e-3)
    _check_equal(blob, ref, 5)
    assert np.isinf(ref[0].tau[3]) and np.all(np.isinf(ref[1].tau[10:20]))
    back = isr_ctx.blob_from_bytes(blob.to_bytes())
    a = isr_ctx.decompress(blob).cpu().numpy()
    b = isr_ctx.decompress(back).cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_elemcut_refusals(isr_ctx):
    from paper_2407_20731_amd import isr
    u = torch.from_numpy(synth.field(10, 5, seed=812)).cuda()
    with pytest.raises(isr.IsrError):
        isr_ctx.compress_elemcut(u, 5, -1.0)
    f = isr_ctx._field(u, 5, 1e-3, "bf16")
    import ctypes as C
    h = C.c_void_p()
    assert isr.load_library().isr_compress_elemcut(isr_ctx._h, C.byref(f), C.byref(h), None) == isr.EINVAL


def test_elemcut_full_size():
    from paper_2407_20731_amd import isr
    E, N, TOL = 65536, 7, 1e-3
    print(f"[case] elemcut full size E={E} N={N}", flush=True)
    u_np = synth.field(E, N, seed=2)
    u = torch.from_numpy(u_np).cuda()
    T = gll_tables(N)
    ids = np.random.default_rng(5).choice(E, size=96, replace=False)
    ids.sort()
    with isr.Context() as ctx:
        blob = ctx.compress_elemcut(u, N, TOL)
        assert blob.status == 0
        arr = blob.arrays()
        plain = ctx.compress(u, N, TOL, "fp64").arrays()
        sample = P.compress_elemcut(u_np, N, TOL, elements=ids)
        for c in range(3):
            h = arr.comps[c]
            assert h["U2"] == exact_sum(norm_terms(u_np[c], T.w3, None)), c
            assert h["rel_err"] <= TOL and h["kept"] >= plain.comps[c]["kept"]
            assert np.array_equal(arr.bitmap[c][ids], sample[c].bitmap), c
            assert abs(h["err2"] - h["dropped"]) <= 1e-12 * h["err2"]
        # component 0: the oracle re-measures the dropped energy and the error
        # of the GPU's kept set, and checks every element's cut is a
        # threshold set inside its budget
        keep = unpack_bitmap(arr.bitmap[0], N + 1)
        coef = forward(u_np[0], T.A)
        en = energies(coef, T.g3, None)
        assert arr.comps[0]["dropped"] == exact_sum(en[~keep])
        recon = inverse(np.where(keep, coef, 0.0), T.V)
        assert arr.comps[0]["err2"] == exact_sum(norm_terms(u_np[0] - recon, T.w3, None))
        assert np.array_equal(arr.values[0].view(np.uint64), coef[keep].view(np.uint64))
        flat = en.reshape(E, -1)
        kf = keep.reshape(E, -1)
        max_drop = np.where(kf, -np.inf, flat).max(axis=1)
        min_keep = np.where(kf, flat, np.inf).min(axis=1)
        assert np.all(max_drop < min_keep)
        U2e = norm_terms(u_np[0], T.w3, None).reshape(E, -1).sum(axis=1)
        drop_e = np.where(kf, 0.0, flat).sum(axis=1)
        assert np.all(drop_e <= (TOL * TOL) * U2e * (1 + 1e-12))
        print(f"[elemcut] kept {[c['kept'] for c in arr.comps]} vs global cut "
              f"{[c['kept'] for c in plain.comps]}", flush=True)
