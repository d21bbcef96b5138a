"""The quantised variant (isr_compress_quantized) on the GPU against the
oracle's (oracle/quantize.py), bit for bit: the cut at the budget's share,
the step, every code, the exact error of the dequantised field and its
decompression; plus its compression ratio after the lossless stage beside
the plain method's at the same tolerance."""

import numpy as np
import pytest

import oracle
import synth
from oracle import quantize as Q

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("order,E,tol,share", [(7, 300, 1e-3, 0.5), (5, 257, 1e-2, 0.25), (9, 40, 1e-4, 0.75),
                                               (3, 101, 1e-3, 0.0), (12, 5, 1e-3, 0.5), (7, 4096, 1e-3, 0.5)])
def test_quantized_equals_oracle(isr_ctx, order, E, tol, share):
    from paper_2407_20731_amd import isr
    print(f"[case] quantized N={order} E={E} tol={tol} share={share}", flush=True)
    u_np = synth.field(E, order, seed=700 + order)
    u = torch.from_numpy(u_np).cuda()
    blob = isr_ctx.compress_quantized(u, order, tol, share)
    assert blob.status == isr.OK
    arr = blob.arrays()
    assert arr.value_kind == 1 and arr.value_bytes == 4
    ref = Q.compress_quantized(u_np, order, tol, share)
    out = isr_ctx.decompress(blob).cpu().numpy()
    for c, r in enumerate(ref):
        h = arr.comps[c]
        assert h["U2"] == r.U2 and h["B"] == r.B and h["tau"] == r.tau and h["kept"] == r.kept
        assert h["dropped"] == r.dropped and h["qstep"] == r.delta
        assert np.array_equal(arr.bitmap[c], r.bitmap)
        assert np.array_equal(arr.values[c].astype(np.float64), r.codes)
        assert h["err2"] == r.err2 and h["rel_err"] == r.rel_err <= tol
        rec = Q.dequantise(r.bitmap, r.codes, r.delta, order)
        assert np.array_equal(out[c].view(np.uint64), rec.view(np.uint64))
    # serialisation round trip keeps the codes and the steps
    back = isr_ctx.blob_from_bytes(blob.to_bytes())
    out2 = isr_ctx.decompress(back).cpu().numpy()
    assert np.array_equal(out.view(np.uint64), out2.view(np.uint64))


def test_quantized_ratio_after_lossless(isr_ctx):
    """Same tolerance, same field: plain FP64 and FP32-value blobs and the
    quantised one, each after the lossless coder (zlib 6, byte-plane shuffle)."""
    from paper_2407_20731_amd import isr
    u = torch.from_numpy(synth.field(4096, 7, seed=77)).cuda()
    nbytes = u.numel() * 8
    res = {}
    for name, blob in (("fp64", isr_ctx.compress(u, 7, 1e-3, "fp64")), ("fp32", isr_ctx.compress(u, 7, 1e-3, "fp32")),
                       ("quantized", isr_ctx.compress_quantized(u, 7, 1e-3, 0.5))):
        raw = blob.to_bytes()
        packed = isr.pack_host(raw, "zlib", 6, True)
        res[name] = ((nbytes - len(raw)) / nbytes, (nbytes - len(packed)) / nbytes, max(blob.stats["rel_err"]))
    print(f"[quantized] (CR lossy, CR with lossless, max rel err): {res}", flush=True)
    assert res["quantized"][1] > res["fp32"][1] and all(v[2] <= 1e-3 for v in res.values())


def test_quantized_refusals(isr_ctx):
    from paper_2407_20731_amd import isr
    u = torch.from_numpy(synth.field(10, 5, seed=78)).cuda()
    for kw in ({"share": 1.0}, {"share": -0.1}):
        with pytest.raises(isr.IsrError):
            isr_ctx.compress_quantized(u, 5, 1e-3, **kw)
    with pytest.raises(isr.IsrError):
        isr_ctx.compress_quantized(u, 5, -1.0)
