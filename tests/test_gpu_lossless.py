"""The hybrid lossless stage on the GPU machine: device blobs queued for lossless
coding on the context's host threads (isr_pack_submit / isr_pack_poll) come
back as packed bytes that decode to exactly the blob's serialized bytes,
while further compressions run; blobs re-uploaded from them decompress to the
same field."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("codec,level,shuffle", [("zlib", 6, True), ("bzip2", 9, False)])
def test_pack_submit_round_trip(codec, level, shuffle):
    from paper_2407_20731_amd import isr
    u = torch.from_numpy(synth.field(1500, 7, seed=81)).cuda()
    with isr.Context(host_threads=4) as ctx:
        blobs = [ctx.compress(u, 7, tol, "bf16") for tol in (1e-3, 1e-2, 1e-4)]
        jobs = [ctx.pack_submit(b, codec, level, shuffle) for b in blobs]
        more = ctx.compress(u, 7, 1e-3, "fp32")  # GPU work while the host codes
        assert more.status == 0
        for b, j in zip(blobs, jobs):
            packed, secs = ctx.pack_poll(j, wait_ms=-1)
            assert secs >= 0.0
            raw = isr.unpack_host(packed)
            assert raw == b.to_bytes()
            cr = (b.stats["in_bytes"] - len(packed)) / b.stats["in_bytes"]
            assert cr > b.stats["cr"]
            back = ctx.blob_from_bytes(raw)
            a = ctx.decompress(b).cpu().numpy()
            c = ctx.decompress(back).cpu().numpy()
            assert np.array_equal(a.view(np.uint64), c.view(np.uint64))
            print(f"[lossless-gpu] {codec}-{level} shuffle={shuffle}: lossy CR {b.stats['cr']:.4f}, "
                  f"with lossless {cr:.4f}, {secs * 1e3:.1f} ms", flush=True)
        with pytest.raises(isr.IsrError) as e:
            ctx.pack_poll(jobs[0])
        assert e.value.code == isr.ENOTFOUND
