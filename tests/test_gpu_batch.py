"""One persistent launch over a batch of snapshots (orders 5, 7, 9, uneven
sizes): every result must equal the same snapshot compressed alone, bit for
bit (the global sums are exact, or fixed-order per lane with the same grids,
so the queue order cannot change them); the FP64 members must equal the
oracle, and the FP32 / BF16 members pass the oracle checks of
tests/mixed_checks.py.  FP32 / BF16 batches run as one streaming pipeline per
snapshot on the scheduler's streams, or with FLAG_BATCH_PERSISTENT as one
persistent launch of the streaming path, with the same results."""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _batch(rng, count, emin, emax, seed0):
    out = []
    for i in range(count):
        N = int(rng.choice([5, 7, 9]))
        E = int(round(np.exp(rng.uniform(np.log(emin), np.log(emax)))))
        out.append((N, E, torch.from_numpy(synth.field(E, N, seed=seed0 + i)).cuda()))
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_batch_equals_alone(isr_ctx, prec):
    rng = np.random.default_rng(11)
    snaps = _batch(rng, 10, 30, 5000, 700)
    snaps.append((7, 4096, torch.from_numpy(synth.field(4096, 7, seed=799)).cuda()))  # sampled window
    # 6,000 identical elements: ties beyond the sort cap, every refinement level
    snaps.append((5, 6000, torch.from_numpy(np.repeat(synth.field(1, 5, seed=5), 6000, axis=1)).cuda()))
    torch.cuda.synchronize()
    print(f"[case] batch prec={prec} sizes={[(N, E) for N, E, _ in snaps]}", flush=True)
    from paper_2407_20731_amd import isr
    with isr.Context(flags=isr.FLAG_BATCH_PERSISTENT) as pctx:
        blobs = pctx.compress_batch([(u, N, 1e-3) for N, E, u in snaps], prec)
        paths = [b.stats["path"] for b in blobs]
        print(f"[batch] {prec} paths {paths}", flush=True)
        if prec != "fp64":
            assert paths.count(2) >= len(blobs) // 2  # the persistent launch (reruns alone aside)
        got = [b.to_bytes() for b in blobs]
    for (N, E, u), g in zip(snaps, got):
        alone = isr_ctx.compress(u, N, 1e-3, prec)
        assert alone.status == 0
        same = g == alone.to_bytes()  # (no assertion diff of MB-sized strings)
        assert same, (N, E)
    if prec != "fp64":
        # the default form: one streaming pipeline per snapshot
        blobs2 = isr_ctx.compress_batch([(u, N, 1e-3) for N, E, u in snaps], prec)
        assert all(b.stats["path"] != 2 for b in blobs2)
        for (N, E, u), g, b2 in zip(snaps, got, blobs2):
            same = g == b2.to_bytes()
            assert same, (N, E)


@pytest.mark.parametrize("shapes", [{5: 2, 7: 1, 9: 0}, {5: 8, 7: 2, 9: 2}, {5: 0, 7: 0, 9: 1}])
def test_batch_persistent_takes_every_shape(shapes):
    """The persistent launch runs whatever tile shape the context holds per
    order (the autotuner's candidates: wave-tile, dense tiles, the large-order
    engine), and every member equals its result alone with the same shapes."""
    from paper_2407_20731_amd import isr
    rng = np.random.default_rng(15)
    snaps = _batch(rng, 9, 30, 2000, 1100)
    torch.cuda.synchronize()
    with isr.Context(flags=isr.FLAG_BATCH_PERSISTENT) as ctx:
        for N, t in shapes.items():
            ctx.set_tile(N, "bf16", t)
        print(f"[case] batch shapes {shapes} sizes={[(N, E) for N, E, _ in snaps]}", flush=True)
        blobs = ctx.compress_batch([(u, N, 1e-3) for N, E, u in snaps], "bf16")
        paths = [b.stats["path"] for b in blobs]
        assert paths.count(2) >= len(blobs) - 1, paths
        for (N, E, u), b in zip(snaps, blobs):
            assert b.status == 0
            same = b.to_bytes() == ctx.compress(u, N, 1e-3, "bf16").to_bytes()
            assert same, (N, E, shapes[N])


def test_batch_fp64_matches_oracle(isr_ctx):
    rng = np.random.default_rng(12)
    snaps = _batch(rng, 6, 20, 400, 800)
    torch.cuda.synchronize()
    blobs = isr_ctx.compress_batch([(u, N, 1e-3) for N, E, u in snaps], "fp64")
    for (N, E, u), b in zip(snaps, blobs):
        arr = b.arrays()
        ref = oracle.compress(u.cpu().numpy(), N, 1e-3)
        for c, rc in enumerate(ref.comps):
            assert arr.comps[c]["tau"] == rc.tau and arr.comps[c]["kept"] == rc.kept
            assert np.array_equal(arr.bitmap[c], rc.bitmap)
            assert np.array_equal(arr.values[c].view(np.uint64), rc.values.view(np.uint64))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_mixed_matches_oracle(isr_ctx, prec):
    """Every member of an FP32 / BF16 batch against the oracle with the checks
    of tests/mixed_checks.py, its decompressed output included: ten snapshots
    in one persistent launch, and the same batch as stream pipelines."""
    from mixed_checks import verify_mixed
    from paper_2407_20731_amd import isr
    rng = np.random.default_rng(14)
    snaps = _batch(rng, 10, 20, 600, 1000)
    torch.cuda.synchronize()
    print(f"[case] batch oracle prec={prec} sizes={[(N, E) for N, E, _ in snaps]}", flush=True)
    refs = [oracle.compress(u.cpu().numpy(), N, 1e-3, keep_arrays=True) for N, E, u in snaps]
    for flags in (isr.FLAG_BATCH_PERSISTENT, 0):
        with isr.Context(flags=flags) as ctx:
            blobs = ctx.compress_batch([(u, N, 1e-3) for N, E, u in snaps], prec)
            paths = [b.stats["path"] for b in blobs]
            if flags:
                assert paths.count(2) >= len(blobs) // 2
            for (N, E, u), b, ref in zip(snaps, blobs, refs):
                assert b.status == 0
                coef = ctx.forward(u, N, prec).cpu().numpy().astype(np.float64)
                out = ctx.decompress(b).cpu().numpy()
                rep = verify_mixed(b.arrays(), b.status, b.stats["repair_iters"], u.cpu().numpy(), N, 1e-3, prec, coef,
                                   ref.comps, out=out)
                print(f"[batch-oracle] {prec} N={N} E={E} path={b.stats['path']}: {rep}", flush=True)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_window_miss_reruns(isr_ctx, prec):
    """A snapshot whose sampled elements are scaled far down misses its
    window inside the persistent launch (every later phase skips it) and is
    rerun on the general pipeline; it and its batch mates equal their results
    alone, byte for byte."""
    rng = np.random.default_rng(13)
    snaps = _batch(rng, 8, 30, 3000, 900)
    u = synth.field(4096, 7, ncomp=2, seed=42)
    u[:, np.arange(4096) % 4 == 0] *= 1e-8
    snaps.insert(3, (7, 4096, torch.from_numpy(u).cuda()))
    torch.cuda.synchronize()
    print(f"[case] batch miss prec={prec} sizes={[(N, E) for N, E, _ in snaps]}", flush=True)
    blobs = isr_ctx.compress_batch([(x, N, 1e-3) for N, E, x in snaps], prec)
    assert blobs[3].stats["path"] == 0
    for (N, E, x), b in zip(snaps, blobs):
        assert b.status == 0
        same = b.to_bytes() == isr_ctx.compress(x, N, 1e-3, prec).to_bytes()
        assert same, (N, E)
