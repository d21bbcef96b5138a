"""Continuous batching behind isr_submit / isr_poll, on the GPU.

Requests of different sizes and orders (element windows of device-resident
pools, FP32 MFMA path, tol 1e-3) are submitted back to back; the scheduler
admits them while stream slots and HBM budget are free and their pipelines
overlap on the device.  Each result must equal the same request compressed
alone (bit-identical: every global sum is exact or fixed-order per lane, so
scheduling cannot change it) and pass the oracle checks of
tests/mixed_checks.py, requests must actually overlap, and a small budget
must bound what is admitted without deadlock.
"""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _pools(orders, n_elem, seed0=500):
    return {N: torch.from_numpy(synth.field(n_elem, N, seed=seed0 + N)).cuda() for N in orders}


def _requests(pools, rng, count, emax):
    reqs = []
    for _ in range(count):
        N = int(rng.choice(sorted(pools)))
        E = int(np.clip(round(np.exp(rng.normal(np.log(600), 0.8))), 40, emax))
        off = int(rng.integers(0, pools[N].shape[1] - E + 1))
        reqs.append((N, off, E))
    return reqs


def test_mix_equals_alone_and_overlaps():
    from paper_2407_20731_amd import isr
    pools = _pools((5, 7, 9), 3000)
    rng = np.random.default_rng(7)
    reqs = _requests(pools, rng, 24, 2500)
    with isr.Context(device=0, max_inflight=6) as ctx:
        torch.cuda.synchronize()
        ids = [ctx.submit(pools[N][:, off:off + E], N, 1e-3, "fp32") for (N, off, E) in reqs]
        mixed = [ctx.poll(r, wait_ms=-1) for r in ids]
        alone = [ctx.compress(pools[N][:, off:off + E], N, 1e-3, "fp32") for (N, off, E) in reqs]
        torch.cuda.synchronize()
        for (N, off, E), m, a in zip(reqs, mixed, alone):
            assert m.status == isr.OK and a.status == isr.OK
            assert m.to_bytes() == a.to_bytes(), (N, off, E)
            assert max(m.stats["rel_err"]) <= 1e-3
        # the served results against the oracle (the smaller requests, to keep
        # the CPU side short)
        from mixed_checks import verify_mixed
        checked = 0
        for (N, off, E), m in zip(reqs, mixed):
            if E > 1000 or checked >= 10:
                continue
            x = pools[N][:, off:off + E]
            u_np = x.cpu().numpy()
            coef = ctx.forward(x, N, "fp32").cpu().numpy().astype(np.float64)
            out = ctx.decompress(m).cpu().numpy()
            ref = oracle.compress(u_np, N, 1e-3, keep_arrays=True)
            verify_mixed(m.arrays(), m.status, m.stats["repair_iters"], u_np, N, 1e-3, "fp32", coef, ref.comps, out=out)
            checked += 1
        assert checked >= 5
        spans = sorted((m.stats["t_start"], m.stats["t_done"]) for m in mixed)
        overlaps = sum(1 for k in range(1, len(spans)) if spans[k][0] < spans[k - 1][1])
        print(f"[serving] {len(spans)} requests, {overlaps} started before the previous one finished", flush=True)
        assert overlaps >= 3


def test_budget_bounds_admission():
    from paper_2407_20731_amd import isr
    pools = _pools((7,), 4000, seed0=600)
    u = pools[7]
    # the whole pool (4000 elements, 2.0 M values per component: candidate
    # lists of 2^20 on the first attempt) needs ~89 MB of scratch + blob, a
    # window of 1500 elements (lists for every value) ~57 MB: one window at a
    # time fits the 80 MB budget
    with isr.Context(device=0, max_inflight=8, budget_bytes=80 << 20) as ctx:
        # one request alone above the budget is refused at submit
        with pytest.raises(isr.IsrError) as e:
            ctx.submit(u, 7, 1e-3, "fp32")
        assert e.value.code == isr.ENOMEM
        torch.cuda.synchronize()
        reqs = [(o, 1500) for o in (0, 500, 1000, 1500, 2000, 2500)]
        ids = [ctx.submit(u[:, o:o + E], 7, 1e-3, "fp32") for (o, E) in reqs]
        outs = [ctx.poll(r, wait_ms=-1) for r in ids]
        for (o, E), b in zip(reqs, outs):
            assert b.status == isr.OK
            ref = ctx.compress(u[:, o:o + E], 7, 1e-3, "fp32")
            assert b.to_bytes() == ref.to_bytes()


def test_poll_unknown_and_pending():
    from paper_2407_20731_amd import isr
    with isr.Context(device=0) as ctx:
        with pytest.raises(isr.IsrError) as e:
            ctx.poll(987654321)
        assert e.value.code == isr.ENOTFOUND
        u = torch.from_numpy(synth.field(2000, 9, seed=9)).cuda()
        torch.cuda.synchronize()
        r = ctx.submit(u, 9, 1e-3, "bf16")
        b = None
        for _ in range(10000):
            b = ctx.poll(r, wait_ms=5)
            if b is not None:
                break
        assert b is not None and b.status == isr.OK


def test_arena_gives_back_empty_chunks():
    """A request that needs most of the budget is admitted after smaller ones
    have left the budget split into chunks with nothing live in them."""
    from paper_2407_20731_amd import isr
    small = synth.field_torch(1000, 7, ncomp=3, seed=51, device="cuda")
    big = synth.field_torch(24000, 7, ncomp=3, seed=52, device="cuda")  # ~0.9 GB of scratch and blob
    with isr.Context(device=0, budget_bytes=1 << 30) as ctx:
        ctx.compress(small, 7, 1e-3, "bf16").free()
        b = ctx.compress(big, 7, 1e-3, "bf16")
        assert b.status == 0
        b.free()


def test_copy_on_submit_lets_the_caller_overwrite():
    """With copy-on-submit the caller overwrites the field on its stream right
    after isr_submit returns, while the request still waits for a slot; the
    result equals compressing the original field."""
    from paper_2407_20731_amd import isr
    u = synth.field_torch(3000, 7, ncomp=3, seed=61, device="cuda")
    keep = u.clone()
    big = synth.field_torch(20000, 9, ncomp=3, seed=62, device="cuda")
    torch.cuda.synchronize()
    with isr.Context(device=0, max_inflight=1) as ctx:
        first = ctx.submit(big, 9, 1e-3, "bf16")  # holds the only slot for a while
        rid = ctx.submit(u, 7, 1e-3, "bf16", copy=True)
        u.fill_(1.0e30)  # same (current) stream: ordered after the copy
        b = ctx.poll(rid, wait_ms=-1)
        ctx.poll(first, wait_ms=-1).free()
        ref = ctx.compress(keep, 7, 1e-3, "bf16")
        assert b.status == isr.OK
        assert b.to_bytes() == ref.to_bytes()
        # a window with a component stride is copied compactly
        pool = synth.field_torch(5000, 5, ncomp=3, seed=63, device="cuda")
        win = pool[:, 1000:3000]
        rid = ctx.submit(win, 5, 1e-3, "fp32", copy=True)
        pool.zero_()
        b2 = ctx.poll(rid, wait_ms=-1)
        pool2 = synth.field_torch(5000, 5, ncomp=3, seed=63, device="cuda")
        assert b2.to_bytes() == ctx.compress(pool2[:, 1000:3000], 5, 1e-3, "fp32").to_bytes()


def test_copy_on_submit_counts_against_the_budget():
    """The copy is part of the request's footprint: a request that fits the
    budget borrowed is refused at submit when its copy would not fit too."""
    from paper_2407_20731_amd import isr
    u = synth.field_torch(2000, 7, ncomp=3, seed=64, device="cuda")  # ~63 MB footprint, 25 MB field
    torch.cuda.synchronize()
    with isr.Context(device=0, budget_bytes=75 << 20) as ctx:
        with pytest.raises(isr.IsrError) as e:
            ctx.submit(u, 7, 1e-3, "fp32", copy=True)
        assert e.value.code == isr.ENOMEM
        b = ctx.poll(ctx.submit(u, 7, 1e-3, "fp32"), wait_ms=-1)
        assert b.status == isr.OK
