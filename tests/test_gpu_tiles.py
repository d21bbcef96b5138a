"""GPU checks of the tile shapes of the FP32 / BF16 streaming passes.

Every compiled shape (wave-tile engine 0, dense tiles of T elements) must
satisfy the same oracle checks as the default one (tests/test_gpu_mixed.py:
U2 to 1e-12, coefficient bound, kept sets within the threshold band, the bound
met, decompress equal to the oracle's reconstruction), on element counts that
give several tiles and a ragged last tile.  The autotuner must time every
candidate, keep the fastest, and write a table a new context reads back.
"""

import os

import numpy as np
import pytest

import synth
from test_gpu_mixed import check_mixed

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# the shapes compiled into the library, per order (0 = wave-tile engine)
SHAPES = {1: [0, 32, 64], 2: [0, 16, 32], 3: [0, 4, 8], 4: [0, 4, 8], 5: [0, 2, 4, 8], 6: [0, 1, 2, 3],
          7: [0, 1, 2], 8: [0, 1, 2], 9: [0, 1, 2], 10: [0, 1], 11: [0, 1]}
CASES = [(o, t) for o, ts in SHAPES.items() for t in ts]


def elements_for(order, tile):
    # three tiles and a ragged fourth, and at least a few hundred values
    t = max(tile, 1)
    E = 3 * t + max(1, t // 2) if t > 1 else 13
    n3 = (order + 1) ** 3
    while E * n3 < 2000:
        E += t
    return E


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("order,tile", CASES)
def test_tile_shape_against_oracle(isr_ctx, prec, order, tile):
    E = elements_for(order, tile)
    tol = 1e-3 if order >= 3 else 1e-2
    print(f"[case] prec={prec} order={order} tile={tile} E={E} tol={tol}", flush=True)
    isr_ctx.set_tile(order, prec, tile)
    try:
        assert isr_ctx.get_tile(order, prec) == tile
        check_mixed(isr_ctx, prec, order, E, tol, seed=300 + order)
    finally:
        isr_ctx.set_tile(order, prec, -1)


def test_tile_shapes_rejected(isr_ctx):
    from paper_2407_20731_amd import isr
    with pytest.raises(isr.IsrError):
        isr_ctx.set_tile(5, "bf16", 3)    # not compiled
    with pytest.raises(isr.IsrError):
        isr_ctx.set_tile(5, "fp64", 2)    # FP64 has one engine
    with pytest.raises(isr.IsrError):
        isr_ctx.set_tile(13, "bf16", 0)   # no streaming path


def test_autotune_round_trip(tmp_path):
    from paper_2407_20731_amd import isr
    path = str(tmp_path / "tiles.txt")
    u = torch.from_numpy(synth.field(3000, 5, seed=41)).cuda()
    with isr.Context(autotune_path=path) as ctx:
        rep = ctx.autotune(u, 5, 1e-3, "bf16", reps=1)
        print(f"[tune] N=5 bf16 E=3000: {rep}", flush=True)
        assert sorted(rep["ms"]) == SHAPES[5]
        assert rep["best"] == min(rep["ms"], key=rep["ms"].get)
        assert ctx.get_tile(5, "bf16") == rep["best"]
        blob = ctx.compress(u, 5, 1e-3, "bf16")
        assert blob.status == 0
    assert os.path.exists(path)
    assert f"5 2 {rep['best']}" in open(path).read().split("\n")
    with isr.Context(autotune_path=path) as ctx2:
        assert ctx2.get_tile(5, "bf16") == rep["best"]
        assert ctx2.get_tile(5, "fp32") in SHAPES[5]  # untouched entry: the built-in choice


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("order,tile", [(3, 8), (5, 2), (5, 4), (7, 0), (7, 1), (9, 0), (9, 1), (11, 1)])
def test_tile_shape_with_jacobians(isr_ctx, prec, order, tile):
    """Per-element Jacobians (affine elements of different sizes) on the
    streaming engines: the norm, energy and error terms carry J_e."""
    E = elements_for(order, tile)
    jac = np.random.default_rng(order + tile).uniform(0.1, 3.0, size=E)
    print(f"[case] prec={prec} order={order} tile={tile} E={E} with Jacobians", flush=True)
    isr_ctx.set_tile(order, prec, tile)
    try:
        check_mixed(isr_ctx, prec, order, E, 1e-3, seed=400 + order, jac_np=jac)
    finally:
        isr_ctx.set_tile(order, prec, -1)
