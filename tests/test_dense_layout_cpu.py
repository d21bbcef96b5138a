"""Host-side check of the dense-tile engine's LDS geometry (no GPU).

The contractions of the dense-tile passes read the rows of the contracted
index past n (the MFMA operand's padded rows) without a lane mask, relying on
every such read staying inside the wave's buffer, whose tail past the dense
slots is zeroed.  This test restates the engine's tile geometry (the pencil
bases of the three axes, the lane -> (pencil, row) map of a 16x16 MFMA tile
with one or two copies of the 1D matrix) for every compiled shape, read from
the shape list in csrc/isr_internal.h, and enumerates every access of every
stage: reads stay below the buffer length the engine reserves, stores of
valid rows stay inside the tile, and the valid (pencil, row) positions of a
stage cover the tile exactly once (the partition that lets the stages run in
place without barriers).
"""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2407_20731_amd", "csrc", "isr_internal.h")


def _shapes():
    text = open(HDR).read()
    m = re.search(r"#define ISR_DENSE_SHAPES\(X\)(.*?)\n(?!\s*X\()", text, re.S)
    assert m, "shape list not found"
    return [(int(a), int(b)) for a, b in re.findall(r"X\((\d+),\s*(\d+)\)", m.group(1))]


def _geometry(N, T):
    n = N + 1
    n2, n3 = n * n, n * n * n
    KP = 8 if n <= 8 else 16
    ncopy = 16 // KP
    gpc = 4 // ncopy
    pb = 16 * ncopy
    tp = T * n2
    nb = (tp + pb - 1) // pb
    s = (T * n3 + 63) // 64
    ldsw = s * 64
    ovr = T * n3 + n2 * (KP - n if KP > n else 0)
    ldsb = (max(ovr, ldsw) + 63) // 64 * 64
    return dict(n=n, n2=n2, n3=n3, KP=KP, gpc=gpc, pb=pb, tp=tp, nb=nb, ldsw=ldsw, ldsb=ldsb)


def _pbase(ax, pi, n, n2, n3):
    if ax == 0:
        return pi * n
    if ax == 1:
        return (pi // n) * n2 + pi % n
    return (pi // n2) * n3 + pi % n2


def test_shape_list_parsed():
    shapes = _shapes()
    assert (5, 2) in shapes and (9, 1) in shapes and len(shapes) >= 20


@pytest.mark.parametrize("N,T", _shapes())
def test_unmasked_reads_stay_in_the_buffer_and_stores_partition_the_tile(N, T):
    g = _geometry(N, T)
    n, n2, n3 = g["n"], g["n2"], g["n3"]
    for ax in range(3):
        st = (1, n, n2)[ax]
        written = {}
        for lane in range(64):
            P, grp = lane & 15, lane >> 4
            hc, a0 = grp // g["gpc"], 4 * (grp % g["gpc"])
            for b in range(g["nb"]):
                pi = g["pb"] * b + 16 * hc + P
                pv = pi < g["tp"]
                p = _pbase(ax, pi, n, n2, n3) + a0 * st if pv else 0
                pair = ax == 0 and n % 2 == 0  # two consecutive floats per access along i
                for m in range(4):
                    off = p + m if pair else p + m * st
                    assert 0 <= off < g["ldsb"], (N, T, ax, lane, b, m, off, g["ldsb"])
                    if pv and a0 + m < n:
                        assert off < T * n3, (N, T, ax, lane, b, m, off)
                        assert off not in written, (N, T, ax, off)
                        written[off] = (pi, a0 + m)
        assert sorted(written) == list(range(T * n3)), (N, T, ax)
