"""The hybrid lossless stage's host coder (isr_pack_host / isr_unpack_host),
on the CPU: round trips of serialized blobs, the packed format read back by
Python's own zlib and bz2 modules (independent decoders), the byte-plane
shuffle of the kept values, the compression ratio of the whole chain
(Sec. IV-C: (original - compressed) / original), and refusals of corrupt
input.  The blobs are written here from the oracle's arrays in the
serialized layout of include/isr.h."""

import bz2
import os
import struct
import zlib

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2407_20731_amd", "libisr.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libisr.so not built")


def serialized_blob(u, order, tol, value_dtype=np.float32):
    """A blob in the serialized layout (version 3) from the oracle's result,
    values stored as value_dtype."""
    ref = oracle.compress(u, order, tol)
    n = order + 1
    E = u.shape[1]
    W = (n ** 3 + 63) // 64
    vb = np.dtype(value_dtype).itemsize
    prec = 0 if vb == 8 else 1
    out = [b"ISR1", struct.pack("<Iiiqiidiiiiii", 3, order, len(ref.comps), E, vb, W, tol, prec, 0, 0, 0, 0, 0)]
    voff = 0
    for rc in ref.comps:
        out.append(struct.pack("<6d2Qd", rc.U2, rc.B, rc.tau, rc.dropped, rc.err2, rc.rel_err, rc.kept, voff, 0.0))
        voff += rc.kept
    for rc in ref.comps:
        out.append(rc.bitmap.astype("<u8").tobytes())
    for rc in ref.comps:
        out.append(rc.elem_ptr.astype("<u8").tobytes())
    for rc in ref.comps:
        out.append(rc.values.astype(value_dtype).tobytes())
    blob = b"".join(out)
    assert len(blob) == 64 + 72 * len(ref.comps) + 8 * len(ref.comps) * E * W + 8 * len(ref.comps) * (E + 1) + voff * vb
    return blob, u.nbytes


def _isr():
    from paper_2407_20731_amd import isr
    return isr


def _chunks(packed):
    """Split a packed blob with the documented layout."""
    assert packed[:4] == b"ISRZ"
    ver, codec, flags, raw_n, K, csz = struct.unpack_from("<IIIQII", packed, 4)
    sizes = struct.unpack_from(f"<{K}Q", packed, 32)
    at = 32 + 8 * K
    chunks = []
    for s in sizes:
        chunks.append(packed[at:at + s])
        at += s
    assert at == len(packed)
    return ver, codec, flags, raw_n, csz, chunks


@pytest.mark.parametrize("codec,level", [("zlib", 1), ("zlib", 6), ("bzip2", 9)])
@pytest.mark.parametrize("shuffle", [False, True])
def test_round_trip_and_independent_decoder(codec, level, shuffle):
    isr = _isr()
    blob, nbytes = serialized_blob(synth.field(300, 7, seed=71), 7, 1e-3)
    packed = isr.pack_host(blob, codec, level, shuffle, threads=3)
    assert isr.unpack_host(packed) == blob
    ver, cdc, flags, raw_n, csz, chunks = _chunks(packed)
    assert ver == 1 and cdc == isr.CODECS[codec] and flags == (1 if shuffle else 0) and raw_n == len(blob)
    dec = zlib.decompress if codec == "zlib" else bz2.decompress
    raw = b"".join(dec(c) for c in chunks)
    assert len(raw) == len(blob)
    if not shuffle:
        assert raw == blob
    else:
        # values section stored byte plane by byte plane
        arr = isr.parse_blob(blob)
        off = len(blob) - sum(c["kept"] for c in arr.comps) * 4
        assert raw[:off] == blob[:off]
        v = np.frombuffer(blob[off:], dtype=np.uint8).reshape(-1, 4)
        assert raw[off:] == v.T.copy().tobytes()
    cr_lossy = (nbytes - len(blob)) / nbytes
    cr_all = (nbytes - len(packed)) / nbytes
    print(f"[lossless] {codec}-{level} shuffle={shuffle}: CR lossy {cr_lossy:.4f}, with lossless {cr_all:.4f}")
    assert cr_all > cr_lossy


def test_multi_chunk_blob_and_thread_counts():
    isr = _isr()
    blob, _ = serialized_blob(synth.field(2500, 7, seed=72), 7, -1.0)  # keep all: several 4 MiB chunks
    a = isr.pack_host(blob, "zlib", 3, True, threads=1)
    b = isr.pack_host(blob, "zlib", 3, True, threads=8)
    assert a == b  # chunks are coded independently: same bytes whatever the threads
    assert len(_chunks(a)[-1]) > 1
    assert isr.unpack_host(b) == blob


def test_fp64_blob_shuffle_round_trip():
    isr = _isr()
    blob, _ = serialized_blob(synth.field(100, 5, seed=73), 5, 1e-3, value_dtype=np.float64)
    assert isr.unpack_host(isr.pack_host(blob, "bzip2", 5, True)) == blob


def test_refusals():
    isr = _isr()
    blob, _ = serialized_blob(synth.field(20, 3, seed=74), 3, 1e-2)
    with pytest.raises(isr.IsrError):
        isr.pack_host(blob, "zlib", 12)  # bad level
    with pytest.raises(isr.IsrError):
        isr.pack_host(b"XXXX" + bytes(100), "zlib", 6, True)  # shuffle needs a blob
    packed = bytearray(isr.pack_host(blob, "zlib", 6))
    with pytest.raises(isr.IsrError):
        isr.unpack_host(bytes(packed[:-3]))  # truncated
    packed[40] ^= 0xFF
    with pytest.raises(isr.IsrError):
        isr.unpack_host(bytes(packed))  # corrupt chunk
