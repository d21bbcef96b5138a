"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and its host-computed tables equal the oracle's bit for bit
(the two are computed independently: binary128 Newton in C++ vs mpmath)."""

import ctypes as C
import os

import numpy as np
import pytest

from oracle.tables import gll_tables

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2407_20731_amd", "libisr.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libisr.so not built")


def _isr():
    from paper_2407_20731_amd import isr
    return isr


def test_every_declared_symbol_is_exported():
    isr = _isr()
    names = isr.exported_symbols()
    assert len(names) >= 15
    lib = C.CDLL(LIB)
    for name in names:
        assert hasattr(lib, name), name


def test_version_string():
    assert _isr().load_library().isr_version().startswith(b"isr ")


@pytest.mark.parametrize("N", range(1, 16))
def test_library_tables_equal_oracle_bit_for_bit(N):
    lib_t = _isr().gll_tables(N)
    T = gll_tables(N)
    for key, ref in (("xi", T.xi), ("w", T.w), ("V", T.V), ("A", T.A), ("gamma", T.gamma),
                     ("w3", T.w3), ("g3", T.g3)):
        got = lib_t[key]
        assert got.shape == ref.shape, key
        bad = np.flatnonzero(got.view(np.uint64).ravel() != ref.view(np.uint64).ravel())
        assert bad.size == 0, (key, N, bad[:5], got.ravel()[bad[:5]], ref.ravel()[bad[:5]])


def test_table_query_rejects_bad_order():
    isr = _isr()
    lib = isr.load_library()
    for order in (0, 16, -3):
        assert lib.isr_gll_tables(order, None, None, None, None, None, None, None) == isr.EINVAL
    assert b"order" in lib.isr_last_error()


def test_null_arguments_are_rejected_without_a_gpu():
    isr = _isr()
    lib = isr.load_library()
    assert lib.isr_destroy(None) == isr.EINVAL
    assert lib.isr_compress(None, None, None, None) == isr.EINVAL
    assert lib.isr_blob_size(None, None) == isr.EINVAL
    assert lib.isr_blob_from_host(None, None, 0, None) == isr.EINVAL
    lib.isr_blob_free(None)  # no-op


def test_parse_blob_rejects_garbage():
    isr = _isr()
    with pytest.raises(ValueError):
        isr.parse_blob(b"XXXX" + bytes(60))
