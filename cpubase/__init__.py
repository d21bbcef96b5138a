"""Fast FP64 CPU baseline (C + OpenMP, ``isr_cpu.c``): the same lossy step as
the GPU library, timed by bench.py on the host cores beside the oracle.

Not part of the GPU library and not used by it.  ``build()`` compiles
``libisr_cpu.so`` in this directory; ``compress()`` marshals NumPy arrays
(the transform tables are inputs: the caller passes the canonical FP64
tables).
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import List

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "isr_cpu.c")
LIB = os.path.join(HERE, "libisr_cpu.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall", SRC,
           "-o", tmp, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


class _Stats(C.Structure):
    _fields_ = [("U2", C.c_double), ("B", C.c_double), ("tau", C.c_double), ("dropped", C.c_double),
                ("err2", C.c_double), ("rel", C.c_double), ("kept", C.c_uint64), ("repair_iters", C.c_int32),
                ("status", C.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} not built (run cpubase.build())")
        lib = C.CDLL(LIB)
        P = C.c_void_p
        lib.isr_cpu_compress.restype = C.c_int
        lib.isr_cpu_compress.argtypes = [P, C.c_int64, C.c_int, C.c_int, C.c_int64, C.c_double, P, P, P, P, P,
                                         C.c_int, P, P, P, C.c_uint64, P]
        _lib = lib
    return _lib


@dataclass
class CpuResult:
    status: int
    stats: List[dict]
    bitmap: np.ndarray      # uint64 [ncomp, E, W]
    elem_ptr: np.ndarray    # uint64 [ncomp, E + 1]
    values: List[np.ndarray]


def compress(u: np.ndarray, order: int, tol: float, A, V, w3, g3, jac=None, threads: int = 0) -> CpuResult:
    """u[ncomp, E, n, n, n] FP64 (contiguous); tables as FP64 arrays."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    ncomp, E = u.shape[0], u.shape[1]
    n = order + 1
    W = (n ** 3 + 63) // 64
    bitmap = np.zeros((ncomp, E, W), dtype=np.uint64)
    elem_ptr = np.zeros((ncomp, E + 1), dtype=np.uint64)
    values = np.empty(u.size, dtype=np.float64)
    st = (_Stats * ncomp)()
    tabs = [np.ascontiguousarray(t, dtype=np.float64) for t in (A, V, w3, g3)]
    jp = None
    if jac is not None:
        jac = np.ascontiguousarray(jac, dtype=np.float64)
        jp = jac.ctypes.data
    p = lambda a: a.ctypes.data  # noqa: E731
    rc = _load().isr_cpu_compress(p(u), E, order, ncomp, 0, float(tol), *(p(t) for t in tabs), jp, int(threads),
                                  p(bitmap), p(elem_ptr), p(values), values.size, st)
    if rc not in (0, -4):
        raise RuntimeError(f"isr_cpu_compress failed with {rc}")
    stats = [{k: getattr(st[c], k) for k, _ in _Stats._fields_} for c in range(ncomp)]
    vals, off = [], 0
    for s in stats:
        vals.append(values[off:off + s["kept"]])
        off += s["kept"]
    return CpuResult(rc, stats, bitmap, elem_ptr, vals)
