"""Python binding of the C ABI in include/isr.h (ctypes; marshalling only).

Every step of the compression runs in the HIP library ``libisr.so`` built in
this directory.  torch is used for device memory and streams only: callers
pass CUDA (HIP) tensors, the binding passes their data pointers and the
current stream.  There is no fallback: if the library is missing or fails to
load, every call raises.

torch is imported before the library is loaded so that the process holds a
single HIP runtime (torch ships one with the same soname).
"""

from __future__ import annotations

import ctypes as C
import os
import struct
import weakref
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np

import torch  # noqa: F401  (must precede loading libisr.so)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libisr.so")

OK, PENDING, EINVAL, ENOMEM, EDEVICE, ETOL, ENOTFOUND = 0, 1, -1, -2, -3, -4, -6
PREC_FP64, PREC_FP32, PREC_BF16 = 0, 1, 2
FLAG_TIMING = 1
FLAG_BATCH_PERSISTENT = 4  # FP32/BF16 batches (>= 8, orders 5/7/9) as one persistent launch
FIELD_COPY = 1  # isr_field.flags: copy-on-submit
MAX_COMP = 8
NPHASE = 9
PHASES = ("pass1", "select1", "pass2", "refine", "pass3", "finalize", "repair", "fallback", "sample")
PRECISIONS = {"fp64": PREC_FP64, "fp32": PREC_FP32, "bf16": PREC_BF16}
_STATUS = {OK: "ISR_OK", PENDING: "ISR_PENDING", EINVAL: "ISR_EINVAL", ENOMEM: "ISR_ENOMEM",
           EDEVICE: "ISR_EDEVICE", ETOL: "ISR_ETOL", ENOTFOUND: "ISR_ENOTFOUND"}


class IsrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class isr_config(C.Structure):
    _fields_ = [("device", C.c_int32), ("flags", C.c_uint32), ("hbm_budget_bytes", C.c_uint64),
                ("max_inflight", C.c_int32), ("host_threads", C.c_int32), ("autotune_path", C.c_char_p)]


class isr_field(C.Structure):
    _fields_ = [("field", C.c_void_p), ("n_elem", C.c_int64), ("order", C.c_int32), ("ncomp", C.c_int32),
                ("comp_stride", C.c_int64), ("tol", C.c_double), ("precision", C.c_int32),
                ("flags", C.c_int32), ("elem_jac", C.c_void_p), ("stream", C.c_void_p)]


class isr_tune_report(C.Structure):
    _fields_ = [("count", C.c_int32), ("tile", C.c_int32 * 16), ("ms", C.c_double * 16), ("best", C.c_int32)]


class isr_stats(C.Structure):
    _fields_ = [("norm2", C.c_double * MAX_COMP), ("budget", C.c_double * MAX_COMP),
                ("tau", C.c_double * MAX_COMP), ("dropped", C.c_double * MAX_COMP),
                ("err2", C.c_double * MAX_COMP), ("rel_err", C.c_double * MAX_COMP),
                ("kept", C.c_uint64 * MAX_COMP), ("in_bytes", C.c_uint64), ("blob_bytes", C.c_uint64),
                ("cr", C.c_double), ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("phase_ms", C.c_float * NPHASE), ("repair_iters", C.c_int32), ("status", C.c_int32),
                ("precision", C.c_int32), ("path", C.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libisr.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
    lib = C.CDLL(path)
    P, I32, I64, U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
    sig = {
        "isr_create": (I32, [C.POINTER(isr_config), C.POINTER(P)]),
        "isr_destroy": (I32, [P]),
        "isr_last_error": (C.c_char_p, []),
        "isr_version": (C.c_char_p, []),
        "isr_compress": (I32, [P, C.POINTER(isr_field), C.POINTER(P), C.POINTER(isr_stats)]),
        "isr_compress_batch": (I32, [P, C.POINTER(isr_field), I32, C.POINTER(P), C.POINTER(isr_stats)]),
        "isr_compress_noalloc": (I32, [P, C.POINTER(isr_field), P, U64, C.POINTER(U64), C.POINTER(isr_stats)]),
        "isr_compress_quantized": (I32, [P, C.POINTER(isr_field), C.c_double, C.POINTER(P), C.POINTER(isr_stats)]),
        "isr_compress_elemcut": (I32, [P, C.POINTER(isr_field), C.POINTER(P), C.POINTER(isr_stats)]),
        "isr_submit": (I32, [P, C.POINTER(isr_field), C.POINTER(U64)]),
        "isr_poll": (I32, [P, U64, I32, C.POINTER(P), C.POINTER(isr_stats)]),
        "isr_decompress": (I32, [P, P, P, I32, P]),
        "isr_forward": (I32, [P, C.POINTER(isr_field), P]),
        "isr_blob_info": (I32, [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I64), C.POINTER(I32)]),
        "isr_blob_size": (I32, [P, C.POINTER(U64)]),
        "isr_blob_to_host": (I32, [P, P, U64]),
        "isr_blob_from_host": (I32, [P, P, U64, C.POINTER(P)]),
        "isr_blob_free": (None, [P]),
        "isr_gll_tables": (I32, [I32] + [P] * 7),
        "isr_get_tile": (I32, [P, I32, I32, C.POINTER(I32)]),
        "isr_pack_host": (I32, [P, U64, I32, I32, C.c_uint32, I32, P, U64, C.POINTER(U64)]),
        "isr_unpack_host": (I32, [P, U64, P, U64, C.POINTER(U64)]),
        "isr_pack_submit": (I32, [P, P, I32, I32, C.c_uint32, C.POINTER(U64)]),
        "isr_pack_poll": (I32, [P, U64, I32, P, U64, C.POINTER(U64), C.POINTER(C.c_double)]),
        "isr_set_tile": (I32, [P, I32, I32, I32]),
        "isr_autotune": (I32, [P, C.POINTER(isr_field), I32, C.POINTER(isr_tune_report)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols() -> List[str]:
    """Names declared in include/isr.h (for the export check)."""
    hdr = os.path.join(os.path.dirname(_HERE), "include", "isr.h")
    import re
    names = re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(isr_\w+)\s*\(", open(hdr).read(), re.M)
    return sorted(set(names))


def _check(rc: int, what: str):
    if rc != OK:
        raise IsrError(rc, f"{what}: {load_library().isr_last_error().decode(errors='replace')}")


def gll_tables(order: int) -> Dict[str, np.ndarray]:
    """The library's own FP64 tables (host only; no GPU needed)."""
    lib = load_library()
    n = order + 1
    out = {k: np.zeros(s) for k, s in (("xi", n), ("w", n), ("V", n * n), ("A", n * n), ("gamma", n),
                                        ("w3", n ** 3), ("g3", n ** 3))}
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
    _check(lib.isr_gll_tables(order, *(ptr(out[k]) for k in ("xi", "w", "V", "A", "gamma", "w3", "g3"))),
           "isr_gll_tables")
    out["V"] = out["V"].reshape(n, n)
    out["A"] = out["A"].reshape(n, n)
    out["w3"] = out["w3"].reshape(n, n, n)
    out["g3"] = out["g3"].reshape(n, n, n)
    return out


CODECS = {"zlib": 1, "bzip2": 2}
PACK_SHUFFLE = 1


def pack_host(blob_bytes: bytes, codec="zlib", level: int = 6, shuffle: bool = False, threads: int = 0) -> bytes:
    """Lossless coding of a serialized blob on host threads (no GPU)."""
    lib = load_library()
    n = C.c_uint64()
    args = (blob_bytes, len(blob_bytes), CODECS[codec], level, PACK_SHUFFLE if shuffle else 0, threads)
    _check(lib.isr_pack_host(*args, None, 0, C.byref(n)), "isr_pack_host")
    buf = C.create_string_buffer(n.value)
    _check(lib.isr_pack_host(*args, buf, n.value, C.byref(n)), "isr_pack_host")
    return buf.raw[:n.value]


def unpack_host(packed: bytes) -> bytes:
    """Inverse of pack_host."""
    lib = load_library()
    n = C.c_uint64()
    _check(lib.isr_unpack_host(packed, len(packed), None, 0, C.byref(n)), "isr_unpack_host")
    buf = C.create_string_buffer(n.value)
    _check(lib.isr_unpack_host(packed, len(packed), buf, n.value, C.byref(n)), "isr_unpack_host")
    return buf.raw[:n.value]


def _stats_dict(st: isr_stats, ncomp: int) -> dict:
    return {
        "norm2": list(st.norm2[:ncomp]), "budget": list(st.budget[:ncomp]), "tau": list(st.tau[:ncomp]),
        "dropped": list(st.dropped[:ncomp]), "err2": list(st.err2[:ncomp]), "rel_err": list(st.rel_err[:ncomp]),
        "kept": list(st.kept[:ncomp]), "in_bytes": st.in_bytes, "blob_bytes": st.blob_bytes, "cr": st.cr,
        "t_submit": st.t_submit, "t_start": st.t_start, "t_done": st.t_done,
        "phase_ms": dict(zip(PHASES, list(st.phase_ms))), "repair_iters": st.repair_iters,
        "status": st.status, "precision": st.precision, "path": st.path,
    }


@dataclass
class BlobArrays:
    order: int
    ncomp: int
    n_elem: int
    value_bytes: int
    words: int
    tol: float
    precision: int
    status: int
    engine: int                # FP32 / BF16: engine whose inverse decompresses it (0 general, 1 wave-tile, 2 dense)
    tile: int                  # its dense tile (engine 2)
    value_kind: int            # 0 coefficient values, 1 quantisation codes (qstep per component)
    comps: List[dict]          # U2, B, tau, dropped, err2, rel_err, kept, voff, qstep
    bitmap: np.ndarray         # uint64 [ncomp, n_elem, W]
    elem_ptr: np.ndarray       # uint64 [ncomp, n_elem + 1]
    values: List[np.ndarray]   # per component


def parse_blob(buf: bytes) -> BlobArrays:
    """Split a serialized blob (layout documented in include/isr.h)."""
    if buf[:4] != b"ISR1":
        raise ValueError("not an ISR1 blob")
    version, = struct.unpack_from("<I", buf, 4)
    if version != 3:
        raise ValueError(f"blob version {version} is not 3")
    order, ncomp, n_elem, vb, W, tol, prec, status, engine, tile, kind = struct.unpack_from("<iiqiidiiiii", buf, 8)
    comps = []
    off = 64
    for _ in range(ncomp):
        U2, B, tau, dropped, err2, rel, kept, voff, qstep = struct.unpack_from("<6d2Qd", buf, off)
        comps.append(dict(U2=U2, B=B, tau=tau, dropped=dropped, err2=err2, rel_err=rel, kept=kept, voff=voff,
                          qstep=qstep))
        off += 72
    nb = ncomp * n_elem * W
    bitmap = np.frombuffer(buf, dtype="<u8", count=nb, offset=off).reshape(ncomp, n_elem, W)
    off += 8 * nb
    npt = ncomp * (n_elem + 1)
    elem_ptr = np.frombuffer(buf, dtype="<u8", count=npt, offset=off).reshape(ncomp, n_elem + 1)
    off += 8 * npt
    vdt = "<f8" if vb == 8 else "<f4"
    values = []
    for c in comps:
        values.append(np.frombuffer(buf, dtype=vdt, count=c["kept"], offset=off + c["voff"] * vb))
    return BlobArrays(order, ncomp, n_elem, vb, W, tol, prec, status, engine, tile, kind, comps, bitmap, elem_ptr,
                      values)


class Blob:
    """A compressed snapshot held in device memory by the library."""

    def __init__(self, ctx: "Context", handle: int, stats: Optional[dict], status: int):
        self._ctx = ctx
        self._h = C.c_void_p(handle)
        self.stats = stats
        self.status = status
        ctx._blobs.add(self)  # freed by Context.close() if still alive then
        lib = load_library()
        o, nc, vb = C.c_int32(), C.c_int32(), C.c_int32()
        ne = C.c_int64()
        _check(lib.isr_blob_info(self._h, C.byref(o), C.byref(nc), C.byref(ne), C.byref(vb)), "isr_blob_info")
        self.order, self.ncomp, self.n_elem, self.value_bytes = o.value, nc.value, ne.value, vb.value

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("blob was freed")
        return self._h

    def nbytes(self) -> int:
        n = C.c_uint64()
        _check(load_library().isr_blob_size(self.handle, C.byref(n)), "isr_blob_size")
        return n.value

    def to_bytes(self) -> bytes:
        n = self.nbytes()
        buf = C.create_string_buffer(n)
        _check(load_library().isr_blob_to_host(self.handle, buf, n), "isr_blob_to_host")
        return buf.raw

    def arrays(self) -> BlobArrays:
        return parse_blob(self.to_bytes())

    def free(self):
        # a blob must not outlive its context (the library frees it into the
        # context's arena)
        if self._h and self._ctx._h:
            load_library().isr_blob_free(self._h)
        self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


class Context:
    def __init__(self, device: int = 0, budget_bytes: int = 0, flags: int = 0, max_inflight: int = 0,
                 autotune_path: Optional[str] = None, host_threads: int = 0):
        lib = load_library()
        cfg = isr_config(device=device, flags=flags, hbm_budget_bytes=budget_bytes, max_inflight=max_inflight,
                         host_threads=host_threads, autotune_path=autotune_path.encode() if autotune_path else None)
        h = C.c_void_p()
        self._blobs = weakref.WeakSet()
        self._h = C.c_void_p(0)
        _check(lib.isr_create(C.byref(cfg), C.byref(h)), "isr_create")
        self._h = h
        self.device = device

    def close(self):
        if self._h:
            for b in list(self._blobs):
                b.free()
            _check(load_library().isr_destroy(self._h), "isr_destroy")
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _field(self, u: "torch.Tensor", order: int, tol: float, precision, jac=None, stream=None,
               n_elem: Optional[int] = None, comp_stride: int = 0) -> isr_field:
        if not isinstance(u, torch.Tensor) or u.dtype != torch.float64 or not u.is_cuda:
            raise TypeError("field must be a float64 CUDA tensor")
        n = order + 1
        if u.dim() != 5 or tuple(u.shape[2:]) != (n, n, n):
            raise ValueError(f"field must be [ncomp, E, {n}, {n}, {n}]")
        ncomp, E = u.shape[0], u.shape[1]
        if u.stride()[1:] != (n ** 3, n * n, n, 1):
            raise ValueError("each component must be contiguous [E, n, n, n]")
        stride = comp_stride or u.stride(0)
        p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        jp = None
        if jac is not None:
            if jac.dtype != torch.float64 or not jac.is_cuda or not jac.is_contiguous() or jac.numel() != E:
                raise ValueError("jac must be a contiguous float64 CUDA tensor of n_elem entries")
            jp = jac.data_ptr()
        return isr_field(field=u.data_ptr(), n_elem=n_elem or E, order=order, ncomp=ncomp,
                         comp_stride=stride, tol=float(tol), precision=p, flags=0,
                         elem_jac=jp, stream=_stream_ptr(stream))

    def get_tile(self, order: int, precision) -> int:
        """Tile shape in use for (order, precision): 0 = wave-tile engine, T = dense tiles of T elements."""
        t = C.c_int32()
        p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        _check(load_library().isr_get_tile(self._h, order, p, C.byref(t)), "isr_get_tile")
        return t.value

    def set_tile(self, order: int, precision, tile: int):
        """Use tile shape `tile` (-1: built-in choice) for later requests of (order, precision)."""
        p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        _check(load_library().isr_set_tile(self._h, order, p, int(tile)), "isr_set_tile")

    def autotune(self, u, order: int, tol: float, precision, reps: int = 3) -> dict:
        """Time every tile shape of (order, precision) on this field; keep the fastest."""
        f = self._field(u, order, tol, precision)
        r = isr_tune_report()
        _check(load_library().isr_autotune(self._h, C.byref(f), int(reps), C.byref(r)), "isr_autotune")
        return {"best": r.best, "ms": {int(r.tile[k]): float(r.ms[k]) for k in range(r.count)}}

    def compress(self, u, order: int, tol: float, precision="fp64", jac=None, stream=None) -> Blob:
        f = self._field(u, order, tol, precision, jac, stream)
        h = C.c_void_p()
        st = isr_stats()
        rc = load_library().isr_compress(self._h, C.byref(f), C.byref(h), C.byref(st))
        if rc not in (OK, ETOL):
            _check(rc, "isr_compress")
        return Blob(self, h.value, _stats_dict(st, f.ncomp), rc)

    def compress_quantized(self, u, order: int, tol: float, share: float = 0.5, stream=None) -> Blob:
        """Quantised variant (FP64 path): cut at (1 - share) of the budget,
        kept coefficients coded as integers with the rest of it."""
        f = self._field(u, order, tol, "fp64", None, stream)
        h = C.c_void_p()
        st = isr_stats()
        rc = load_library().isr_compress_quantized(self._h, C.byref(f), float(share), C.byref(h), C.byref(st))
        if rc not in (OK, ETOL):
            _check(rc, "isr_compress_quantized")
        return Blob(self, h.value, _stats_dict(st, f.ncomp), rc)

    def compress_elemcut(self, u, order: int, tol: float, jac=None, stream=None) -> Blob:
        """Per-element cut (FP64 path): every element cut alone at its own
        share of the budget."""
        f = self._field(u, order, tol, "fp64", jac, stream)
        h = C.c_void_p()
        st = isr_stats()
        rc = load_library().isr_compress_elemcut(self._h, C.byref(f), C.byref(h), C.byref(st))
        if rc not in (OK, ETOL):
            _check(rc, "isr_compress_elemcut")
        return Blob(self, h.value, _stats_dict(st, f.ncomp), rc)

    def compress_noalloc(self, u, order: int, tol: float, out, precision="fp64", stream=None):
        """Allocation-free compression into `out` (a uint8 CUDA tensor of at
        least the worst-case blob size, 256-byte aligned).  Returns
        (status, blob bytes, stats dict); the serialized blob is out[:bytes]."""
        f = self._field(u, order, tol, precision, None, stream)
        if not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != torch.uint8 or not out.is_contiguous():
            raise TypeError("out must be a contiguous uint8 CUDA tensor")
        n = C.c_uint64()
        st = isr_stats()
        rc = load_library().isr_compress_noalloc(self._h, C.byref(f), C.c_void_p(out.data_ptr()), out.numel(),
                                                 C.byref(n), C.byref(st))
        if rc not in (OK, ETOL):
            _check(rc, "isr_compress_noalloc")
        return rc, n.value, _stats_dict(st, f.ncomp)

    def compress_batch(self, fields: Sequence[tuple], precision="fp64", stream=None) -> List[Blob]:
        """fields: sequence of (u, order, tol)."""
        fs = (isr_field * len(fields))(*[self._field(u, o, t, precision, None, stream) for (u, o, t) in fields])
        hs = (C.c_void_p * len(fields))()
        sts = (isr_stats * len(fields))()
        rc = load_library().isr_compress_batch(self._h, fs, len(fields), hs, sts)
        if rc not in (OK, ETOL):
            _check(rc, "isr_compress_batch")
        return [Blob(self, hs[i], _stats_dict(sts[i], fs[i].ncomp), sts[i].status) for i in range(len(fields))]

    def submit(self, u, order: int, tol: float, precision="fp64", stream=None, copy: bool = False) -> int:
        """Queue a compression; with copy=True the library copies the field at
        submit (copy-on-submit) and the caller may overwrite it at once (on
        the same stream)."""
        f = self._field(u, order, tol, precision, None, stream)
        f.flags = FIELD_COPY if copy else 0
        req = C.c_uint64()
        _check(load_library().isr_submit(self._h, C.byref(f), C.byref(req)), "isr_submit")
        return req.value

    def poll(self, req: int, wait_ms: int = 0):
        """Returns None while pending, else the Blob (raises on errors)."""
        h = C.c_void_p()
        st = isr_stats()
        rc = load_library().isr_poll(self._h, req, wait_ms, C.byref(h), C.byref(st))
        if rc == PENDING:
            return None
        if rc not in (OK, ETOL):
            _check(rc, "isr_poll")
        nc = 0
        b = Blob(self, h.value, None, rc)
        b.stats = _stats_dict(st, b.ncomp)
        return b

    def decompress(self, blob: Blob, out=None, dtype=torch.float64, stream=None):
        n = blob.order + 1
        if out is None:
            out = torch.empty((blob.ncomp, blob.n_elem, n, n, n), dtype=dtype, device=f"cuda:{self.device}")
        prec = PREC_FP64 if out.dtype == torch.float64 else PREC_FP32
        if not out.is_contiguous() or out.numel() != blob.ncomp * blob.n_elem * n ** 3:
            raise ValueError("output must be a contiguous [ncomp, E, n, n, n] tensor")
        _check(load_library().isr_decompress(self._h, blob.handle, C.c_void_p(out.data_ptr()), prec,
                                             C.c_void_p(_stream_ptr(stream))), "isr_decompress")
        return out

    def forward(self, u, order: int, precision="fp64", stream=None):
        f = self._field(u, order, 0.0, precision, None, stream)
        n = order + 1
        dt = torch.float64 if f.precision == PREC_FP64 else torch.float32
        out = torch.empty((f.ncomp, f.n_elem, n, n, n), dtype=dt, device=u.device)
        _check(load_library().isr_forward(self._h, C.byref(f), C.c_void_p(out.data_ptr())), "isr_forward")
        return out

    def pack_submit(self, blob: Blob, codec="zlib", level: int = 6, shuffle: bool = False) -> int:
        """Queue the blob for lossless coding on the context's host threads."""
        job = C.c_uint64()
        _check(load_library().isr_pack_submit(self._h, blob.handle, CODECS[codec], level,
                                              PACK_SHUFFLE if shuffle else 0, C.byref(job)), "isr_pack_submit")
        return job.value

    def pack_poll(self, job: int, wait_ms: int = 0):
        """None while pending, else (packed bytes, seconds from submit to done)."""
        lib = load_library()
        n = C.c_uint64()
        secs = C.c_double()
        rc = lib.isr_pack_poll(self._h, job, wait_ms, None, 0, C.byref(n), C.byref(secs))
        if rc == PENDING:
            return None
        _check(rc, "isr_pack_poll")
        buf = C.create_string_buffer(n.value)
        _check(lib.isr_pack_poll(self._h, job, 0, buf, n.value, C.byref(n), C.byref(secs)), "isr_pack_poll")
        return buf.raw[:n.value], secs.value

    def blob_from_bytes(self, buf: bytes) -> Blob:
        h = C.c_void_p()
        _check(load_library().isr_blob_from_host(self._h, buf, len(buf), C.byref(h)), "isr_blob_from_host")
        return Blob(self, h.value, None, OK)
