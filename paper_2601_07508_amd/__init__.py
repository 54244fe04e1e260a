"""Python binding of libmmp: exact C = A B mod p on MI355X.

Argument marshalling only.  Every step of the product runs in the HIP
library (``libmmp.so``, built by ``build.py``); tensors are torch CUDA
tensors of dtype float64 holding integers in [0, p), and streams are torch
CUDA streams.  If the library is missing this module raises ImportError:
there is no CPU fallback.

The functions mirror the C-ABI declared in ``include/mmp.h``.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmmp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2601_07508_amd/build.py "
                      "(or __graft_entry__.build()) first")

_lib = ctypes.CDLL(LIB_PATH)

_u64, _i64, _int, _vp, _dbl, _sz = (ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.c_double, ctypes.c_size_t)

FORM_AUTO, FORM_FP64_WORDS, FORM_INT8_WORDS = 0, 1, 2

STATUS = {0: "MMP_OK", -1: "MMP_EINVAL", -2: "MMP_EBOUND", -3: "MMP_ERANGE", -4: "MMP_ENOMEM",
          -5: "MMP_EHIP", -6: "MMP_EBUSY", -7: "MMP_ENOTFOUND", -8: "MMP_ETIMEOUT"}


class MmpOpts(ctypes.Structure):
    _fields_ = [("form", _int), ("force_kblock", _i64), ("validate_entries", _int), ("tile", _int),
                ("strict_fmod", _int), ("reserved", _int * 7)]


class MmpPlan(ctypes.Structure):
    _fields_ = [("p", _u64), ("u", _int), ("v", _int), ("form", _int), ("alpha", _u64), ("beta", _u64),
                ("lambda_", _i64), ("kblock", _i64), ("slots", _int), ("lazy", _int), ("tile", _int),
                ("bm", _int), ("bn", _int), ("bk", _int), ("digits_a", _int), ("digits_b", _int),
                ("kblock_int8", _i64), ("q", _dbl), ("est_seconds", _dbl), ("workspace_bytes", _sz)]

    def as_dict(self):
        d = {f[0]: getattr(self, f[0]) for f in self._fields_}
        d["lambda"] = d.pop("lambda_")
        return d


class MmpJob(ctypes.Structure):
    _fields_ = [("p", _u64), ("u", _int), ("v", _int), ("m", _i64), ("n", _i64), ("k", _i64),
                ("A", _vp), ("lda", _i64), ("B", _vp), ("ldb", _i64), ("C", _vp), ("ldc", _i64)]


_lib.mm_modp.argtypes = [_u64, _int, _int, _i64, _i64, _i64, _vp, _vp, _vp]
_lib.mm_modp.restype = _int
_lib.mm_modp_async.argtypes = [ctypes.POINTER(MmpOpts), _u64, _int, _int, _i64, _i64, _i64, _vp, _i64,
                               _vp, _i64, _vp, _i64, _vp]
_lib.mm_modp_async.restype = _int
_lib.mmp_plan.argtypes = [_u64, _int, _int, _i64, _i64, _i64, ctypes.POINTER(MmpOpts),
                          ctypes.POINTER(MmpPlan)]
_lib.mmp_plan.restype = _int
_lib.mmp_footprint.argtypes = [ctypes.POINTER(MmpJob), ctypes.POINTER(MmpPlan)]
_lib.mmp_footprint.restype = _sz
_lib.mmp_strerror.argtypes = [_int]
_lib.mmp_strerror.restype = ctypes.c_char_p
_lib.mmp_last_hip_error.argtypes = []
_lib.mmp_last_hip_error.restype = _int


class MmpError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = f"{where}: {STATUS.get(status, status)} ({_lib.mmp_strerror(status).decode()})"
        if status == -5:
            msg += f", hipError {_lib.mmp_last_hip_error()}"
        super().__init__(msg)


def _check(status: int, where: str):
    if status != 0:
        raise MmpError(status, where)


def lib() -> ctypes.CDLL:
    """The loaded C library (for tests of the raw C-ABI)."""
    return _lib


def strerror(status: int) -> str:
    return _lib.mmp_strerror(status).decode()


def _opts(form=FORM_AUTO, force_kblock=0, validate_entries=False, tile=0, strict_fmod=False):
    o = MmpOpts()
    o.form = form
    o.force_kblock = force_kblock
    o.validate_entries = 1 if validate_entries else 0
    o.tile = tile
    o.strict_fmod = 1 if strict_fmod else 0
    return o


def plan(p: int, m: int, n: int, k: int, u: int = 0, v: int = 0, **opts) -> dict:
    """The planner's decisions for one product (host only; see mmp_plan)."""
    out = MmpPlan()
    o = _opts(**opts)
    _check(_lib.mmp_plan(p, u, v, m, n, k, ctypes.byref(o), ctypes.byref(out)), "mmp_plan")
    return out.as_dict()


def footprint(p: int, m: int, n: int, k: int, u: int = 0, v: int = 0, **opts) -> int:
    pl = MmpPlan()
    o = _opts(**opts)
    _check(_lib.mmp_plan(p, u, v, m, n, k, ctypes.byref(o), ctypes.byref(pl)), "mmp_plan")
    job = MmpJob()
    job.p, job.u, job.v, job.m, job.n, job.k = p, pl.u, pl.v, m, n, k
    return int(_lib.mmp_footprint(ctypes.byref(job), ctypes.byref(pl)))


def _check_mat(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D tensor with unit column stride")


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def mm_modp_async(A, B, C, p: int, u: int = 0, v: int = 0, stream=None, **opts):
    """C = A B mod p on ``stream`` (default: torch's current stream), asynchronous."""
    _check_mat(A, "A")
    _check_mat(B, "B")
    _check_mat(C, "C")
    m, k = A.shape
    k2, n = B.shape
    if k2 != k or tuple(C.shape) != (m, n):
        raise ValueError("shape mismatch")
    o = _opts(**opts)
    st = _lib.mm_modp_async(ctypes.byref(o), p, u, v, m, n, k, A.data_ptr(), max(A.stride(0), 1),
                            B.data_ptr(), max(B.stride(0), 1), C.data_ptr(), max(C.stride(0), 1),
                            _stream_ptr(stream))
    _check(st, "mm_modp_async")
    return C


def mm_modp(A, B, p: int, u: int = 0, v: int = 0, out=None, stream=None, **opts):
    """Returns C = A B mod p (float64 CUDA tensor), enqueued on ``stream``."""
    import torch
    m, n = A.shape[0], B.shape[1]
    C = out if out is not None else torch.empty((m, n), dtype=torch.float64, device=A.device)
    return mm_modp_async(A, B, C, p, u, v, stream=stream, **opts)


def mm_modp_sync(A, B, C, p: int, u: int = 0, v: int = 0):
    """The synchronous, contiguous, null-stream entry point ``mm_modp``."""
    _check_mat(A, "A")
    _check_mat(B, "B")
    _check_mat(C, "C")
    m, k = A.shape
    n = B.shape[1]
    for t in (A, B, C):
        if not t.is_contiguous():
            raise ValueError("mm_modp needs contiguous matrices")
    _check(_lib.mm_modp(p, u, v, m, n, k, A.data_ptr(), B.data_ptr(), C.data_ptr()), "mm_modp")
    return C
