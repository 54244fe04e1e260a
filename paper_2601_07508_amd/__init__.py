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


class MmpOperand(ctypes.Structure):
    _fields_ = [("planes", _vp), ("p", _u64), ("side", _int), ("digits", _int), ("rows", _i64), ("cols", _i64),
                ("kp", _i64)]


class MmpOpts(ctypes.Structure):
    _fields_ = [("form", _int), ("validate_entries", _int), ("tile", _int), ("strict_fmod", _int),
                ("force_kblock", _i64), ("workspace", _vp), ("workspace_bytes", _sz), ("extended_block", _int),
                ("splits", _int), ("centered_words", _int), ("batch_launch", _int),
                ("prepared_a", ctypes.POINTER(MmpOperand)), ("prepared_b", ctypes.POINTER(MmpOperand))]


class MmpPlan(ctypes.Structure):
    _fields_ = [("p", _u64), ("u", _int), ("v", _int), ("form", _int), ("alpha", _u64), ("beta", _u64),
                ("lambda_", _i64), ("kblock", _i64), ("slots", _int), ("lazy", _int), ("extended", _int),
                ("tile", _int),
                ("bm", _int), ("bn", _int), ("bk", _int), ("digits_a", _int), ("digits_b", _int),
                ("kblock_int8", _i64), ("q", _dbl), ("est_seconds", _dbl), ("splits", _int),
                ("workspace_bytes", _sz), ("centered", _int), ("biased", _int)]

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
_lib.mm_modp_static.argtypes = list(_lib.mm_modp_async.argtypes)
_lib.mm_modp_static.restype = _int
STATIC_SCRATCH_BYTES = 256 << 20  # MMP_STATIC_SCRATCH_BYTES
_lib.mmp_plan.argtypes = [_u64, _int, _int, _i64, _i64, _i64, ctypes.POINTER(MmpOpts),
                          ctypes.POINTER(MmpPlan)]
_lib.mmp_plan.restype = _int
_lib.mmp_footprint.argtypes = [ctypes.POINTER(MmpJob), ctypes.POINTER(MmpPlan)]
_lib.mmp_footprint.restype = _sz
_lib.mmp_strerror.argtypes = [_int]
_lib.mmp_strerror.restype = ctypes.c_char_p
_lib.mmp_last_hip_error.argtypes = []
_lib.mmp_last_hip_error.restype = _int


_lib.mm_modp_batched.argtypes = [ctypes.POINTER(MmpJob), _int, ctypes.POINTER(MmpOpts), _vp]
_lib.mm_modp_batched.restype = _int
_lib.mmp_workspace_batched.argtypes = [ctypes.POINTER(MmpJob), _int, ctypes.POINTER(MmpOpts)]
_lib.mmp_workspace_batched.restype = _sz
_lib.mm_modp_crt.argtypes = [ctypes.POINTER(MmpOpts), _vp, _i64, _vp, _i64, _i64, _i64, _i64, _int,
                             ctypes.POINTER(_u64), _int, ctypes.POINTER(_vp), _i64, _vp]
_lib.mm_modp_crt.restype = _int
_lib.mmp_workspace_crt.argtypes = [_i64, _i64, _i64, _int, _int, ctypes.POINTER(MmpOpts)]
_lib.mmp_workspace_crt.restype = _sz


_lib.mmp_autotune.argtypes = [_u64, _i64, _i64, _i64, ctypes.POINTER(MmpOpts), ctypes.POINTER(MmpPlan),
                              ctypes.POINTER(_int)]
_lib.mmp_autotune.restype = _int
_lib.mmp_tune_cache_clear.argtypes = []
_lib.mmp_tune_cache_clear.restype = _int
_lib.mmp_tune_cache_save.argtypes = [ctypes.c_char_p]
_lib.mmp_tune_cache_save.restype = _int
_lib.mmp_tune_cache_load.argtypes = [ctypes.c_char_p]
_lib.mmp_tune_cache_load.restype = _int


class MmpInt8Bound(ctypes.Structure):
    _fields_ = [("digits", _int), ("weight_max", _int), ("weight_min", _int), ("lo", _i64), ("hi", _i64),
                ("term_max", _i64), ("term_min", _i64), ("witness_max", _i64 * 2), ("witness_min", _i64 * 2),
                ("kblock", _i64)]

    def as_dict(self):
        d = {f[0]: getattr(self, f[0]) for f in self._fields_}
        d["witness_max"] = tuple(self.witness_max)
        d["witness_min"] = tuple(self.witness_min)
        return d


_lib.mmp_int8_bound.argtypes = [_u64, _int, ctypes.POINTER(MmpInt8Bound)]
_lib.mmp_int8_bound.restype = _int
_lib.mmp_int8_interval_bound.argtypes = [_int, _i64, _i64, ctypes.POINTER(MmpInt8Bound)]
_lib.mmp_int8_interval_bound.restype = _int


class MmpTimer(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", _i64), ("total_ms", _dbl)]


_lib.mmp_timers_enable.argtypes = [_int]
_lib.mmp_timers_enable.restype = _int
_lib.mmp_timers_read.argtypes = [ctypes.POINTER(MmpTimer), _int, _int]
_lib.mmp_timers_read.restype = _int


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


def timers_enable(on: bool = True) -> None:
    """Start (or stop) recording per-phase kernel times (see mmp_timers_enable)."""
    _lib.mmp_timers_enable(1 if on else 0)


def timers_read(reset: bool = True) -> dict:
    """{phase: (launches, total_ms)} of the recorded launches; waits for them."""
    n = _lib.mmp_timers_read(None, 0, 0)
    buf = (MmpTimer * max(n, 1))()
    n = _lib.mmp_timers_read(buf, len(buf), 1 if reset else 0)
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(min(n, len(buf)))}


def lib() -> ctypes.CDLL:
    """The loaded C library (for tests of the raw C-ABI)."""
    return _lib


def strerror(status: int) -> str:
    return _lib.mmp_strerror(status).decode()


def _opts(form=FORM_AUTO, force_kblock=0, validate_entries=False, tile=0, strict_fmod=False,
          workspace=None, extended_block=False, splits=0, centered_words=False, prepared_a=None,
          prepared_b=None, batch_launch=0):
    o = MmpOpts()
    o.batch_launch = batch_launch
    if prepared_a is not None:  # a PreparedOperand (its struct lives as long as it does)
        o.prepared_a = ctypes.pointer(prepared_a.desc)
    if prepared_b is not None:
        o.prepared_b = ctypes.pointer(prepared_b.desc)
    o.splits = splits
    o.extended_block = 1 if extended_block else 0
    o.centered_words = 1 if centered_words else 0
    o.form = form
    o.force_kblock = force_kblock
    o.validate_entries = 1 if validate_entries else 0
    o.tile = tile
    o.strict_fmod = 1 if strict_fmod else 0
    if workspace is not None:  # a device tensor owned by the caller
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    return o


def plan(p: int, m: int, n: int, k: int, u: int = 0, v: int = 0, **opts) -> dict:
    """The planner's decisions for one product (host only; see mmp_plan)."""
    out = MmpPlan()
    o = _opts(**opts)
    _check(_lib.mmp_plan(p, u, v, m, n, k, ctypes.byref(o), ctypes.byref(out)), "mmp_plan")
    return out.as_dict()


def int8_bound(p: int = 0, entry_bits: int = 0) -> dict:
    """The INT8-digit form's exact int32 block for residues mod p, or for the
    integers below 2^entry_bits of mm_modp_crt (host only; see mmp_int8_bound)."""
    out = MmpInt8Bound()
    _check(_lib.mmp_int8_bound(p, entry_bits, ctypes.byref(out)), "mmp_int8_bound")
    return out.as_dict()


def int8_interval_bound(digits: int, lo: int, hi: int) -> dict:
    """The same for entries whose digit values lie in [lo, hi] (mmp_int8_interval_bound)."""
    out = MmpInt8Bound()
    _check(_lib.mmp_int8_interval_bound(digits, lo, hi, ctypes.byref(out)), "mmp_int8_interval_bound")
    return out.as_dict()


def autotune(p: int, m: int, n: int, k: int, **opts):
    """Times the candidate plans on the device; returns (plan, candidates timed)."""
    out = MmpPlan()
    tried = _int()
    o = _opts(**opts)
    _check(_lib.mmp_autotune(p, m, n, k, ctypes.byref(o), ctypes.byref(out), ctypes.byref(tried)), "mmp_autotune")
    return out.as_dict(), tried.value


def tune_cache_clear():
    _lib.mmp_tune_cache_clear()


def tune_cache_save(path: str):
    _check(_lib.mmp_tune_cache_save(path.encode()), "mmp_tune_cache_save")


def tune_cache_load(path: str) -> int:
    n = _lib.mmp_tune_cache_load(path.encode())
    if n < 0:
        raise MmpError(n, "mmp_tune_cache_load")
    return n


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


def mm_modp_static(A, B, C, p: int, u: int = 0, v: int = 0, stream=None, **opts):
    """mm_modp_async with the library's fixed device workspace (mm_modp_static):
    no allocation; calls that overlap on one device race."""
    _check_mat(A, "A")
    _check_mat(B, "B")
    _check_mat(C, "C")
    m, k = A.shape
    k2, n = B.shape
    if k2 != k or tuple(C.shape) != (m, n):
        raise ValueError("shape mismatch")
    o = _opts(**opts)
    st = _lib.mm_modp_static(ctypes.byref(o), p, u, v, m, n, k, A.data_ptr(), max(A.stride(0), 1),
                             B.data_ptr(), max(B.stride(0), 1), C.data_ptr(), max(C.stride(0), 1),
                             _stream_ptr(stream))
    _check(st, "mm_modp_static")
    return C


def crt_limbs(moduli) -> int:
    """64-bit limbs that hold every integer below the product of ``moduli``."""
    M = 1
    for m in moduli:
        M *= int(m)
    return max(1, ((M - 1).bit_length() + 63) // 64)


def crt_reconstruct(residues, moduli, limbs: int = 0, out=None, stream=None):
    """The integers X in [0, prod(moduli)) with X = residues[t] mod moduli[t]
    entry by entry (see mmp_crt_reconstruct).  ``residues``: equally shaped
    float64 CUDA matrices.  Returns a (limbs, m, n) int64 CUDA tensor holding
    the 64-bit limbs, least significant first (reinterpret as unsigned)."""
    import torch
    if len(residues) != len(moduli) or not residues:
        raise ValueError("one residue matrix per modulus")
    for c in residues:
        _check_mat(c, "residue")
    m, n = residues[0].shape
    ldc = max(residues[0].stride(0), 1)
    if any(tuple(c.shape) != (m, n) or max(c.stride(0), 1) != ldc for c in residues):
        raise ValueError("residue matrices must share shape and leading dimension")
    limbs = limbs or crt_limbs(moduli)
    if out is None:
        out = torch.empty((limbs, m, n), dtype=torch.int64, device=residues[0].device)
    if not isinstance(out, torch.Tensor) or out.dtype not in (torch.int64, torch.uint64) or not out.is_cuda:
        raise TypeError("out must be an int64/uint64 CUDA tensor")
    if out.dim() != 3 or tuple(out.shape[:2]) != (limbs, m) or out.shape[2] < n or out.stride(2) != 1 \
            or out.stride(0) != m * out.stride(1):
        raise ValueError("out must be (limbs, m, >= n) with planes of m rows")
    ptrs = (_vp * len(residues))(*[c.data_ptr() for c in residues])
    mods = (_u64 * len(moduli))(*[int(x) for x in moduli])
    _check(_lib.mmp_crt_reconstruct(ptrs, ldc, mods, len(moduli), m, n, out.data_ptr(), max(out.stride(1), 1),
                                    limbs, _stream_ptr(stream)), "mmp_crt_reconstruct")
    return out


class PreparedOperand:
    """The INT8 digit planes of one operand (see mmp_prepare_operand); pass it
    as ``prepared_a=`` / ``prepared_b=`` to mm_modp_async.  Holds the planes'
    device memory and the matrix it was made from."""

    def __init__(self, M, p: int, side: int, stream=None):
        import torch
        _check_mat(M, "M")
        rows, cols = M.shape
        nbytes = _lib.mmp_operand_bytes(p, side, rows, cols)
        if nbytes == 0:
            raise MmpError(-1, "mmp_operand_bytes")
        self.planes = torch.empty(nbytes, dtype=torch.int8, device=M.device)
        self.source = M
        self.desc = MmpOperand()
        _check(_lib.mmp_prepare_operand(p, side, M.data_ptr(), rows, cols, max(M.stride(0), 1),
                                        self.planes.data_ptr(), nbytes, ctypes.byref(self.desc),
                                        _stream_ptr(stream)), "mmp_prepare_operand")


def prepare_operand(M, p: int, side: int, stream=None) -> PreparedOperand:
    """Digit planes of M (side 0: an A, side 1: a B) for reuse across products."""
    return PreparedOperand(M, p, side, stream)


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


def _jobs_array(jobs):
    """jobs: list of (A, B, C, p, u, v) with float64 CUDA tensors."""
    arr = (MmpJob * max(len(jobs), 1))()
    for i, (A, B, C, p, u, v) in enumerate(jobs):
        for t, name in ((A, "A"), (B, "B"), (C, "C")):
            _check_mat(t, name)
        m, k = A.shape
        k2, n = B.shape
        if k2 != k or tuple(C.shape) != (m, n):
            raise ValueError(f"job {i}: shape mismatch")
        j = arr[i]
        j.p, j.u, j.v, j.m, j.n, j.k = p, u, v, m, n, k
        j.A, j.lda = A.data_ptr(), max(A.stride(0), 1)
        j.B, j.ldb = B.data_ptr(), max(B.stride(0), 1)
        j.C, j.ldc = C.data_ptr(), max(C.stride(0), 1)
    return arr


def workspace_batched(jobs, **opts) -> int:
    arr = _jobs_array(jobs)
    o = _opts(**opts)
    return int(_lib.mmp_workspace_batched(arr, len(jobs), ctypes.byref(o)))


def mm_modp_batched(jobs, stream=None, **opts):
    """Runs every job (A, B, C, p, u, v) -> C = A B mod p, batched on one stream."""
    arr = _jobs_array(jobs)
    o = _opts(**opts)
    _check(_lib.mm_modp_batched(arr, len(jobs), ctypes.byref(o), _stream_ptr(stream)), "mm_modp_batched")


def _check_u64(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype not in (torch.int64, torch.uint64) or not t.is_cuda:
        raise TypeError(f"{name} must be an int64/uint64 CUDA tensor of non-negative integers")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D tensor with unit column stride")


def workspace_crt(m, n, k, entry_bits, nprimes, **opts) -> int:
    o = _opts(**opts)
    return int(_lib.mmp_workspace_crt(m, n, k, entry_bits, nprimes, ctypes.byref(o)))


def mm_modp_crt(A, B, primes, outs, entry_bits: int, stream=None, **opts):
    """outs[i] = A B mod primes[i]; A, B int64 CUDA tensors of entries < 2^entry_bits."""
    _check_u64(A, "A")
    _check_u64(B, "B")
    m, k = A.shape
    k2, n = B.shape
    if k2 != k or len(outs) != len(primes):
        raise ValueError("shape mismatch")
    ldc = None
    for C in outs:
        _check_mat(C, "C")
        if tuple(C.shape) != (m, n):
            raise ValueError("output shape mismatch")
        if ldc is not None and C.stride(0) != ldc:
            raise ValueError("outputs must share one leading dimension")
        ldc = C.stride(0)
    pr = (_u64 * len(primes))(*primes)
    cs = (_vp * len(outs))(*[C.data_ptr() for C in outs])
    o = _opts(**opts)
    _check(_lib.mm_modp_crt(ctypes.byref(o), A.data_ptr(), max(A.stride(0), 1), B.data_ptr(),
                            max(B.stride(0), 1), m, n, k, entry_bits, pr, len(primes), cs, max(ldc or n, 1),
                            _stream_ptr(stream)), "mm_modp_crt")


# ------------------------------------------------------------------ serving

class MmpServerStats(ctypes.Structure):
    _fields_ = [("submitted", _i64), ("completed", _i64), ("failed", _i64), ("rejected", _i64),
                ("launches", _i64), ("max_batch", _i64), ("queued", _i64), ("running", _i64),
                ("used_bytes", _sz), ("peak_used_bytes", _sz), ("resident_bytes", _sz),
                ("max_inflight", _i64), ("max_running", _i64)]


SERVER_DRY_RUN = 1
SERVER_FAIL_LAUNCHES = 2
SUBMIT_NOQUEUE = 1

_lib.mmp_server_create.argtypes = [ctypes.POINTER(_vp), _int, _sz, _int, _int]
_lib.mmp_server_create.restype = _int
_lib.mmp_server_destroy.argtypes = [_vp]
_lib.mmp_server_destroy.restype = _int
_lib.mmp_register_operand.argtypes = [_vp, _vp, _i64, _i64, _i64, _u64, _int, ctypes.POINTER(_u64)]
_lib.mmp_register_operand.restype = _int
_lib.mmp_crt_reconstruct.argtypes = [ctypes.POINTER(_vp), _i64, ctypes.POINTER(_u64), _int, _i64, _i64, _vp, _i64,
                                     _int, _vp]
_lib.mmp_crt_reconstruct.restype = _int
_lib.mmp_operand_bytes.argtypes = [_u64, _int, _i64, _i64]
_lib.mmp_operand_bytes.restype = _sz
_lib.mmp_prepare_operand.argtypes = [_u64, _int, _vp, _i64, _i64, _i64, _vp, _sz, ctypes.POINTER(MmpOperand), _vp]
_lib.mmp_prepare_operand.restype = _int
_lib.mmp_unregister_operand.argtypes = [_vp, _u64]
_lib.mmp_unregister_operand.restype = _int
_lib.mmp_submit.argtypes = [_vp, ctypes.POINTER(MmpJob), _int, ctypes.POINTER(_u64)]
_lib.mmp_submit_after.argtypes = [_vp, ctypes.POINTER(MmpJob), _int, _vp, ctypes.POINTER(_u64)]
_lib.mmp_submit_after.restype = _int
_lib.mmp_submit.restype = _int
_lib.mmp_poll.argtypes = [_vp, _u64, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_dbl)]
_lib.mmp_poll.restype = _int
_lib.mmp_wait.argtypes = [_vp, _u64, _dbl, ctypes.POINTER(_int), ctypes.POINTER(_dbl)]
_lib.mmp_wait.restype = _int
_lib.mmp_server_stats.argtypes = [_vp, ctypes.POINTER(MmpServerStats)]
_lib.mmp_server_stats.restype = _int


class Server:
    """Continuous-batching request server (see mmp_server_create).

    Tensors passed to submit() are kept referenced until their ticket is
    reported done, so their memory cannot be released while in flight.
    submit() orders the request after the work queued so far on torch's
    current stream (mmp_submit_after: the server's launch stream waits for
    an event recorded there), so A, B and C may still be in production on it;
    the host does not block.  register_operand() is synchronous and first
    waits for torch's current stream.
    """

    def __init__(self, hbm_budget: int, max_slots: int = 64, device: int = 0, dry_run: bool = False,
                 fail_launches: bool = False):
        self._h = _vp()
        flags = (SERVER_DRY_RUN if dry_run else 0) | (SERVER_FAIL_LAUNCHES if fail_launches else 0)
        _check(_lib.mmp_server_create(ctypes.byref(self._h), device, hbm_budget, max_slots, flags),
               "mmp_server_create")
        self._keep = {}

    def close(self):
        if self._h:
            _check(_lib.mmp_server_destroy(self._h), "mmp_server_destroy")
            self._h = _vp()
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def register_operand(self, M, p: int, side: int) -> int:
        import torch
        _check_mat(M, "M")
        torch.cuda.current_stream(M.device).synchronize()
        h = _u64()
        _check(_lib.mmp_register_operand(self._h, M.data_ptr(), M.shape[0], M.shape[1], max(M.stride(0), 1),
                                         p, side, ctypes.byref(h)), "mmp_register_operand")
        self._keep[("operand", h.value)] = M
        return h.value

    def unregister_operand(self, handle: int):
        _check(_lib.mmp_unregister_operand(self._h, handle), "mmp_unregister_operand")
        self._keep.pop(("operand", handle), None)

    def submit_raw(self, job: MmpJob, noqueue: bool = False, keep=None, stream=None) -> int:
        """A raw job: mmp_submit_after on a torch stream, or mmp_submit (no
        ordering) with stream=None."""
        t = _u64()
        flags = SUBMIT_NOQUEUE if noqueue else 0
        if stream is None:
            _check(_lib.mmp_submit(self._h, ctypes.byref(job), flags, ctypes.byref(t)), "mmp_submit")
        else:  # torch's default stream is the null stream (handle 0)
            _check(_lib.mmp_submit_after(self._h, ctypes.byref(job), flags, _vp(stream.cuda_stream),
                                         ctypes.byref(t)), "mmp_submit_after")
        if keep is not None:
            self._keep[t.value] = keep
        return t.value

    def submit(self, A, B, C, p: int, u: int = 0, v: int = 0, noqueue: bool = False, stream=None,
               ordered: bool = True) -> int:
        """Queues C = A B mod p after the work on `stream` (default: torch's
        current stream); ordered=False skips the ordering when the caller has
        already synchronised the device work that writes A, B and C."""
        import torch
        arr = _jobs_array([(A, B, C, p, u, v)])
        s = None
        if ordered:
            s = stream if stream is not None else torch.cuda.current_stream(C.device)
        return self.submit_raw(arr[0], noqueue, keep=(A, B, C), stream=s)

    def poll(self, ticket: int):
        """None while running; else (status, latency_s)."""
        done, st, lat = _int(), _int(), _dbl()
        _check(_lib.mmp_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(st), ctypes.byref(lat)), "mmp_poll")
        if not done.value:
            return None
        self._keep.pop(ticket, None)
        return st.value, lat.value

    def wait(self, ticket: int, timeout_s: float = -1.0):
        st, lat = _int(), _dbl()
        _check(_lib.mmp_wait(self._h, ticket, timeout_s, ctypes.byref(st), ctypes.byref(lat)), "mmp_wait")
        self._keep.pop(ticket, None)
        return st.value, lat.value

    def stats(self) -> dict:
        s = MmpServerStats()
        _check(_lib.mmp_server_stats(self._h, ctypes.byref(s)), "mmp_server_stats")
        return {f[0]: getattr(s, f[0]) for f in s._fields_}
