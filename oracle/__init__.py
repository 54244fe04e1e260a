"""Exact CPU oracle for C = A B mod p.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing here is imported by the GPU
library or its Python binding, and nothing here imports them.

Two independent parts:

* ``mm_modp`` / ``mm_modp_entries``: the definition of the problem
  (Section 1, eq. goal), C[i][j] = sum_l A[i][l] B[l][j] mod p, computed with
  128-bit integer products and sums in plain C (``mmp_oracle.c``), OpenMP over
  rows.  Because the multiword method is exact (Section 3.2, Prop. UVMW), this
  definition is what every GPU result must equal bit for bit.
* ``paper_algorithms``: the paper's floating-point algorithms (Algs. 1-6)
  emulated step by step in IEEE binary64 on the CPU, used to pin the paper's
  block-size bound (a block one larger than the bound fails on worst-case
  inputs) and to reproduce the bitsize limits of Table tab.summary.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mmp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", _SRC, "-o", _LIB + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        u64, i64 = ctypes.c_uint64, ctypes.c_int64
        vp = ctypes.c_void_p
        lib.oracle_mm_modp.argtypes = [u64, i64, i64, i64, vp, vp, vp]
        lib.oracle_mm_modp.restype = ctypes.c_int
        lib.oracle_mm_modp_entries.argtypes = [u64, i64, i64, i64, vp, vp, i64, vp, vp, vp]
        lib.oracle_mm_modp_entries.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _u64(x) -> np.ndarray:
    a = np.asarray(x)
    if a.dtype == np.float64:
        if not np.all(np.floor(a) == a) or (a.size and a.min() < 0):
            raise ValueError("oracle inputs must be non-negative integers")
        a = a.astype(np.uint64)
    return np.ascontiguousarray(a, dtype=np.uint64)


def threads() -> int:
    return int(_load().oracle_threads())


def mm_modp(p: int, A, B) -> np.ndarray:
    """C = A B mod p exactly; A (m x k), B (k x n) integer arrays; returns uint64."""
    A = _u64(A)
    B = _u64(B)
    m, k = A.shape
    k2, n = B.shape
    if k != k2:
        raise ValueError("inner dimensions differ")
    C = np.zeros((m, n), dtype=np.uint64)
    rc = _load().oracle_mm_modp(int(p), m, n, k, A.ctypes.data, B.ctypes.data, C.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_mm_modp failed: {rc}")
    return C


def mm_modp_entries(p: int, A, B, rows, cols) -> np.ndarray:
    """Selected outputs C[rows[t], cols[t]] of A B mod p; returns uint64."""
    A = _u64(A)
    B = _u64(B)
    m, k = A.shape
    _, n = B.shape
    r = np.ascontiguousarray(rows, dtype=np.int64)
    c = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.zeros(r.shape[0], dtype=np.uint64)
    rc = _load().oracle_mm_modp_entries(int(p), m, n, k, A.ctypes.data, B.ctypes.data,
                                        r.shape[0], r.ctypes.data, c.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_mm_modp_entries failed: {rc}")
    return out
