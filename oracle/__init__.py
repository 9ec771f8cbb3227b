"""ORACLE -- test infrastructure only, never part of the product path.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library must never call it.

What it computes is the plain definition of the product in Z[y] (Section 1,
problem statement; Section 2, c_i = sum_{l+m=i} a_l b_m), by schoolbook:

* ``polymul`` / ``polymul_rows``: the C schoolbook in ``schoolbook.c`` (OpenMP
  over output coefficients, 64x64->128-bit word products), reading and writing
  the fixed-width two's complement layout of Section 2.3.
* ``polymul_mod``: every c_i mod q (q odd, below 2^61) by the same definition
  over Z/qZ, for checking all coefficients of products too large for the exact
  schoolbook.
* ``pyint``: pure-Python integer helpers (encoding, evaluation mod q) and an
  independent Kronecker-substitution product used to pin the C code.

It shares no code with the GPU path (no limbs, primes or transforms here).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "schoolbook.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C schoolbook into ``oracle/liboracle.so`` with gcc + OpenMP."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-mtune=generic", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-Wall", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.oracle_polymul_rows.argtypes = [
            u64p, ctypes.c_int64, ctypes.c_int32, u64p, ctypes.c_int64, ctypes.c_int32,
            u64p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, ctypes.c_int]
        lib.oracle_polymul_rows.restype = ctypes.c_int
        lib.oracle_polymul_mod.argtypes = [
            u64p, ctypes.c_int64, ctypes.c_int32, u64p, ctypes.c_int64, ctypes.c_int32,
            ctypes.c_uint64, u64p, ctypes.c_int]
        lib.oracle_polymul_mod.restype = ctypes.c_int
        lib.oracle_threads.argtypes = [ctypes.c_int]
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(arr: np.ndarray):
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _words(arr, nwords: int) -> np.ndarray:
    a = np.asarray(arr)
    if a.dtype == np.int64:
        a = a.view(np.uint64)
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a.reshape(-1, nwords)


def out_bits(da: int, Na: int, db: int, Nb: int) -> int:
    """Two's complement width that always holds c_i: |c_i| <= min(da,db) 2^(Na+Nb-2)
    (Relation (citighterbound) with the term count made exact)."""
    t = min(da, db)
    return Na + Nb - 1 + (t).bit_length() if t > 0 else 1


def polymul(a, da: int, Na: int, b, db: int, Nb: int, wc: int | None = None,
            nthreads: int = 0) -> np.ndarray:
    """All da+db-1 coefficients of a*b as a (da+db-1, wc) uint64 array."""
    return polymul_rows(a, da, Na, b, db, Nb, None, wc, nthreads)


def polymul_rows(a, da: int, Na: int, b, db: int, Nb: int, rows, wc: int | None = None,
                 nthreads: int = 0) -> np.ndarray:
    """Selected output coefficients (``rows`` = list of indices, None = all)."""
    lib = _load()
    wa, wb = (Na + 63) // 64, (Nb + 63) // 64
    if wc is None:
        wc = (out_bits(da, Na, db, Nb) + 63) // 64
    A = _words(a, wa)
    B = _words(b, wb)
    assert A.shape[0] == da and B.shape[0] == db
    if rows is None:
        n = max(da + db - 1, 0) if (da and db) else 0
        rp = None
        nr = 0
    else:
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        n = r.shape[0]
        rp = r.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        nr = n
    C = np.zeros((n, wc), dtype=np.uint64)
    if n == 0:
        return C
    rc = lib.oracle_polymul_rows(_ptr(A), da, Na, _ptr(B), db, Nb, _ptr(C), wc, rp, nr, nthreads)
    if rc != 0:
        raise ValueError("oracle_polymul_rows failed")
    return C


def polymul_mod(a, da: int, Na: int, b, db: int, Nb: int, q: int,
                nthreads: int = 0) -> np.ndarray:
    """c_i mod q for all da+db-1 coefficients of a*b (residues in [0, q)), by the
    schoolbook convolution of the operands' residues; q odd, below 2^61."""
    lib = _load()
    wa, wb = (Na + 63) // 64, (Nb + 63) // 64
    A = _words(a, wa)
    B = _words(b, wb)
    assert A.shape[0] == da and B.shape[0] == db
    n = da + db - 1 if (da and db) else 0
    C = np.zeros(n, dtype=np.uint64)
    if n == 0:
        return C
    if lib.oracle_polymul_mod(_ptr(A), da, Na, _ptr(B), db, Nb, q, _ptr(C), nthreads) != 0:
        raise ValueError("oracle_polymul_mod failed")
    return C


def threads(nthreads: int = 0) -> int:
    """Threads an OpenMP region of the oracle uses for the given request (0 = default)."""
    return _load().oracle_threads(nthreads)
