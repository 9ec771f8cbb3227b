"""ORACLE -- test infrastructure only.  Pure-Python integer references.

* ``decode`` / ``encode``: the coefficient layout of Section 2.3 (ceil(N/w)
  words per coefficient, two's complement, Relation (definingN) for the range),
  written independently of the GPU library and of ``schoolbook.c``.
* ``kronecker``: the same product by Kronecker substitution, a(2^s) * b(2^s) as
  one Python big-integer product, then unpacking signed base-2^s digits.  It is
  a different algorithm from the schoolbook (Python's big-integer multiply),
  used as an independent pin of the C oracle.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def decode(words, N: int) -> list[int]:
    """(d, ceil(N/64)) uint64 words -> list of Python ints (sign from bit N-1)."""
    w = (N + 63) // 64
    arr = np.asarray(words)
    if arr.dtype == np.int64:
        arr = arr.view(np.uint64)
    arr = arr.reshape(-1, w)
    out = []
    mask = (1 << N) - 1
    for row in arr:
        v = 0
        for k in range(w - 1, -1, -1):
            v = (v << 64) | int(row[k])
        v &= mask
        if v >> (N - 1):
            v -= 1 << N
        out.append(v)
    return out


def encode(vals: Sequence[int], nwords: int) -> np.ndarray:
    """list of Python ints -> (len, nwords) uint64 two's complement (mod 2^(64*nwords))."""
    out = np.zeros((len(vals), nwords), dtype=np.uint64)
    mod = 1 << (64 * nwords)
    for i, v in enumerate(vals):
        u = v % mod
        for k in range(nwords):
            out[i, k] = (u >> (64 * k)) & 0xFFFFFFFFFFFFFFFF
    return out


def kronecker(a: Sequence[int], b: Sequence[int]) -> list[int]:
    """Product via Kronecker substitution y -> 2^s with a digit width s large enough
    that every signed c_i fits in (-2^(s-1), 2^(s-1))."""
    if not a or not b:
        return []
    ha = max(abs(x) for x in a)
    hb = max(abs(y) for y in b)
    bound = min(len(a), len(b)) * ha * hb          # |c_i| <= bound
    s = bound.bit_length() + 2
    A = 0
    for x in reversed(a):
        A = (A << s) + x
    B = 0
    for y in reversed(b):
        B = (B << s) + y
    P = A * B
    n = len(a) + len(b) - 1
    out = []
    half = 1 << (s - 1)
    base = 1 << s
    for _ in range(n):
        digit = P % base             # in [0, 2^s)
        if digit >= half:
            digit -= base            # signed digit in [-2^(s-1), 2^(s-1))
        out.append(digit)
        P = (P - digit) >> s
    assert P == 0
    return out


def eval_mod(coeffs: Sequence[int], r: int, q: int) -> int:
    """Horner evaluation of sum_i coeffs[i] r^i mod q."""
    acc = 0
    for x in reversed(coeffs):
        acc = (acc * r + x) % q
    return acc
