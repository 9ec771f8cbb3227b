"""Host pins of the recovery's Chinese remaindering in matrix form (no GPU needed).

For np <= 20 primes the recovery computes c_{i,j} = sum_k y_k (P/p_k) - t P (Section 4,
the Chinese remaindering of each c_{i,j}: y_k = u_k - p_k with u_k = r_k (P/p_k)^{-1} mod
p_k as the lazy product leaves it, in [0, 2 p_k), and t = round(sum_k y_k / p_k), summed in
single precision as round(sum_k u_k / p_k) - np) as int8 products on the matrix cores: the
terms' balanced
bytes times a digit matrix A the host builds (``zpm_crt_matrix``).  This test models that
computation on the CPU with the library's A, in the kernel's lane order:

* the operand fragments of v_mfma_i32_16x16x64_i8 (lane l supplies row l mod 16 of A and
  column l mod 16 of B, each with the 16 consecutive slots 16 (l / 16) + b of a 64-slot
  step; D row 4 (l / 16) + i, column l mod 16 to lane l) -- the layout a probe on gfx950
  confirmed;
* the terms: y_k + 0x80808080 with every byte flipped, i.e. balanced signed bytes, t in
  byte 0 of term np, lane group g supplying term 4 g + w of step 0 and 16 + g + 4 w of
  step 1 as its word w;
* each lane group's fold of its digit sums into consecutive 32-bit words and a carry.

The reconstruction must equal c exactly for random c with |c| < P / (2 (1 + 2^-12)) (the
planner's bound) and at its extremes, for every np from 1 to 20, with P from the
library's own prime table and u_k drawn from both halves of [0, 2 p_k); the single-precision
quotient sum must round to the same t, with an error below 2^-15.  A's entries must be
signed bytes and every digit sum must fit the int32 accumulator.
"""
import ctypes
import random
from fractions import Fraction

import numpy as np
import pytest

from paper_1612_05778_amd import _native as nat


def primes(np_):
    out = []
    for k in range(np_):
        p, r = ctypes.c_uint32(), ctypes.c_uint32()
        assert nat.zpm_prime(k, ctypes.byref(p), ctypes.byref(r)) == nat.ZPM_OK
        out.append(p.value)
    return out


def matrix(np_):
    cap = 16 * 2 * 64 * 16
    buf = (ctypes.c_int8 * cap)()
    tiles = ctypes.c_int32()
    assert nat.zpm_crt_matrix(np_, buf, cap, ctypes.byref(tiles)) == nat.ZPM_OK
    TN = tiles.value
    frag = np.frombuffer(bytes(buf), dtype=np.int8)[:TN * 2 * 64 * 16].astype(np.int64)
    return TN, frag.reshape(TN, 2, 64, 16)


def term(st, g, w):
    """The term lane group g supplies as word w of step st."""
    return 4 * g + w if st == 0 else 16 + g + 4 * w


def stage(y, t, np_):
    """One value's terms as the kernel encodes them: y_q's balanced bytes (the bytes of
    y_q + 0x80808080, each flipped), t in byte 0 of term np."""
    return [((v + 0x80808080) & 0xFFFFFFFF) ^ 0x80808080 for v in y] + [t & 0xFF]


def mfma_model(A_frag, words, TN):
    """D for 16 values: A fragments (TN, 2, 64, 16) and each value's staged words."""
    nterms = len(words[0])
    D = np.zeros((TN, 16, 16), dtype=np.int64)          # tile, row, column (value)
    for st in range(2):
        B = np.zeros((64, 16), dtype=np.int64)         # slot, value
        for v in range(16):
            for g in range(4):
                for w in range(4):
                    q = term(st, g, w)
                    if q >= nterms:
                        continue
                    x = words[v][q]
                    for a in range(4):
                        b = ((x >> (8 * a)) & 255)
                        B[16 * g + 4 * w + a, v] = b - 256 if b >= 128 else b
        for T in range(TN):
            A = np.zeros((16, 64), dtype=np.int64)
            for lane in range(64):
                A[lane % 16, 16 * (lane // 16):16 * (lane // 16) + 16] = A_frag[T, st, lane]
            D[T] += A @ B
    return D


def fold(D, TN, v):
    """Lane groups g = 0..3 of column v: TN words and a carry each, summed."""
    total = 0
    for g in range(4):
        a, num = 0, 0
        for T in range(TN):
            for i in range(4):
                a += int(D[T, 4 * g + i, v]) << (8 * i)
            num += (a & 0xFFFFFFFF) << (32 * T)
            a >>= 32
        num += a << (32 * TN)
        total += num << (32 * TN * g)
    return total


@pytest.mark.parametrize("np_", list(range(1, 21)))
def test_matrix_crt_reconstructs(np_):
    ps = primes(np_)
    P = 1
    for p in ps:
        P *= p
    TN, A = matrix(np_)
    rng = random.Random(np_)
    cmax = P * 4096 // (2 * 4097) - 1          # the planner keeps |c| below this
    vals = [cmax, -cmax, 0, 1, -1] + [x for x in (2**31, -(2**31)) if abs(x) < cmax] + \
           [rng.randrange(-cmax, cmax + 1) for _ in range(57)]
    for chunk in range(0, len(vals), 16):
        cs = vals[chunk:chunk + 16]
        cs = cs + [0] * (16 - len(cs))
        words = []
        for c in cs:
            us = []
            for p in ps:
                Bk = P // p
                u = (c % p) * pow(Bk % p, -1, p) % p
                us.append(u + p if rng.random() < 0.5 else u)   # the lazy product's range
            y = [u - p for u, p in zip(us, ps)]
            f = sum(Fraction(yk, p) for yk, p in zip(y, ps))
            t = round(f)
            assert abs(t) <= np_
            # the kernel's single-precision sum of u_k / p_k, less np, rounds to the same t
            f32 = np.float32(0)
            for u, p in zip(us, ps):
                f32 = np.float32(f32 + np.float32(u) * np.float32(1.0 / p))
            # (its error stays far below the 2^-13 the bound leaves between c / P and 1/2)
            assert int(np.rint(f32)) - np_ == t and abs(Fraction(float(f32)) - np_ - f) < Fraction(1, 2**15)
            words.append(stage(y, t, np_))
        D = mfma_model(A, words, TN)
        assert np.abs(D).max() < 2**31
        for v, c in enumerate(cs):
            assert fold(D, TN, v) == c, (np_, c)


def test_matrix_rejects():
    buf = (ctypes.c_int8 * 16)()
    tiles = ctypes.c_int32()
    assert nat.zpm_crt_matrix(0, buf, 16, ctypes.byref(tiles)) == nat.ZPM_EINVAL
    assert nat.zpm_crt_matrix(21, buf, 16, ctypes.byref(tiles)) == nat.ZPM_EINVAL
    assert nat.zpm_crt_matrix(18, buf, 16, ctypes.byref(tiles)) == nat.ZPM_EINVAL
