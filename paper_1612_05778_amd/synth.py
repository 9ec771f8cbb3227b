"""Seeded synthetic workloads (random dense polynomials, as in the experiments of
Section 4: "random and dense" inputs with a stated degree and coefficient size).

This module only draws random numbers and writes them in the coefficient
layout of Section 2.3 (ceil(N/64) little-endian 64-bit words per coefficient,
two's complement).  It contains none of the multiplication method.

Generator: ``numpy.random.Generator(PCG64(seed))``; for a product the operand
``a`` is drawn before ``b``.

Workloads (sizes of the named configurations):

* ``int64_1k``   d = 1024 coefficients, uniform signed 64-bit (N = 64), seed 1.
* ``bits4096_64k`` d = 2^16, magnitude uniform in [0, 2^4096), uniform sign
  (N = 4097, 65 words), seed 2.
* ``bits16384_256k`` d = 2^18, magnitude uniform in [0, 2^16384), uniform sign
  (N = 16385, 257 words), seed 3.
* ``batch4096``  4096 products, degree log-uniform in [63, 8191], magnitude bits
  log-uniform in [32, 2048], seed 4.
* ``served``     Poisson arrivals, degree log-uniform in [15, 65535], bits
  log-uniform in [16, 8192], seed 5: a pool of distinct requests
  (``served_pool``) and arrival times (``served_arrivals``) that cycle through it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _negate_rows(mag: np.ndarray) -> np.ndarray:
    """Two's complement negation of each row of unsigned multi-word integers."""
    d, w = mag.shape
    out = ~mag
    # add one: the carry runs through the low words that were zero in ``mag``
    nz = mag != 0
    first = np.where(nz.any(axis=1), nz.argmax(axis=1), w)   # first nonzero word
    cols = np.arange(w)[None, :]
    low = cols < first[:, None]
    out[low] = 0                                              # ~0 + carry -> 0, carry on
    rows = np.nonzero(first < w)[0]
    out[rows, first[rows]] = (~mag[rows, first[rows]]) + np.uint64(1)
    return out


def signed_words(rng: np.random.Generator, d: int, mag_bits: int) -> tuple[np.ndarray, int]:
    """d coefficients with magnitude uniform in [0, 2^mag_bits) and uniform sign.

    Returns (words (d, ceil(N/64)) uint64, N) with N = mag_bits + 1.  The
    magnitude words are drawn first (row-major), then the d signs.
    """
    N = mag_bits + 1
    w = (N + 63) // 64
    mw = (mag_bits + 63) // 64
    mag = np.zeros((d, w), dtype=np.uint64)
    if mw:
        mag[:, :mw] = rng.integers(0, 2**64, size=(d, mw), dtype=np.uint64)
        top = mag_bits - 64 * (mw - 1)          # bits used in the top magnitude word
        if top < 64:
            mag[:, mw - 1] &= np.uint64((1 << top) - 1)
    sign = rng.integers(0, 2, size=d).astype(bool)
    out = mag.copy()
    if sign.any():
        out[sign] = _negate_rows(mag[sign])
    return out, N


def int64_words(rng: np.random.Generator, d: int) -> tuple[np.ndarray, int]:
    """d coefficients uniform over all signed 64-bit integers (N = 64)."""
    v = rng.integers(-2**63, 2**63, size=d, dtype=np.int64)
    return v.view(np.uint64).reshape(d, 1).copy(), 64


@dataclass
class Product:
    a: np.ndarray
    Na: int
    b: np.ndarray
    Nb: int

    @property
    def da(self) -> int:
        return self.a.shape[0]

    @property
    def db(self) -> int:
        return self.b.shape[0]


def int64_1k(seed: int = 1, d: int = 1024) -> Product:
    r = rng_for(seed)
    a, Na = int64_words(r, d)
    b, Nb = int64_words(r, d)
    return Product(a, Na, b, Nb)


def dense(seed: int, d: int, mag_bits: int) -> Product:
    r = rng_for(seed)
    a, Na = signed_words(r, d, mag_bits)
    b, Nb = signed_words(r, d, mag_bits)
    return Product(a, Na, b, Nb)


def bits4096_64k(seed: int = 2) -> Product:
    return dense(seed, 1 << 16, 4096)


def bits16384_256k(seed: int = 3) -> Product:
    return dense(seed, 1 << 18, 16384)


def _log_uniform_int(r: np.random.Generator, lo: int, hi: int, n: int) -> np.ndarray:
    x = np.floor(np.exp(r.uniform(math.log(lo), math.log(hi + 1), size=n))).astype(np.int64)
    return np.clip(x, lo, hi)


def batch_sizes(seed: int = 4, n: int = 4096, deg=(63, 8191), bits=(32, 2048)):
    """(degrees, magnitude bits) of a batch: all degrees first, then all bit sizes."""
    r = rng_for(seed)
    degs = _log_uniform_int(r, deg[0], deg[1], n)
    nbits = _log_uniform_int(r, bits[0], bits[1], n)
    return r, degs, nbits


def batch(seed: int = 4, n: int = 4096, deg=(63, 8191), bits=(32, 2048)) -> list[Product]:
    """``n`` independent products; for product t both operands have deg_t + 1
    coefficients of bits_t-bit magnitude; a then b are drawn per product."""
    r, degs, nbits = batch_sizes(seed, n, deg, bits)
    out = []
    for t in range(n):
        a, Na = signed_words(r, int(degs[t]) + 1, int(nbits[t]))
        b, Nb = signed_words(r, int(degs[t]) + 1, int(nbits[t]))
        out.append(Product(a, Na, b, Nb))
    return out


def batch_uneven(seed: int = 4, n: int = 256, deg=(63, 8191), bits=(32, 2048)) -> list[Product]:
    """Variant with independent (degree, bits) for a and b."""
    r = rng_for(seed)
    da = _log_uniform_int(r, deg[0], deg[1], n) + 1
    db = _log_uniform_int(r, deg[0], deg[1], n) + 1
    na = _log_uniform_int(r, bits[0], bits[1], n)
    nb = _log_uniform_int(r, bits[0], bits[1], n)
    out = []
    for t in range(n):
        a, Na = signed_words(r, int(da[t]), int(na[t]))
        b, Nb = signed_words(r, int(db[t]), int(nb[t]))
        out.append(Product(a, Na, b, Nb))
    return out


@dataclass
class Request:
    t_arrival: float     # seconds since stream start
    prod: Product


def served_stream(seed: int = 5, n: int = 1000, rate: float = 100.0,
                  deg=(15, 65535), bits=(16, 8192)) -> list[Request]:
    """Open-loop Poisson arrival stream: exponential inter-arrival times at ``rate``
    requests/s; per request degree and bit size log-uniform as stated."""
    r = rng_for(seed)
    gaps = r.exponential(1.0 / rate, size=n)
    degs = _log_uniform_int(r, deg[0], deg[1], n)
    nbits = _log_uniform_int(r, bits[0], bits[1], n)
    t = np.cumsum(gaps)
    out = []
    for k in range(n):
        a, Na = signed_words(r, int(degs[k]) + 1, int(nbits[k]))
        b, Nb = signed_words(r, int(degs[k]) + 1, int(nbits[k]))
        out.append(Request(float(t[k]), Product(a, Na, b, Nb)))
    return out


def served_sizes(seed: int = 5, n: int = 1000, deg=(15, 65535), bits=(16, 8192)):
    """Sizes only (degrees, bits) of ``served_stream`` with the same seed."""
    r = rng_for(seed)
    r.exponential(1.0, size=n)
    return _log_uniform_int(r, deg[0], deg[1], n), _log_uniform_int(r, bits[0], bits[1], n)


def served_pool(seed: int = 5, n_pool: int = 1024, deg=(15, 65535),
                bits=(16, 8192)) -> list[Product]:
    """``n_pool`` distinct requests of the served distribution (degree and magnitude
    bits log-uniform as stated; a then b drawn per request).  Generator stream
    ``PCG64([seed, 1])``: all degrees, then all bit sizes, then the operands."""
    r = np.random.Generator(np.random.PCG64([seed, 1]))
    degs = _log_uniform_int(r, deg[0], deg[1], n_pool)
    nbits = _log_uniform_int(r, bits[0], bits[1], n_pool)
    out = []
    for t in range(n_pool):
        a, Na = signed_words(r, int(degs[t]) + 1, int(nbits[t]))
        b, Nb = signed_words(r, int(degs[t]) + 1, int(nbits[t]))
        out.append(Product(a, Na, b, Nb))
    return out


def served_arrivals(seed: int = 5, n: int = 22000) -> np.ndarray:
    """Arrival times of an open-loop Poisson stream at rate 1 (divide by the rate in
    requests/s): cumulative sums of unit exponential gaps, stream ``PCG64([seed, 2])``.
    Request k carries pool entry ``k % n_pool``."""
    r = np.random.Generator(np.random.PCG64([seed, 2]))
    return np.cumsum(r.exponential(1.0, size=n))
