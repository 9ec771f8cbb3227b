"""64-bit machine-word primes (zpm_mul_p64): bit-exact parity with the oracle.

Small and ragged shapes for every prime count (1, 2, 3) and a range of K cover:
a y-transform of one pass and of two passes with four-step twiddles (column tiles 1 and
16), x-transforms of 4 to 1024 points, limbs wider than 64 bits, a single coefficient,
squares, extreme coefficients and bits above N.  Seeded random shapes with random
feasible (K, np) follow, and zpm_mul (31-bit primes) must give the same words.  At the
full 2^16 x 4097-bit size, the default plan and the paper's two-prime configuration
(K = 128, M = 33) must reproduce the oracle's stored digest of the whole product.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1612_05778_amd import _native as nat
from paper_1612_05778_amd import api, synth
from tests.gpu_util import dev, host, words_for
from tests.test_gpu_fullsize import check_digest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def check(ctx, A, da, Na, B, db, Nb, K=0, np_=0, square=False):
    print(f"[p64] da={da} Na={Na} db={db} Nb={Nb} K={K} np={np_} square={square}", flush=True)
    ta = dev(A)
    tb = ta if square else dev(B)
    got = host(ctx.mul_p64(ta, Na, tb, Nb, K=K, np=np_))
    ref = oracle.polymul(A, da, Na, B, db, Nb, wc=got.shape[1])
    bad = np.nonzero((got != ref).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} coefficients differ, first at {bad[:8].tolist()}"
    return got


CASES = [
    # da, Na, db, Nb, K, np
    (1, 2, 1, 2, 0, 0),              # one coefficient each: L = 1, no y pass
    (3, 70, 2, 65, 4, 1),
    (40, 64, 30, 90, 4, 1),
    (5, 100, 7, 130, 8, 2),
    (9, 200, 9, 201, 4, 3),
    (17, 130, 3, 150, 2, 3),         # limbs of 75 bits (two words)
    (300, 20, 260, 33, 2, 1),        # two y passes
    (2100, 8, 2000, 10, 2, 1),       # two y passes, 16-wide column tiles
    (2, 1100, 3, 1000, 512, 1),      # 1024-point x-transforms
    (1000, 513, 1001, 700, 0, 0),
    (4097, 257, 3000, 300, 0, 0),
    (700, 900, 650, 1000, 64, 3),
    (2000, 2000, 1500, 64, 128, 2),
    (5000, 300, 6000, 200, 0, 2),
    (3, 5000, 2, 4000, 0, 0),
]


@pytest.mark.parametrize("da,Na,db,Nb,K,np_", CASES)
def test_p64_shapes(ctx, da, Na, db, Nb, K, np_):
    r = np.random.default_rng(da * 7 + db)
    a, _ = synth.signed_words(r, da, Na - 1)
    b, _ = synth.signed_words(r, db, Nb - 1)
    check(ctx, a, da, Na, b, db, Nb, K, np_)


@pytest.mark.parametrize("d,N,K,np_", [(257, 300, 0, 0), (1000, 64, 16, 1), (3001, 777, 0, 3)])
def test_p64_square(ctx, d, N, K, np_):
    p = synth.dense(300 + d, d, N - 1)
    got = check(ctx, p.a, d, N, p.a, d, N, K, np_, square=True)
    two = host(ctx.mul_p64(dev(p.a), N, dev(p.a), N, K=K, np=np_))
    assert np.array_equal(got, two), "square differs from the product of two copies"


def test_p64_extremes_and_high_bits(ctx):
    N = 300
    lo, hi = -(1 << (N - 1)), (1 << (N - 1)) - 1
    A = words_for([lo] * 257, N)
    check(ctx, A, 257, N, A, 257, N)
    B = words_for([hi if i % 2 else lo for i in range(100)], N)
    check(ctx, A, 257, N, B, 100, N, K=32, np_=3)
    # bits above N - 1 in the top word are not part of the value
    r = np.random.default_rng(11)
    a, _ = synth.signed_words(r, 500, 200)
    b, _ = synth.signed_words(r, 400, 150)
    clean = host(ctx.mul_p64(dev(a), 201, dev(b), 151))
    a2, b2 = a.copy(), b.copy()
    a2[:, -1] ^= (r.integers(0, 2**63, size=500, dtype=np.int64).astype(np.uint64) << np.uint64(9))
    b2[:, -1] ^= (r.integers(0, 2**63, size=400, dtype=np.int64).astype(np.uint64) << np.uint64(23))
    dirty = host(ctx.mul_p64(dev(a2), 201, dev(b2), 151))
    assert np.array_equal(clean, dirty)


def test_p64_random_shapes_and_agreement(ctx):
    r = np.random.default_rng(64)
    done = 0
    while done < 24:
        da, db = (int(math.exp(r.uniform(0, math.log(5000)))) for _ in range(2))
        Na, Nb = (max(2, int(math.exp(r.uniform(math.log(2), math.log(2500))))) for _ in range(2))
        if da * db * ((Na + 63) // 64) * ((Nb + 63) // 64) > 3e7:
            continue
        K = int(r.choice([0, 2, 4, 8, 16, 32, 64, 128, 256, 512]))
        np_ = int(r.choice([0, 1, 2, 3]))
        try:
            api.plan_p64(da, Na, db, Nb, K=K, np=np_)
        except nat.ZpmError:
            continue
        a, _ = synth.signed_words(r, da, Na - 1)
        b, _ = synth.signed_words(r, db, Nb - 1)
        got = check(ctx, a, da, Na, b, db, Nb, K, np_)
        if done % 4 == 0:
            other = host(ctx.mul(dev(a), Na, dev(b), Nb))
            assert np.array_equal(got, other), "64-bit and 31-bit prime paths disagree"
        done += 1


def test_p64_errors(ctx):
    a = dev(words_for([1, 2, 3], 64))
    with pytest.raises(nat.ZpmError):
        ctx.mul_p64(a, 64, a, 64, np=4)
    with pytest.raises(nat.ZpmError):
        ctx.mul_p64(a, 64, a, 64, K=3)
    # 4097-bit coefficients need K >= 64 with three primes
    with pytest.raises(nat.ZpmError):
        api.plan_p64(1 << 16, 4097, 1 << 16, 4097, K=32)


@pytest.mark.parametrize("K,np_", [(128, 2), (0, 0)])
def test_p64_bits4096_64k(ctx, K, np_):
    prod = synth.bits4096_64k()
    pl = api.plan_p64(prod.da, prod.Na, prod.db, prod.Nb, K=K, np=np_)
    print(f"[p64 fullsize] d=2^16 N=4097 K={pl['K']} M={pl['M']} np={pl['np']}", flush=True)
    out = ctx.mul_p64(dev(prod.a), prod.Na, dev(prod.b), prod.Nb, K=K, np=np_)
    torch.cuda.synchronize()
    got = host(out)
    del out
    torch.cuda.empty_cache()
    assert check_digest("bits4096_64k", got)


@pytest.mark.parametrize("K", [64, 128])
def test_p64_square_fixed_shapes(ctx, K):
    """Squares on the compile-time x-kernels (K = 64, 128) and the fixed innermost y pass:
    sampled rows against the oracle and every word against the 31-bit prime path."""
    d, N = 4097, 20 * K
    p = synth.dense(64 + K, d, N - 1)
    pl = api.plan_p64(d, N, d, N, K=K)
    assert pl["pass_log2n"][-1] == 9
    print(f"[p64 square] K={K} d={d} N={N} np={pl['np']}", flush=True)
    A = dev(p.a)
    got = host(ctx.mul_p64(A, N, A, N, K=K))
    other = host(ctx.mul(A, N, A, N))
    assert np.array_equal(got, other), "64-bit and 31-bit prime squares disagree"
    rows = [0, 1, d - 1, d, 2 * d - 3, 2 * d - 2, 1234, 5000]
    ref = oracle.polymul_rows(p.a, d, N, p.a, d, N, rows, wc=got.shape[1])
    assert np.array_equal(got[rows], ref)
