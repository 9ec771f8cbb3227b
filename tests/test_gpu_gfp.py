"""One generalized Fermat prime (zpm_mul_gfp): bit-exact parity with the oracle.

The shapes reach every prime (k = 8, 16, 32), every K from 2 to k (x-transforms of 4 to
64 points, whose roots are powers of the radix), y-transforms of zero to four passes
(with and without twiddles between them), limbs of one to many 16-bit chunks, unequal
degrees and bit sizes, a single coefficient, squares, extreme coefficients and bits
above N.  Seeded random shapes follow, and zpm_mul (31-bit primes and CRT) must give the
same words.  At 2^16 x 4097 bits the whole product must reproduce the oracle's stored
digest.
"""
import numpy as np
import pytest

import oracle
from oracle import pyint
from paper_1612_05778_amd import api, synth
from tests.gpu_util import dev, host, words_for
from tests.test_gpu_fullsize import check_digest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def check(ctx, A, da, Na, B, db, Nb, K=0, k=0, square=False):
    print(f"[gfp] da={da} Na={Na} db={db} Nb={Nb} K={K} k={k} square={square}", flush=True)
    ta = dev(A)
    tb = ta if square else dev(B)
    got = host(ctx.mul_gfp(ta, Na, tb, Nb, K=K, k=k))
    ref = oracle.polymul(A, da, Na, B, db, Nb, wc=got.shape[1])
    bad = np.nonzero((got != ref).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} coefficients differ, first at {bad[:8].tolist()}"
    return got


CASES = [
    # da, Na, db, Nb, K, k
    (1, 2, 1, 2, 0, 0),            # one coefficient each: L = 1, no y pass
    (2, 3, 1, 5, 2, 8),            # L = 2
    (3, 40, 2, 33, 2, 8),
    (9, 64, 8, 64, 4, 8),
    (17, 90, 20, 70, 8, 8),        # 16-point x-transforms, root r
    (40, 200, 30, 150, 0, 8),
    (300, 60, 260, 33, 4, 8),      # three y passes of the 8-digit prime (16, 8, 8 points)
    (700, 64, 900, 100, 8, 8),
    (5, 100, 7, 130, 2, 16),
    (33, 300, 31, 290, 16, 16),    # 32-point x-transforms
    (129, 180, 140, 200, 4, 16),
    (1000, 150, 1001, 130, 8, 16),
    (3, 500, 2, 400, 32, 32),      # 64-point x-transforms, root r
    (64, 700, 65, 650, 16, 32),
    (257, 800, 300, 500, 0, 32),
    (2100, 300, 2000, 256, 0, 32),  # three y passes (32, 16, 16 points)
    (4097, 257, 3000, 300, 0, 0),
    (5000, 40, 6000, 33, 2, 8),    # four 16-point passes
]


@pytest.mark.parametrize("da,Na,db,Nb,K,k", CASES)
def test_gfp_shapes(ctx, da, Na, db, Nb, K, k):
    r = np.random.default_rng(da * 11 + db)
    a, _ = synth.signed_words(r, da, Na - 1)
    b, _ = synth.signed_words(r, db, Nb - 1)
    check(ctx, a, da, Na, b, db, Nb, K, k)


@pytest.mark.parametrize("d,N,K,k", [(257, 300, 0, 0), (1000, 64, 8, 8), (301, 900, 0, 32),
                                     (2, 33, 2, 16)])
def test_gfp_square(ctx, d, N, K, k):
    p = synth.dense(500 + d, d, N - 1)
    got = check(ctx, p.a, d, N, p.a, d, N, K, k, square=True)
    two = host(ctx.mul_gfp(dev(p.a), N, dev(p.a), N, K=K, k=k))
    assert np.array_equal(got, two), "square differs from the product of two copies"


@pytest.mark.parametrize("k", [8, 16, 32])
def test_gfp_extremes_and_high_bits(ctx, k):
    # all coefficients -2^(N-1): the largest |c_i| and the longest carries
    for d, N in [(50, 100), (7, 61)]:
        vals = [-(1 << (N - 1))] * d
        W = words_for(vals, N)
        got = check(ctx, W, d, N, W, d, N, 0, k)
        t = [min(i + 1, 2 * d - 1 - i, d) for i in range(2 * d - 1)]
        assert pyint.decode(got, 64 * got.shape[1]) == [ti << (2 * N - 2) for ti in t]
    # max positive against -1, and alternating signs
    d, N = 40, 97
    A = words_for([(1 << (N - 1)) - 1] * d, N)
    B = words_for([-1] * d, N)
    check(ctx, A, d, N, B, d, N, 0, k)
    alt = words_for([(-1) ** i * ((1 << (N - 1)) - 1 - i) for i in range(d)], N)
    check(ctx, alt, d, N, A, d, N, 0, k)
    # bits above N are ignored (sign extension from bit N-1)
    r = np.random.default_rng(77 + k)
    d, N = 33, 70
    A = r.integers(0, 2**63, size=(d, 2), dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    B = r.integers(0, 2**63, size=(d, 2), dtype=np.uint64)
    check(ctx, A, d, N, B, d, N, 0, k)


def test_gfp_random_shapes_match_zpm_mul(ctx):
    rng = np.random.default_rng(2024)
    for it in range(12):
        da = int(np.exp(rng.uniform(0, np.log(3000))))
        db = int(np.exp(rng.uniform(0, np.log(3000))))
        Na = int(np.exp(rng.uniform(np.log(2), np.log(1200))))
        Nb = int(np.exp(rng.uniform(np.log(2), np.log(1200))))
        k = int(rng.choice([0, 8, 16, 32]))
        try:
            pl = api.plan_gfp(da, Na, db, Nb, 0, k)
        except RuntimeError:
            continue
        K = int(rng.choice([kk for kk in (2, 4, 8, 16, 32) if kk <= pl["k"]]))
        try:
            api.plan_gfp(da, Na, db, Nb, K, pl["k"])
        except RuntimeError:
            K = 0
        a, _ = synth.signed_words(rng, da, Na - 1)
        b, _ = synth.signed_words(rng, db, Nb - 1)
        got = check(ctx, a, da, Na, b, db, Nb, K, pl["k"])
        assert np.array_equal(got, host(ctx.mul(dev(a), Na, dev(b), Nb)))


def test_gfp_bits4096_64k(ctx):
    prod = synth.bits4096_64k()
    print("[gfp] d=2^16 N=4097", flush=True)
    got = host(ctx.mul_gfp(dev(prod.a), prod.Na, dev(prod.b), prod.Nb))
    assert check_digest("bits4096_64k", got)
