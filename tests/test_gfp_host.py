"""Host-side pins of the generalized Fermat prime variant (no GPU needed).

* Each prime p = r^k + 1 of the library is prime (a Miller-Rabin written here, and
  sympy), r has the stated sparse form below 2^29, p's bit length is as reported, and
  2^21 divides p - 1 (so the y-transforms up to 2^21 points have roots, Section 2.1's
  condition on the primitive roots of unity).
* r is a primitive 2k-th root of unity mod p (r^k = -1): the premise that makes products
  by its powers digit rotations (Relation (FurerHypothesis) and Section 3.1's table of
  generalized Fermat primes).
* The root omega of order L the library returns, checked with Python integers: its order
  is exactly L, and omega^(L/2k) = r (L >= 2k) or omega = r^(2k/L), so that every y-pass
  of n <= 2k points has root r^(2k/n).
* The planner: p > 4 max(da, db) K 2^(2M) exactly (Relation (recoveryModulo)), K <= k a
  power of two, K M >= N, pass lengths summing to log2 L, each at most 2k and 32 points.
"""
import random

import pytest
import sympy

from paper_1612_05778_amd import _native as nat
from paper_1612_05778_amd import api

FORMS = {8: [(-1, 25)], 16: [(-1, 9), (-1, 7)], 32: [(-1, 14), (-1, 13)]}


def miller_rabin(n: int, rounds: int = 24) -> bool:
    if n < 4:
        return n in (2, 3)
    if n % 2 == 0:
        return False
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    rng = random.Random(n & 0xFFFFFFFF)
    for _ in range(rounds):
        a = rng.randrange(2, n - 1)
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def value(digits, r, p):
    return sum(d * r**l for l, d in enumerate(digits)) % p


@pytest.mark.parametrize("k", [8, 16, 32])
def test_prime(k):
    r, log2p = api.gfp_prime(k)
    assert r == 2**29 + sum(g * 2**s for g, s in FORMS[k])
    p = r**k + 1
    assert p.bit_length() == log2p
    assert miller_rabin(p) and sympy.isprime(p)
    v2 = ((p - 1) & -(p - 1)).bit_length() - 1
    assert v2 >= 21
    assert pow(r, k, p) == p - 1 and pow(r, 2 * k, p) == 1


def test_prime_rejects_other_k():
    r, lp = api.ctypes.c_int32(), api.ctypes.c_int32()
    assert nat.zpm_gfp_prime(64, api.ctypes.byref(r), api.ctypes.byref(lp)) == nat.ZPM_EINVAL


@pytest.mark.parametrize("k", [8, 16, 32])
@pytest.mark.parametrize("logL", [0, 1, 2, 4, 5, 6, 7, 9, 12, 17, 21])
def test_root(k, logL):
    r, _ = api.gfp_prime(k)
    p = r**k + 1
    d = api.gfp_root(k, logL)
    assert all(abs(x) <= r // 2 for x in d), "digits are not balanced"
    w = value(d, r, p)
    L = 1 << logL
    assert pow(w, L, p) == 1
    if L > 1:
        assert pow(w, L // 2, p) == p - 1, "omega is not of order exactly L"
    if L >= 2 * k:
        assert pow(w, L // (2 * k), p) == r
    else:
        assert w == pow(r, 2 * k // L, p)


@pytest.mark.parametrize("shape", [(1, 2, 1, 2), (5, 64, 3, 100), (1000, 200, 700, 180),
                                   (65536, 4097, 65536, 4097), (3000, 1000, 2500, 700),
                                   (40, 400, 41, 3000), (2**20, 40, 2**20, 40)])
@pytest.mark.parametrize("k", [0, 8, 16, 32])
def test_plan(shape, k):
    da, Na, db, Nb = shape
    pl = nat.GfpInfo()
    rc = nat.zpm_plan_gfp(da, Na, db, Nb, 0, k, api.ctypes.byref(pl))
    if rc == nat.ZPM_EUNSUPPORTED:
        # no K <= k of this prime satisfies the bound: confirm with exact integers
        for kk in ([k] if k else [8, 16, 32]):
            r, _ = api.gfp_prime(kk)
            p = r**kk + 1
            K = 2
            while K <= kk:
                M = max(2, -(-max(Na, Nb) // K))
                assert not (p > 4 * max(da, db) * K * 2 ** (2 * M)) or (M + 15) // 16 > 32
                K *= 2
        return
    assert rc == nat.ZPM_OK
    d = pl.as_dict()
    r, log2p = api.gfp_prime(d["k"])
    p = r ** d["k"] + 1
    K, M = d["K"], d["M"]
    assert 2 <= K <= d["k"] and K & (K - 1) == 0
    assert K * M >= max(Na, Nb) and M >= 2
    assert p > 4 * max(da, db) * K * 2 ** (2 * M)
    L = 1 << d["log2_L"]
    assert L >= da + db - 1 and (L == 1 or L // 2 < da + db - 1)
    assert sum(d["pass_log2n"]) == d["log2_L"]
    assert all(1 <= x <= 5 and (1 << x) <= 2 * d["k"] for x in d["pass_log2n"])
    assert d["workspace_bytes"] == 2 * K * L * d["k"] * 4
    if k:
        assert d["k"] == k
