"""Host side of the 64-bit machine-word prime variant (no GPU): prime table and planner.

The primes are checked with a Miller-Rabin test written here (the first twelve primes
as bases, deterministic below 3.3e24), not the library's; the planner's choices are
checked against the bound P > 4 max(da, db) K 2^(2M) of Section 2.2 computed with
Python integers, and for minimality of the prime count.
"""
import pytest

from paper_1612_05778_amd import _native as nat
from paper_1612_05778_amd import api

BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    if n < 2:
        return False
    for q in BASES:
        if n % q == 0:
            return n == q
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in BASES:
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


def test_miller_rabin_pins():
    # known values: 2^61 - 1 is a Mersenne prime; 2^62 - 57 is the largest prime below 2^62
    assert is_prime(2**61 - 1) and is_prime(2**62 - 57)
    assert not is_prime(2**62 - 1) and not is_prime(3215031751)   # strong pseudoprime to 2, 3, 5, 7
    assert [n for n in range(60) if is_prime(n)] == [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41,
                                                      43, 47, 53, 59]


def test_prime64_table():
    step = 1 << 21
    want, c = [], (2**62 - 1) // step
    while len(want) < 3:
        if is_prime(c * step + 1):
            want.append(c * step + 1)
        c -= 1
    got = [api.prime64(k) for k in range(3)]
    assert [p for p, _ in got] == want        # the three largest, largest first, none skipped
    for p, root in got:
        assert p < 2**62 and (p - 1) % step == 0
        assert pow(root, step, p) == 1 and pow(root, step // 2, p) == p - 1   # order exactly 2^21
    with pytest.raises(nat.ZpmError):
        api.prime64(3)


SHAPES = [(1, 2, 1, 2), (3, 70, 2, 65), (1000, 513, 1001, 700), (65536, 4097, 65536, 4097),
          (1 << 20, 64, 1 << 20, 64), (2, 1100, 3, 1000), (4097, 257, 3000, 300), (7, 9000, 5, 8000)]


def prime_product(np_):
    P = 1
    for k in range(np_):
        P *= api.prime64(k)[0]
    return P


@pytest.mark.parametrize("da,Na,db,Nb", SHAPES)
def test_plan_p64_bound_and_shape(da, Na, db, Nb):
    d, N = max(da, db), max(Na, Nb, 2)
    for K in (0, 2, 8, 64, 128, 512):
        for np_ in (0, 1, 2, 3):
            try:
                pl = api.plan_p64(da, Na, db, Nb, K=K, np=np_)
            except nat.ZpmError:
                continue
            if K:
                assert pl["K"] == K
            if np_:
                assert pl["np"] == np_
            K_, M, n = pl["K"], pl["M"], pl["np"]
            assert K_ & (K_ - 1) == 0 and 2 <= K_ <= 512 and 1 <= n <= 3
            assert K_ * M >= N and M == max(2, -(-N // K_))
            P = prime_product(n)
            assert P > 4 * d * K_ * 2 ** (2 * M)
            if not np_ and n > 1:          # the fewest primes that cover the bound
                assert prime_product(n - 1) <= 4 * d * K_ * 2 ** (2 * M)
            assert pl["log2P"] == P.bit_length()
            L = 1 << pl["log2_L"]
            assert L >= da + db - 1 and (L == 1 or L // 2 < da + db - 1)
            assert sum(pl["pass_log2n"]) == pl["log2_L"] and all(1 <= x <= 9 for x in pl["pass_log2n"])
            assert pl["workspace_bytes"] == n * 2 * K_ * L * 8
            assert (2 * K_ << pl["log2_tx"]) * 2 <= 8192 and pl["log2_tx"] <= pl["log2_L"]
            assert ((2 * K_ - 1) << pl["log2_ti"]) * (2 * n + 1) <= 16384


def test_plan_p64_limits():
    with pytest.raises(nat.ZpmError):
        api.plan_p64(1 << 20, 64, (1 << 20) + 2, 64)          # da + db - 1 > 2^21
    with pytest.raises(nat.ZpmError):
        api.plan_p64(1000, 60000, 1000, 60000)                 # M > 92 even at K = 512
    with pytest.raises(nat.ZpmError):
        api.plan_p64(10, 64, 10, 64, np=4)
    with pytest.raises(nat.ZpmError):
        api.plan_p64(10, 64, 10, 64, K=1024)
    with pytest.raises(nat.ZpmError):
        api.plan_p64(0, 64, 10, 64)
    # the paper's two-prime configuration for d = 2^16, N = 4097
    pl = api.plan_p64(1 << 16, 4097, 1 << 16, 4097, K=128, np=2)
    assert (pl["M"], pl["log2P"]) == (33, 124)
