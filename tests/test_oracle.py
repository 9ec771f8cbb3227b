"""Pins of the oracle (CPU only).

The oracle is the plain definition c_i = sum_{l+m=i} a_l b_m (Section 1 and
Section 2).  Each test below checks it against something that is not a retyping
of that formula:

* exhaustive and random brute force against a Kronecker-substitution product
  done with Python's own big-integer multiply (a different algorithm);
* closed forms: (y+1)^n squared has the binomial coefficients C(2n, i)
  (Vandermonde), constant extreme polynomials have c_i = t_i * a * b with t_i
  the number of index pairs;
* evaluation identities at any size: A(r) B(r) = C(r) mod random primes q, and
  exactly at y = 1 and y = -1;
* algebraic invariants (commutativity, negation, monomial shift) and the
  coefficient bound |c_i| <= min(da, db) 2^(Na+Nb-2) of Relation (citighterbound);
* planted mistakes in a copy of the oracle's output (dropped term, wrong sign,
  index shift, flipped bit) to show each pin would catch that kind of error.
"""
import itertools
import math
import random

import numpy as np
import pytest

import oracle
from oracle import pyint
from paper_1612_05778_amd import synth


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _mul_ints(a, Na, b, Nb):
    A = pyint.encode(a, (Na + 63) // 64)
    B = pyint.encode(b, (Nb + 63) // 64)
    C = oracle.polymul(A, len(a), Na, B, len(b), Nb)
    return pyint.decode(C, 64 * C.shape[1]) if len(C) else []


def _rand_poly(rng, d, N):
    return [rng.randint(-(1 << (N - 1)), (1 << (N - 1)) - 1) for _ in range(d)]


def test_exhaustive_tiny_against_kronecker():
    # every pair of polynomials with <= 2 coefficients of N = 3 bits, and d = 1..3 at N = 2
    for N, d in ((3, 1), (3, 2), (2, 3)):
        vals = range(-(1 << (N - 1)), 1 << (N - 1))
        for a in itertools.product(vals, repeat=d):
            for b in itertools.product(vals, repeat=d if N == 3 else 1):
                assert _mul_ints(list(a), N, list(b), N) == pyint.kronecker(list(a), list(b))


@pytest.mark.parametrize("seed", range(4))
def test_random_small_against_kronecker(seed):
    rng = random.Random(seed)
    edge_N = [1, 2, 3, 31, 32, 33, 63, 64, 65, 127, 128, 129, 511]
    for _ in range(60):
        da, db = rng.randint(1, 64), rng.randint(1, 64)
        Na = rng.choice(edge_N + [rng.randint(1, 512)])
        Nb = rng.choice(edge_N + [rng.randint(1, 512)])
        a, b = _rand_poly(rng, da, Na), _rand_poly(rng, db, Nb)
        assert _mul_ints(a, Na, b, Nb) == pyint.kronecker(a, b)


def test_ignores_bits_above_N():
    # bits >= N in the top word are not part of the value (sign-extension from bit N-1)
    rng = np.random.default_rng(7)
    for N in (1, 5, 64, 70, 130):
        w = (N + 63) // 64
        a = rng.integers(0, 2**64, size=(9, w), dtype=np.uint64)
        b = rng.integers(0, 2**64, size=(5, w), dtype=np.uint64)
        C = oracle.polymul(a, 9, N, b, 5, N)
        assert pyint.decode(C, 64 * C.shape[1]) == pyint.kronecker(pyint.decode(a, N), pyint.decode(b, N))


def test_binomial_closed_form():
    n = 300
    row = [math.comb(n, i) for i in range(n + 1)]
    N = max(x.bit_length() for x in row) + 1
    c = _mul_ints(row, N, row, N)
    assert c == [math.comb(2 * n, i) for i in range(2 * n + 1)]


@pytest.mark.parametrize("da,db,N", [(1, 1, 1), (5, 3, 2), (17, 40, 64), (33, 33, 65), (7, 2, 4097)])
def test_extreme_constant_polynomials(da, db, N):
    lo, hi = -(1 << (N - 1)), (1 << (N - 1)) - 1
    t = [min(i + 1, da + db - 1 - i, da, db) for i in range(da + db - 1)]
    # maximum magnitude and maximum carry: every product is +2^(2N-2)
    assert _mul_ints([lo] * da, N, [lo] * db, N) == [ti << (2 * N - 2) for ti in t]
    # mixed signs
    assert _mul_ints([hi] * da, N, [-1] * db, N) == [-ti * hi for ti in t]
    # the stated output width holds the extreme case exactly
    Nout = oracle.out_bits(da, N, db, N)
    assert max(t) << (2 * N - 2) <= (1 << (Nout - 1)) - 1


def _eval_checks(prod, C, Nout, nprimes=3, seed=0):
    """A(r)B(r) = C(r) mod q for random 61-bit primes; exact at r = +1, -1."""
    a = pyint.decode(prod.a, prod.Na)
    b = pyint.decode(prod.b, prod.Nb)
    c = pyint.decode(C, 64 * C.shape[1])
    rng = random.Random(seed)
    qs = [2305843009213693951, 2305843009213693921, 2305843009213693907][:nprimes]
    for q in qs:
        r = rng.randrange(2, q - 1)
        if pyint.eval_mod(a, r, q) * pyint.eval_mod(b, r, q) % q != pyint.eval_mod(c, r, q):
            return False
    if sum(a) * sum(b) != sum(c):
        return False
    alt = lambda v: sum(x if i % 2 == 0 else -x for i, x in enumerate(v))
    if alt(a) * alt(b) != alt(c):
        return False
    bound = min(prod.da, prod.db) << (prod.Na + prod.Nb - 2)
    return all(abs(x) <= bound for x in c) and all(-(1 << (Nout - 1)) <= x < (1 << (Nout - 1)) for x in c)


def test_eval_identity_mid_size():
    prod = synth.dense(11, 1024, 1024)
    C = oracle.polymul(prod.a, prod.da, prod.Na, prod.b, prod.db, prod.Nb)
    assert _eval_checks(prod, C, oracle.out_bits(prod.da, prod.Na, prod.db, prod.Nb))


def test_int64_1k_against_kronecker():
    prod = synth.int64_1k()
    C = oracle.polymul(prod.a, prod.da, prod.Na, prod.b, prod.db, prod.Nb)
    assert C.shape == (2047, 3)      # 138-bit output coefficients -> 3 words
    assert pyint.decode(C, 192) == pyint.kronecker(pyint.decode(prod.a, 64), pyint.decode(prod.b, 64))


def test_rows_subset_matches_full():
    prod = synth.dense(12, 300, 200)
    full = oracle.polymul(prod.a, prod.da, prod.Na, prod.b, prod.db, prod.Nb)
    rows = [0, 1, 150, 298, 299, 300, 598]
    part = oracle.polymul_rows(prod.a, prod.da, prod.Na, prod.b, prod.db, prod.Nb, rows)
    assert np.array_equal(part, full[rows])


def test_invariants():
    rng = random.Random(5)
    a, b = _rand_poly(rng, 37, 90), _rand_poly(rng, 21, 70)
    ab = _mul_ints(a, 90, b, 70)
    assert _mul_ints(b, 70, a, 90) == ab                                  # commutativity
    assert _mul_ints([-x for x in a], 91, b, 70) == [-x for x in ab]     # negation
    assert _mul_ints([0] * 5 + a, 90, b, 70) == [0] * 5 + ab              # y^5 * a
    assert _mul_ints([0] * 4, 3, b, 70) == [0] * (4 + 21 - 1)             # zero


def test_planted_mistakes_are_caught():
    """Corrupt copies of a correct oracle output; the pins above must reject each."""
    prod = synth.dense(13, 200, 300)
    C = oracle.polymul(prod.a, prod.da, prod.Na, prod.b, prod.db, prod.Nb)
    Nout = oracle.out_bits(prod.da, prod.Na, prod.db, prod.Nb)
    assert _eval_checks(prod, C, Nout)
    a = pyint.decode(prod.a, prod.Na)
    b = pyint.decode(prod.b, prod.Nb)
    c = pyint.decode(C, 64 * C.shape[1])
    w = C.shape[1]
    bad = []
    x = list(c); x[57] -= a[20] * b[37]; bad.append(x)                     # dropped term
    x = list(c); x[57] = -x[57]; bad.append(x)                             # wrong sign
    bad.append(c[1:] + [0])                                                # index shift
    x = list(c); x[123] ^= 1 << 200; bad.append(x)                         # one bit
    x = list(c); x[0] += 2 * a[0] * b[0]; bad.append(x)                   # sign of a term
    for x in bad:
        assert not _eval_checks(prod, pyint.encode(x, w), Nout)


def test_synth_encoding():
    r = synth.rng_for(99)
    words, N = synth.signed_words(r, 500, 130)
    assert words.shape == (500, 3) and N == 131
    vals = pyint.decode(words, N)
    assert all(abs(v) < (1 << 130) for v in vals)
    assert any(v < 0 for v in vals) and any(v > 0 for v in vals)
    # words above bit N-1 are pure sign extension
    top = words[:, 2] >> np.uint64(2)
    neg = np.array([v < 0 for v in vals])
    assert np.all(top[neg] == np.uint64((1 << 62) - 1)) and np.all(top[~neg] == 0)
    # the same seed gives the same stream
    w2, _ = synth.signed_words(synth.rng_for(99), 500, 130)
    assert np.array_equal(words, w2)
    # negative zero is encoded as zero
    z = synth._negate_rows(np.zeros((2, 3), dtype=np.uint64))
    assert not z.any()


def test_synth_config_shapes():
    p = synth.int64_1k()
    assert p.a.shape == (1024, 1) and p.Na == 64
    degs, bits = synth.served_sizes(5, 1000)
    assert degs.min() >= 15 and degs.max() <= 65535 and bits.min() >= 16 and bits.max() <= 8192
    _, degs, bits = synth.batch_sizes(4, 4096)
    assert degs.min() >= 63 and degs.max() <= 8191 and bits.min() >= 32 and bits.max() <= 2048


def test_stored_digest_matches_oracle():
    """tests/golden/digests.json holds digests written by tests/golden/make_digests.py
    from the generators and the oracle; the small one is recomputed here."""
    import hashlib
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "digests.json")
    ref = json.load(open(path))["int64_1k"]
    p = synth.int64_1k(1)
    c = oracle.polymul(p.a, p.da, p.Na, p.b, p.db, p.Nb, wc=ref["wc"])
    assert hashlib.sha256(c.tobytes()).hexdigest() == ref["sha256"]


# ---- the residue oracle (every c_i mod q, for products too large for the exact one) ----
QS = [2305843009213693951, 2305843009213693921]   # primes below 2^61


@pytest.mark.parametrize("seed", range(3))
def test_polymul_mod_against_exact(seed):
    """Residues equal the exact product reduced mod q (the exact oracle is pinned above),
    over ragged sizes, edge widths, negative values and bits above N."""
    rng = np.random.default_rng(100 + seed)
    for _ in range(12):
        da, db = int(rng.integers(1, 90)), int(rng.integers(1, 90))
        Na = int(rng.choice([1, 2, 63, 64, 65, 130, 1000, int(rng.integers(1, 700))]))
        Nb = int(rng.choice([1, 3, 64, 129, 257, int(rng.integers(1, 700))]))
        a = rng.integers(0, 2**64, size=(da, (Na + 63) // 64), dtype=np.uint64)
        b = rng.integers(0, 2**64, size=(db, (Nb + 63) // 64), dtype=np.uint64)
        C = oracle.polymul(a, da, Na, b, db, Nb)
        c = pyint.decode(C, 64 * C.shape[1])
        for q in QS + [3, 1000003]:
            got = oracle.polymul_mod(a, da, Na, b, db, Nb, q)
            assert got.tolist() == [x % q for x in c]


def test_polymul_mod_closed_forms():
    # (y+1)^n squared: binomials C(2n, i) mod q, with n past the 32-term reduction period
    n = 700
    row = [math.comb(n, i) for i in range(n + 1)]
    N = max(x.bit_length() for x in row) + 1
    A = pyint.encode(row, (N + 63) // 64)
    for q in QS:
        got = oracle.polymul_mod(A, n + 1, N, A, n + 1, N, q)
        assert got.tolist() == [math.comb(2 * n, i) % q for i in range(2 * n + 1)]
    # extreme constants: all -2^(N-1) gives c_i = t_i 2^(2N-2); 2^(N-1)-1 against -1
    da, db, N = 300, 170, 4097
    t = [min(i + 1, da + db - 1 - i, da, db) for i in range(da + db - 1)]
    lo = pyint.encode([-(1 << (N - 1))] * da, 65)
    lo_b = pyint.encode([-(1 << (N - 1))] * db, 65)
    hi = pyint.encode([(1 << (N - 1)) - 1] * da, 65)
    m1 = pyint.encode([-1] * db, 65)
    for q in QS:
        assert oracle.polymul_mod(lo, da, N, lo_b, db, N, q).tolist() == \
            [(ti << (2 * N - 2)) % q for ti in t]
        assert oracle.polymul_mod(hi, da, N, m1, db, N, q).tolist() == \
            [(-ti * ((1 << (N - 1)) - 1)) % q for ti in t]


def test_polymul_mod_evaluation_and_planted():
    """sum_i c_i r^i = a(r) b(r) mod q on a mid-size product; a changed residue, a
    shifted index or a dropped term fails it."""
    prod = synth.dense(21, 3000, 2000)
    a = pyint.decode(prod.a, prod.Na)
    b = pyint.decode(prod.b, prod.Nb)
    rng = random.Random(3)
    for q in QS:
        c = oracle.polymul_mod(prod.a, prod.da, prod.Na, prod.b, prod.db, prod.Nb, q).tolist()
        r = rng.randrange(2, q - 1)
        lhs = pyint.eval_mod(a, r, q) * pyint.eval_mod(b, r, q) % q
        assert pyint.eval_mod(c, r, q) == lhs
        bad = [list(c) for _ in range(3)]
        bad[0][1234] = (bad[0][1234] + 1) % q
        bad[1] = c[1:] + [0]
        bad[2][2999] = (bad[2][2999] - a[2999] * b[0]) % q
        for x in bad:
            assert pyint.eval_mod(x, r, q) != lhs
