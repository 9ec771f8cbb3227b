"""Parity at full size, in the launch configuration bench.py times (default plan).

The oracle cannot redo a whole 2^16 x 4096-bit product in test time, so:

* sampled output coefficients (first, last, middle and random indices) are
  recomputed by the oracle one by one and compared bit for bit;
* every coefficient is covered by the evaluation identities
  a(r) b(r) = c(r) mod q for 61-bit primes q and random r, and exactly at
  y = 1 and y = -1 (a wrong coefficient passes one modular check with
  probability about (da + db) / q);
* every coefficient satisfies |c_i| <= min(da, db) 2^(Na+Nb-2) and its words
  above Nout bits are pure sign extension;
* tests/golden/digests.json (written by tests/golden/make_digests.py from the
  generators and the oracle alone) holds, for bits4096_64k, the SHA-256 of the
  oracle's complete output: the whole device output must have that digest, every
  coefficient bit for bit.  For bits16384_256k it holds the SHA-256 of c_i mod q for
  every coefficient and two primes q below 2^61 (the oracle's modular schoolbook),
  which the device output reduced mod q must reproduce, and the digests of 256 exact
  oracle rows, which the device's rows must reproduce.  A missing entry fails.
"""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1612_05778_amd import synth
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu

Q = [2305843009213693951, 2305843009213693921]


def to_ints(words: np.ndarray) -> list[int]:
    return [int.from_bytes(row.tobytes(), "little", signed=True) for row in words]


def eval_mod(vals, r, q):
    acc = 0
    for x in reversed(vals):
        acc = (acc * r + x) % q
    return acc


DIGESTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "digests.json")


def digest_entry(name):
    if not os.path.exists(DIGESTS):
        pytest.fail(f"{DIGESTS} is missing")
    ref = json.load(open(DIGESTS)).get(name)
    if ref is None:
        pytest.fail(f"{DIGESTS} has no entry for {name}")
    return ref


def check_digest(name, got):
    ref = digest_entry(name)
    assert got.shape[1] == ref["wc"], "output width differs from the digested one"
    assert hashlib.sha256(got.tobytes()).hexdigest() == ref["sha256"], \
        f"{name}: device output differs from the oracle's full output"
    print(f"[fullsize] {name}: every coefficient matches the oracle digest", flush=True)
    return True


def check_residues_and_rows(name, prod, got, c):
    """Every coefficient mod two primes against the oracle's modular schoolbook, and the
    stored exact rows, both from the digest file."""
    ref = digest_entry(name)
    assert got.shape[1] == ref["wc"], "output width differs from the digested one"
    assert (ref["da"], ref["Na"], ref["db"], ref["Nb"]) == (prod.da, prod.Na, prod.db, prod.Nb)
    for q, want in ref["residue_sha256"].items():
        res = np.array([x % int(q) for x in c], dtype=np.uint64)
        assert hashlib.sha256(res.tobytes()).hexdigest() == want, \
            f"{name}: some coefficient differs from the oracle mod {q}"
    rows = ref["rows"]
    assert len(rows) >= 256
    bad = [r for r, h in zip(rows, ref["row_sha256"])
           if hashlib.sha256(got[r].tobytes()).hexdigest() != h]
    assert not bad, f"{name}: rows {bad[:8]} differ from the stored oracle rows"
    print(f"[fullsize] {name}: all {len(c)} coefficients match the oracle mod "
          f"{len(ref['residue_sha256'])} primes; {len(rows)} stored oracle rows exact", flush=True)


def full_checks(prod, got, nsample, seed, name=None):
    da, db = prod.da, prod.db
    nout = da + db - 1
    rng = np.random.default_rng(seed)
    rows = sorted(set([0, 1, da - 1, da, nout // 2, nout - 2, nout - 1] +
                      rng.choice(nout, size=nsample, replace=False).tolist()))
    print(f"[fullsize] oracle on {len(rows)} sampled rows", flush=True)
    ref = oracle.polymul_rows(prod.a, da, prod.Na, prod.b, db, prod.Nb, rows, wc=got.shape[1])
    assert np.array_equal(got[rows], ref), "sampled coefficients differ from the oracle"
    print("[fullsize] evaluation identities", flush=True)
    a = to_ints(prod.a)
    b = to_ints(prod.b)
    # inputs are sign-extended encodings, so from_bytes(signed) gives their values
    c = to_ints(got)
    if name is not None:
        check_residues_and_rows(name, prod, got, c)
    bound = min(da, db) << (prod.Na + prod.Nb - 2)
    nb = oracle.out_bits(da, prod.Na, db, prod.Nb)
    assert all(-bound <= x <= bound for x in c)
    assert all(-(1 << (nb - 1)) <= x < (1 << (nb - 1)) for x in c)
    assert sum(a) * sum(b) == sum(c)
    alt = lambda v: sum(v[0::2]) - sum(v[1::2])
    assert alt(a) * alt(b) == alt(c)
    r = int(rng.integers(2, 2**61))
    for q in Q:
        assert eval_mod(a, r, q) * eval_mod(b, r, q) % q == eval_mod(c, r, q)


@pytest.fixture(scope="module")
def ctx():
    from paper_1612_05778_amd.api import Context
    c = Context(0)
    yield c
    c.close()


def test_bits4096_64k(ctx):
    prod = synth.bits4096_64k()
    print("[fullsize] d=2^16 N=4097 on GPU", flush=True)
    out = ctx.mul(dev(prod.a), prod.Na, dev(prod.b), prod.Nb)
    torch.cuda.synchronize()
    got = host(out)
    del out
    assert check_digest("bits4096_64k", got)
    full_checks(prod, got, 40, 7)


def test_bits16384_256k(ctx):
    prod = synth.bits16384_256k()
    print("[fullsize] d=2^18 N=16385 on GPU", flush=True)
    out = ctx.mul(dev(prod.a), prod.Na, dev(prod.b), prod.Nb)
    torch.cuda.synchronize()
    got = host(out)
    del out
    torch.cuda.empty_cache()
    full_checks(prod, got, 8, 8, name="bits16384_256k")
