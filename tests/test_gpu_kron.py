"""Kronecker reshaping: wide coefficients cut into chunks, y -> z^S, joined with carries.

Moderate sizes are computed both ways (reshaped with several chunk widths, and
directly) and against the oracle; coefficients too wide for a direct plan go through
zpm_mul's fallback and are checked against the oracle (all coefficients where that
takes seconds, sampled coefficients plus evaluation identities otherwise).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import pyint
from paper_1612_05778_amd import api, synth
from tests.gpu_util import dev, host, words_for

pytestmark = pytest.mark.gpu

Q = [2305843009213693951, 2305843009213693921]


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def oracle_check(p, got, rows=None):
    if rows is None:
        ref = oracle.polymul(p.a, p.da, p.Na, p.b, p.db, p.Nb, wc=got.shape[1])
        bad = np.nonzero((got != ref).any(axis=1))[0]
    else:
        ref = oracle.polymul_rows(p.a, p.da, p.Na, p.b, p.db, p.Nb, rows, wc=got.shape[1])
        bad = np.nonzero((got[rows] != ref).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} coefficients differ, first at {bad[:8].tolist()}"


@pytest.mark.parametrize("da,ba,db,bb", [(50, 3000, 50, 3000), (37, 1500, 80, 2600),
                                          (1, 5000, 9, 700), (300, 257, 200, 640)])
def test_reshaped_equals_direct_and_oracle(ctx, da, ba, db, bb):
    r = np.random.default_rng(da * 1000 + db)
    a, Na = synth.signed_words(r, da, ba)
    b, Nb = synth.signed_words(r, db, bb)
    p = synth.Product(a, Na, b, Nb)
    A, B = dev(a), dev(b)
    direct = ctx.mul(A, Na, B, Nb)
    for w in (256, 512, 2048, 0):
        print(f"[kron] da={da} Na={Na} db={db} Nb={Nb} chunk {w}", flush=True)
        got = ctx.mul_kronecker(A, Na, B, Nb, chunk_bits=w)
        torch.cuda.synchronize()
        assert torch.equal(got, direct), f"chunk {w}: differs from the direct product"
    oracle_check(p, host(direct))


def test_reshaped_extremes_and_square(ctx):
    N = 2000
    lo, hi = -(1 << (N - 1)), (1 << (N - 1)) - 1
    A = words_for([lo] * 33, N)
    B = words_for([hi, -1, lo, 0, 1] * 4, N)
    p = synth.Product(A, N, B, N)
    got = host(ctx.mul_kronecker(dev(A), N, dev(B), N, chunk_bits=256))
    oracle_check(p, got)
    TA = dev(A)
    sq = host(ctx.mul_kronecker(TA, N, TA, N, chunk_bits=512))
    oracle_check(synth.Product(A, N, A, N), sq)


def test_wide_coefficients_through_mul(ctx):
    r = np.random.default_rng(5)
    a, Na = synth.signed_words(r, 8, 300000)
    b, Nb = synth.signed_words(r, 6, 200000)
    print(f"[kron] wide: 8 x {Na} bits times 6 x {Nb} bits", flush=True)
    got = host(ctx.mul(dev(a), Na, dev(b), Nb))
    oracle_check(synth.Product(a, Na, b, Nb), got)


def test_wide_262k_sampled(ctx):
    r = np.random.default_rng(6)
    a, Na = synth.signed_words(r, 32, 262144)
    b, Nb = synth.signed_words(r, 32, 262144)
    print(f"[kron] 32 x {Na} bits squared-size product", flush=True)
    got = host(ctx.mul(dev(a), Na, dev(b), Nb))
    p = synth.Product(a, Na, b, Nb)
    oracle_check(p, got, rows=[0, 1, 31, 32, 62])
    av = [int.from_bytes(x.tobytes(), "little", signed=True) for x in a]
    bv = [int.from_bytes(x.tobytes(), "little", signed=True) for x in b]
    cv = [int.from_bytes(x.tobytes(), "little", signed=True) for x in got]
    rr = 123456789123
    for q in Q:
        ea = sum(x * pow(rr, i, q) for i, x in enumerate(av)) % q
        eb = sum(x * pow(rr, i, q) for i, x in enumerate(bv)) % q
        ec = sum(x * pow(rr, i, q) for i, x in enumerate(cv)) % q
        assert ea * eb % q == ec
