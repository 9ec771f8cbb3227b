"""Parity of the HIP path (through the C-ABI) with the oracle: bit-exact on every
output word.  Integer work, so the tolerance is zero.

Sizes: small cases that span several tiles with ragged tails, the 1024 x 64-bit
workload in full, degenerate inputs (single coefficients, one-bit and extreme
coefficients, zero polynomials, unequal degrees and sizes), and several forced
plans (K, np) for the same input, which must give identical bytes.
"""
import random
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import pyint
from paper_1612_05778_amd import synth
from tests.gpu_util import dev, host, words_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1612_05778_amd.api import Context
    c = Context(0)
    yield c
    c.close()


def run(ctx, A, da, Na, B, db, Nb, **kw):
    print(f"[case] da={da} Na={Na} db={db} Nb={Nb} {kw}", flush=True)
    out = ctx.mul(dev(A), Na, dev(B), Nb, **kw)
    torch.cuda.synchronize()
    return host(out)


def check(ctx, A, da, Na, B, db, Nb, **kw):
    got = run(ctx, A, da, Na, B, db, Nb, **kw)
    ref = oracle.polymul(A, da, Na, B, db, Nb, wc=got.shape[1])
    assert got.shape == ref.shape
    bad = np.nonzero((got != ref).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} coefficients differ, first at {bad[:8].tolist()}"
    return got


def test_int64_1k_full(ctx):
    p = synth.int64_1k()
    check(ctx, p.a, p.da, p.Na, p.b, p.db, p.Nb)


@pytest.mark.parametrize("seed", range(6))
def test_random_small(ctx, seed):
    rng = random.Random(100 + seed)
    for _ in range(8):
        da, db = rng.randint(1, 300), rng.randint(1, 300)
        Na = rng.choice([1, 2, 3, 31, 32, 33, 63, 64, 65, 100, 129, 257, 700])
        Nb = rng.choice([1, 2, 3, 31, 32, 33, 63, 64, 65, 100, 129, 257, 700])
        r = synth.rng_for(seed * 1000 + da)
        A, _ = synth.signed_words(r, da, Na - 1) if Na > 1 else (r.integers(0, 2, (da, 1), dtype=np.uint64), 1)
        B, _ = synth.signed_words(r, db, Nb - 1) if Nb > 1 else (r.integers(0, 2, (db, 1), dtype=np.uint64), 1)
        check(ctx, A, da, Na, B, db, Nb)


def test_ignores_bits_above_N(ctx):
    rng = np.random.default_rng(3)
    for N in (5, 64, 70, 130):
        w = (N + 63) // 64
        A = rng.integers(0, 2**64, size=(37, w), dtype=np.uint64)
        B = rng.integers(0, 2**64, size=(29, w), dtype=np.uint64)
        check(ctx, A, 37, N, B, 29, N)


@pytest.mark.parametrize("da,db,N", [(1, 1, 1), (1, 1, 64), (2, 1, 3), (1, 700, 65), (5, 3, 2),
                                     (17, 40, 64), (33, 33, 65), (64, 64, 4097), (300, 257, 129)])
def test_extreme_constants(ctx, da, db, N):
    lo, hi = -(1 << (N - 1)), (1 << (N - 1)) - 1
    for a_val, b_val in ((lo, lo), (hi, -1), (hi, hi), (lo, hi), (-1, -1)):
        A = words_for([a_val] * da, N)
        B = words_for([b_val] * db, N)
        check(ctx, A, da, N, B, db, N)


def test_alternating_and_zero(ctx):
    N = 200
    vals = [(-1) ** i * ((1 << (N - 1)) - 1 - i) for i in range(150)]
    A = words_for(vals, N)
    B = words_for(list(reversed(vals)), N)
    check(ctx, A, 150, N, B, 150, N)
    Z = words_for([0] * 77, 64)
    got = check(ctx, A, 150, N, Z, 77, 64)
    assert not got.any()


def test_binomial(ctx):
    import math
    n = 500
    row = [math.comb(n, i) for i in range(n + 1)]
    N = max(x.bit_length() for x in row) + 1
    A = words_for(row, N)
    got = run(ctx, A, n + 1, N, A, n + 1, N)
    assert pyint.decode(got, 64 * got.shape[1]) == [math.comb(2 * n, i) for i in range(2 * n + 1)]


# The recovery normalises carries either one lane per coefficient (outputs of at most
# 8 * TI 32-bit words, TI coefficients per workgroup) or one wave per coefficient with a
# scan.  With K = 16 the tile is 8 coefficients, so 50 x 1021-bit operands (outputs of
# 64 words) take the first branch and 50 x 1022-bit ones (66 words) the second; the rest
# reach each branch with long serial chains (K = 2, tiles of 64) or tiles of 4.
@pytest.mark.parametrize("d,N,K", [(50, 1021, 16), (50, 1022, 16), (100, 1000, 2),
                                   (200, 64, 0), (40, 6000, 0), (30, 24000, 0)])
def test_carry_branches(ctx, d, N, K):
    r = synth.rng_for(7 * d + N)
    A, _ = synth.signed_words(r, d, N - 1)
    B, _ = synth.signed_words(r, d + 3, N - 1)
    check(ctx, A, d, N, B, d + 3, N, K=K)


def test_plans_agree(ctx):
    p = synth.dense(21, 777, 900)
    ref = None
    for K, np_ in [(0, 0), (2, 0), (4, 0), (8, 0), (16, 0), (32, 0), (64, 0), (128, 0), (16, 30)]:
        got = check(ctx, p.a, p.da, p.Na, p.b, p.db, p.Nb, K=K, np=np_)
        if ref is None:
            ref = got
        assert np.array_equal(got, ref)


def test_wider_output_is_sign_extended(ctx):
    p = synth.dense(22, 100, 300)
    wc = (oracle.out_bits(100, p.Na, 100, p.Nb) + 63) // 64 + 3
    check(ctx, p.a, 100, p.Na, p.b, 100, p.Nb, wc=wc)


def test_empty_and_invalid(ctx):
    from paper_1612_05778_amd import _native as nat
    A = dev(words_for([1, 2, 3], 8))
    E = torch.empty((0, 1), dtype=torch.int64, device="cuda")
    out = ctx.mul(E, 8, A, 8)
    assert out.shape[0] == 0
    with pytest.raises(nat.ZpmError):
        ctx.mul(A, 8, A, 8, wc=0)
    # output overlapping an input is rejected before any launch
    big = torch.zeros((8, 1), dtype=torch.int64, device="cuda")
    rc = nat.zpm_mul(ctx.handle, big.data_ptr(), 3, 8, A.data_ptr(), 3, 8, big.data_ptr(), 1, None)
    assert rc == nat.ZPM_EINVAL


def test_repeat_is_deterministic(ctx):
    p = synth.dense(23, 2000, 1000)
    a, b = dev(p.a), dev(p.b)
    o1 = host(ctx.mul(a, p.Na, b, p.Nb))
    o2 = host(ctx.mul(a, p.Na, b, p.Nb))
    assert np.array_equal(o1, o2)
    rows = [0, 1, 999, 1999, 2000, 3998]
    ref = oracle.polymul_rows(p.a, p.da, p.Na, p.b, p.db, p.Nb, rows, wc=o1.shape[1])
    assert np.array_equal(o1[rows], ref)


def test_current_stream_is_used(ctx):
    """Without an explicit stream the binding enqueues on torch's current stream: under a
    side stream the product follows that stream's earlier work (a copy into the operand)
    and precedes its later work (a copy of the result)."""
    from paper_1612_05778_amd import api
    p = synth.int64_1k()
    a, b = dev(p.a), dev(p.b)
    za = torch.zeros_like(a)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    print("[case] int64_1k on a side stream", flush=True)
    with torch.cuda.stream(s):
        assert api._stream_handle(None) == s.cuda_stream
        za.copy_(a)
        out = ctx.mul(za, p.Na, b, p.Nb)
        res = out.clone()
    s.synchronize()
    assert api._stream_handle(None) == torch.cuda.current_stream().cuda_stream
    ref = oracle.polymul(p.a, p.da, p.Na, p.b, p.db, p.Nb, wc=res.shape[1])
    assert np.array_equal(host(res), ref)
