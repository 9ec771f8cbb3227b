"""Squares: one operand passed twice is converted and transformed once.

Every case passes the same device tensor as a and b and compares with the oracle
bit for bit, and with the product of two distinct copies (the unsquared path).
Plans cover the register x-kernel (K <= 32) and the LDS x-kernel (K = 64, 128),
with and without column passes, and ragged sizes; squares also run inside batches
next to ordinary products and through the server.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1612_05778_amd import api, synth
from tests.gpu_util import dev, host, words_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def square_check(ctx, A, d, N, **kw):
    print(f"[square] d={d} N={N} {kw}", flush=True)
    ta = dev(A)
    got = ctx.mul(ta, N, ta, N, **kw)
    two = ctx.mul(ta, N, dev(A), N, **kw)            # distinct copies: unsquared path
    torch.cuda.synchronize()
    assert torch.equal(got, two), "square differs from the product of two copies"
    ref = oracle.polymul(A, d, N, A, d, N, wc=got.shape[1])
    bad = np.nonzero((host(got) != ref).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} coefficients differ, first at {bad[:8].tolist()}"


@pytest.mark.parametrize("d,bits,K", [
    (1, 63, 0), (7, 200, 0), (300, 513, 0), (1000, 64, 0), (2500, 1500, 0),
    (5000, 300, 0),                       # column passes
    (700, 900, 64), (3000, 2000, 128),    # x-transforms in LDS
    (900, 700, 32), (6000, 1000, 32),     # x-transforms one half at a time
    (4097, 257, 8), (3, 5000, 0),
])
def test_square_random(ctx, d, bits, K):
    p = synth.dense(100 + d, d, bits)
    square_check(ctx, p.a, d, p.Na, K=K)


def test_square_extremes_and_binomial(ctx):
    N = 300
    lo = -(1 << (N - 1))
    A = words_for([lo] * 257, N)
    square_check(ctx, A, 257, N)
    n = 200
    from math import comb
    A = words_for([comb(n, i) for i in range(n + 1)], 200)
    ta = dev(A)
    got = host(ctx.mul(ta, 200, ta, 200))
    from oracle import pyint
    vals = pyint.decode(got, 64 * got.shape[1])
    assert vals == [comb(2 * n, i) for i in range(2 * n + 1)]


def test_squares_in_batch_and_server(ctx):
    prods = synth.batch(4, 12, deg=(63, 2047), bits=(32, 600))
    ops = [(dev(p.a), p.Na, dev(p.b), p.Nb) for p in prods]
    items = []
    for k, (a, Na, b, Nb) in enumerate(ops):
        items.append((a, Na, a, Na) if k % 2 == 0 else (a, Na, b, Nb))
    got = ctx.mul_batch(items)
    torch.cuda.synchronize()
    for k, (it, g) in enumerate(zip(items, got)):
        p = prods[k]
        B, Nb = (p.a, p.Na) if k % 2 == 0 else (p.b, p.Nb)
        ref = oracle.polymul(p.a, p.da, p.Na, B, B.shape[0], Nb, wc=g.shape[1])
        assert np.array_equal(host(g), ref), f"batched product {k} differs"
    srv = api.Server(ctx, hbm_budget=1 << 30, n_streams=2)
    sub = [srv.submit(*it) for it in items]
    for t, _ in sub:
        assert srv.wait(t, 60)[0] == 0
    srv.close()
    for k, ((_, o), g) in enumerate(zip(sub, got)):
        assert torch.equal(o, g), f"served product {k} differs from the batched one"
