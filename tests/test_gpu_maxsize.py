"""The longest product the prime tables allow: da + db - 1 = 2^21, the order of every
prime's root of unity, so the y-transform has its maximum length.  Both the 31-bit and
the 64-bit prime paths run it; the output is checked by oracle rows at sampled indices
(first, last, middle, the operand boundary and random ones) and, over every coefficient,
by the evaluation identities at y = 1, y = -1 and at a random point modulo two 61-bit
primes, plus the coefficient bound.
"""
import numpy as np
import pytest
import torch

from paper_1612_05778_amd import api, synth
from tests.gpu_util import dev, host
from tests.test_gpu_fullsize import full_checks

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def prod():
    r = np.random.default_rng(21)
    da, db = 1 << 20, (1 << 20) + 1
    a, Na = synth.signed_words(r, da, 63)
    b, Nb = synth.signed_words(r, db, 40)
    return synth.Product(a, Na, b, Nb)


@pytest.mark.parametrize("path", ["p31", "p64"])
def test_max_transform_length(ctx, prod, path):
    if path == "p31":
        pl = api.plan(prod.da, prod.Na, prod.db, prod.Nb)
    else:
        pl = api.plan_p64(prod.da, prod.Na, prod.db, prod.Nb)
    assert pl["log2_L"] == 21
    print(f"[maxsize] {path} da={prod.da} db={prod.db} K={pl['K']} np={pl['np']}", flush=True)
    A, B = dev(prod.a), dev(prod.b)
    out = ctx.mul(A, prod.Na, B, prod.Nb) if path == "p31" else ctx.mul_p64(A, prod.Na, B, prod.Nb)
    torch.cuda.synchronize()
    got = host(out)
    del out, A, B
    torch.cuda.empty_cache()
    assert got.shape[0] == 1 << 21
    full_checks(prod, got, 24, 5)
