"""Random shapes against the oracle: uneven degrees and widths, default and forced plans.

Seeded draws of (da, Na, db, Nb) spread log-uniformly over small and mid sizes, each
multiplied with the planner's choice and with a random feasible forced K (which moves
the product between the register and LDS x-kernels and changes the y split and the
column tiles), plus the batch of all of them.  Every coefficient is compared with the
oracle.  Sizes are capped so the oracle takes well under a second per case.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1612_05778_amd import _native as nat
from paper_1612_05778_amd import api, synth
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


def draws(seed, n):
    r = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        da, db = (int(math.exp(r.uniform(0, math.log(6000)))) for _ in range(2))
        Na, Nb = (int(math.exp(r.uniform(math.log(2), math.log(3000)))) for _ in range(2))
        if da * db * ((Na + 63) // 64) * ((Nb + 63) // 64) > 3e7:
            continue
        out.append((da, max(Na, 2), db, max(Nb, 2)))
    return r, out


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def test_random_shapes(ctx):
    r, shapes = draws(2024, 40)
    items, prods = [], []
    for k, (da, Na, db, Nb) in enumerate(shapes):
        a, _ = synth.signed_words(r, da, Na - 1)
        b, _ = synth.signed_words(r, db, Nb - 1)
        p = synth.Product(a, Na, b, Nb)
        A, B = dev(a), dev(b)
        want = None
        Ks = [0] + [int(r.choice([2, 4, 8, 16, 32, 64, 128]))]
        for K in Ks:
            try:
                api.plan(da, Na, db, Nb, K=K)
            except nat.ZpmError:
                continue
            print(f"[shape {k}] da={da} Na={Na} db={db} Nb={Nb} K={K}", flush=True)
            got = host(ctx.mul(A, Na, B, Nb, K=K))
            if want is None:
                want = oracle.polymul(a, da, Na, b, db, Nb, wc=got.shape[1])
            bad = np.nonzero((got != want).any(axis=1))[0]
            assert bad.size == 0, f"shape {k} K={K}: {bad.size} coefficients differ"
        items.append((A, Na, B, Nb))
        prods.append(want)
    print(f"[batch] {len(items)} products", flush=True)
    outs = ctx.mul_batch(items)
    torch.cuda.synchronize()
    for k, (o, want) in enumerate(zip(outs, prods)):
        assert np.array_equal(host(o), want), f"batched shape {k} differs"
