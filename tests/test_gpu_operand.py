"""Resident operand: b transformed once, then multiplied by several a.

Each product must equal, word for word, the ordinary product of the same a and b
and the oracle; sizes cover a's below the bounds (shorter and narrower than the
plan), the register and LDS x-kernels, plans with and without column passes, and
the bounds themselves; a beyond the bounds is refused.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1612_05778_amd import _native as nat
from paper_1612_05778_amd import api, synth
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("db,Nb,da_max,Na_max,K", [
    (300, 513, 400, 600, 0),
    (2000, 257, 3000, 300, 0),        # column passes
    (700, 900, 800, 1000, 64),        # x-transforms in LDS
    (900, 700, 1200, 800, 32),        # x-transforms one half at a time
    (4000, 600, 5000, 700, 32),
    (5000, 64, 5000, 64, 0),
    (1, 4000, 50, 4000, 0),
])
def test_operand_products(ctx, db, Nb, da_max, Na_max, K):
    pb = synth.dense(7 + db, db, Nb - 1)
    B = dev(pb.b)
    print(f"[operand] db={db} Nb={Nb} bounds ({da_max}, {Na_max}) K={K}", flush=True)
    op = api.Operand(ctx, B, Nb, da_max, Na_max, K=K)
    info = op.info()
    assert info["db"] == db and info["da"] == da_max
    rng = np.random.default_rng(db)
    sizes = [(da_max, Na_max), (max(1, da_max // 3), max(2, Na_max // 2)),
             (int(rng.integers(1, da_max + 1)), int(rng.integers(2, Na_max + 1)))]
    for da, Na in sizes:
        pa = synth.dense(int(rng.integers(1 << 20)), da, Na - 1)
        A = dev(pa.a)
        got = op.mul(A, Na)
        ref = ctx.mul(A, Na, B, Nb)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), f"a ({da}, {Na}): differs from the ordinary product"
        if da * db <= 2_000_000:
            want = oracle.polymul(pa.a, da, Na, pb.b, db, Nb, wc=got.shape[1])
            assert np.array_equal(host(got), want), f"a ({da}, {Na}): differs from the oracle"
    a_big = dev(synth.dense(3, da_max + 1, 10).a)
    with pytest.raises(nat.ZpmError):
        op.mul(a_big, 11)
    op.close()


def test_operand_reuse_after_other_work(ctx):
    pb = synth.dense(11, 1500, 400)
    B = dev(pb.b)
    op = api.Operand(ctx, B, pb.Nb, 1500, pb.Nb)
    pa = synth.dense(12, 1500, 400)
    A = dev(pa.a)
    first = op.mul(A, pa.Na)
    other = synth.dense(13, 4000, 700)
    ctx.mul(dev(other.a), other.Na, dev(other.b), other.Nb)   # reuses the context workspace
    again = op.mul(A, pa.Na)
    torch.cuda.synchronize()
    assert torch.equal(first, again)
    op.close()
