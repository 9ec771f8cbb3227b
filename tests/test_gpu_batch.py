"""Batched products in one persistent launch (zpm_mul_batch), bit-exact against the
oracle and against the one-at-a-time path; forced plans agree; graph replays agree.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1612_05778_amd import synth
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1612_05778_amd.api import Context
    c = Context(0)
    yield c
    c.close()


def small_mix(seed=40, n=120):
    prods = synth.batch(seed, n, deg=(1, 400), bits=(1, 700))
    prods += synth.batch_uneven(seed + 1, n // 2, deg=(1, 300), bits=(1, 500))
    # degenerate members: single coefficients, one-bit coefficients, extreme values
    r = synth.rng_for(seed + 2)
    a, Na = synth.signed_words(r, 1, 64)
    b, Nb = synth.signed_words(r, 1, 3)
    prods.append(synth.Product(a, Na, b, Nb))
    prods.append(synth.Product(np.ones((5, 1), dtype=np.uint64), 1, np.ones((3, 1), dtype=np.uint64), 1))
    lo = np.full((17, 2), np.uint64(0), dtype=np.uint64)
    lo[:, 1] = np.uint64(1 << 63)       # -2^127 with N = 128
    prods.append(synth.Product(lo, 128, lo.copy(), 128))
    return prods


def to_dev(prods):
    return [(dev(p.a), p.Na, dev(p.b), p.Nb) for p in prods]


def check_all(prods, outs):
    torch.cuda.synchronize()
    for i, (p, o) in enumerate(zip(prods, outs)):
        got = host(o)
        ref = oracle.polymul(p.a, p.da, p.Na, p.b, p.db, p.Nb, wc=got.shape[1])
        assert np.array_equal(got, ref), f"product {i} (da={p.da} Na={p.Na} db={p.db} Nb={p.Nb}) differs"


def test_batch_matches_oracle(ctx):
    prods = small_mix()
    print(f"[batch] {len(prods)} products", flush=True)
    outs = ctx.mul_batch(to_dev(prods))
    ctx.sync()
    check_all(prods, outs)


def test_batch_forced_plans_agree(ctx):
    prods = small_mix(50, 40)
    items = to_dev(prods)
    ref = [host(o) for o in ctx.mul_batch(items)]
    ctx.sync()
    for K in (4, 8, 16):     # K = 2 would need more than the 16 primes a batch plan may use
        print(f"[batch] K={K}", flush=True)
        outs = ctx.mul_batch(items, K=K)
        ctx.sync()
        for r, o in zip(ref, outs):
            assert np.array_equal(r, host(o))


def test_batch_equals_plain_path(ctx):
    prods = synth.batch(4, 48)          # the first products of the 4096-product workload
    items = to_dev(prods)
    outs = ctx.mul_batch(items)
    ctx.sync()
    for (a, Na, b, Nb), o in zip(items, outs):
        plain = ctx.mul(a, Na, b, Nb)
        torch.cuda.synchronize()
        assert np.array_equal(host(plain), host(o))
    check_all(prods[:6], outs[:6])


def test_batch_graph_replays(ctx):
    prods = small_mix(60, 30)
    items = to_dev(prods)
    eager = [host(o) for o in ctx.mul_batch(items)]
    ctx.sync()
    outs = [torch.empty((p.da + p.db - 1, e.shape[1]), dtype=torch.int64, device="cuda")
            for p, e in zip(prods, eager)]
    for rep in range(4):
        for o in outs:
            o.fill_(0x5A5A)
        ctx.mul_batch(items, graph=True, outs=outs)
        ctx.sync()
        for e, o in zip(eager, outs):
            assert np.array_equal(e, host(o)), f"replay {rep} differs"
        # eager work between replays
        x = ctx.mul(items[0][0], items[0][1], items[1][2], items[1][3])
        torch.cuda.synchronize()
        del x


def test_batch_graph_back_to_back(ctx):
    """Two graph batches with different job arrays, enqueued one right after the other on
    one stream with no host synchronisation in between (each call captures a new graph and
    rewrites the pinned descriptors the previous graph's copies read): both must equal
    their eager results, on every repetition."""
    p1, p2 = small_mix(70, 30), small_mix(80, 44)
    i1, i2 = to_dev(p1), to_dev(p2)
    e1 = [host(o) for o in ctx.mul_batch(i1)]
    e2 = [host(o) for o in ctx.mul_batch(i2)]
    ctx.sync()
    for rep in range(3):
        o1 = ctx.mul_batch(i1, graph=True)
        o2 = ctx.mul_batch(i2, graph=True)
        o3 = ctx.mul_batch(i1, graph=True)
        ctx.sync()
        for e, o in list(zip(e1, o1)) + list(zip(e2, o2)) + list(zip(e1, o3)):
            assert np.array_equal(e, host(o)), f"back-to-back graph batch differs (rep {rep})"


def test_persistent_single_launch(ctx):
    """ZPM_BATCH_PERSISTENT: every stage of every product in one persistent launch, tasks
    taken from a ticket counter in stage order (its schedule is modelled on the CPU in
    test_persistent_model.py).  Must equal the grouped launches and the oracle, on
    repeated calls and with a square and forced limb counts in the mix."""
    prods = small_mix()
    items = to_dev(prods)
    items.append((items[0][0], items[0][1], items[0][0], items[0][1]))   # a square
    prods.append(synth.Product(prods[0].a, prods[0].Na, prods[0].a, prods[0].Na))
    print(f"[batch] persistent launch of {len(items)} products", flush=True)
    ref = [host(o) for o in ctx.mul_batch(items)]
    ctx.sync()
    for rep in range(3):
        outs = ctx.mul_batch(items, persistent=True)
        ctx.sync()
        for i, (r, o) in enumerate(zip(ref, outs)):
            assert np.array_equal(r, host(o)), f"persistent product {i} differs (rep {rep})"
    check_all(prods, outs)
    outs = ctx.mul_batch(items, persistent=True, K=4)
    ctx.sync()
    check_all(prods, outs)


def test_persistent_flag_combination_is_rejected(ctx):
    from paper_1612_05778_amd import _native as nat
    jobs = (nat.Job * 1)()
    assert nat.zpm_mul_batch_ex(ctx.handle, jobs, 0, nat.ZPM_BATCH_PERSISTENT | nat.ZPM_BATCH_GRAPH,
                                0, None) == nat.ZPM_EINVAL


def test_batch_empty_and_invalid(ctx):
    from paper_1612_05778_amd import _native as nat
    outs = ctx.mul_batch([])
    assert outs == []
    a = dev(np.ones((3, 1), dtype=np.uint64))
    e = torch.empty((0, 1), dtype=torch.int64, device="cuda")
    outs = ctx.mul_batch([(a, 8, e, 8), (a, 8, a, 8)])
    ctx.sync()
    assert outs[0].shape[0] == 0
    assert host(outs[1])[:, 0].tolist() == [1, 2, 3, 2, 1]
    jobs = (nat.Job * 1)()
    jobs[0].a, jobs[0].da, jobs[0].Na = a.data_ptr(), 3, 8
    jobs[0].b, jobs[0].db, jobs[0].Nb = a.data_ptr(), 3, 8
    jobs[0].c, jobs[0].wc = None, 1
    assert nat.zpm_mul_batch(ctx.handle, jobs, 1, 0, None) == nat.ZPM_EINVAL
