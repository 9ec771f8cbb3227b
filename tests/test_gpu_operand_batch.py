"""Resident operands in batches and in the server.

A batch of products against resident operands (zpm_mul_operand_batch) must give,
word for word, what zpm_mul_operand gives for each product alone, and a sample must
match the oracle.  The operands cover a plan with column passes, two with 18 primes
(more than the batch planner itself takes), and the register and LDS row kernels.
Graph replays must follow the current contents of a.  Plans beyond the batch kernels
(K = 32 in registers, more than 20 primes) are refused by the batch call and run alone
in the server.  A server fed a mix of ordinary and operand requests must give the same
words as the products computed alone.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1612_05778_amd import _native as nat
from paper_1612_05778_amd import api, synth
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu

# (db, Nb, da_max, Na_max, K)
OPERANDS = [
    (300, 257, 400, 300, 0),
    (2000, 257, 3000, 300, 0),      # column passes
    (100, 2000, 100, 2000, 0),      # K = 8, 18 primes
    (700, 900, 800, 1000, 64),      # x-transforms in LDS
    (200, 400, 300, 500, 0),        # K = 2, 18 primes
]


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def operands(ctx):
    ops = []
    for k, (db, Nb, da_max, Na_max, K) in enumerate(OPERANDS):
        pb = synth.dense(40 + k, db, Nb - 1)
        B = dev(pb.b)
        op = api.Operand(ctx, B, Nb, da_max, Na_max, K=K)
        ops.append((pb, op))
    yield ops
    for _, op in ops:
        op.close()


def items_for(operands, seed, per_op):
    rng = np.random.default_rng(seed)
    items, host_a = [], []
    for k, (pb, op) in enumerate(operands):
        db, Nb, da_max, Na_max, _ = OPERANDS[k]
        sizes = [(da_max, Na_max)] + [(int(rng.integers(1, da_max + 1)), int(rng.integers(2, Na_max + 1)))
                                      for _ in range(per_op - 1)]
        for da, Na in sizes:
            pa = synth.dense(int(rng.integers(1 << 30)), da, Na - 1)
            items.append((dev(pa.a), Na, op))
            host_a.append((pa, k))
    order = rng.permutation(len(items))
    return [items[i] for i in order], [host_a[i] for i in order]


def test_operand_batch_equals_alone_and_oracle(ctx, operands):
    nps = [op.info()["np"] for _, op in operands]
    print(f"[operand batch] operands {OPERANDS}, primes {nps}", flush=True)
    assert max(nps) > 16, "no operand plan with more than 16 primes"
    items, host_a = items_for(operands, 3, 5)
    got = ctx.mul_operand_batch(items)
    ref = [op.mul(a, Na) for (a, Na, op) in items]
    torch.cuda.synchronize()
    for k, (g, r) in enumerate(zip(got, ref)):
        assert torch.equal(g, r), f"job {k}: batch differs from zpm_mul_operand"
    for k in range(0, len(items), 3):
        pa, j = host_a[k]
        pb = operands[j][0]
        if pa.da * pb.db > 2_000_000:
            continue
        want = oracle.polymul(pa.a, pa.da, pa.Na, pb.b, pb.db, pb.Nb, wc=got[k].shape[1])
        assert np.array_equal(host(got[k]), want), f"job {k}: differs from the oracle"


def test_operand_batch_graph_follows_inputs(ctx, operands):
    items, _ = items_for(operands[:3], 4, 3)
    outs = [torch.empty_like(o) for o in ctx.mul_operand_batch(items)]
    rng = np.random.default_rng(9)
    for rep in range(3):
        # new contents in the same tensors: the replayed graph must read them
        for a, Na, _ in items:
            fresh = synth.dense(int(rng.integers(1 << 30)), a.shape[0], Na - 1)
            a.copy_(dev(fresh.a))
        print(f"[operand graph] replay {rep}", flush=True)
        ctx.mul_operand_batch(items, graph=True, outs=outs)
        torch.cuda.synchronize()
        ref = [op.mul(a, Na) for (a, Na, op) in items]
        torch.cuda.synchronize()
        for k, (g, r) in enumerate(zip(outs, ref)):
            assert torch.equal(g, r), f"replay {rep}, job {k}: differs from zpm_mul_operand"


def test_operand_batch_refusals(ctx, operands):
    pb = synth.dense(70, 900, 699)
    B = dev(pb.b)
    wide = api.Operand(ctx, B, 700, 1200, 800, K=32)    # register row kernel with K = 32
    a = dev(synth.dense(71, 100, 99).a)
    with pytest.raises(nat.ZpmError) as e:
        ctx.mul_operand_batch([(a, 100, wide)])
    assert e.value.code == nat.ZPM_EUNSUPPORTED
    pm = synth.dense(73, 300, 512)
    many = api.Operand(ctx, dev(pm.b), 513, 400, 600)     # 21 primes
    assert many.info()["np"] > 20
    with pytest.raises(nat.ZpmError) as e:
        ctx.mul_operand_batch([(a, 100, many)])
    assert e.value.code == nat.ZPM_EUNSUPPORTED
    many.close()
    _, op = operands[0]
    job, out = op.job(a, 100)
    jobs = (nat.OperandJob * 1)(job)
    assert nat.zpm_mul_operand_batch(ctx.handle, jobs, 1, nat.ZPM_BATCH_PERSISTENT, None) == nat.ZPM_ENOTIMPL
    # an operand of another context, and an a beyond the operand's bounds
    other = api.Context(0)
    try:
        assert nat.zpm_mul_operand_batch(other.handle, jobs, 1, 0, None) == nat.ZPM_EINVAL
    finally:
        other.close()
    big = dev(synth.dense(72, OPERANDS[0][2] + 1, 10).a)
    bjob, _ = op.job(big, 11)
    bjobs = (nat.OperandJob * 1)(bjob)
    assert nat.zpm_mul_operand_batch(ctx.handle, bjobs, 1, 0, None) == nat.ZPM_EINVAL
    torch.cuda.synchronize()
    wide.close()


def test_server_mixes_operand_and_ordinary_requests(ctx, operands):
    pb = synth.dense(80, 900, 699)
    wide = api.Operand(ctx, dev(pb.b), 700, 1200, 800, K=32)   # runs alone in the server
    items, _ = items_for(operands, 5, 8)
    pm = synth.dense(82, 300, 512)
    many = api.Operand(ctx, dev(pm.b), 513, 400, 600)      # 21 primes: runs alone too
    items += [(dev(synth.dense(81 + k, 300 + 97 * k, 500).a), 501, wide) for k in range(4)]
    items += [(dev(synth.dense(90 + k, 100 + 70 * k, 599).a), 600, many) for k in range(4)]
    pool = synth.served_pool(6, 60, (15, 1023), (16, 1024))
    plain = [(dev(p.a), p.Na, dev(p.b), p.Nb) for p in pool]
    order = np.random.default_rng(7).permutation(len(items) + len(plain))
    srv = api.Server(ctx, hbm_budget=1 << 30, n_streams=3, large_bits=2e6)
    print(f"[server operands] {len(items)} operand and {len(plain)} ordinary requests", flush=True)
    tickets = []
    for i in order:
        if i < len(items):
            a, Na, op = items[i]
            tickets.append(("op", i) + srv.submit_operand(a, Na, op))
        else:
            a, Na, b, Nb = plain[i - len(items)]
            tickets.append(("plain", i - len(items)) + srv.submit(a, Na, b, Nb))
    for _, _, t, _ in tickets:
        st, _ = srv.wait(t, timeout=60)
        assert st == 0, f"ticket {t} ended with {st}"
    stats = srv.stats()
    srv.close()
    assert stats["completed"] == len(tickets) and stats["failed"] == 0
    assert stats["batches"] < len(tickets), "no request shared a batch"
    for kind, i, _, out in tickets:
        if kind == "op":
            a, Na, op = items[i]
            ref = op.mul(a, Na)
        else:
            a, Na, b, Nb = plain[i]
            ref = ctx.mul(a, Na, b, Nb)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"{kind} request {i} differs from the product alone"
    wide.close()
    many.close()
