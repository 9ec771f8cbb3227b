"""Serving by continuous batching on the device: each result is the same alone and in
the mix.

Requests of the served distribution (degree and bits log-uniform, seed 5), scaled
down so the test takes seconds, arrive on a Poisson clock fast enough that new
requests land while earlier batches run.  Every output must equal, word for word,
the same product computed alone by zpm_mul after the server is gone; a sample is
also checked against the oracle.  The same stream through a server in single-product
mode, a server whose pool holds one request at a time, and a server sharing its
context with direct zpm_mul calls must give the same words.
"""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_1612_05778_amd import api, synth

from .gpu_util import dev, host

pytestmark = pytest.mark.gpu

DEG, BITS = (15, 2047), (16, 1024)


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def stream_inputs():
    pool = synth.served_pool(5, 160, DEG, BITS)
    ops = [(dev(p.a), p.Na, dev(p.b), p.Nb) for p in pool]
    return pool, ops


def run_stream(srv, ops, rate, t_arr):
    outs, tickets = [], []
    t0 = time.perf_counter()
    for k, (a, Na, b, Nb) in enumerate(ops):
        while time.perf_counter() - t0 < t_arr[k] / rate:
            pass
        t, o = srv.submit(a, Na, b, Nb)
        tickets.append(t)
        outs.append(o)
    for t in tickets:
        st, lat = srv.wait(t, timeout=60)
        assert st == 0, f"ticket {t} ended with {st}"
    return outs


def alone(ctx, ops):
    res = [ctx.mul(a, Na, b, Nb) for (a, Na, b, Nb) in ops]
    torch.cuda.synchronize()
    return res


def test_mix_equals_alone_and_oracle(ctx, stream_inputs):
    pool, ops = stream_inputs
    print(f"served mix: {len(ops)} requests, deg {DEG}, bits {BITS}", flush=True)
    t_arr = synth.served_arrivals(5, len(ops))
    srv = api.Server(ctx, hbm_budget=1 << 30, n_streams=3, large_bits=2e6)
    outs = run_stream(srv, ops, rate=4000.0, t_arr=t_arr)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(ops) and st["failed"] == 0
    assert st["batches"] < len(ops), "no request shared a batch"
    assert st["hbm_peak"] <= st["hbm_budget"]
    ref = alone(ctx, ops)
    for k, (o, r) in enumerate(zip(outs, ref)):
        assert torch.equal(o, r), f"request {k} differs from the product computed alone"
    for k in range(0, len(pool), 16):
        p = pool[k]
        want = oracle.polymul(p.a, p.da, p.Na, p.b, p.db, p.Nb, wc=outs[k].shape[1])
        assert np.array_equal(host(outs[k]), want), f"request {k} differs from the oracle"


def test_single_product_mode_same_words(ctx, stream_inputs):
    _, ops = stream_inputs
    t_arr = synth.served_arrivals(5, len(ops))
    srv = api.Server(ctx, hbm_budget=1 << 30, n_streams=2, single_product=True)
    outs = run_stream(srv, ops[:60], rate=4000.0, t_arr=t_arr)
    st = srv.stats()
    srv.close()
    assert st["batches"] == 60
    ref = alone(ctx, ops[:60])
    for k, (o, r) in enumerate(zip(outs, ref)):
        assert torch.equal(o, r), f"request {k} differs (single-product mode)"


def test_tight_pool_admits_one_at_a_time(ctx, stream_inputs):
    _, ops = stream_inputs
    big = sorted(range(len(ops)), key=lambda k: ops[k][0].shape[0] * ops[k][1])[-8:]
    sel = [ops[k] for k in big]
    fp = max(api.plan(a.shape[0], Na, b.shape[0], Nb)["workspace_bytes"] for a, Na, b, Nb in sel)
    srv = api.Server(ctx, hbm_budget=int(fp * 2.5), n_streams=4)
    outs = run_stream(srv, sel, rate=1e6, t_arr=np.arange(len(sel), dtype=float))
    st = srv.stats()
    srv.close()
    assert st["hbm_peak"] <= st["hbm_budget"]
    assert st["admission_waits"] >= 1
    for k, (o, r) in enumerate(zip(outs, alone(ctx, sel))):
        assert torch.equal(o, r), f"request {k} differs (tight pool)"


def test_server_and_direct_calls_share_a_context(ctx, stream_inputs):
    _, ops = stream_inputs
    srv = api.Server(ctx, hbm_budget=1 << 30, n_streams=2)
    tickets = [srv.submit(a, Na, b, Nb) for (a, Na, b, Nb) in ops[:40]]
    direct = [ctx.mul(a, Na, b, Nb) for (a, Na, b, Nb) in ops[40:60]]
    for t, _ in tickets:
        assert srv.wait(t, timeout=60)[0] == 0
    srv.close()
    torch.cuda.synchronize()
    ref = alone(ctx, ops[:60])
    for k in range(40):
        assert torch.equal(tickets[k][1], ref[k])
    for k in range(20):
        assert torch.equal(direct[k], ref[40 + k])


def test_bad_requests_on_device(ctx):
    srv = api.Server(ctx, hbm_budget=1 << 24, n_streams=1)
    a = torch.zeros((3000, 64), dtype=torch.int64, device="cuda")
    with pytest.raises(api.nat.ZpmError) as e:       # workspace beyond a 16 MiB pool
        srv.submit(a, 4096, a, 4096)
    assert e.value.code == api.nat.ZPM_ENOMEM
    e0 = torch.zeros((0, 1), dtype=torch.int64, device="cuda")
    t, o = srv.submit(e0, 64, a[:5, :1].contiguous(), 64)
    assert srv.wait(t, 5) == (0, 0.0) and o.numel() == 0
    srv.close()
