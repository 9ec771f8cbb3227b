#!/usr/bin/env python3
"""Benchmark: exact dense Z[y] products on one MI355X.

A step is one whole product (every stage of the method) of the named workload
with inputs already resident in HBM.  Default workload: d = 2^16 coefficients
per operand, magnitudes uniform in [0, 2^4096) with uniform signs (N = 4097),
seed 2.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

The cpu_baseline leg times the oracle (plain schoolbook, all host threads) on a
bounded sample of output coefficients of the same workload and extrapolates by
the number of coefficient pairs; it is a reported baseline only.

More legs follow the main line's timing: ``square`` and ``resident_operand`` (the same
operands), ``p64`` (64-bit machine-word primes) and ``gfp`` (one generalized Fermat
prime) on the same product, ``latency`` (d = 1024 signed 64-bit coefficients, median and
p99 per call), ``large`` (d = 2^18, 16384-bit magnitudes), ``batched`` (4096 products of
uneven size, one at a time through zpm_mul against tuned zpm_mul_batch with graph
replay), ``operand_batch`` (1024 products of 512 x 1025-bit coefficients with one factor
held as a resident operand: zpm_mul_operand_batch against zpm_mul_batch and against
zpm_mul_operand one at a time) and ``served`` (an open-loop Poisson stream through the continuous-batching
server at a stated fraction of its saturated throughput, with p50/p99 latency, and the
same stream through the single-product baseline).  Batched, served and large legs state
their roofline fraction T*/T, T* being the sum over each product's kernels of
max(algorithmic bytes / HBM peak, algorithmic ops / ALU peak).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

METRIC = "output coeff-bits/s (exact) at d=2^16,N=4096; batched vs plain; p99 latency"

WORKLOADS = {
    "int64_1k": dict(d=1024, mag_bits=None, seed=1),
    "bits4096_64k": dict(d=1 << 16, mag_bits=4096, seed=2),
    "bits16384_256k": dict(d=1 << 18, mag_bits=16384, seed=3),
}


def make_workload(name: str):
    from paper_1612_05778_amd import synth
    if name == "int64_1k":
        return synth.int64_1k()
    w = WORKLOADS[name]
    return synth.dense(w["seed"], w["d"], w["mag_bits"])


def cpu_baseline(prod, target_s: float) -> dict:
    """Oracle throughput on a bounded sample of output rows, extrapolated by pair count."""
    import oracle
    from paper_1612_05778_amd.workmodel import product_bits
    da, db = prod.da, prod.db
    nout = da + db - 1
    threads = oracle.threads(0)
    rng = np.random.default_rng(12345)

    def pairs(i):
        return min(i + 1, da, db, nout - i)

    n = max(threads, 8)
    t_total, p_total, rows_done = 0.0, 0, 0
    while True:
        rows = np.sort(rng.choice(nout, size=min(n, nout), replace=False))
        t0 = time.perf_counter()
        oracle.polymul_rows(prod.a, da, prod.Na, prod.b, db, prod.Nb, rows)
        dt = time.perf_counter() - t0
        t_total += dt
        p_total += int(sum(pairs(int(i)) for i in rows))
        rows_done += len(rows)
        if t_total >= target_s or rows_done >= nout:
            break
        # grow the next batch towards the time target
        rate = max(dt / len(rows), 1e-6)
        n = int(min(nout, max(n, (target_s - t_total) / rate)))
    full_pairs = da * db
    est = t_total * full_pairs / p_total
    bits = product_bits(da, prod.Na, db, prod.Nb)
    return {
        "value": bits / est, "unit": "coeff-bits/s", "cores": threads, "kind": "oracle",
        "sample": f"{rows_done} random output coefficients of the same product "
                  f"({p_total} of {full_pairs} coefficient pairs) in {t_total:.1f} s; "
                  f"full-product time extrapolated by pair count: {est:.1f} s",
    }


KERNEL_SOURCES = ("stages.hpp", "kernels.hip", "kernels.hpp", "zpm_internal.hpp")


def kernel_sources_sha256() -> str:
    """Digest of the device sources of the single-product kernels."""
    import hashlib
    h = hashlib.sha256()
    base = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1612_05778_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(base, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/<workload>_traffic.json: FETCH_SIZE x its copy-calibrated factor plus
    WRITE_SIZE x its factor), or None when there is none or the kernel sources have
    changed since the counters were taken."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        f"{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        doc = json.load(f)
    if doc.get("sources_sha256") != kernel_sources_sha256():
        return None
    k = doc.get("kernels", {}).get(kernel)
    return None if k is None else k["fetch_bytes"] + k["write_bytes"]


def batch_leg(ctx, reps: int) -> dict:
    """The 4096-product batch (degree log-uniform in [63, 8191], magnitude bits
    log-uniform in [32, 2048], seed 4): one product at a time through zpm_mul against
    zpm_mul_batch (tuned per size class, graph replay); outputs must be identical."""
    import torch
    from paper_1612_05778_amd import _native as nat
    from paper_1612_05778_amd import synth
    from paper_1612_05778_amd.batchio import PackedBatch
    print("[bench] batch leg: generating 4096 products", file=sys.stderr, flush=True)
    pb = PackedBatch(synth.batch(4, 4096))
    st = torch.cuda.current_stream()
    h = st.cuda_stream
    bits = pb.bits()
    t0 = time.perf_counter()
    nat.check(nat.zpm_tune(ctx.handle, pb.jobs, pb.n, None, h), "zpm_tune")
    tune_s = time.perf_counter() - t0
    print(f"[bench] batch leg: tuned in {tune_s:.1f} s; timing plain path", file=sys.stderr, flush=True)

    def plain():
        for i in range(pb.n):
            j = pb.jobs[i]
            nat.check(nat.zpm_mul(ctx.handle, j.a, j.da, j.Na, j.b, j.db, j.Nb, j.c, j.wc, h), "zpm_mul")

    def timed(fn, k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(st)
        for _ in range(k):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    plain()
    torch.cuda.synchronize()
    ref = pb.outputs.clone()
    plain_ms = timed(plain, 2)
    print("[bench] batch leg: timing batched path", file=sys.stderr, flush=True)
    pb.outputs.zero_()

    def batched():
        nat.check(nat.zpm_mul_batch(ctx.handle, pb.jobs, pb.n, nat.ZPM_BATCH_GRAPH, h), "zpm_mul_batch")

    batched()
    torch.cuda.synchronize()
    same = bool(torch.equal(pb.outputs, ref))
    batch_ms = timed(batched, reps)
    print("[bench] batch leg: timing the persistent launch", file=sys.stderr, flush=True)
    pb.outputs.zero_()

    def persistent():
        nat.check(nat.zpm_mul_batch(ctx.handle, pb.jobs, pb.n, nat.ZPM_BATCH_PERSISTENT, h),
                  "zpm_mul_batch")

    persistent()
    torch.cuda.synchronize()
    same_persistent = bool(torch.equal(pb.outputs, ref))
    persistent_ms = timed(persistent, reps)
    nl = nat.c_i64()
    nat.zpm_batch_schedule(pb.jobs, pb.n, 0, ctypes.byref(nl), None, 0)
    ts = sum(t_star_of(pb.jobs[i].da, pb.jobs[i].Na, pb.jobs[i].db, pb.jobs[i].Nb)
             for i in range(pb.n)) * 1e3
    return {"workload": "batch4096", "products": pb.n, "out_bits": bits,
            "value": bits / (batch_ms / 1e3), "ms": batch_ms, "launches": nl.value,
            "plain_value": bits / (plain_ms / 1e3), "plain_ms": plain_ms,
            "speedup": plain_ms / batch_ms, "identical_to_plain": same,
            "persistent_ms": persistent_ms, "persistent_value": bits / (persistent_ms / 1e3),
            "persistent_identical_to_plain": same_persistent,
            "t_star_ms": ts, "roofline_frac": ts / batch_ms, "plain_roofline_frac": ts / plain_ms,
            "tune_s": tune_s, "tuned_classes": len(ctx.tune_table())}


def operand_batch_leg(ctx, reps: int, n: int = 1024, d: int = 512, mag: int = 1024) -> dict:
    """One factor b held as a resident operand times n different a of the same shape (d
    coefficients, magnitudes uniform below 2^mag, uniform signs; seeds 21 and 22):
    zpm_mul_operand_batch (graph replay) against zpm_mul_batch of the same products,
    which converts and transforms b in every product, and against zpm_mul_operand one
    product at a time.  All three outputs must be identical."""
    import torch
    from paper_1612_05778_amd import _native as nat
    from paper_1612_05778_amd import synth
    from paper_1612_05778_amd.api import Operand, out_words
    print(f"[bench] operand batch leg: {n} x {d} coefficients of {mag + 1} bits",
          file=sys.stderr, flush=True)
    N = mag + 1
    w = (N + 63) // 64
    pb = synth.dense(21, d, mag)
    r = synth.rng_for(22)
    A = torch.empty((n, d, w), dtype=torch.int64)
    for i in range(n):
        words, _ = synth.signed_words(r, d, mag)
        A[i] = torch.from_numpy(words.view(np.int64))
    A = A.cuda()
    B = torch.from_numpy(np.ascontiguousarray(pb.b).view(np.int64)).cuda()
    wc = out_words(d, N, d, N)
    C = torch.zeros((n, 2 * d - 1, wc), dtype=torch.int64, device="cuda")
    op = Operand(ctx, B, N, d, N)
    jobs = (nat.Job * n)()
    ojobs = (nat.OperandJob * n)()
    for i in range(n):
        jobs[i].a, jobs[i].da, jobs[i].Na = A[i].data_ptr(), d, N
        jobs[i].b, jobs[i].db, jobs[i].Nb = B.data_ptr(), d, N
        jobs[i].c, jobs[i].wc = C[i].data_ptr(), wc
        ojobs[i].a, ojobs[i].da, ojobs[i].Na, ojobs[i].op = A[i].data_ptr(), d, N, op._h
        ojobs[i].c, ojobs[i].wc = C[i].data_ptr(), wc
    st = torch.cuda.current_stream()
    h = st.cuda_stream
    bits = float(n * (2 * d - 1) * (64 * wc))

    def timed(fn, k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        e0.record(st)
        for _ in range(k):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    def plain_batch():
        nat.check(nat.zpm_mul_batch(ctx.handle, jobs, n, nat.ZPM_BATCH_GRAPH, h), "zpm_mul_batch")

    def operand_batch():
        nat.check(nat.zpm_mul_operand_batch(ctx.handle, ojobs, n, nat.ZPM_BATCH_GRAPH, h),
                  "zpm_mul_operand_batch")

    def one_by_one():
        for i in range(n):
            nat.check(nat.zpm_mul_operand(ctx.handle, ojobs[i].a, d, N, op._h, ojobs[i].c, wc, h),
                      "zpm_mul_operand")

    def served(use_operand):
        # all n requests submitted at once to a server (4 streams), until the last ends
        from paper_1612_05778_amd.api import Server
        srv = Server(ctx, hbm_budget=4 << 30, n_streams=4)
        tk = nat.c_u64()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tickets = []
        for i in range(n):
            if use_operand:
                nat.check(nat.zpm_server_submit_operand(srv._h, ctypes.byref(ojobs[i]), ctypes.byref(tk)),
                          "zpm_server_submit_operand")
            else:
                nat.check(nat.zpm_server_submit(srv._h, ctypes.byref(jobs[i]), ctypes.byref(tk)),
                          "zpm_server_submit")
            tickets.append(tk.value)
        t_sub = time.perf_counter() - t0
        stt, lat = nat.c_i32(), ctypes.c_double()
        for t in tickets:
            nat.check(nat.zpm_server_wait(srv._h, t, 60.0, ctypes.byref(stt), ctypes.byref(lat)),
                      "zpm_server_wait")
            if stt.value != 0:
                raise RuntimeError(f"served request ended with {stt.value}")
        dt = time.perf_counter() - t0
        mean_batch = srv.stats()["mean_batch"]
        srv.close()
        return dt * 1e3, mean_batch, t_sub * 1e3

    batch_ms = timed(plain_batch, reps)
    ref = C.clone()
    C.zero_()
    single_ms = timed(one_by_one, 2)
    same_single = bool(torch.equal(C, ref))
    C.zero_()
    op_ms = timed(operand_batch, reps)
    same = bool(torch.equal(C, ref))
    served(True)                                   # first use of the server's plans
    C.zero_()
    srv_op_ms, srv_op_batch, srv_op_sub = served(True)
    same_served = bool(torch.equal(C, ref))
    srv_ms, srv_batch, srv_sub = served(False)
    info = op.info()
    op.close()
    return {"workload": f"operand{d}x{N}_batch{n}", "products": n, "out_bits": bits,
            "ms": op_ms, "value": bits / (op_ms / 1e3),
            "plan": {"K": info["K"], "np": info["np"], "log2_L": info["log2_L"]},
            "batch_ms": batch_ms, "vs_batch": batch_ms / op_ms,
            "single_ms": single_ms, "vs_single": single_ms / op_ms,
            "identical_to_batch": same, "single_identical_to_batch": same_single,
            # wall-clock from the first submission to the last completion; the Python
            # submission loop alone takes submit_ms of it
            "served_operand_ms": srv_op_ms, "served_operand_submit_ms": srv_op_sub,
            "served_operand_mean_batch": srv_op_batch, "served_identical_to_batch": same_served,
            "served_plain_ms": srv_ms, "served_plain_submit_ms": srv_sub,
            "served_plain_mean_batch": srv_batch}


def t_star_of(da: int, Na: int, db: int, Nb: int) -> float:
    """Roofline time (s) of one product under the planner's single-product plan: the sum
    over its kernels of max(algorithmic bytes / HBM peak, algorithmic ops / ALU peak)."""
    from paper_1612_05778_amd.api import plan as get_plan
    from paper_1612_05778_amd.workmodel import t_star
    try:
        pl = get_plan(da, Na, db, Nb)
    except RuntimeError:
        return 0.0
    return t_star(pl)


def served_leg(ctx, n_req: int, n_warm: int, load: float, budget: int, streams: int,
               n_single: int, large_bits: float = 0.0, large_streams: int = 0,
               fixed_rate: float = 0.0, min_batch: int = 0, linger_s: float = 0.0) -> dict:
    """Open-loop Poisson stream of the served distribution (degree log-uniform in
    [15, 65535], magnitude bits log-uniform in [16, 8192], seed 5) through the
    continuous-batching server.  The offered load is ``load`` times the server's
    saturated throughput on the same request pool, measured first.  Latency runs
    from each request's scheduled arrival to its completion.  The same stream (its
    first ``n_single`` requests) also runs through a single-product server, the
    unbatched baseline.  Every output must equal the product computed alone."""
    import torch
    from paper_1612_05778_amd import _native as nat
    from paper_1612_05778_amd import api, synth
    from paper_1612_05778_amd.batchio import PackedBatch
    from paper_1612_05778_amd.workmodel import product_bits

    n_pool = 1024
    print(f"[bench] served leg: generating a pool of {n_pool} requests", file=sys.stderr, flush=True)
    pool = synth.served_pool(5, n_pool)
    pb = PackedBatch(pool)
    bits = [product_bits(p.da, p.Na, p.db, p.Nb) for p in pool]
    tstar = [t_star_of(p.da, p.Na, p.db, p.Nb) for p in pool]
    mean_bits = float(np.mean(bits))
    big = float(large_bits or (1 << 26))
    h = torch.cuda.current_stream().cuda_stream
    for rep in range(2):               # the first pass builds tables and plan constants
        t0 = time.perf_counter()
        for i in range(pb.n):
            j = pb.jobs[i]
            nat.check(nat.zpm_mul(ctx.handle, j.a, j.da, j.Na, j.b, j.db, j.Nb, j.c, j.wc, h), "zpm_mul")
        torch.cuda.synchronize()
        plain_s = time.perf_counter() - t0
    ref = pb.outputs.clone()

    cap_t = (nat.c_u64 * 8192)()
    cap_s = (nat.c_i32 * 8192)()
    cap_l = (ctypes.c_double * 8192)()
    cap_n = nat.c_i64()

    def saturated(srv):
        pb.outputs.zero_()
        torch.cuda.synchronize()
        t = nat.c_u64()
        w0 = time.perf_counter()
        for i in range(pb.n):
            nat.check(nat.zpm_server_submit(srv._h, ctypes.byref(pb.jobs[i]), ctypes.byref(t)), "submit")
        left = pb.n
        while left:
            nat.check(nat.zpm_server_completions(srv._h, cap_t, cap_s, cap_l, 8192, ctypes.byref(cap_n)),
                      "completions")
            for k in range(cap_n.value):
                if cap_s[k] != 0:
                    raise RuntimeError(f"served request failed with {cap_s[k]}")
            left -= cap_n.value
        return sum(bits) / (time.perf_counter() - w0)

    def stream(srv, n_total, warm, rate):
        arr = synth.served_arrivals(5, n_total) / rate
        owner = {}                     # ticket -> request index
        busy = [0] * n_pool            # ticket in flight per pool entry
        lag = np.zeros(n_total)
        lat = np.full(n_total, np.nan)
        guard_waits = 0
        t = nat.c_u64()

        def drain():
            nat.check(nat.zpm_server_completions(srv._h, cap_t, cap_s, cap_l, 8192, ctypes.byref(cap_n)),
                      "completions")
            for k in range(cap_n.value):
                r = owner.pop(cap_t[k])
                if cap_s[k] != 0:
                    raise RuntimeError(f"served request {r} failed with {cap_s[k]}")
                lat[r] = lag[r] + cap_l[k]
                if busy[r % n_pool] == cap_t[k]:
                    busy[r % n_pool] = 0

        t_start = time.perf_counter()
        for k in range(n_total):
            if k == warm:
                srv.reset_stats()
                t_meas = time.perf_counter()
            due = t_start + arr[k]
            while True:
                now = time.perf_counter()
                if now >= due:
                    break
                if due - now > 50e-6:
                    drain()
            e = k % n_pool
            while busy[e]:             # the entry's previous request still writes its output
                guard_waits += 1
                drain()
            lag[k] = time.perf_counter() - due
            nat.check(nat.zpm_server_submit(srv._h, ctypes.byref(pb.jobs[e]), ctypes.byref(t)), "submit")
            owner[t.value] = k
            busy[e] = t.value
        while owner:
            drain()
        span = time.perf_counter() - t_meas
        st = srv.stats()
        m = lat[warm:]
        rb = np.array([bits[k % n_pool] for k in range(warm, n_total)])
        done_bits = float(rb.sum())
        done_tstar = float(sum(tstar[k % n_pool] for k in range(warm, n_total)))

        def pct(x):
            if not len(x):
                return {"n": 0}
            return {"n": int(len(x)), "p50_ms": float(np.percentile(x, 50)) * 1e3,
                    "p99_ms": float(np.percentile(x, 99)) * 1e3}
        return {"requests": n_total - warm, "warmup_requests": warm,
                "offered_req_per_s": rate, "offered_bits_per_s": rate * mean_bits,
                "throughput_bits_per_s": done_bits / span,
                "roofline_frac": done_tstar / span,
                "p50_ms": float(np.percentile(m, 50)) * 1e3, "p99_ms": float(np.percentile(m, 99)) * 1e3,
                "max_ms": float(np.max(m)) * 1e3, "mean_ms": float(np.mean(m)) * 1e3,
                "small": pct(m[rb < big]), "large": pct(m[rb >= big]),
                "server_p50_ms": st["p50_s"] * 1e3, "server_p99_ms": st["p99_s"] * 1e3,
                "max_submit_lag_ms": float(np.max(lag[warm:])) * 1e3,
                "batches": st["batches"], "mean_batch": st["mean_batch"],
                "admission_waits": st["admission_waits"], "hbm_peak_bytes": st["hbm_peak"],
                "inflight_peak": st["inflight_peak"], "pool_reuse_waits": guard_waits}

    srv = api.Server(ctx, hbm_budget=budget, n_streams=streams, large_bits=large_bits,
                     large_streams=large_streams, min_batch=min_batch, linger_s=linger_s)
    print("[bench] served leg: saturated throughput", file=sys.stderr, flush=True)
    saturated(srv)
    cap = saturated(srv)
    torch.cuda.synchronize()
    same_sat = bool(torch.equal(pb.outputs, ref))
    rate = fixed_rate or load * cap / mean_bits
    print(f"[bench] served leg: capacity {cap:.3g} bits/s; offered {rate:.0f} req/s for "
          f"{n_warm}+{n_req} requests", file=sys.stderr, flush=True)
    pb.outputs.zero_()
    torch.cuda.synchronize()
    res = stream(srv, n_warm + n_req, n_warm, rate)
    srv.close()
    torch.cuda.synchronize()
    res["identical_to_alone"] = same_sat and bool(torch.equal(pb.outputs, ref))
    out = {"workload": "served", "pool_requests": n_pool, "pool_mean_out_bits": mean_bits,
           "hbm_budget_bytes": budget, "streams": streams, "load": load,
           "large_bits": big, "large_streams": large_streams or max(1, streams // 2),
           "min_batch": min_batch or 4, "linger_us": (linger_s or 150e-6) * 1e6,
           "saturated_bits_per_s": cap, "plain_sequential_bits_per_s": sum(bits) / plain_s,
           "saturated_roofline_frac": cap / sum(bits) * sum(tstar),
           "plain_sequential_roofline_frac": sum(tstar) / plain_s,
           **res}
    if n_single:
        print(f"[bench] served leg: single-product baseline, {n_single} requests", file=sys.stderr,
              flush=True)
        srv = api.Server(ctx, hbm_budget=budget, n_streams=streams, large_bits=large_bits,
                         large_streams=large_streams, single_product=True)
        saturated(srv)
        cap1 = saturated(srv)
        w = max(1, n_single // 10)
        base = stream(srv, n_single + w, w, rate)
        srv.close()
        out["single_product"] = {"saturated_bits_per_s": cap1,
                                 "saturated_roofline_frac": cap1 / sum(bits) * sum(tstar),
                                 **{k: base[k] for k in (
            "requests", "throughput_bits_per_s", "roofline_frac", "p50_ms", "p99_ms", "max_ms",
            "mean_ms", "small", "large")}}
    return out


def latency_leg(ctx, n: int = 400) -> dict:
    """Latency of the small single product (d = 1024 coefficients of signed 64-bit
    integers each, seed 1): one call at a time, each bracketed by events on its stream;
    then the same with the host kept ahead of the device (device time alone)."""
    import torch
    from paper_1612_05778_amd import synth
    from paper_1612_05778_amd.workmodel import product_bits
    prod = synth.int64_1k()
    a = torch.from_numpy(prod.a.view(np.int64).copy()).cuda()
    b = torch.from_numpy(prod.b.view(np.int64).copy()).cuda()
    out = ctx.mul(a, prod.Na, b, prod.Nb)
    for _ in range(20):
        ctx.mul(a, prod.Na, b, prod.Nb, out=out)
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev[0].record(st)
    for i in range(n):
        ctx.mul(a, prod.Na, b, prod.Nb, out=out)
        ev[i + 1].record(st)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - w0) / n
    lat = sorted(ev[i].elapsed_time(ev[i + 1]) * 1e3 for i in range(n))
    # the same calls queued behind a device-side wait, so that the host is ahead of the
    # device throughout: the intervals are the device's own time per product, free of
    # host delays (which the run above includes whenever the host is the slower side)
    torch.cuda.synchronize()
    torch.cuda._sleep(int(2.4e9 * 40e-6 * n))      # about 40 us of the shader clock per call
    ev[0].record(st)
    for i in range(n):
        ctx.mul(a, prod.Na, b, prod.Nb, out=out)
        ev[i + 1].record(st)
    torch.cuda.synchronize()
    dev_lat = sorted(ev[i].elapsed_time(ev[i + 1]) * 1e3 for i in range(n))
    bits = product_bits(prod.da, prod.Na, prod.db, prod.Nb)
    med = lat[n // 2]
    return {"workload": "int64_1k", "calls": n, "median_us": med,
            "p99_us": lat[min(n - 1, int(0.99 * n))], "min_us": lat[0],
            "host_wall_us_per_call": wall * 1e6, "value": bits / (med / 1e6),
            "device_median_us": dev_lat[n // 2],
            "device_p99_us": dev_lat[min(n - 1, int(0.99 * n))],
            "t_star_us": t_star_of(prod.da, prod.Na, prod.db, prod.Nb) * 1e6}


def large_leg(ctx, steps: int) -> dict:
    """The large product (d = 2^18 coefficients of 16384-bit magnitudes, seed 3)."""
    import torch
    from paper_1612_05778_amd.api import plan as get_plan
    from paper_1612_05778_amd.workmodel import product_bits
    print("[bench] large leg: generating 2^18 x 16385-bit operands", file=sys.stderr, flush=True)
    prod = make_workload("bits16384_256k")
    a = torch.from_numpy(prod.a.view(np.int64)).cuda()
    b = torch.from_numpy(prod.b.view(np.int64)).cuda()
    da, Na, db, Nb = prod.da, prod.Na, prod.db, prod.Nb
    del prod
    pl = get_plan(da, Na, db, Nb)
    out = ctx.mul(a, Na, b, Nb)
    ctx.mul(a, Na, b, Nb, out=out)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(steps):
        ctx.mul(a, Na, b, Nb, out=out)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    bits = product_bits(da, Na, db, Nb)
    ts = t_star_of(da, Na, db, Nb) * 1e3
    del a, b, out
    torch.cuda.empty_cache()
    return {"workload": "bits16384_256k", "d": da, "N": Na, "steps": steps, "ms": ms,
            "value": bits / (ms / 1e3), "plan": {k: pl[k] for k in ("K", "M", "np", "log2_L", "col_log2n")},
            "t_star_ms": ts, "roofline_frac": ts / ms}


def gfp_leg(ctx, a, b, prod, steps: int, product_ms: float) -> dict:
    """The single generalized Fermat prime variant on the same operands."""
    import torch
    from paper_1612_05778_amd.api import plan_gfp
    from paper_1612_05778_amd.workmodel import INT32_PEAK, gfp_work, product_bits
    info = plan_gfp(prod.da, prod.Na, prod.db, prod.Nb)
    print(f"[bench] gfp k={info['k']} K={info['K']} M={info['M']} passes={info['pass_log2n']}",
          file=sys.stderr, flush=True)
    out = ctx.mul_gfp(a, prod.Na, b, prod.Nb)
    ctx.mul_gfp(a, prod.Na, b, prod.Nb, out=out)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(steps):
        ctx.mul_gfp(a, prod.Na, b, prod.Nb, out=out)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ctx.profile_begin()
    for _ in range(steps):
        ctx.mul_gfp(a, prod.Na, b, prod.Nb, out=out)
    torch.cuda.synchronize()
    kern = ctx.profile_end()
    k2 = info["k"] ** 2
    kin = {}
    for name, (n, t) in kern.items():
        w = gfp_work(info, name)
        per = t / steps
        kin[name] = {"launches_per_step": n / steps, "ms_per_step": per,
                     "generic_products": w["products"], "algorithmic_bytes": w["bytes"],
                     "GBps": w["bytes"] / (per / 1e3) / 1e9 if w["bytes"] else None,
                     "digit_mads_per_s": w["products"] * k2 / (per / 1e3) if w["products"] else None,
                     "mad_frac_of_int32_peak": (w["products"] * k2 / (per / 1e3) / INT32_PEAK
                                                if w["products"] else None)}
    bits = product_bits(prod.da, prod.Na, prod.db, prod.Nb)
    del out
    torch.cuda.empty_cache()
    return {"k": info["k"], "r": info["r"], "log2p": info["log2p"], "K": info["K"], "M": info["M"],
            "log2_L": info["log2_L"], "y_passes_log2n": info["pass_log2n"], "ms": ms,
            "value": bits / (ms / 1e3), "vs_product": product_ms / ms, "kernels": kin}


P64_CONFIGS = {"default": ((0, 0),), "paper": ((128, 2),), "both": ((0, 0), (128, 2))}


def copy_bandwidth(mib: int = 1024, reps: int = 5) -> float:
    """Achieved HBM bytes/s (read + write) of a plain device copy of `mib` MiB."""
    import torch
    n = mib << 17
    src = torch.ones(n, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n * 8 / (ms / 1e3)


def p64_bytes(pl: dict, prod) -> dict:
    """Algorithmic HBM bytes per step of each 64-bit-prime kernel group: every residue
    read and written once per pass; the first forward pass reads only the d nonzero rows,
    the last inverse pass writes only the da + db - 1 output rows."""
    np_, K, L = pl["np"], pl["K"], 1 << pl["log2_L"]
    nout = prod.da + prod.db - 1
    wa, wb = (prod.Na + 63) // 64, (prod.Nb + 63) // 64
    wc = (pl["nout_bits"] + 63) // 64
    col = 8 * np_ * 2 * K * L                     # one full pass over the spectra
    npass = len(pl["pass_log2n"])
    rows_in = 8 * np_ * K * (prod.da + prod.db)   # nonzero limb rows of a and b
    last_out = 8 * np_ * 2 * K * nout
    return {
        "p64_convert_in": 8 * (prod.da * wa + prod.db * wb) + rows_in,
        "p64_y_fwd": (rows_in + col + 2 * col * (npass - 1)) if npass else 0,
        "p64_x_convolve": 2 * col,
        "p64_y_inv": (2 * col * (npass - 1) + col + last_out) if npass else 0,
        "p64_recover": last_out + 8 * nout * wc,
    }


def p64_leg(ctx, a, b, prod, steps: int, product_ms: float, configs=((0, 0), (128, 2))) -> dict:
    """The 64-bit machine-word prime variant on the same operands: the planner's choice and
    the paper's own two-prime configuration (K = 128, M = 33 for N = 4097)."""
    import torch
    from paper_1612_05778_amd.api import plan_p64
    from paper_1612_05778_amd.workmodel import product_bits
    bits = product_bits(prod.da, prod.Na, prod.db, prod.Nb)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    res = []
    for K, np_ in configs:
        try:
            pl = plan_p64(prod.da, prod.Na, prod.db, prod.Nb, K=K, np=np_)
        except RuntimeError:
            continue
        print(f"[bench] p64 K={pl['K']} M={pl['M']} np={pl['np']}", file=sys.stderr, flush=True)
        out = ctx.mul_p64(a, prod.Na, b, prod.Nb, K=K, np=np_)
        for _ in range(2):
            ctx.mul_p64(a, prod.Na, b, prod.Nb, K=K, np=np_, out=out)
        torch.cuda.synchronize()
        ctx.profile_begin()
        e0.record(stream)
        for _ in range(steps):
            ctx.mul_p64(a, prod.Na, b, prod.Nb, K=K, np=np_, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        kernels = ctx.profile_end()
        ms = e0.elapsed_time(e1) / steps
        alg = p64_bytes(pl, prod)
        kin = {}
        for k, (n, t) in kernels.items():
            kin[k] = {"launches_per_step": n / steps, "ms_per_step": t / steps,
                      "algorithmic_bytes": alg.get(k)}
            if alg.get(k):
                kin[k]["GBps"] = alg[k] / (t / steps / 1e3) / 1e9
                kin[k]["hbm_frac"] = alg[k] / (t / steps / 1e3) / 8.0e12
        res.append({"K": pl["K"], "M": pl["M"], "np": pl["np"], "log2_L": pl["log2_L"],
                    "y_passes_log2n": pl["pass_log2n"], "ms": ms, "value": bits / (ms / 1e3),
                    "vs_product": product_ms / ms, "kernels": kin})
        del out
        torch.cuda.empty_cache()
    return {"plans": res}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="bits4096_64k", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the cpu_baseline leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain leg")
    ap.add_argument("--only-product", action="store_true",
                    help="time the product alone: no square, resident-operand, batched, served "
                         "or cpu_baseline legs (for profiling the product's kernels)")
    ap.add_argument("--no-p64", action="store_true", help="skip the 64-bit prime leg")
    ap.add_argument("--only-p64", action="store_true",
                    help="time the 64-bit prime variant alone (for profiling its kernels)")
    ap.add_argument("--p64-config", default="both", choices=["default", "paper", "both"],
                    help="64-bit prime plans to time: the planner's, the paper's two-prime one, or both")
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--no-served", action="store_true", help="skip the served (Poisson) leg")
    ap.add_argument("--served-requests", type=int, default=20000)
    ap.add_argument("--served-warmup", type=int, default=2000)
    ap.add_argument("--served-load", type=float, default=0.7,
                    help="offered load as a fraction of the server's saturated throughput")
    ap.add_argument("--served-budget-gib", type=float, default=16.0)
    ap.add_argument("--served-streams", type=int, default=4)
    ap.add_argument("--served-min-batch", type=int, default=0,
                    help="small requests a batch waits for while the device is busy (0 = library default)")
    ap.add_argument("--served-linger-us", type=float, default=0.0,
                    help="longest such wait in microseconds (0 = library default, < 0 = none)")
    ap.add_argument("--served-rate", type=float, default=0.0,
                    help="offered requests/s (0 = --served-load times the saturated throughput)")
    ap.add_argument("--served-large-streams", type=int, default=0,
                    help="streams large requests may hold (0 = library default)")
    ap.add_argument("--served-large-bits", type=float, default=0.0,
                    help="output bits from which a request runs alone (0 = library default)")
    ap.add_argument("--served-single", type=int, default=3000,
                    help="requests of the single-product baseline (0 = skip)")
    ap.add_argument("--no-latency", action="store_true", help="skip the int64_1k latency leg")
    ap.add_argument("--no-large", action="store_true", help="skip the bits16384_256k leg")
    ap.add_argument("--large-steps", type=int, default=5)
    ap.add_argument("--no-gfp", action="store_true", help="skip the generalized Fermat prime leg")
    ap.add_argument("--only-gfp", action="store_true",
                    help="time the generalized Fermat prime variant alone (for profiling)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design note, not a measured configuration.",
              file=sys.stderr)
        return 2

    import torch
    from paper_1612_05778_amd.api import Context, plan as get_plan
    from paper_1612_05778_amd.workmodel import (INT32_PEAK, HBM_PEAK, MFMA_I8_PEAK, kernel_time,
                                                kernel_work, product_bits)

    print(f"[bench] workload {args.workload}: generating", file=sys.stderr, flush=True)
    if args.copy_mib:
        n = args.copy_mib << 17                     # int64 elements
        src = torch.ones(n, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    prod = make_workload(args.workload)
    a = torch.from_numpy(prod.a.view(np.int64).copy()).cuda()
    b = torch.from_numpy(prod.b.view(np.int64).copy()).cuda()
    pl = get_plan(prod.da, prod.Na, prod.db, prod.Nb)
    ctx = Context(0)
    stream = torch.cuda.current_stream()
    out = ctx.mul(a, prod.Na, b, prod.Nb)             # allocates tables + workspace
    for _ in range(args.warmup):
        ctx.mul(a, prod.Na, b, prod.Nb, out=out)
    torch.cuda.synchronize()
    print(f"[bench] plan K={pl['K']} M={pl['M']} np={pl['np']} L=2^{pl['log2_L']}; timing "
          f"{args.steps} steps", file=sys.stderr, flush=True)

    # per-kernel breakdown: every kernel bracketed by events (a few microseconds each,
    # so this run is not the headline timing)
    ctx.profile_begin()
    for _ in range(args.steps):
        ctx.mul(a, prod.Na, b, prod.Nb, out=out)
    torch.cuda.synchronize()
    kernels = ctx.profile_end()
    dom = max(kernels, key=lambda k: kernels[k][1])

    # timed region: events around the dominant kernel only, for its live duration
    ctx.profile_begin(kinds=[dom])
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.mul(a, prod.Na, b, prod.Nb, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    kernels_timed = ctx.profile_end()
    ctx.sync()
    ms = e0.elapsed_time(e1) / args.steps
    bits = product_bits(prod.da, prod.Na, prod.db, prod.Nb)
    value = bits / (ms / 1e3)

    # dominant kernel and its roofline
    kinfo = {}
    for name, (launches, tot) in kernels.items():
        if name == dom:
            launches, tot = kernels_timed[name]
        work = kernel_work(pl, name)
        per = tot / launches
        kinfo[name] = {"launches_per_step": launches / args.steps, "avg_ms": per,
                       "share": tot / (ms * args.steps), **work,
                       "timed_in": "timed region" if name == dom else "breakdown run"}
    d = kinfo[dom]
    from paper_1612_05778_amd import _native as nat
    from paper_1612_05778_amd.workmodel import OPS_BFLY_DIF as OPS_BFLY
    bfly = ctypes.c_double()
    nat.check(nat.zpm_butterfly_ceiling(0, 4096, ctypes.byref(bfly)), "zpm_butterfly_ceiling")
    ceiling = {"kernel": "register-resident forward butterflies (add_lz, mul_shoup_lz: values "
                         "in [0, 2p)), 8 pairs per thread, 8 workgroups of 256 per CU",
               "butterflies_per_s": bfly.value,
               "int32_ops_per_s": bfly.value * OPS_BFLY,
               "vs_derived_peak": bfly.value * OPS_BFLY / INT32_PEAK}
    if d["ops"]:
        achieved = d["ops"] / (d["avg_ms"] / 1e3)
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": INT32_PEAK / 1e12,
                "unit": "Tops/s (int32 VALU)", "frac": achieved / INT32_PEAK,
                "peak_measured": bfly.value * OPS_BFLY / 1e12,
                "frac_measured": achieved / (bfly.value * OPS_BFLY),
                "traffic": measured_traffic(args.workload, dom), "traffic_unit": "bytes/launch",
                "algorithmic_bytes": d["bytes"],
                "kernel": dom}
    else:
        achieved = d["bytes"] / (d["avg_ms"] / 1e3)
        roof = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": achieved / HBM_PEAK, "traffic": measured_traffic(args.workload, dom),
                "traffic_unit": "bytes/launch", "algorithmic_bytes": d["bytes"], "kernel": dom}
    for v in kinfo.values():
        if v["ops"]:
            v["int32_Tops"] = v["ops"] / (v["avg_ms"] / 1e3) / 1e12
        if v.get("mfma_ops"):
            v["int8_mfma_Tops"] = v["mfma_ops"] / (v["avg_ms"] / 1e3) / 1e12
            v["int8_mfma_frac"] = v["mfma_ops"] / (v["avg_ms"] / 1e3) / MFMA_I8_PEAK
        v["GBps"] = v["bytes"] / (v["avg_ms"] / 1e3) / 1e9
        v["roofline_frac"] = kernel_time(v) / (v["avg_ms"] / 1e3)

    # per-step distribution (a second run of the same steps, one event pair per step)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record(stream)
    for s_ in range(args.steps):
        ctx.mul(a, prod.Na, b, prod.Nb, out=out)
        ev[s_ + 1].record(stream)
    torch.cuda.synchronize()
    per_step = sorted(ev[s_].elapsed_time(ev[s_ + 1]) for s_ in range(args.steps))
    step_stats = {"median_ms": per_step[len(per_step) // 2],
                  "p99_ms": per_step[min(len(per_step) - 1, int(0.99 * len(per_step)))],
                  "min_ms": per_step[0]}

    # the whole path against its roofline: T* = sum over kernels of max(bytes / BW, ops / ALU)
    copy_bw = copy_bandwidth()

    def t_star(bw):
        return 1e3 * sum(v["launches_per_step"] * kernel_time(v, bw) for v in kinfo.values())
    path = {"t_star_ms": t_star(HBM_PEAK), "frac": t_star(HBM_PEAK) / ms,
            "t_star_measured_copy_ms": t_star(copy_bw), "frac_measured_copy": t_star(copy_bw) / ms,
            "copy_GBps": copy_bw / 1e9, "alu_peak_Tops": INT32_PEAK / 1e12}

    # host <-> device transfers of the operands and the product (pinned host buffers);
    # not part of the timed region
    ha = torch.empty(a.shape, dtype=a.dtype, pin_memory=True)
    hb = torch.empty(b.shape, dtype=b.dtype, pin_memory=True)
    hc = torch.empty(out.shape, dtype=out.dtype, pin_memory=True)
    ha.copy_(a); hb.copy_(b)
    torch.cuda.synchronize()
    e0.record(stream)
    a.copy_(ha, non_blocking=True)
    b.copy_(hb, non_blocking=True)
    e1.record(stream)
    torch.cuda.synchronize()
    h2d = e0.elapsed_time(e1)
    e0.record(stream)
    hc.copy_(out, non_blocking=True)
    e1.record(stream)
    torch.cuda.synchronize()
    d2h = e0.elapsed_time(e1)
    pcie = {"h2d_ms": h2d, "d2h_ms": d2h, "value_with_transfers": bits / ((ms + h2d + d2h) / 1e3)}
    del ha, hb, hc

    line = {
        "metric": METRIC, "value": value, "unit": "coeff-bits/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "d": prod.da, "N": prod.Na,
                   "plan": {k: pl[k] for k in ("K", "M", "np", "log2_L", "log2_L1", "col_log2n", "W")},
                   "wall_ms_per_step": wall * 1e3 / args.steps},
        "roofline": roof,
        "alu_ceiling": ceiling,
        "path_roofline": path,
        "step_ms": step_stats,
        "transfers": pcie,
        "kernels": kinfo,
    }
    if args.only_gfp:
        print(json.dumps({"workload": args.workload,
                          "gfp": gfp_leg(ctx, a, b, prod, args.steps, ms)}), flush=True)
        ctx.close()
        return 0
    if args.only_p64:
        print(json.dumps({"workload": args.workload,
                          "p64": p64_leg(ctx, a, b, prod, args.steps, ms, P64_CONFIGS[args.p64_config])}), flush=True)
        ctx.close()
        return 0
    if args.only_product:
        args.no_batch = args.no_served = args.no_cpu = True
        print(json.dumps(line), flush=True)
        ctx.close()
        return 0
    # the same workload squared (a passed twice): one conversion and forward transform
    sq = ctx.mul(a, prod.Na, a, prod.Na)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.mul(a, prod.Na, a, prod.Na, out=sq)
    e1.record(stream)
    torch.cuda.synchronize()
    sq_ms = e0.elapsed_time(e1) / args.steps
    line["square"] = {"ms": sq_ms, "value": bits / (sq_ms / 1e3), "vs_product": ms / sq_ms}
    del sq
    # b transformed once (resident operand), then products with a
    from paper_1612_05778_amd.api import Operand
    op = Operand(ctx, b, prod.Nb, prod.da, prod.Na)
    op.mul(a, prod.Na, out=out)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        op.mul(a, prod.Na, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    op_ms = e0.elapsed_time(e1) / args.steps
    line["resident_operand"] = {"ms": op_ms, "value": bits / (op_ms / 1e3), "vs_product": ms / op_ms}
    op.close()
    if not args.no_p64:
        line["p64"] = p64_leg(ctx, a, b, prod, args.steps, ms, P64_CONFIGS[args.p64_config])
    if not args.no_gfp:
        line["gfp"] = gfp_leg(ctx, a, b, prod, args.steps, ms)
    if not args.no_latency:
        line["latency"] = latency_leg(ctx)
    if not args.no_large:
        del a, b
        torch.cuda.empty_cache()
        line["large"] = large_leg(ctx, args.large_steps)
    if not args.no_batch:
        line["batched"] = batch_leg(ctx, args.batch_reps)
        line["operand_batch"] = operand_batch_leg(ctx, args.batch_reps)
    if not args.no_served:
        line["served"] = served_leg(ctx, args.served_requests, args.served_warmup, args.served_load,
                                    int(args.served_budget_gib * (1 << 30)), args.served_streams,
                                    args.served_single, args.served_large_bits,
                                    args.served_large_streams, args.served_rate,
                                    args.served_min_batch, args.served_linger_us * 1e-6)
    if not args.no_cpu:
        print("[bench] cpu_baseline: timing the oracle on a sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(prod, args.cpu_seconds)
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
