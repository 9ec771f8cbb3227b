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
    nl = nat.c_i64()
    nat.zpm_batch_schedule(pb.jobs, pb.n, 0, ctypes.byref(nl), None, 0)
    return {"workload": "batch4096", "products": pb.n, "out_bits": bits,
            "value": bits / (batch_ms / 1e3), "ms": batch_ms, "launches": nl.value,
            "plain_value": bits / (plain_ms / 1e3), "plain_ms": plain_ms,
            "speedup": plain_ms / batch_ms, "identical_to_plain": same,
            "tune_s": tune_s, "tuned_classes": len(ctx.tune_table())}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="bits4096_64k", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the cpu_baseline leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain leg")
    ap.add_argument("--batch-reps", type=int, default=5)
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
    from paper_1612_05778_amd.workmodel import INT32_PEAK, HBM_PEAK, kernel_work, product_bits

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

    ctx.profile_begin()
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
    kernels = ctx.profile_end()
    ctx.sync()
    ms = e0.elapsed_time(e1) / args.steps
    bits = product_bits(prod.da, prod.Na, prod.db, prod.Nb)
    value = bits / (ms / 1e3)

    # dominant kernel and its roofline
    kinfo = {}
    for name, (launches, tot) in kernels.items():
        work = kernel_work(pl, name)
        per = tot / launches
        kinfo[name] = {"launches_per_step": launches / args.steps, "avg_ms": per,
                       "share": tot / (ms * args.steps), **work}
    dom = max(kinfo, key=lambda k: kinfo[k]["avg_ms"] * kinfo[k]["launches_per_step"])
    d = kinfo[dom]
    if d["ops"]:
        achieved = d["ops"] / (d["avg_ms"] / 1e3)
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": INT32_PEAK / 1e12,
                "unit": "Tops/s (int32 VALU)", "frac": achieved / INT32_PEAK, "traffic": None,
                "kernel": dom}
    else:
        achieved = d["bytes"] / (d["avg_ms"] / 1e3)
        roof = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": achieved / HBM_PEAK, "traffic": None, "kernel": dom}
    for v in kinfo.values():
        if v["ops"]:
            v["int32_Tops"] = v["ops"] / (v["avg_ms"] / 1e3) / 1e12
        v["GBps"] = v["bytes"] / (v["avg_ms"] / 1e3) / 1e9

    line = {
        "metric": METRIC, "value": value, "unit": "coeff-bits/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "d": prod.da, "N": prod.Na,
                   "plan": {k: pl[k] for k in ("K", "M", "np", "log2_L", "log2_L1", "col_log2n", "W")},
                   "wall_ms_per_step": wall * 1e3 / args.steps},
        "roofline": roof,
        "kernels": kinfo,
    }
    if not args.no_batch:
        line["batched"] = batch_leg(ctx, args.batch_reps)
    if not args.no_cpu:
        print("[bench] cpu_baseline: timing the oracle on a sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(prod, args.cpu_seconds)
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
