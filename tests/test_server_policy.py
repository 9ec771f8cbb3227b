"""Admission and batching policy of the serving loop, against a simulated device.

zpm_server_create_simulated runs the same worker, lanes, pool allocator and
bookkeeping as a device-backed server, but a batch only "runs" for a modelled time
and nothing is computed (no device, outputs untouched).  Checked here: every ticket
is reported exactly once; the pool budget is never exceeded and a request larger
than the pool is rejected; requests wait for pool memory instead of overcommitting;
small requests are not held behind large ones; one lane is served in arrival order;
a device error fails in-flight and queued requests and later submissions instead of
hanging; bad jobs are refused; destroy drains what was submitted; concurrent
submitters are safe.
"""
import ctypes
import threading
import time

import pytest

from paper_1612_05778_amd import _native as nat
from paper_1612_05778_amd import api

FAKE = 0x1000   # never dereferenced by the simulated device


def job(d, N, wc=None):
    j = nat.Job()
    j.a = j.b = j.c = FAKE
    j.da = j.db = d
    j.Na = j.Nb = N
    j.wc = api.out_words(d, N, d, N) if (d and wc is None) else (wc or 1)
    return j


def footprint(d, N):
    return api.plan(d, N, d, N)["workspace_bytes"]


def sim(budget, streams=2, rate=1e11, overhead=20e-6, fail_after=-1, max_batch=0, large_bits=0.0):
    return api.Server(None, hbm_budget=budget, n_streams=streams, max_batch=max_batch,
                      large_bits=large_bits,
                      simulate={"bits_per_s": rate, "overhead_s": overhead, "fail_after": fail_after})


def drain(s, tickets, timeout=20.0):
    got = {}
    t_end = time.time() + timeout
    while len(got) < len(tickets):
        for t, st, lat in s.completions():
            assert t not in got, "ticket reported twice"
            got[t] = (st, lat, len(got))
        assert time.time() < t_end, f"{len(tickets) - len(got)} tickets never finished"
        time.sleep(1e-4)
    assert set(got) == set(tickets)
    return got


def test_all_finish_once_and_stats():
    s = sim(1 << 30)
    ts = [s.submit_job(job(16 + 7 * i, 32 + 13 * i)) for i in range(300)]
    got = drain(s, ts)
    assert all(v[0] == 0 for v in got.values())
    st = s.stats()
    assert st["submitted"] == st["completed"] == 300 and st["failed"] == 0
    assert 0 < st["p50_s"] <= st["p99_s"] <= st["max_s"]
    assert st["inflight"] == 0 and st["queued"] == 0 and st["hbm_in_use"] == 0
    assert 1 <= st["mean_batch"] and st["batches"] <= 300
    # consumed: polling again finds nothing
    with pytest.raises(nat.ZpmError) as e:
        s.poll(ts[0])
    assert e.value.code == nat.ZPM_ENOTFOUND
    s.close()


def test_budget_respected_and_admission_waits():
    fp = footprint(4000, 2000)
    budget = int(fp * 1.5)          # one such request at a time
    s = sim(budget, streams=4, rate=2e10)
    ts = [s.submit_job(job(4000, 2000)) for _ in range(6)]
    got = drain(s, ts)
    st = s.stats()
    assert all(v[0] == 0 for v in got.values())
    assert st["hbm_peak"] <= budget
    assert st["hbm_peak"] >= fp
    assert st["admission_waits"] >= 1
    assert st["inflight_peak"] == 1
    # a request whose workspace alone exceeds the pool is refused at submission
    with pytest.raises(nat.ZpmError) as e:
        s.submit_job(job(40000, 8000))
    assert e.value.code == nat.ZPM_ENOMEM
    assert s.stats()["rejected"] == 1
    s.close()


def test_small_requests_pass_large_ones():
    # large: ~0.3 s each on the simulated device; small: microseconds
    s = sim(8 << 30, streams=2, rate=1e10, large_bits=1e8)
    big = [s.submit_job(job(30000, 8000)) for _ in range(3)]
    time.sleep(0.01)
    small = [s.submit_job(job(20, 64)) for _ in range(50)]
    got = drain(s, big + small, timeout=30)
    last_small = max(got[t][2] for t in small)
    first_big = min(got[t][2] for t in big)
    assert last_small < first_big, "small requests waited behind large ones"
    assert max(got[t][1] for t in small) < 0.2
    s.close()


def test_large_stream_limit():
    # four long large requests, two of them at a time at most; small ones keep flowing
    s = api.Server(None, hbm_budget=8 << 30, n_streams=3, large_bits=1e8, large_streams=2,
                   simulate={"bits_per_s": 1e10, "overhead_s": 1e-5})
    big = [s.submit_job(job(30000, 8000)) for _ in range(4)]
    time.sleep(0.02)
    st = s.stats()
    assert st["inflight"] == 2 and st["queued"] == 2
    small = [s.submit_job(job(20, 64)) for _ in range(10)]
    got = drain(s, big + small, timeout=30)
    assert max(got[t][2] for t in small) < min(got[t][2] for t in big)
    s.close()


def test_one_stream_serves_a_lane_in_order():
    s = sim(1 << 30, streams=1, rate=1e9, max_batch=4)
    ts = [s.submit_job(job(50 + (i % 7) * 10, 100)) for i in range(40)]
    got = drain(s, ts)
    order = sorted(ts, key=lambda t: got[t][2])
    assert order == ts
    st = s.stats()
    assert st["batches"] >= 10 and st["mean_batch"] <= 4
    s.close()


def test_device_error_fails_requests_and_submissions():
    s = sim(1 << 30, streams=2, rate=1e9, overhead=1e-3, fail_after=2, max_batch=2)
    ts = [s.submit_job(job(100, 500)) for _ in range(20)]
    got = drain(s, ts)
    codes = [got[t][0] for t in ts]
    assert codes.count(0) >= 1
    assert nat.ZPM_EDEVICE in codes
    assert all(c in (0, nat.ZPM_EDEVICE) for c in codes)
    with pytest.raises(nat.ZpmError) as e:
        s.submit_job(job(10, 10))
    assert e.value.code == nat.ZPM_EDEVICE
    assert s.stats()["failed"] == codes.count(nat.ZPM_EDEVICE)
    s.close()


def test_bad_and_empty_jobs():
    s = sim(1 << 30)
    with pytest.raises(nat.ZpmError) as e:
        s.submit_job(job(10, 100, wc=1))               # output too narrow
    assert e.value.code == nat.ZPM_EINVAL
    j = job(10, 100)
    j.c = None
    with pytest.raises(nat.ZpmError):
        s.submit_job(j)
    j = job(10, 100)
    j.Na = 0
    with pytest.raises(nat.ZpmError):
        s.submit_job(j)
    t = s.submit_job(job(0, 100))                      # empty product: done at once
    assert s.poll(t) == (0, 0.0)
    with pytest.raises(nat.ZpmError) as e:
        s.poll(123456789)
    assert e.value.code == nat.ZPM_ENOTFOUND
    # a request against a resident operand needs one (a simulated server has no
    # context, so no operand can belong to it)
    oj = nat.OperandJob()
    oj.a, oj.da, oj.Na, oj.op, oj.c, oj.wc = FAKE, 10, 100, None, FAKE, 4
    tk = nat.c_u64()
    assert nat.zpm_server_submit_operand(s._h, ctypes.byref(oj), ctypes.byref(tk)) == nat.ZPM_EINVAL
    assert nat.zpm_server_submit_operand(s._h, None, ctypes.byref(tk)) == nat.ZPM_EINVAL
    s.close()


def test_wait_timeout_then_result():
    s = sim(4 << 30, streams=1, rate=1e9)
    t = s.submit_job(job(20000, 4000))                 # ~1 s simulated
    with pytest.raises(nat.ZpmError) as e:
        s.wait(t, timeout=0.01)
    assert e.value.code == nat.ZPM_EBUSY
    st, lat = s.wait(t, timeout=30)
    assert st == 0 and lat > 0.01
    s.close()


def test_single_product_mode_runs_one_per_batch():
    s = api.Server(None, hbm_budget=1 << 30, n_streams=2, single_product=True,
                   simulate={"bits_per_s": 1e11, "overhead_s": 1e-4})
    ts = [s.submit_job(job(30 + i, 100)) for i in range(40)]
    drain(s, ts)
    st = s.stats()
    assert st["batches"] == 40 and st["mean_batch"] == 1
    s.close()


def test_destroy_drains_submitted_work():
    s = sim(1 << 30, streams=2, rate=1e10)
    for i in range(100):
        s.submit_job(job(200 + i, 300))
    t0 = time.time()
    s.close()                                          # returns after every request finished
    assert time.time() - t0 < 20


def test_concurrent_submitters():
    s = sim(1 << 30, streams=3, rate=1e11)
    out, errs = [], []

    def worker(k):
        try:
            for i in range(100):
                out.append(s.submit_job(job(16 + ((k * 100 + i) % 200), 64)))
        except Exception as e:   # noqa: BLE001
            errs.append(e)

    th = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert not errs
    assert len(set(out)) == 400
    got = drain(s, out)
    assert all(v[0] == 0 for v in got.values())
    s.close()


def test_config_rejected():
    for cfg in ({"n_streams": 17}, {"max_batch": 5000}, {"large_bits": -1.0}, {"single": 2},
                {"n_streams": 2, "large_streams": 3}, {"large_streams": -1}, {"min_batch": -2},
                {"linger_s": 2.0}):
        c = nat.ServerConfig(1 << 20, cfg.get("n_streams", 0), cfg.get("max_batch", 0),
                             cfg.get("large_bits", 0.0), cfg.get("single", 0),
                             cfg.get("large_streams", 0), cfg.get("min_batch", 0),
                             cfg.get("linger_s", 0.0))
        h = nat.c_vp()
        assert nat.zpm_server_create_simulated(ctypes.byref(c), 1e9, 0.0, -1, ctypes.byref(h)) \
            == nat.ZPM_EINVAL


def test_small_requests_coalesce_while_busy():
    # a long request occupies one stream; three small ones arriving meanwhile wait
    # (min_batch 4) until a fourth joins them, and run as one batch
    s = api.Server(None, hbm_budget=1 << 30, n_streams=2, min_batch=4, linger_s=0.5,
                   simulate={"bits_per_s": 1e8, "overhead_s": 1e-3})
    big = s.submit_job(job(2000, 400))          # about 1.6e6 bits: 16 ms simulated
    time.sleep(0.002)
    small = []
    for _ in range(3):
        small.append(s.submit_job(job(16, 32)))
        time.sleep(0.002)
    time.sleep(0.02)                             # the long one has finished; three wait
    assert s.stats()["batches"] == 1
    small.append(s.submit_job(job(16, 32)))
    drain(s, [big] + small)
    st = s.stats()
    assert st["batches"] == 2 and st["mean_batch"] == 2.5
    s.close()


def test_linger_expires_and_idle_device_does_not_wait():
    s = api.Server(None, hbm_budget=1 << 30, n_streams=2, min_batch=8, linger_s=0.03,
                   simulate={"bits_per_s": 1e8, "overhead_s": 1e-3})
    # idle device: a lone small request starts at once
    t0 = time.time()
    drain(s, [s.submit_job(job(16, 32))])
    assert time.time() - t0 < 0.025
    # busy device: two small requests wait for the linger time, then run together
    big = s.submit_job(job(4000, 400))          # about 3.2e6 bits: 32 ms simulated
    time.sleep(0.002)
    small = [s.submit_job(job(16, 32)) for _ in range(2)]
    got = drain(s, [big] + small)
    assert all(v[0] == 0 for v in got.values())
    st = s.stats()
    assert st["batches"] == 3 and st["completed"] == 4
    s.close()
