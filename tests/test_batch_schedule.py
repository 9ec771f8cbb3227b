"""Host-side schedule of batched products (CPU only, no kernels run).

zpm_batch_schedule returns the launches zpm_mul_batch makes.  Checked here: levels
come in order and the first level is convert-in only; every live product has exactly
one convert-in, one row-convolution and one recovery segment, and as many inverse as
forward column-pass segments; LDS stays within one workgroup's 64 KiB; the number of
launches does not grow with the number of products; a forced K shows up as the
convolution variant; bad arguments are rejected.
"""
import ctypes

import numpy as np

from paper_1612_05778_amd import _native as nat
from paper_1612_05778_amd import api, synth


def jobs_for(sizes):
    jobs = (nat.Job * max(len(sizes), 1))()
    for i, (da, Na, db, Nb) in enumerate(sizes):
        jobs[i].da, jobs[i].Na, jobs[i].db, jobs[i].Nb = da, Na, db, Nb
        jobs[i].wc = (api.out_bits(da, Na, db, Nb) + 63) // 64 if da and db else 1
    return jobs


def schedule(sizes, K=0):
    jobs = jobs_for(sizes)
    n = nat.c_i64()
    buf = (nat.c_i64 * (6 * 4096))()
    rc = nat.zpm_batch_schedule(jobs, len(sizes), K, ctypes.byref(n), buf, 4096)
    assert rc == 0, rc
    return np.array(buf[: 6 * n.value], dtype=np.int64).reshape(-1, 6)


def workload(n):
    _, degs, bits = synth.batch_sizes(4, n)
    return [(int(d) + 1, int(b) + 1, int(d) + 1, int(b) + 1) for d, b in zip(degs, bits)]


def test_levels_and_segments():
    sizes = workload(512) + [(1, 1, 1, 1), (0, 5, 3, 5), (3, 64, 8192, 2049)]
    live = sum(1 for s in sizes if s[0] and s[2])
    L = schedule(sizes)
    level, kind, nseg = L[:, 0], L[:, 1], L[:, 3]
    assert np.all(np.diff(level) >= 0), "levels out of order"
    assert set(kind[level == 0]) == {0}
    for k in (0, 2, 4):
        assert nseg[kind == k].sum() == live
    assert nseg[kind == 1].sum() == nseg[kind == 3].sum()
    assert np.all(L[:, 4] > 0) and np.all(L[:, 5] <= 65536)
    # a product's recovery comes after its convolution: last level is recovery only
    assert set(kind[level == level.max()]) == {4}


def test_launch_count_independent_of_batch_size():
    sizes = workload(4096)
    few = schedule(sizes[:256])
    many = schedule(sizes)
    assert len(many) <= 5 * 40            # levels x compiled variants, not products
    assert many[many[:, 1] == 0, 3].sum() == 4096
    assert len(few) <= len(many)


def test_forced_K_and_invalid():
    sizes = [(300, 500, 200, 400)] * 3
    for K in (4, 8, 16):
        L = schedule(sizes, K)
        conv = L[L[:, 1] == 2]
        # variant: log2 K of the register kernel, + 32 when the inner factor is the
        # full 2^(12 - log2 K) (the compile-time kernel)
        pl = api.plan(300, 500, 200, 400, K=K)
        full = 32 if pl["log2_L1"] == 12 - int(np.log2(K)) else 0
        assert len(conv) == 1 and conv[0, 2] == int(np.log2(K)) + full and conv[0, 3] == 3
    jobs = jobs_for([(3, 8, 3, 8)])
    jobs[0].wc = 0
    n = nat.c_i64()
    assert nat.zpm_batch_schedule(jobs, 1, 0, ctypes.byref(n), None, 0) == nat.ZPM_EINVAL
    # K = 2 needs 17 primes here, beyond the batch limit of 16
    jobs = jobs_for(sizes)
    assert nat.zpm_batch_schedule(jobs, 3, 2, ctypes.byref(n), None, 0) == nat.ZPM_EUNSUPPORTED
