"""Products that reach the kernels with compile-time transform shapes.

Long products use the row kernel with the inner y-factor L1 = 2^(12 - log2 K) fixed at
compile time, and column passes of 2^1 ... 2^10 points with fixed tile widths.  Every K
of the register row kernels (2, 4, 8, 16) is run with a column pass of each length, as
a product, as a square, and as a product whose first operand is longer than half the
transform (the forward pass then reads both halves of each column; otherwise only the
lower one), and compared with the oracle at sampled output indices (the first, last and
middle coefficients, the operand boundary and random ones).  Small products run alone
with a shortened inner factor (the planner's row-group floor) must give the words of
the forced-K plan and of the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1612_05778_amd import api, synth
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


CASES = [(K, logn) for K in (2, 4, 8, 16) for logn in range(1, 11)
         if (12 - (K.bit_length() - 1)) + logn <= 21]


def sampled(prod, got, seed, n=40):
    nout = prod.da + prod.db - 1
    rng = np.random.default_rng(seed)
    rows = sorted(set([0, 1, prod.da - 1, prod.da, nout // 2, nout - 2, nout - 1] +
                      rng.choice(nout, size=min(n, nout), replace=False).tolist()))
    ref = oracle.polymul_rows(prod.a, prod.da, prod.Na, prod.b, prod.db, prod.Nb, rows,
                              wc=got.shape[1])
    bad = [r for r, g, w in zip(rows, got[rows], ref) if not np.array_equal(g, w)]
    assert not bad, f"rows {bad[:8]} differ from the oracle"


@pytest.mark.parametrize("K,logn", CASES)
def test_fixed_shapes(ctx, K, logn):
    logL1 = 12 - (K.bit_length() - 1)
    logL = logL1 + logn
    d = (1 << (logL - 2)) + 1                  # da + db - 1 = 2^(logL-1) + 1: L = 2^logL
    N = 17 * K                                 # M = 17
    r = np.random.default_rng(K * 100 + logn)
    a, _ = synth.signed_words(r, d, N - 1)
    b, _ = synth.signed_words(r, d, N - 1)
    prod = synth.Product(a, N, b, N)
    pl = api.plan(d, N, d, N, K=K)
    assert (pl["log2_L"], pl["log2_L1"], pl["col_log2n"]) == (logL, logL1, [logn])
    print(f"[fixed] K={K} L1=2^{logL1} pass=2^{logn} tile={pl['col_tile']} d={d}", flush=True)
    A, B = dev(a), dev(b)
    got = host(ctx.mul(A, N, B, N, K=K))
    sampled(prod, got, logn)
    sq = synth.Product(a, N, a, N)
    got_sq = host(ctx.mul(A, N, A, N, K=K))
    sampled(sq, got_sq, logn + 1)
    # a longer than half the transform (its forward pass reads both halves), b shorter
    da2, db2 = (1 << (logL - 1)) + 3, 1 << (logL - 2)
    a2, _ = synth.signed_words(r, da2, N - 1)
    b2, _ = synth.signed_words(r, db2, N - 1)
    pl2 = api.plan(da2, N, db2, N, K=K)
    assert (pl2["log2_L"], pl2["col_log2n"]) == (logL, [logn])
    sampled(synth.Product(a2, N, b2, N), host(ctx.mul(dev(a2), N, dev(b2), N, K=K)), logn + 2)
    del A, B
    torch.cuda.empty_cache()


# the LDS row kernel (K >= 64) with the planner's inner factor: 4 K L1 = 8192 words
LDS_CASES = [(K, logn) for K in (64, 128, 256) for logn in (5, 7, 9)]


@pytest.mark.parametrize("K,logn", LDS_CASES)
def test_fixed_shapes_lds_kernel(ctx, K, logn):
    logL1 = 13 - 2 - (K.bit_length() - 1)
    logL = logL1 + logn
    d = (1 << (logL - 2)) + 1
    N = 3 * K                                  # M = 3
    r = np.random.default_rng(K + logn)
    a, _ = synth.signed_words(r, d, N - 1)
    b, _ = synth.signed_words(r, d, N - 1)
    prod = synth.Product(a, N, b, N)
    pl = api.plan(d, N, d, N, K=K)
    assert (pl["log2_L"], pl["log2_L1"], pl["col_log2n"]) == (logL, logL1, [logn])
    print(f"[fixed lds] K={K} L1=2^{logL1} pass=2^{logn} d={d}", flush=True)
    A, B = dev(a), dev(b)
    sampled(prod, host(ctx.mul(A, N, B, N, K=K)), logn)
    sampled(synth.Product(a, N, a, N), host(ctx.mul(A, N, A, N, K=K)), logn + 1)
    if logn == 7:
        op = api.Operand(ctx, B, N, d, N, K=K)   # b's spectra resident, then a * b
        sampled(prod, host(op.mul(A, N)), logn + 2)
        op.close()
    del A, B
    torch.cuda.empty_cache()


def _ceil_log2(x):
    return (x - 1).bit_length()


# Single products now take 16-column tiles; the 8-column compiled passes of 2^8 to 2^10
# points are reached by batches whose tuned tile is 8.  A tuning table that sets (K, 8)
# for the product's size class is loaded, and the batch must give the same words as the
# single product (16-column passes) and the oracle at sampled rows.
@pytest.mark.parametrize("K,logn", [(16, 8), (16, 9), (8, 10)])
def test_batch_eight_column_passes(K, logn, tmp_path):
    from paper_1612_05778_amd import _native as nat
    from paper_1612_05778_amd.api import Context
    ctx = Context(0)    # its own context: the loaded tuning table must not leak
    logL1 = 12 - (K.bit_length() - 1)
    logL = logL1 + logn
    d = (1 << (logL - 2)) + 1
    N = 17 * K
    r = np.random.default_rng(K * 31 + logn)
    a, _ = synth.signed_words(r, d, N - 1)
    b, _ = synth.signed_words(r, d, N - 1)
    cls = (_ceil_log2(2 * d - 1) << 8) | _ceil_log2((N + 31) // 32)
    path = tmp_path / "tune.json"
    path.write_text('{"version": %d, "classes": {"%d": [%d, 8]}}' % (nat.zpm_version(), cls, K))
    ctx.tune_load(str(path))
    assert ctx.tune_table()[cls] == (K, 8)
    print(f"[batch tile 8] K={K} pass=2^{logn} d={d} class={cls}", flush=True)
    A, B = dev(a), dev(b)
    got = host(ctx.mul_batch([(A, N, B, N)])[0])
    single = host(ctx.mul(A, N, B, N, K=K))
    assert np.array_equal(got, single), "8-column batch passes differ from the single product"
    sampled(synth.Product(a, N, b, N), got, logn + 5)
    ctx.close()
    del A, B
    torch.cuda.empty_cache()


# Small products that run alone shorten a deep inner factor so that the row kernel has
# at least 128 workgroups; the forced-K product keeps the cost model's split.  Both must
# give the same words, and match the oracle (every row of the smallest, sampled rows
# otherwise); ragged sizes and unequal operands included.
@pytest.mark.parametrize("da,Na,db,Nb", [
    (1024, 64, 1024, 64), (4096, 64, 4096, 64), (2048, 128, 2048, 128), (16384, 64, 16384, 64),
    (512, 1024, 512, 1024), (3001, 77, 1900, 51), (1500, 300, 20, 900),
])
def test_small_products_split_inner_factor(ctx, da, Na, db, Nb):
    r = np.random.default_rng(da + 7 * Na)
    a, Na = synth.signed_words(r, da, Na - 1)
    b, Nb = synth.signed_words(r, db, Nb - 1)
    pl = api.plan(da, Na, db, Nb)
    base = api.plan(da, Na, db, Nb, K=pl["K"])
    print(f"[alone split] {da}x{Na} * {db}x{Nb}: K={pl['K']} np={pl['np']} "
          f"L1=2^{pl['log2_L1']} passes={pl['col_log2n']} (cost model: L1=2^{base['log2_L1']} "
          f"passes={base['col_log2n']})", flush=True)
    A, B = dev(a), dev(b)
    got = host(ctx.mul(A, Na, B, Nb))
    forced = host(ctx.mul(A, Na, B, Nb, K=pl["K"]))
    assert np.array_equal(got, forced), "the split plan and the cost model's differ"
    prod = synth.Product(a, Na, b, Nb)
    if da * db <= 1 << 21:
        want = oracle.polymul(a, da, Na, b, db, Nb, wc=got.shape[1])
        assert np.array_equal(got, want), "differs from the oracle"
    else:
        sampled(prod, got, da)
    del A, B
    torch.cuda.empty_cache()
