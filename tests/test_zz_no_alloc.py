"""zpm_mul_noalloc, the product entry point that allocates nothing, through the C-ABI.

Its residue workspace is the library's fixed device array instead of the context's
buffer; everything else is zpm_mul's path.  Checked here:
* two calls in a row on one reserved context, the second with a smaller product, give
  the same words as zpm_mul on another context, and sampled rows match the oracle
  (Section 1's product c_i = sum a_l b_m);
* a square (one operand passed twice) likewise;
* device free memory is unchanged by the calls;
* a product whose workspace exceeds the array fails with ZPM_ETOOBIG, one whose
  tables are not resident with ZPM_ENOMEM, both with c untouched, and one whose
  coefficients need Kronecker reshaping with ZPM_ENOTIMPL.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1612_05778_amd import _native as nat
from paper_1612_05778_amd import api, synth
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _noalloc(ctx, A, Na, B, Nb, out):
    return nat.zpm_mul_noalloc(ctx.handle, A.data_ptr(), A.shape[0], Na, B.data_ptr(), B.shape[0],
                               Nb, out.data_ptr(), out.shape[1], None)


def _out(p, fill=0):
    wc = api.out_words(p.da, p.Na, p.db, p.Nb)
    return torch.full((p.da + p.db - 1, wc), fill, dtype=torch.int64, device="cuda")


def _oracle_rows(p, got):
    rows = sorted({0, 1, p.da - 1, p.da, p.da + p.db - 2, (p.da + p.db - 1) // 2})
    ref = oracle.polymul_rows(p.a, p.da, p.Na, p.b, p.db, p.Nb, rows, wc=got.shape[1])
    assert np.array_equal(got[rows], ref), "rows differ from the oracle"


def test_noalloc_two_calls_match_mul():
    plain = api.Context(0)
    ctx = api.Context(0)
    big = synth.dense(401, 3000, 999)
    small = synth.dense(402, 700, 300)
    sq = synth.dense(403, 1200, 640)
    prods = [big, small]
    for p in prods + [sq]:
        assert api.plan(p.da, p.Na, p.db, p.Nb)["workspace_bytes"] <= nat.zpm_noalloc_max_bytes()
    ctx.reserve(0, 2 * big.da - 1, max(p.Na for p in prods + [sq]), max_plans=4)
    ins = [(dev(p.a), dev(p.b)) for p in prods]
    A3 = dev(sq.a)
    outs = [_out(p) for p in prods]
    out3 = _out(sq)
    # zpm_mul's results first: this also loads every kernel the products use
    refs = [host(plain.mul(A, p.Na, B, p.Nb)) for p, (A, B) in zip(prods, ins)]
    ref3 = host(plain.mul(A3, sq.Na, A3, sq.Na))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for p, (A, B), o in zip(prods, ins, outs):      # the second call is the smaller product
        assert _noalloc(ctx, A, p.Na, B, p.Nb, o) == nat.ZPM_OK
    assert _noalloc(ctx, A3, sq.Na, A3, sq.Na, out3) == nat.ZPM_OK
    ctx.sync()
    assert torch.cuda.mem_get_info()[0] == free0, "zpm_mul_noalloc allocated device memory"
    for p, ref, o in zip(prods, refs, outs):
        got = host(o)
        assert np.array_equal(got, ref), "zpm_mul_noalloc differs from zpm_mul"
        _oracle_rows(p, got)
    got3 = host(out3)
    assert np.array_equal(got3, ref3)
    rows = [0, sq.da - 1, 2 * sq.da - 2]
    assert np.array_equal(got3[rows], oracle.polymul_rows(sq.a, sq.da, sq.Na, sq.a, sq.da, sq.Na,
                                                          rows, wc=got3.shape[1]))
    # the larger product again, after the smaller one left its residues in the array
    o = _out(big, 0x5A5A)
    A, B = ins[0]
    assert _noalloc(ctx, A, big.Na, B, big.Nb, o) == nat.ZPM_OK
    assert np.array_equal(host(o), host(outs[0]))
    ctx.close()
    plain.close()


def test_noalloc_limits():
    ctx = api.Context(0)
    # tables not resident (fresh context, nothing reserved): ZPM_ENOMEM, c untouched
    p = synth.dense(404, 500, 200)
    A, B = dev(p.a), dev(p.b)
    o = _out(p, 0x3C3C)
    assert _noalloc(ctx, A, p.Na, B, p.Nb, o) == nat.ZPM_ENOMEM
    # beyond the scratch array: ZPM_ETOOBIG, c untouched
    big = synth.dense(405, 20000, 2999)
    assert api.plan(big.da, big.Na, big.db, big.Nb)["workspace_bytes"] > nat.zpm_noalloc_max_bytes()
    ctx.reserve(0, 2 * big.da - 1, big.Na, max_plans=2)
    A2, B2 = dev(big.a), dev(big.b)
    o2 = _out(big, 0x3C3C)
    assert _noalloc(ctx, A2, big.Na, B2, big.Nb, o2) == nat.ZPM_ETOOBIG
    torch.cuda.synchronize()
    assert (host(o) == np.uint64(0x3C3C)).all() and (host(o2) == np.uint64(0x3C3C)).all()
    # coefficients too wide for a direct plan (zpm_mul would reshape them): ZPM_ENOTIMPL
    wide = synth.dense(406, 2, 300000)
    with pytest.raises(RuntimeError):
        api.plan(wide.da, wide.Na, wide.db, wide.Nb)
    Aw, Bw = dev(wide.a), dev(wide.b)
    ow = _out(wide, 0x3C3C)
    assert _noalloc(ctx, Aw, wide.Na, Bw, wide.Nb, ow) == nat.ZPM_ENOTIMPL
    # after the reservation the small product runs
    assert _noalloc(ctx, A, p.Na, B, p.Nb, o) == nat.ZPM_OK
    ctx.sync()
    _oracle_rows(p, host(o))
    ctx.close()
