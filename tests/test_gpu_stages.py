"""Intermediate stages, through zpm_mul_ex's workspace dump (stop_after), against their
definitions evaluated here with Python integers from the inputs alone.

After convert-in (Section 2, BivariateRepresentation): column j < K of prime k holds
a_{i,j} mod p_k for i < da, where a_{i,j} is the unsigned field of bits [jM, (j+1)M)
of the N-bit two's complement coefficient a_i for j < K - 1, and the top limb is the
signed field from bit (K - 1)M, so that a_i = sum_j a_{i,j} 2^(M j); columns K + j hold
b's limbs.

After the inverse column passes: column j < 2K - 1 holds c_{i,j} (2K L) 2^-32 mod p_k
for i < da + db - 1, with c_{i,j} = sum over j1 + j2 = j and l of a_{l,j1} b_{i-l,j2},
the coefficients of A(x, y) B(x, y) before x = 2^M is substituted (Section 2.1); the
transforms are unnormalised and the pointwise product is a Montgomery product, and the
recovery applies 2^32 / (2K L).  Residues are compared mod p_k (the kernels keep them
below 2 p_k).

Shapes: the register row kernel without and with a column pass, and the LDS row
kernel; the full product is checked against the oracle as well.
"""
import numpy as np
import pytest

import oracle
from oracle import pyint
from paper_1612_05778_amd import api, synth

from .gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def limbs(vals, K, M):
    """a_{i,j}: unsigned M-bit fields, the top one signed (Section 2)."""
    out = []
    for v in vals:
        row = []
        for j in range(K):
            if j < K - 1:
                row.append((v >> (M * j)) & ((1 << M) - 1))
            else:
                row.append(v >> (M * j))      # Python's shift of a negative value floors
        assert sum(x << (M * j) for j, x in enumerate(row)) == v
        out.append(row)
    return out


@pytest.mark.parametrize("da,ba,db,bb,K", [
    (40, 300, 30, 250, 4),          # register row kernel, no column pass
    (1100, 100, 1000, 120, 2),      # a column pass
    (24, 2000, 20, 1800, 64),       # LDS row kernel, a column pass
])
def test_stage_dumps_match_definitions(ctx, da, ba, db, bb, K):
    r = np.random.default_rng(da * 7 + db)
    a, Na = synth.signed_words(r, da, ba)
    b, Nb = synth.signed_words(r, db, bb)
    A, B = dev(a), dev(b)
    va, vb = pyint.decode(a, Na), pyint.decode(b, Nb)
    info = api.plan(da, Na, db, Nb, K)
    K, M, npr, L = info["K"], info["M"], info["np"], 1 << info["log2_L"]
    print(f"[stages] da={da} Na={Na} db={db} Nb={Nb} K={K} M={M} np={npr} L={L} "
          f"ncol={info['ncol']}", flush=True)
    ps = [api.prime(k)[0] for k in range(npr)]
    la, lb = limbs(va, K, M), limbs(vb, K, M)

    ws1, _ = ctx.mul_stage(A, Na, B, Nb, 1, K=K, np=npr)
    w1 = ws1.cpu().numpy()
    for k, p in enumerate(ps):
        want_a = np.array([[x % p for x in row] for row in la], dtype=object).T   # (K, da)
        want_b = np.array([[x % p for x in row] for row in lb], dtype=object).T
        got_a = (w1[k, :K, :da] % p).astype(object)
        got_b = (w1[k, K:, :db] % p).astype(object)
        assert max(w1[k, :K, :da].max(), w1[k, K:, :db].max()) < 2 * p, \
            "convert-in left a residue at or above 2p"
        assert (got_a == want_a).all(), f"prime {k}: a's limb residues differ"
        assert (got_b == want_b).all(), f"prime {k}: b's limb residues differ"

    ws4, _ = ctx.mul_stage(A, Na, B, Nb, 4, K=K, np=npr)
    w4 = ws4.cpu().numpy()
    nout = da + db - 1
    # c_{i,j} over the integers for every i of short products, else the ends and a sample
    rows = list(range(nout)) if nout <= 300 else \
        sorted({0, 1, nout - 2, nout - 1, *r.choice(nout, 120, replace=False).tolist()})
    c = {}
    for i in rows:
        ci = [0] * (2 * K - 1)
        for l in range(max(0, i - db + 1), min(da, i + 1)):
            rowa, rowb = la[l], lb[i - l]
            for j1 in range(K):
                x = rowa[j1]
                if x:
                    for j2 in range(K):
                        ci[j1 + j2] += x * rowb[j2]
        c[i] = ci
    for k, p in enumerate(ps):
        f = (2 * K * L) * pow(2, -32, p) % p
        for i in rows:
            got = [int(w4[k, j, i]) % p for j in range(2 * K - 1)]
            want = [(c[i][j] * f) % p for j in range(2 * K - 1)]
            assert got == want, f"prime {k}, row {i}: c_ij residues differ"

    out = ctx.mul(A, Na, B, Nb, K=K, np=npr)
    want = oracle.polymul(a, da, Na, b, db, Nb, wc=out.shape[1])
    assert np.array_equal(host(out), want), "the full product differs from the oracle"
