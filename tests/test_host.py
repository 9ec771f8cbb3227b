"""Host-side logic of the HIP library (CPU only, no kernels run).

* The C-ABI library loads and exports every function ``include/zpm.h`` declares.
* The prime table: the 48 largest primes c 2^21 + 1 below 2^30 (enumerated here with
  sympy), the stored root has order 2^21.
* The planner (DetermineBase + RecoveryPrime of Section 2.3): K M >= N, the prime
  product P exceeds 2 d K 2^(2M) (1 + 2^-12) with d = min(da, db), and no fewer primes
  would (Relation (recoveryModulo) for c_{i,j} itself), L >= da+db-1, 2K and L divide
  p - 1, CRT words hold P; checked with Python integers.
* The bound's premise: every c_{i,j} of the limb products is below min(da, db) K 2^(2M)
  in magnitude, checked on extreme and random operands with Python integers.
* Output width (Relation (citighterbound)) agrees with the extreme cases.
"""
import os
import re

import pytest
import sympy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def nat():
    from paper_1612_05778_amd import _native
    return _native


def test_exports_match_header(nat):
    hdr = open(os.path.join(ROOT, "include", "zpm.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    declared = set(re.findall(r"\b(zpm_[a-z_0-9]+)\s*\(", hdr))
    assert declared, "no declarations found"
    for name in sorted(declared):
        assert hasattr(nat.lib, name), f"{name} declared in zpm.h but not exported"
    assert nat.zpm_version() >= 100


def test_error_codes_and_host_argument_checks(nat):
    """The boundary's error codes have their own texts, and calls with a null context
    or bad sizes are refused on the host, before any device is touched."""
    texts = {c: nat.zpm_strerror(c).decode() for c in
             (nat.ZPM_OK, nat.ZPM_EINVAL, nat.ZPM_ENOMEM, nat.ZPM_EDEVICE, nat.ZPM_ERANGE,
              nat.ZPM_EUNSUPPORTED, nat.ZPM_ENOTIMPL, nat.ZPM_EBUSY, nat.ZPM_ENOTFOUND)}
    assert len(set(texts.values())) == len(texts), texts
    assert "range" in texts[nat.ZPM_ERANGE] and "not implemented" in texts[nat.ZPM_ENOTIMPL]
    assert nat.zpm_reserve(None, 1 << 20, 1 << 10, 64, 0) == nat.ZPM_EINVAL
    assert nat.zpm_set_option(None, nat.ZPM_OPT_CHECK_INPUTS, 1) == nat.ZPM_EINVAL
    assert nat.zpm_mul(None, None, 1, 64, None, 1, 64, None, 3, None) == nat.ZPM_EINVAL
    assert nat.zpm_mul_batch_ex(None, None, 0, 0, 0, None) == nat.ZPM_EINVAL
    assert nat.zpm_mul_operand_batch(None, None, 0, 0, None) == nat.ZPM_EINVAL
    assert nat.zpm_server_submit_operand(None, None, None) == nat.ZPM_EINVAL


def test_prime_table(nat):
    from paper_1612_05778_amd import api
    ps = []
    for k in range(48):
        p, r = api.prime(k)
        assert p < 2**30 and sympy.isprime(p) and (p - 1) % 2**21 == 0
        assert pow(r, 2**20, p) == p - 1          # order exactly 2^21
        ps.append(p)
    assert ps == sorted(ps, reverse=True) and len(set(ps)) == 48
    expect = [c * 2**21 + 1 for c in range(2**9 - 1, 0, -1) if sympy.isprime(c * 2**21 + 1)][:48]
    assert ps == expect
    with pytest.raises(Exception):
        api.prime(48)


PLAN_CASES = [
    (1024, 64, 1024, 64),          # signed 64-bit, 1024 coefficients
    (65536, 4097, 65536, 4097),    # 4096-bit magnitudes, 2^16 coefficients
    (262144, 16385, 262144, 16385),
    (64, 33, 8192, 2049),
    (1, 1, 1, 1),
    (1, 5000, 3, 7),
    (16, 8193, 16, 8193),
    (5000, 2, 7, 300),
]


@pytest.mark.parametrize("da,Na,db,Nb", PLAN_CASES)
def test_plan_invariants(nat, da, Na, db, Nb):
    from paper_1612_05778_amd import api
    pl = api.plan(da, Na, db, Nb)
    K, M, np_ = pl["K"], pl["M"], pl["np"]
    N = max(Na, Nb, 2)
    assert K >= 2 and M >= 2 and K & (K - 1) == 0 and K * M >= N
    d = min(da, db)
    P = 1
    for k in range(np_):
        P *= api.prime(k)[0]
    assert 4096 * P > 4097 * 2 * d * K * 2 ** (2 * M)
    if np_ <= 24:                       # every count up to 24 has compiled kernels
        P1 = P // api.prime(np_ - 1)[0]
        assert not 4096 * P1 > 4097 * 2 * d * K * 2 ** (2 * M), "fewer primes would do"
    L = 1 << pl["log2_L"]
    assert L >= da + db - 1 and (L == 1 or L // 2 < da + db - 1)
    assert max(L, 2 * K) <= 2**21
    assert pl["log2P"] == P.bit_length()
    assert 32 * pl["W"] >= P.bit_length() + 1
    # y-transform split: inner factor times the column passes is L
    assert pl["log2_L1"] + sum(pl["col_log2n"]) == pl["log2_L"]
    assert pl["workspace_bytes"] == 4 * np_ * 2 * K * L
    assert pl["nout_bits"] == api.out_bits(da, Na, db, Nb)
    check_col_tiles(pl)


def check_col_tiles(pl):
    """Column-pass tiles the kernels accept: each of the 256 threads owns one inner index
    and steps by 256 / T, the tile fits LDS, and it does not exceed the pass stride."""
    S = 1 << pl["log2_L"]
    for logn, T in zip(pl["col_log2n"], pl["col_tile"]):
        S >>= logn
        assert 1 <= T <= 256 and T & (T - 1) == 0, pl
        assert T * (1 << logn) <= 16384 and T <= S, pl


def test_col_tiles_for_every_K(nat):
    from paper_1612_05778_amd import api
    for (da, Na) in [(777, 901), (5000, 64), (65536, 4097), (3000, 700), (100000, 200)]:
        for logK in range(1, 11):
            try:
                pl = api.plan(da, Na, da, Na, K=1 << logK)
            except nat.ZpmError:
                continue
            check_col_tiles(pl)


def test_forced_plans(nat):
    from paper_1612_05778_amd import api
    for K in (2, 4, 8, 16, 32, 64):
        pl = api.plan(300, 500, 200, 400, K=K)
        assert pl["K"] == K and pl["K"] * pl["M"] >= 500
    pl = api.plan(300, 500, 200, 400, K=8, np=40)
    assert pl["np"] == 40
    with pytest.raises(nat.ZpmError):
        api.plan(300, 500, 200, 400, K=2, np=1)     # one prime cannot hold 2^(2*250)
    with pytest.raises(nat.ZpmError):
        api.plan(0, 5, 3, 5)


def test_small_products_alone_get_more_row_groups(nat):
    """Products that run alone with a deep inner y-factor (2^10 or more, x-transforms in
    registers) shorten it until the row kernel has at least 128 workgroups (np per inner
    block of rows); K and the primes stay the cost model's, and a forced K keeps its split."""
    from paper_1612_05778_amd import api
    for (da, Na) in [(1024, 64), (4096, 64), (2048, 128), (16384, 64), (512, 1024), (3001, 77)]:
        pl = api.plan(da, Na, da, Na)
        base = api.plan(da, Na, da, Na, K=pl["K"])
        assert base["log2_L1"] >= 10 and base["ncol"] <= 1, base
        assert (pl["K"], pl["M"], pl["np"], pl["log2_L"]) == \
            (base["K"], base["M"], base["np"], base["log2_L"])
        assert pl["log2_L1"] < base["log2_L1"] and pl["ncol"] == 1, pl
        assert pl["log2_L1"] + pl["col_log2n"][0] == pl["log2_L"]
        groups = pl["np"] << (pl["log2_L"] - pl["log2_L1"])
        assert groups >= 128 and (pl["log2_L1"] == 5 or groups < 256), pl
        assert pl["workspace_bytes"] == base["workspace_bytes"]
        check_col_tiles(pl)
    # shallow inner factors, large K, and products that fill the device keep their plan
    for (da, Na) in [(256, 256), (128, 4096), (64, 2048), (65536, 4096), (65536, 64)]:
        pl = api.plan(da, Na, da, Na)
        assert pl == api.plan(da, Na, da, Na, K=pl["K"]), pl


def test_out_bits_extremes(nat):
    from paper_1612_05778_amd import api
    for da, Na, db, Nb in [(1, 1, 1, 1), (3, 64, 5, 64), (4, 10, 4, 10), (1024, 64, 1024, 64),
                           (65536, 4097, 65536, 4097)]:
        nb = api.out_bits(da, Na, db, Nb)
        t = min(da, db)
        extreme = t * 2 ** (Na + Nb - 2)             # (-2^(Na-1)) (-2^(Nb-1)) summed t times
        assert extreme <= 2 ** (nb - 1) - 1
        assert nb == Na + Nb - 1 + t.bit_length()
    assert api.out_bits(1024, 64, 1024, 64) == 138
    assert api.out_bits(65536, 4097, 65536, 4097) == 8210


def test_kronecker_plans(nat):
    from paper_1612_05778_amd import api
    # too wide for one product, fine after reshaping
    with pytest.raises(nat.ZpmError):
        api.plan(32, 262145, 32, 262145)
    for (da, Na, db, Nb, w) in [(32, 262145, 32, 262145, 0), (8, 300000, 5, 200000, 0),
                                (50, 3000, 70, 2000, 512), (1, 70000, 1, 70000, 1024),
                                (100, 64, 100, 64, 256)]:
        k = api.kronecker_plan(da, Na, db, Nb, w)
        cw = k["chunk_bits"]
        assert cw % 64 == 0 and 256 <= cw <= 16384 and (w == 0 or cw == w)
        sa, sb = -(-Na // cw), -(-Nb // cw)
        assert (k["s_a"], k["s_b"], k["S"]) == (sa, sb, sa + sb - 1)
        assert k["da2"] == k["S"] * (da - 1) + sa and k["db2"] == k["S"] * (db - 1) + sb
        assert k["N2"] == cw + 1
        inner = k["inner"]
        assert inner["da"] == k["da2"] and inner["Na"] == cw + 1
        assert k["wc2"] == -(-nat.zpm_out_bits(k["da2"], cw + 1, k["db2"], cw + 1) // 64)
        assert k["da2"] + k["db2"] - 1 <= 1 << 21
    for bad in (100, -64):
        with pytest.raises(nat.ZpmError):
            api.kronecker_plan(10, 1000, 10, 1000, bad)


def test_from_to_ints_roundtrip(nat):
    from paper_1612_05778_amd import api
    vals = [0, 1, -1, 2**63, -(2**63), 2**200 - 7, -(2**200), 12345]
    t, N = api.from_ints(vals, device="cpu")
    assert N == 202 and t.shape == (len(vals), 4)
    assert api.to_ints(t) == vals
    t, N = api.from_ints([5, -3], 300, device="cpu")
    assert N == 300 and api.to_ints(t) == [5, -3]
    with pytest.raises(ValueError):
        api.from_ints([2**10], 10, device="cpu")


def limbs(x, N, K, M):
    """The limb split of Section 2: K limbs of M bits, the lower ones unsigned and the
    top one the signed rest (x is an N-bit two's complement value, K M >= N)."""
    out = []
    for j in range(K - 1):
        out.append((x >> (M * j)) & ((1 << M) - 1))
    out.append(x >> (M * (K - 1)))
    assert sum(a << (M * j) for j, a in enumerate(out)) == x
    return out


@pytest.mark.parametrize("da,db,N,K", [(3, 5, 40, 4), (7, 2, 33, 8), (4, 4, 64, 2), (6, 9, 17, 16)])
def test_cij_bound(da, db, N, K):
    """|c_{i,j}| < min(da, db) K 2^(2M) for c_{i,j} = sum a_{l,k} b_{m,h} over l + m = i,
    k + h = j: the premise of the planner's prime bound."""
    import random
    rng = random.Random(da * 100 + db * 10 + K)
    M = max(2, -(-N // K))
    lo, hi = -(1 << (N - 1)), (1 << (N - 1)) - 1
    cases = [([lo] * da, [lo] * db), ([hi] * da, [hi] * db), ([lo] * da, [hi] * db)]
    cases += [([rng.randint(lo, hi) for _ in range(da)], [rng.randint(lo, hi) for _ in range(db)])
              for _ in range(20)]
    bound = min(da, db) * K * 2 ** (2 * M)
    worst = 0
    for a, b in cases:
        A = [limbs(x, N, K, M) for x in a]
        B = [limbs(x, N, K, M) for x in b]
        for i in range(da + db - 1):
            for j in range(2 * K - 1):
                c = sum(A[l][k] * B[i - l][j - k] for l in range(max(0, i - db + 1), min(da, i + 1))
                        for k in range(max(0, j - K + 1), min(K, j + 1)))
                worst = max(worst, abs(c))
    assert worst < bound
    assert worst > bound // 16          # the extreme cases come close to it
