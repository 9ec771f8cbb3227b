"""Algorithmic work per kernel launch, for roofline reporting.

Counts are what the method itself must do for a plan (Section 3.3: K
transforms of length L along y for each operand and 2K inverse ones; along x,
per y-frequency, a cyclic and a negacyclic convolution of length K, i.e. three
K-point transforms each, plus the twist by theta^j before the negacyclic
forward transforms and the untwist after its inverse), not what a particular
kernel happens to execute (the kernels run the x part as 2K-point transforms
whose first stage is the twist):

* values are kept in [0, 2p) (every prime is below 2^30) and reduced only that far;
* one forward (DIF) radix-2 butterfly = 8 int32 VALU operations: u + v reduced below
  2p (add, sub, min), u - v + 2p (2), its Shoup product with the twiddle (mul_hi,
  mul_lo and a multiply-add); one inverse (DIT) butterfly = 9: the Shoup product (3),
  u + v and u - v reduced below 2p (3 each);
* one pointwise product = 6 (Montgomery product up to one p; the normalisation by
  2^32 / (2K L) is taken by the recovery's first Shoup product, counted there);
* one four-step twiddle or twist product = 3 (Shoup product up to one p);
* convert-in, per limb residue: 2 per 32-bit word of the limb (a multiply-add with
  the table entry 2^(32 t) mod p and its carry) plus 6 for the final reduction;
* CRT of one value c_{i,j} from np residues (Section 2.2, the recovery through
  the Chinese remaindering of Section 4): 6 per residue (its Shoup product with
  (P/p_k)^{-1}), 2 per word of each of the np products y_k (P/p_k) summed over W
  words (multiply-add and carry), and 4 per word for the quotient correction and
  the shifted accumulation at 2^(Mj).  Up to 20 primes the kernel forms the sum
  sum_k y_k (P/p_k) - t P on the int8 matrix cores: each 32 x 32-bit word product
  is 16 byte products, 2 int8 operations each, counted against the int8 matrix
  peak instead of the int32 one.

HBM bytes are the compulsory reads and writes of each launch (every element in
and out once).
"""
from __future__ import annotations

import math

OPS_BFLY_DIF = 8
OPS_BFLY_DIT = 9
OPS_POINTWISE = 6
OPS_TWIDDLE = 3
INT32_PEAK = 256 * 64 * 2.4e9      # 256 CUs x 64 lanes x 2.4 GHz: int32 VALU op/s
HBM_PEAK = 8.0e12                   # bytes/s
MFMA_I8_PEAK = 5.0e15               # dense int8 matrix operations/s (published)
CRT_MFMA_NP = 20                    # prime counts whose CRT sum runs on the matrix cores


def kernel_work(plan: dict, name: str) -> dict:
    """{'ops': int32 ops per launch, 'bytes': HBM bytes per launch} for one kernel kind."""
    K, np_ = plan["K"], plan["np"]
    L = 1 << plan["log2_L"]
    logL1 = plan["log2_L1"]
    da, db = plan["da"], plan["db"]
    nout = da + db - 1
    logx = int(math.log2(2 * K))
    if name == "convolve_rows":
        logK = logx - 1
        # forward: the inner y factor on both operands' K rows, four K-point transforms
        # per position (cyclic and negacyclic, a and b); inverse: the inner y factor on
        # 2K rows, two K-point transforms per position
        dif = np_ * L * K * (logL1 + 2 * logK)
        dit = np_ * L * K * (logL1 + logK)
        twists = np_ * L * 3 * K               # theta^j on both operands, theta^-j after
        pw = np_ * 2 * K * L
        words_in = np_ * 2 * K * L
        return {"ops": dif * OPS_BFLY_DIF + dit * OPS_BFLY_DIT + twists * OPS_TWIDDLE
                + pw * OPS_POINTWISE, "bytes": 4 * 2 * words_in}
    if name in ("col_pass_fwd", "col_pass_inv"):
        # per launch = one pass; the mean over the passes.  The first forward pass
        # reads only the rows below da (db) of a's (b's) columns, the rest being zero.
        cols = plan["col_log2n"]
        npass = max(len(cols), 1)
        logn = sum(cols) / npass
        bfly = np_ * K * L * logn
        tw = np_ * 2 * K * L
        full = 4 * np_ * 2 * K * L
        if name == "col_pass_fwd":
            first_read = 4 * np_ * K * (min(da, L) + min(db, L))
            read = (first_read + (npass - 1) * full) / npass
        else:
            read = full
        ob = OPS_BFLY_DIF if name == "col_pass_fwd" else OPS_BFLY_DIT
        return {"ops": bfly * ob + tw * OPS_TWIDDLE, "bytes": read + full}
    if name == "bivariate_representation":
        # per launch = one operand; the mean of the two
        w = ((plan["Na"] + 63) // 64 * da + (plan["Nb"] + 63) // 64 * db) / 2
        d = (da + db) / 2
        words = (plan["M"] + 31) // 32
        return {"ops": d * K * np_ * (2 * words + 6), "bytes": 8 * w + 4 * np_ * K * d}
    if name == "recovering_product":
        wc = (plan["nout_bits"] + 63) // 64
        W = plan["W"]
        nvals = (2 * K - 1) * nout
        byts = 4 * np_ * (2 * K - 1) * nout + 8 * nout * wc
        if np_ <= CRT_MFMA_NP:
            return {"ops": nvals * (6 * np_ + 4 * W), "mfma_ops": nvals * np_ * W * 32,
                    "bytes": byts}
        return {"ops": nvals * (6 * np_ + 2 * np_ * W + 4 * W), "bytes": byts}
    return {"ops": 0, "bytes": 0}


def kernel_time(w: dict, bw: float = None, alu: float = None) -> float:
    """Roofline time (s) of one launch: the largest of its HBM, int32 VALU and int8
    matrix times."""
    return max(w["bytes"] / (bw or HBM_PEAK), (w.get("ops") or 0) / (alu or INT32_PEAK),
               (w.get("mfma_ops") or 0) / MFMA_I8_PEAK)


KERNELS = ("bivariate_representation", "col_pass_fwd", "convolve_rows", "col_pass_inv",
           "recovering_product")


def launches(plan: dict, name: str, square: bool = False) -> int:
    """Launches of one kernel kind in one product of this plan."""
    if name == "bivariate_representation":
        return 1 if square else 2
    if name in ("col_pass_fwd", "col_pass_inv"):
        return len(plan["col_log2n"])
    return 1


def t_star(plan: dict, bw: float = None, alu: float = None, square: bool = False) -> float:
    """Roofline time (s) of one product: the sum over its launches of
    max(bytes / bandwidth, ops / ALU rate, int8 matrix ops / matrix rate)."""
    bw = bw or HBM_PEAK
    alu = alu or INT32_PEAK
    t = 0.0
    for k in KERNELS:
        n = launches(plan, k, square)
        if n:
            t += n * kernel_time(kernel_work(plan, k), bw, alu)
    return t


def gfp_work(info: dict, name: str) -> dict:
    """Algorithmic work of the generalized Fermat prime variant per product: generic
    products in Z/pZ (k^2 digit multiply-adds each) and HBM bytes, per kernel group.
    Products: the twiddles between y-passes (on every column of each pass but the
    innermost, both directions) and the 2K L pointwise products."""
    k, K = info["k"], info["K"]
    L = 1 << info["log2_L"]
    da, db = info["da"], info["db"]
    nout = da + db - 1
    npass = info["npass"]
    el = 4 * k                                   # bytes of one element
    full = el * 2 * K * L
    wc = (info["nout_bits"] + 63) // 64
    if name == "gfp_convert_in":
        words = ((info["Na"] + 63) // 64) * da + ((info["Nb"] + 63) // 64) * db
        return {"products": 0, "bytes": 8 * words + el * K * (da + db)}
    if name == "gfp_y_fwd":
        rows = el * K * (da + db)
        return {"products": 2 * K * L * max(npass - 1, 0),
                "bytes": (rows + full + 2 * full * (npass - 1)) if npass else 0}
    if name == "gfp_x_convolve":
        return {"products": 2 * K * L, "bytes": 2 * full}
    if name == "gfp_y_inv":
        return {"products": 2 * K * L * max(npass - 1, 0),
                "bytes": (2 * full * (npass - 1) + full + el * 2 * K * nout) if npass else 0}
    if name == "gfp_recover":
        return {"products": 0, "bytes": el * 2 * K * nout + 8 * nout * wc}
    return {"products": 0, "bytes": 0}


def product_bits(da: int, Na: int, db: int, Nb: int) -> int:
    """Output coefficient-bits of one product: (da + db - 1) * Nout."""
    t = min(da, db)
    nout_bits = Na + Nb - 1 + t.bit_length()
    return (da + db - 1) * nout_bits
