"""Algorithmic work per kernel launch, for roofline reporting.

Counts are what the method itself must do for a plan (Section 3.3: K
transforms of length L along y for each operand and 2K inverse ones; along x,
per y-frequency, a cyclic and a negacyclic convolution of length K, i.e. three
K-point transforms each, plus the twist by theta^j before the negacyclic
forward transforms and the untwist after its inverse), not what a particular
kernel happens to execute (the kernels run the x part as 2K-point transforms
whose first stage is the twist):

* one radix-2 butterfly = 11 int32 VALU operations (Shoup product: 2 mul_lo,
  1 mul_hi, 1 sub, 2 for the final reduction; modular add 3; modular sub 2);
* one pointwise product = 13 (Montgomery product 7, Shoup scaling 6);
* one four-step twiddle product = 6 (Shoup product with reduction).

HBM bytes are the compulsory reads and writes of each launch (every element in
and out once).
"""
from __future__ import annotations

import math

OPS_BFLY = 11
OPS_POINTWISE = 13
OPS_TWIDDLE = 6
INT32_PEAK = 256 * 64 * 2.4e9      # 256 CUs x 64 lanes x 2.4 GHz: int32 VALU op/s
HBM_PEAK = 8.0e12                   # bytes/s


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
        bfly = np_ * L * K * (2 * logL1 + 3 * logK)
        twists = np_ * L * 3 * K               # theta^j on both operands, theta^-j after
        pw = np_ * 2 * K * L
        words_in = np_ * 2 * K * L
        return {"ops": bfly * OPS_BFLY + twists * OPS_TWIDDLE + pw * OPS_POINTWISE,
                "bytes": 4 * 2 * words_in}
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
        return {"ops": bfly * OPS_BFLY + tw * OPS_TWIDDLE, "bytes": read + full}
    if name == "bivariate_representation":
        # per launch = one operand; the mean of the two
        w = ((plan["Na"] + 63) // 64 * da + (plan["Nb"] + 63) // 64 * db) / 2
        d = (da + db) / 2
        return {"ops": 0, "bytes": 8 * w + 4 * np_ * K * d}
    if name == "recovering_product":
        wc = (plan["nout_bits"] + 63) // 64
        return {"ops": 0, "bytes": 4 * np_ * (2 * K - 1) * nout + 8 * nout * wc}
    return {"ops": 0, "bytes": 0}


def product_bits(da: int, Na: int, db: int, Nb: int) -> int:
    """Output coefficient-bits of one product: (da + db - 1) * Nout."""
    t = min(da, db)
    nout_bits = Na + Nb - 1 + t.bit_length()
    return (da + db - 1) * nout_bits
