"""Writes digests.json: the SHA-256 of the oracle's full output for the named
workloads, so that a device run can be compared on every coefficient without
re-running a schoolbook product that takes many CPU-minutes.

Only the seeded generators and the oracle are used.  Output layout: the
(da+db-1, wc) little-endian uint64 words of the product, two's complement,
wc = ceil(out_bits / 64).

For bits16384_256k (2^18 coefficients of 16385 bits: about 4.5e15 word products,
out of reach of the exact schoolbook) the entry holds instead
* for each of two primes q below 2^61, the SHA-256 of the residues c_i mod q of all
  da+db-1 coefficients (little-endian uint64, from oracle.polymul_mod), and
* the exact oracle output of ROWS16K_COUNT seeded output rows (the first and last 32,
  da-1, da, the middle one and random ones): the row list and, per row, the SHA-256
  of its wc words.

    python -m tests.golden.make_digests [workload ...]   (default: int64_1k only;
    bits4096_64k takes about 53 CPU-minutes on 8 threads, bits16384_256k about 8)
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1612_05778_amd import synth  # noqa: E402

WORKLOADS = {"int64_1k": lambda: synth.int64_1k(1), "bits4096_64k": lambda: synth.bits4096_64k(2),
             "bits16384_256k": lambda: synth.bits16384_256k(3)}

RESIDUE_PRIMES = [2305843009213693951, 2305843009213693921]
ROWS16K_COUNT = 256


def rows16k(da: int, db: int) -> list[int]:
    """The seeded output rows whose exact values are stored for bits16384_256k."""
    import numpy as np
    nout = da + db - 1
    fixed = list(range(32)) + list(range(nout - 32, nout)) + [da - 1, da, nout // 2]
    rng = np.random.default_rng(16384)
    rest = [int(x) for x in rng.choice(nout, size=ROWS16K_COUNT, replace=False)]
    out = sorted(set(fixed))
    for x in rest:
        if len(out) >= ROWS16K_COUNT:
            break
        if x not in out:
            out.append(x)
    return sorted(out)


def digest_residues(p) -> dict:
    wc = (oracle.out_bits(p.da, p.Na, p.db, p.Nb) + 63) // 64
    t0 = time.time()
    res = {}
    for q in RESIDUE_PRIMES:
        r = oracle.polymul_mod(p.a, p.da, p.Na, p.b, p.db, p.Nb, q)
        res[str(q)] = hashlib.sha256(r.tobytes()).hexdigest()
    t1 = time.time()
    rows = rows16k(p.da, p.db)
    c = oracle.polymul_rows(p.a, p.da, p.Na, p.b, p.db, p.Nb, rows, wc=wc)
    t2 = time.time()
    return {"da": p.da, "Na": p.Na, "db": p.db, "Nb": p.Nb, "wc": wc,
            "residue_sha256": res,
            "rows": rows,
            "row_sha256": [hashlib.sha256(c[r].tobytes()).hexdigest() for r in range(len(rows))],
            "oracle_seconds": round(t2 - t0, 1), "residue_seconds": round(t1 - t0, 1),
            "oracle_threads": oracle.threads()}


def digest(name: str) -> dict:
    p = WORKLOADS[name]()
    if name == "bits16384_256k":
        return digest_residues(p)
    wc = (oracle.out_bits(p.da, p.Na, p.db, p.Nb) + 63) // 64
    t0 = time.time()
    c = oracle.polymul(p.a, p.da, p.Na, p.b, p.db, p.Nb, wc=wc)
    dt = time.time() - t0
    return {"da": p.da, "Na": p.Na, "db": p.db, "Nb": p.Nb, "wc": wc,
            "sha256": hashlib.sha256(c.tobytes()).hexdigest(),
            "oracle_seconds": round(dt, 1), "oracle_threads": oracle.threads()}


def main(argv):
    path = os.path.join(HERE, "digests.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    for name in argv or ["int64_1k"]:
        print(f"oracle: {name}", flush=True)
        out[name] = digest(name)
        print(json.dumps(out[name]), flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:])
