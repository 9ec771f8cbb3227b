"""Writes digests.json: the SHA-256 of the oracle's full output for the named
workloads, so that a device run can be compared on every coefficient without
re-running a schoolbook product that takes many CPU-minutes.

Only the seeded generators and the oracle are used.  Output layout: the
(da+db-1, wc) little-endian uint64 words of the product, two's complement,
wc = ceil(out_bits / 64).

    python -m tests.golden.make_digests [workload ...]
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

WORKLOADS = {"int64_1k": lambda: synth.int64_1k(1), "bits4096_64k": lambda: synth.bits4096_64k(2)}


def digest(name: str) -> dict:
    p = WORKLOADS[name]()
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
    for name in argv or list(WORKLOADS):
        print(f"oracle: {name}", flush=True)
        out[name] = digest(name)
        print(json.dumps(out[name]), flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:])
