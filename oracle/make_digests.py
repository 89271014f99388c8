"""Write ``tests/golden/cost_digests.json``: SHA-256 digests of whole cost
diagonals computed by the oracle, for comparison with the GPU's diagonals
at full size.

TEST INFRASTRUCTURE. Calls only the oracle (and the seeded input generator).

For each workload of ``workloads.instances.DIGEST_WORKLOADS`` the diagonal
C(x), x = 0 .. 2^n - 1 (Section 3.2, eq. knaesatobj, or the k-SAT predicate
of Section 2.2) is evaluated by ``oracle.cost_at`` in chunks of 2^24
consecutive states, in natural index order. Each chunk's values, as
little-endian uint8 when m <= 255 and uint16 otherwise (the GPU cost types),
are hashed on their own (the first 16 hex digits of their SHA-256 locate a
mismatch) and into one SHA-256 of the whole diagonal. The zero count is
stored beside them. n = 33 takes several minutes on 8 threads.

    python -m oracle.make_digests [name ...]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

import oracle
from workloads import instances as inst

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "tests", "golden", "cost_digests.json")
WORKLOADS = os.path.join(ROOT, "tests", "golden", "workloads.json")
CHUNK_LOG2 = 24


def seed_of(name):
    if name in inst.SINGLE_WORKLOADS:
        with open(WORKLOADS) as f:
            return json.load(f)[name]["seed"]
    return 0


def digest(name):
    n, k, r, pred = inst.DIGEST_WORKLOADS[name]
    m = inst.clause_count(n, r)
    seed = seed_of(name)
    cl = inst.instance(n, k, m, seed)
    dtype = np.uint8 if m <= 255 else np.uint16
    lg = min(CHUNK_LOG2, n)
    whole = hashlib.sha256()
    chunks, zeros, total = [], 0, 0
    t0 = time.time()
    for i in range(1 << (n - lg)):
        xs = np.arange(i << lg, (i + 1) << lg, dtype=np.uint64)
        c = oracle.cost_at(cl, n, xs, predicate=pred)
        assert c.min() >= 0 and c.max() <= m
        b = c.astype("<u1" if dtype == np.uint8 else "<u2").tobytes()
        whole.update(b)
        chunks.append(hashlib.sha256(b).hexdigest()[:16])
        zeros += int((c == 0).sum())
        total += int(c.sum(dtype=np.int64))
    rec = {"n": n, "k": k, "r": r, "m": m, "seed": seed, "predicate": pred,
           "dtype": "uint8" if dtype == np.uint8 else "uint16", "chunk_log2": lg,
           "sha256": whole.hexdigest(), "chunks": chunks, "num_zeros": zeros, "sum": total,
           "oracle_seconds": round(time.time() - t0, 1), "oracle_threads": oracle.num_threads()}
    print(name, {k_: v for k_, v in rec.items() if k_ != "chunks"}, flush=True)
    return rec


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names or list(inst.DIGEST_WORKLOADS):
        data[name] = digest(name)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
