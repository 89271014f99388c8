"""Write ``tests/golden/workloads.json``: the satisfiable seed of every fixed
single-instance workload and the oracle's readout on it.

TEST INFRASTRUCTURE. Calls only the oracle (and the seeded input generator).

For each workload (n, k, r, p, ramp angles) the seeds 0, 1, 2, ... are tried in
order and the first instance with at least one NAE solution is kept (the paper
evaluates satisfiable instances only, Section 3.3; the satisfiability check is
an exact brute-force count here). The oracle then evaluates p_succ, E[C] and
the norm at the workload's angles. Large n takes minutes (n = 30 holds a
16 GiB FP64 state), so workloads can be chosen on the command line; existing
entries for other workloads are kept.

    python -m oracle.make_golden nae3_n12_p3 nae3_n22_p12 ...
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

import oracle
from workloads import instances as inst

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "tests", "golden", "workloads.json")


def first_satisfiable(n, k, m, start=0):
    seed = start
    while True:
        cl = inst.instance(n, k, m, seed)
        sols = oracle.count_solutions(cl, n)
        if sols > 0:
            return seed, cl, sols
        seed += 1


def angles(recipe, p):
    """'ramp' is the workload's linear ramp; 'ramp_min' negates every beta,
    which under exp(-i beta H_B) turns the ramp towards lower cost."""
    g, b = inst.ramp_angles(p)
    if recipe == "ramp_min":
        b = -b
    return g, b


def run(name, old=None):
    n, k, r, p, recipe = inst.SINGLE_WORKLOADS[name]
    m = inst.clause_count(n, r)
    t0 = time.time()
    if old and old.get("m") == m and "seed" in old:
        seed = old["seed"]
        cl = inst.instance(n, k, m, seed)
        sols = old["num_solutions"]
    else:
        seed, cl, sols = first_satisfiable(n, k, m)
    cost = oracle.cost(cl, n)
    rec = {"n": n, "k": k, "r": r, "m": m, "p": p, "seed": seed, "num_solutions": sols,
           "oracle_threads": oracle.num_threads(), "results": {}}
    for rcp in ("ramp", "ramp_min"):
        g, b = angles(rcp, p)
        ps, e, norm = oracle.qaoa(cost, n, g, b)
        rec["results"][rcp] = {"p_success": ps, "expected_cost": e, "norm": norm}
    del cost
    rec["oracle_seconds"] = round(time.time() - t0, 1)
    print(name, rec, flush=True)
    return rec


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names or list(inst.SINGLE_WORKLOADS):
        data[name] = run(name, data.get(name))
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
