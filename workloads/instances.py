"""Seeded synthetic inputs: random k-NAE-SAT instances and QAOA angles.

This module is shared by the GPU path's tests and benchmark and by the oracle's
tests. It holds no QAOA or cost arithmetic: it only draws clauses and angles.

Random clause model F_k(n, m) (Section 2.3): every clause picks k distinct
variables uniformly and negates each with probability 1/2, clauses i.i.d.
CNF(n, k, r) (Definition 3.1) draws m ~ Poisson(r n); the fixed workloads use
m = floor(r n + 1/2) instead. Literals are DIMACS-style: +(v+1) is x_v and
-(v+1) is NOT x_v.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def clause_count(n: int, r) -> int:
    """m = floor(r * n + 1/2), computed exactly from the decimal value of r
    (for r = 2.1 this is (21 n + 5) div 10)."""
    fr = Fraction(str(r))
    return int((fr * n + Fraction(1, 2)) // 1)


def random_clauses(n: int, k: int, m: int, rng: np.random.Generator) -> np.ndarray:
    """m clauses of F_k(n, m) as an int32 [m, k] literal array."""
    if not (1 <= k <= n):
        raise ValueError(f"need 1 <= k <= n, got k={k}, n={n}")
    out = np.empty((m, k), dtype=np.int32)
    for i in range(m):
        v = rng.choice(n, k, replace=False)
        neg = rng.integers(0, 2, k)
        out[i] = np.where(neg == 1, -(v + 1), v + 1)
    return out


def instance(n: int, k: int, m: int, seed: int) -> np.ndarray:
    """The instance drawn from PCG64(seed): clauses first in the stream."""
    return random_clauses(n, k, m, np.random.Generator(np.random.PCG64(seed)))


def poisson_instance(n: int, k: int, r: float, seed: int) -> np.ndarray:
    """CNF(n, k, r) of Definition 3.1: m ~ Poisson(r n), then F_k(n, m)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = int(rng.poisson(r * n))
    return random_clauses(n, k, m, rng)


def cnf_instance(n: int, k: int, r: float, seed: int) -> np.ndarray:
    """CNF(n, k, r) of Definition 3.1 drawn with whole-array operations (for
    large ensembles): m ~ Poisson(r n); a clause's k distinct variables are
    the first k of an independent uniform permutation of the n variables;
    signs Bernoulli(1/2). Same distribution as poisson_instance, different
    random stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = int(rng.poisson(r * n))
    if not (1 <= k <= n):
        raise ValueError(f"need 1 <= k <= n, got k={k}, n={n}")
    v = rng.permuted(np.tile(np.arange(n, dtype=np.int32), (m, 1)), axis=1)[:, :k]
    neg = rng.integers(0, 2, (m, k))
    return np.where(neg == 1, -(v + 1), v + 1).astype(np.int32)


def ramp_angles(p: int):
    """Linear ramp gamma_l = 0.5 l / p, beta_l = 0.5 (1 - l / p), l = 1 .. p."""
    l = np.arange(1, p + 1, dtype=np.float64)
    return 0.5 * l / p, 0.5 * (1.0 - l / p)


def random_angles(p: int, rng: np.random.Generator):
    """gamma_l, beta_l ~ U(0, pi), drawn gamma first."""
    g = rng.uniform(0.0, np.pi, p)
    b = rng.uniform(0.0, np.pi, p)
    return g, b


# ---------------------------------------------------------------------------
# Fixed workloads. Each is seeded; the satisfiable-instance seeds for the
# single-instance workloads are chosen once by ``oracle/make_golden.py`` and
# stored in ``tests/golden/workloads.json``.
# ---------------------------------------------------------------------------

SINGLE_WORKLOADS = {
    # name: (n, k, r, p, angle recipe)
    "nae3_n12_p3": (12, 3, 2.1, 3, "ramp"),
    "nae3_n24_p10": (24, 3, 2.1, 10, "ramp"),
    "nae3_n28_p10": (28, 3, 2.1, 10, "ramp"),
    "nae3_n30_p10": (30, 3, 2.1, 10, "ramp"),
    "nae3_n22_p12": (22, 3, 2.1, 12, "ramp"),
}


def batched_workload(count: int = 512, seed: int = 0, n_lo: int = 10, n_hi: int = 20, p: int = 5):
    """Ragged batch: k ~ U{3, 5}; n ~ U{n_lo .. n_hi}; m = round(2.1 n) for
    k = 3 and 9 n for k = 5; p layers with angles U(0, pi). Instance i draws
    from PCG64(seed * 1_000_003 + i): k, n, then clauses, then angles."""
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(seed * 1_000_003 + i))
        k = int(rng.choice([3, 5]))
        n = int(rng.integers(n_lo, n_hi + 1))
        m = clause_count(n, 2.1 if k == 3 else 9.0)
        cl = random_clauses(n, k, m, rng)
        g, b = random_angles(p, rng)
        out.append({"n": n, "k": k, "m": m, "p": p, "clauses": cl, "gammas": g, "betas": b})
    return out


def serving_workload(count: int = 2000, seed: int = 0, rate: float = 200.0,
                     n_lo: int = 14, n_hi: int = 26, p_lo: int = 2, p_hi: int = 20):
    """Poisson request stream: exponential gaps of mean 1/rate seconds; each
    request is a random 3- or 5-NAE-SAT instance (r = 2.1 or 9.0) with
    n ~ U{n_lo .. n_hi}, p ~ U{p_lo .. p_hi} and angles U(0, pi)."""
    arr_rng = np.random.Generator(np.random.PCG64(seed))
    gaps = arr_rng.exponential(1.0 / rate, count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64((seed + 1) * 7_000_003 + i))
        k = int(rng.choice([3, 5]))
        n = int(rng.integers(n_lo, n_hi + 1))
        p = int(rng.integers(p_lo, p_hi + 1))
        m = clause_count(n, 2.1 if k == 3 else 9.0)
        cl = random_clauses(n, k, m, rng)
        g, b = random_angles(p, rng)
        out.append({"arrival_s": float(t[i]), "n": n, "k": k, "m": m, "p": p,
                    "clauses": cl, "gammas": g, "betas": b})
    return out


# Cost diagonals compared in full against the oracle, by chunk digests
# (``oracle/make_digests.py`` writes ``tests/golden/cost_digests.json``):
# name: (n, k, r, predicate). Names that are single workloads above use that
# workload's satisfiable seed; the others use seed 0.
DIGEST_WORKLOADS = {
    "nae3_n24_p10": (24, 3, 2.1, "nae"),
    "nae3_n28_p10": (28, 3, 2.1, "nae"),
    "nae3_n30_p10": (30, 3, 2.1, "nae"),
    "sat3_n30": (30, 3, 4.2, "sat"),        # k-SAT predicate, m = 126
    "nae5_n30_u16": (30, 5, 9.0, "nae"),    # m = 270 > 255: uint16 diagonal
    "nae3_n33": (33, 3, 2.1, "nae"),        # 64-bit basis indices (n > 32), 8 GiB
}
