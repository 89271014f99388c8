"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: the cost diagonal is compared bit for bit; p_succ to an absolute
1e-5 and E[C] to a relative 1e-5 (complex64 state, FP32 arithmetic with FP64
final sums). Where p_succ is not tiny its relative error is checked too, and
the norm must stay within 1e-5 of 1.
"""
import math
import os

import numpy as np
import pytest

import oracle
from workloads import instances as inst

pytestmark = pytest.mark.gpu

P_ABS = 1e-5
E_REL = 1e-5


@pytest.fixture(scope="module")
def q():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2401_02852_amd as q
    q.load_library()
    return q


def gpu_cost(q, cl, n, count=False):
    return q.build_cost_diagonal(cl, n, count_solutions=count)


def check_result(got, ref, what=""):
    ps, e, norm = got
    rps, re_, rnorm = ref
    assert abs(ps - rps) <= P_ABS, f"{what} p_succ {ps} vs {rps}"
    assert abs(e - re_) <= E_REL * max(abs(re_), 1e-12) + 1e-9, f"{what} E[C] {e} vs {re_}"
    assert abs(norm - 1.0) <= 1e-5, f"{what} norm {norm}"
    if rps > 1e-3:
        assert abs(ps - rps) <= 1e-4 * rps, f"{what} relative p_succ {ps} vs {rps}"


# ---------------------------------------------------------------------------
# Cost diagonal: bit-exact
# ---------------------------------------------------------------------------

COST_CASES = [
    # n, k, m, seed
    (1, 1, 1, 0), (2, 2, 3, 1), (3, 3, 0, 2), (4, 2, 9, 3), (5, 3, 11, 4), (6, 4, 13, 5),
    (7, 1, 4, 6), (9, 5, 30, 7), (12, 3, 25, 8), (13, 5, 117, 9), (16, 3, 34, 10),
    (17, 7, 200, 11), (20, 5, 180, 12), (20, 3, 42, 13),
]


@pytest.mark.parametrize("n,k,m,seed", COST_CASES)
def test_cost_bit_exact(q, n, k, m, seed):
    cl = inst.instance(n, k, m, seed).reshape(m, k)
    c, sols = gpu_cost(q, cl, n, count=True)
    ref = oracle.cost(cl, n)
    assert np.array_equal(c.cpu().numpy().astype(np.int64), ref)
    assert sols == int((ref == 0).sum())


def test_cost_uint16_bit_exact(q):
    import torch
    n, k, m = 15, 3, 300   # m > 255 forces uint16
    cl = inst.instance(n, k, m, 21)
    c = gpu_cost(q, cl, n)
    assert c.dtype == torch.uint16
    ref = oracle.cost(cl, n)
    assert np.array_equal(c.cpu().numpy().astype(np.int64), ref)


def test_cost_uint16_forced_small_m(q):
    import torch
    n, k, m = 11, 3, 23
    cl = inst.instance(n, k, m, 22)
    out = torch.empty(1 << n, dtype=torch.uint16, device="cuda")
    c = q.build_cost_diagonal(cl, n, out=out)
    assert np.array_equal(c.cpu().numpy().astype(np.int64), oracle.cost(cl, n))


def test_cost_repeated_variables(q):
    n = 8
    cl = np.array([[1, -1, 2], [3, 3, -4], [2, 4, 4], [5, 6, 7], [-8, -8, -8]], dtype=np.int32)
    c = gpu_cost(q, cl, n)
    assert np.array_equal(c.cpu().numpy().astype(np.int64), oracle.cost(cl, n))


@pytest.mark.parametrize("n", [33, 34])
def test_cost_wide_index_sampled(q, n):
    """n > 32 uses 64-bit basis indices: check sampled states at the top of
    the range (uint8, 8 or 16 GiB)."""
    import torch
    free, _ = torch.cuda.mem_get_info()
    if free < (1 << n) + (1 << 30):
        pytest.skip("not enough device memory")
    k, m = 3, 40
    cl = inst.instance(n, k, m, 30 + n)
    c = gpu_cost(q, cl, n)
    rng = np.random.default_rng(n)
    xs = np.concatenate([rng.integers(0, 1 << n, 2000, dtype=np.uint64),
                         np.arange((1 << n) - 64, 1 << n, dtype=np.uint64)])
    got = c[torch.from_numpy(xs.astype(np.int64)).cuda()].cpu().numpy().astype(np.int64)
    assert np.array_equal(got, oracle.cost_at(cl, n, xs))
    del c
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# QAOA readout
# ---------------------------------------------------------------------------

def run_pair(q, cl, n, m, g, b, **kw):
    c = gpu_cost(q, cl, n)
    got = q.qaoa_run(c, n, m, g, b, **kw)
    ref = oracle.qaoa(oracle.cost(cl, n), n, g, b)
    return got, ref


ANGLE_SETS = ["ramp", "ramp_min", "random", "large_beta"]


def angles(kind, p, seed):
    rng = np.random.default_rng(seed)
    if kind == "ramp":
        return inst.ramp_angles(p)
    if kind == "ramp_min":
        g, b = inst.ramp_angles(p)
        return g, -b
    if kind == "random":
        return rng.uniform(0, np.pi, p), rng.uniform(0, np.pi, p)
    # |tan(beta)| > 1 on every layer: exercises the swapped butterfly form
    return rng.uniform(-2, 2, p), rng.uniform(0.9, 2.2, p) * rng.choice([-1, 1], p)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 11, 13, 14])
@pytest.mark.parametrize("kind", ANGLE_SETS)
def test_qaoa_resident(q, n, kind):
    k = min(3, n)
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, k, m, 100 + n)
    g, b = angles(kind, 4, n)
    got, ref = run_pair(q, cl, n, m, g, b)
    check_result(got, ref, f"n={n} {kind}")


@pytest.mark.parametrize("p", [17, 18])
def test_qaoa_resident_table_paths(q, p):
    """n = 11, m = 23: 17 layers of 24-entry tables plus their mixer forms
    (425 slots) travel in the kernel arguments, 18 layers (450) are copied
    to the device first; both against the oracle."""
    n = 11
    m = inst.clause_count(n, 2.1)
    assert p * (m + 1) + p == (425 if p == 17 else 450)
    cl = inst.instance(n, 3, m, 300)
    g, b = angles("random", p, 7 + p)
    got, ref = run_pair(q, cl, n, m, g, b)
    check_result(got, ref, f"n={n} p={p}")


@pytest.mark.parametrize("n", [15, 17, 20, 22])
@pytest.mark.parametrize("kind", ANGLE_SETS)
@pytest.mark.parametrize("p", [1, 2, 5])
def test_qaoa_sweeps(q, n, kind, p):
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 200 + n)
    g, b = angles(kind, p, n + p)
    got, ref = run_pair(q, cl, n, m, g, b)
    check_result(got, ref, f"n={n} p={p} {kind}")


@pytest.mark.parametrize("tb", [12, 13, 14])
@pytest.mark.parametrize("n", [16, 21, 25])
def test_qaoa_tile_sizes(q, tb, n, monkeypatch):
    """Every tile size the planner can choose, with 1, 2 and 3 high groups."""
    monkeypatch.setenv("QNAE_TILE_BITS", str(tb))
    ctx = q.Context()
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 300 + n)
    g, b = angles("random", 3, tb + n)
    c = gpu_cost(q, cl, n)
    got = q.qaoa_run(c, n, m, g, b, ctx=ctx)
    ref = oracle.qaoa(oracle.cost(cl, n), n, g, b)
    check_result(got, ref, f"tb={tb} n={n}")
    ctx.close()


def test_qaoa_k5_uint16(q):
    n, k = 16, 5
    m = 300
    cl = inst.instance(n, k, m, 41)
    g, b = angles("random", 3, 41)
    got, ref = run_pair(q, cl, n, m, g, b)
    check_result(got, ref, "u16")


@pytest.mark.parametrize("n", [6, 18])
def test_qaoa_p0_and_degenerate(q, n):
    """p = 0 reads out |+>; m = 0 gives C = 0 (p_succ = 1); k = 1 clauses are
    always violated (p_succ = 0)."""
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 7)
    c = gpu_cost(q, cl, n)
    got = q.qaoa_run(c, n, m, [], [])
    ref = oracle.qaoa(oracle.cost(cl, n), n, [], [])
    check_result(got, ref, "p=0")
    empty = np.zeros((0, 3), dtype=np.int32)
    c0 = gpu_cost(q, empty, n)
    r0 = q.qaoa_run(c0, n, 0, [0.3, 0.9], [0.2, -0.7])
    assert abs(r0.p_success - 1) < 1e-5 and r0.expected_cost == 0.0
    k1 = np.array([[1], [-2], [3]], dtype=np.int32)
    c1 = gpu_cost(q, k1, n)
    r1 = q.qaoa_run(c1, n, 3, [0.3, 0.9], [0.2, -0.7])
    assert r1.p_success == 0.0 and abs(r1.expected_cost - 3) < 3e-5


@pytest.mark.parametrize("n", [10, 14, 19])
def test_final_state_matches_oracle(q, n):
    import torch
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 55)
    g, b = angles("random", 3, 55)
    c = gpu_cost(q, cl, n)
    st = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    got = q.qaoa_run(c, n, m, g, b, state=st)
    ref_state = oracle.state(oracle.cost(cl, n), n, g, b)
    diff = np.abs(st.cpu().numpy().astype(np.complex128) - ref_state)
    assert diff.max() < 2e-6 * 2 ** (-n / 2) * 64
    check_result(got, oracle.qaoa(oracle.cost(cl, n), n, g, b), "state")


def test_repeat_deterministic(q):
    n = 21
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 3)
    c = gpu_cost(q, cl, n)
    g, b = angles("random", 4, 3)
    r = [q.qaoa_run(c, n, m, g, b) for _ in range(3)]
    assert r[0] == r[1] == r[2]


# ---------------------------------------------------------------------------
# Full-size workloads (stored oracle results; 28 and 30 qubits)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["nae3_n12_p3", "nae3_n22_p12", "nae3_n24_p10", "nae3_n28_p10", "nae3_n30_p10"])
def test_workloads_vs_stored_oracle(q, golden, name):
    import torch
    rec = golden[name]
    n, k, m, p = rec["n"], rec["k"], rec["m"], rec["p"]
    cl = inst.instance(n, k, m, rec["seed"])
    c, sols = gpu_cost(q, cl, n, count=True)
    assert sols == rec["num_solutions"]
    # integer identities of the full diagonal: total cost and the flip symmetry
    assert int(c.to(torch.int64).sum().item()) == m * 2 ** (n + 1 - k)
    assert torch.equal(c, c.flip(0))
    # sampled states against the oracle, one by one
    rng = np.random.default_rng(n)
    xs = rng.integers(0, 1 << n, 4096, dtype=np.uint64)
    got = c[torch.from_numpy(xs.astype(np.int64)).cuda()].cpu().numpy().astype(np.int64)
    assert np.array_equal(got, oracle.cost_at(cl, n, xs))
    for recipe, ref in rec["results"].items():
        g, b = inst.ramp_angles(p)
        if recipe == "ramp_min":
            b = -b
        r = q.qaoa_run(c, n, m, g, b)
        check_result(r, (ref["p_success"], ref["expected_cost"], ref["norm"]), f"{name}/{recipe}")
    del c
    torch.cuda.empty_cache()


def test_n30_workload_every_tile_shape(q, golden):
    """The n = 30 workload (the benchmark's step) under every tile shape the
    autotuner may choose (and every group split), against the stored oracle
    values: the timed launch configuration is covered whichever shape it
    keeps."""
    import torch
    rec = golden["nae3_n30_p10"]
    n, k, m, p = rec["n"], rec["k"], rec["m"], rec["p"]
    free, _ = torch.cuda.mem_get_info()
    if free < (10 << 30):
        pytest.skip("not enough device memory")
    cl = inst.instance(n, k, m, rec["seed"])
    ctx = q.Context()
    c = q.build_cost_diagonal(cl, n, ctx=ctx)
    ref = rec["results"]["ramp_min"]
    g, b = inst.ramp_angles(p)
    shapes = [(tb, low, page, 0) for tb in (12, 13, 14) for low in (4, 5, 6) for page in (18, 64)]
    shapes += [(tb, 4, 18, split) for tb in (12, 13, 14) for split in (1, 2, 3)]
    for tb, low, page, split in shapes:
        ctx.set_tune(n, {"tile_bits": tb, "low_run_bits": low, "page_bit": page, "split": split})
        r = q.qaoa_run(c, n, m, g, -b, ctx=ctx)
        check_result(r, (ref["p_success"], ref["expected_cost"], ref["norm"]), f"shape {tb}/{low}/{page}/{split}")
    ctx.close()
    del c
    torch.cuda.empty_cache()


def test_u16_costs_every_tile_size(q):
    """16-bit cost values (m = 300) at n = 25 under 12-, 13- and 14-bit tiles
    (three qubit groups with 13- and 14-bit tiles) and each group split, in
    every sweep kind (first, middle, boundary, final; tiles through layout
    L1 and not), against the oracle's readout: the uint16 cost reads and
    their packing into registers."""
    import torch
    n, m, p = 25, 300, 2
    cl = inst.instance(n, 3, m, 6)
    ctx = q.Context()
    c = q.build_cost_diagonal(cl, n, ctx=ctx)
    assert str(c.dtype) == "torch.uint16"
    rng = np.random.default_rng(25)
    g, b = rng.uniform(0, 0.1, p), np.array([0.35, 1.3])
    ref = oracle.qaoa(oracle.cost(cl, n), n, g, b)
    for tb, split in [(12, 0), (13, 0), (13, 1), (13, 3), (14, 0), (14, 1), (14, 2)]:
        ctx.set_tune(n, {"tile_bits": tb, "low_run_bits": 4, "page_bit": 18, "split": split}, "u16")
        check_result(q.qaoa_run(c, n, m, g, b, ctx=ctx), ref, f"shape {tb}/4/18/{split}")
    ctx.close()
    del c
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [24, 30, 33, 34])
def test_ring_closed_form_at_scale(q, n):
    """k = 2 ring of all-positive clauses at p = 1:
    E[C] = n/2 (1 + sin(4 beta) sin(2 gamma) / 2) (graph closed form).
    n = 33 and 34 (the largest n the library takes): 2^33 and 2^34
    amplitudes (64 and 128 GiB of state, 8 and 16 GiB of cost) through 64-bit
    indices in every sweep kind, on a context of their own that is closed
    afterwards."""
    import torch
    if n > 33:
        free, _ = torch.cuda.mem_get_info()
        if free < (150 << 30):
            pytest.skip("not enough device memory for a 2^34-amplitude state")
    ctx = q.Context(0) if n > 32 else None
    try:
        cl = np.array([[i + 1, (i + 1) % n + 1] for i in range(n)], dtype=np.int32)
        c = q.build_cost_diagonal(cl, n, ctx=ctx)
        for g, b in [(0.37, 0.21), (-1.1, 0.6), (2.0, 1.2)]:
            r = q.qaoa_run(c, n, n, [g], [b], ctx=ctx)
            ref = n / 2 * (1 + 0.5 * math.sin(4 * b) * math.sin(2 * g))
            assert abs(r.expected_cost - ref) <= E_REL * ref
            assert abs(r.norm - 1) < 1e-5
            if n % 2:  # odd ring: no 2-colouring, no state satisfies every clause
                assert r.p_success == 0.0
        del c
    finally:
        if ctx is not None:
            ctx.close()
        torch.cuda.empty_cache()


def test_default_context_per_thread(q):
    """Calls on one context must not overlap, so each thread's default
    context is its own: two threads solving at once (n = 18 and 20, tiled
    path) give the same results as one thread solving both in turn."""
    import threading
    a = q.default_context()
    assert q.default_context() is a
    jobs = []
    for n, seed in ((18, 1), (20, 2)):
        m = inst.clause_count(n, 2.1)
        cl = inst.instance(n, 3, m, seed)
        g, b = inst.ramp_angles(6)
        jobs.append((n, m, cl, g, -b))
    c0 = q.Context()  # untuned, like the threads' new default contexts
    alone = []
    for n, m, cl, g, b in jobs:
        alone.append(tuple(q.qaoa_run(q.build_cost_diagonal(cl, n, ctx=c0), n, m, g, b, ctx=c0)))
    got, ctxs, errors = [None, None], [None, None], []

    def worker(i):
        try:
            n, m, cl, g, b = jobs[i]
            ctxs[i] = q.default_context()
            for _ in range(5):
                got[i] = tuple(q.qaoa_run(q.build_cost_diagonal(cl, n), n, m, g, b))
        except Exception as e:  # reported on the main thread
            errors.append(e)

    th = [threading.Thread(target=worker, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    assert ctxs[0] is not ctxs[1] and a not in ctxs
    for g_, a_ in zip(got, alone):
        assert g_ == a_


@pytest.mark.parametrize("case", ["gamma0_tan", "gamma0_cot", "gamma0_mixed", "beta0", "beta_half_pi"])
def test_random_assignment_special_cases_n30(q, golden, case):
    """App. B at full size: with every gamma = 0 the state stays |+> up to a
    global phase (X_j |+> = |+>), and with every beta = 0 (or beta = pi/2,
    where the mixer is a phase times the global flip, under which the NAE
    cost is symmetric) only phases act. Either way |psi(x)|^2 = 2^-n, so
    p_succ = #solutions / 2^n and E[C] = m 2^(1-k). The gamma = 0 cases run
    the tan form (|tan beta| <= 1), the cot form (|tan beta| > 1, X tracked
    as a relabelling with complemented cost reads) and both mixed."""
    import torch
    rec = golden["nae3_n30_p10"]
    n, k, m = rec["n"], rec["k"], rec["m"]
    free, _ = torch.cuda.mem_get_info()
    if free < (10 << 30):
        pytest.skip("not enough device memory")
    rng = np.random.default_rng(7)
    p = 6
    if case == "gamma0_tan":
        g, b = np.zeros(p), rng.uniform(-0.7, 0.7, p)
    elif case == "gamma0_cot":
        g, b = np.zeros(p), rng.uniform(0.9, 2.2, p) * rng.choice([-1, 1], p)
    elif case == "gamma0_mixed":
        g, b = np.zeros(p), np.array([0.3, 1.2, -0.9, 2.0, -0.2, 1.5])
    elif case == "beta0":
        g, b = rng.uniform(-3, 3, p), np.zeros(p)
    else:
        g, b = rng.uniform(-3, 3, p), np.array([np.pi / 2, 0.0, -np.pi / 2, np.pi / 2, 0.0, np.pi / 2])
    cl = inst.instance(n, k, m, rec["seed"])
    c = gpu_cost(q, cl, n)
    r = q.qaoa_run(c, n, m, g, b)
    want_p = rec["num_solutions"] / 2 ** n
    want_e = m * 2.0 ** (1 - k)
    assert abs(r.p_success - want_p) <= 1e-5 * want_p, (r, want_p)
    assert abs(r.expected_cost - want_e) <= E_REL * want_e, (r, want_e)
    assert abs(r.norm - 1.0) <= 1e-5
    del c
    torch.cuda.empty_cache()
