"""Sampling outcomes of the final state (Section 4.2, instance running time)
on the GPU, against the oracle's inverse cumulative distribution.

A draw is a floating-point decision: the GPU state is complex64, the oracle's
complex128, so outcomes are compared where the oracle's cumulative
distribution leaves a margin of 1e-5 (the p_succ tolerance: both are partial
sums of |psi|^2); every outcome must lie within that margin of its cell."""
import numpy as np
import pytest

import oracle
from workloads import instances as inst

pytestmark = pytest.mark.gpu
EPS = 1e-5


@pytest.fixture(scope="module")
def q():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2401_02852_amd as q
    q.load_library()
    return q


def check_against_oracle(psi_o, u, got):
    prob = np.abs(psi_o) ** 2
    cum = np.cumsum(prob) / prob.sum()
    lo = np.concatenate([[0.0], cum[:-1]])
    x = got.astype(np.int64)
    assert np.all(lo[x] - EPS <= u) and np.all(u <= cum[x] + EPS), "outcome outside its cell"
    ref = oracle.sample(psi_o, int(np.log2(len(psi_o))), u).astype(np.int64)
    clear = (lo[ref] + EPS < u) & (u < cum[ref] - EPS)
    assert np.array_equal(x[clear], ref[clear])
    return int(clear.sum())


@pytest.mark.parametrize("n", [1, 3, 8, 12, 13, 17, 20])
def test_sample_matches_oracle(q, n):
    import torch
    rng = np.random.default_rng(n)
    k = min(3, n)
    m = 2 * n + 1
    cl = inst.instance(n, k, m, 77 + n)
    g, b = rng.uniform(0, np.pi, 3), rng.uniform(0, np.pi, 3)
    c = q.build_cost_diagonal(cl, n)
    st = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    q.qaoa_run(c, n, m, g, b, state=st)
    u = rng.random(3000)
    got, costs = q.sample(st, n, u, cost=c)
    cost_o = oracle.cost(cl, n)
    psi_o = oracle.state(cost_o, n, g, b)
    clear = check_against_oracle(psi_o, u, got)
    if n <= 12:
        assert clear > 2000
    assert np.array_equal(costs, cost_o[got.astype(np.int64)])


def test_sample_uniform_state_full_size(q):
    """|+> at n = 30 (8 GiB): every probability is 2^-30 exactly, all sums are
    exact, so each draw is floor(u 2^30)."""
    import torch
    n = 30
    free, _ = torch.cuda.mem_get_info()
    if free < (9 << 30) + (1 << 30):
        pytest.skip("not enough device memory")
    c = torch.zeros(1 << n, dtype=torch.uint8, device="cuda")
    st = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    q.qaoa_run(c, n, 0, [], [], state=st)
    rng = np.random.default_rng(2)
    u = np.concatenate([rng.random(20000), [0.0, 1 - 2 ** -53, 0.5, 2 ** -30, 2 ** -30 * (2 ** 30 - 1)]])
    got, _ = q.sample(st, n, u)
    assert np.array_equal(got, np.floor(u * 2 ** n).astype(np.uint64))
    del st, c
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [22, 23, 25, 26])
def test_sample_exact_sums_every_chunk_shape(q, n):
    """Amplitudes (a + ib) 2^-10 with integers a, b in [0, 7]: every
    probability is a multiple of 2^-20 below 2^-13 and every partial sum is
    exact in FP64 whatever its order, so each draw is the oracle's exactly.
    n = 22..26 gives tile-prefix chunks of 1, 2, 8 and 16 tiles (4096
    amplitudes each); runs of zero tiles at the start, across the middle
    chunk boundary and at the end exercise the skip over empty tiles."""
    import torch
    rng = np.random.default_rng(200 + n)
    N = 1 << n
    a = rng.integers(0, 8, N).astype(np.float32)
    b = rng.integers(0, 8, N).astype(np.float32)
    psi = ((a + 1j * b) * np.float32(2.0 ** -10)).astype(np.complex64)
    psi[: 3 << 12] = 0
    psi[N // 2 - 5000: N // 2 + 9000] = 0
    psi[N - (1 << 12):] = 0
    st = torch.from_numpy(psi).to("cuda")
    u = np.concatenate([rng.random(20000), [0.0, 1 - 2 ** -53, 0.5]])
    got, _ = q.sample(st, n, u)
    ref = oracle.sample(psi.astype(np.complex128), n, u)
    assert np.array_equal(got, ref)
    del st
    torch.cuda.empty_cache()


def test_sample_workload_n30_statistics(q, golden):
    """The n = 30 workload with the ramp (beta negated): the share of
    satisfying draws and the mean cost of the draws agree with the oracle's
    p_succ and E[C] within 5 standard errors; draw costs equal the oracle's
    cost at those states."""
    import torch
    rec = golden["nae3_n30_p10"]
    n, m = rec["n"], rec["m"]
    free, _ = torch.cuda.mem_get_info()
    if free < (9 << 30) + (1 << 30):
        pytest.skip("not enough device memory")
    cl = inst.instance(n, 3, m, rec["seed"])
    g, b = inst.ramp_angles(rec["p"])
    c = q.build_cost_diagonal(cl, n)
    st = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    q.qaoa_run(c, n, m, g, -b, state=st)
    S = 200_000
    got, costs = q.sample(st, n, np.random.default_rng(3).random(S), cost=c)
    ref = rec["results"]["ramp_min"]
    ps = ref["p_success"]
    share = float((costs == 0).mean())
    assert abs(share - ps) <= 5 * np.sqrt(ps * (1 - ps) / S)
    mean = float(costs.mean())
    assert abs(mean - ref["expected_cost"]) <= 5 * costs.std() / np.sqrt(S)
    pick = np.arange(0, S, 97)
    assert np.array_equal(costs[pick], oracle.cost_at(cl, n, got[pick]))
    del st, c
    torch.cuda.empty_cache()


def test_running_time_mean(q):
    """Running times are i.i.d. geometric with success probability p_succ:
    their mean matches 1/p_succ of the oracle within 5 standard errors."""
    import torch
    n, p = 14, 3
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 12)
    g, b = inst.ramp_angles(p)
    c = q.build_cost_diagonal(cl, n)
    st = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    q.qaoa_run(c, n, m, g, -b, state=st)
    ps = oracle.qaoa(oracle.cost(cl, n), n, g, -b)[0]
    _, costs = q.sample(st, n, np.random.default_rng(4).random(400_000), cost=c)
    hits = np.flatnonzero(costs == 0)
    runs = np.diff(np.concatenate([[-1], hits]))
    assert q.running_time(costs) == runs[0]
    assert abs(runs.mean() - 1 / ps) <= 5 * np.sqrt((1 - ps) / ps ** 2 / len(runs))


def test_sample_edge_cases(q):
    import torch
    z = torch.zeros(1 << 10, dtype=torch.complex64, device="cuda")
    with pytest.raises(q.QNAEError, match="zero norm"):
        q.sample(z, 10, [0.5])
    got, costs = q.sample(z, 10, [])
    assert got.shape == (0,)
    # mass on two outcomes only
    z[5] = 0.6
    z[1000] = 0.8j
    got, _ = q.sample(z, 10, [0.0, 0.3599, 0.3601, 0.999999])
    assert list(got) == [5, 5, 1000, 1000]
    with pytest.raises(q.QNAEError, match="uniforms"):
        q.sample(z, 10, [1.0])
