"""Half-state simulation (global-flip symmetry of NAE, Section 2.2) against
the FP64 oracle: the half cost diagonal bit-exact, readouts and the kept
lower half of the final state within the parity tolerances."""
import numpy as np
import pytest

import oracle
from workloads import instances as inst

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2401_02852_amd as q
    q.load_library()
    return q


def check(got, ref, what=""):
    assert abs(got.p_success - ref[0]) <= 1e-5, what
    assert abs(got.expected_cost - ref[1]) <= 1e-5 * max(ref[1], 1e-12) + 1e-9, what
    assert abs(got.norm - 1.0) <= 1e-5, what


@pytest.mark.parametrize("n,k,m", [(2, 2, 3), (9, 3, 20), (15, 3, 32), (18, 5, 160), (16, 3, 300)])
def test_half_cost_bit_exact(q, n, k, m):
    cl = inst.instance(n, k, m, 5 * n + k)
    c, sols = q.build_cost_diagonal_z2(cl, n, count_solutions=True)
    ref = oracle.cost(cl, n)
    assert np.array_equal(c.cpu().numpy().astype(np.int64), ref[: 1 << (n - 1)])
    assert sols == int((ref == 0).sum())


def test_half_cost_wide_sampled(q):
    """n = 33: variables up to index 32 need 64-bit compares although the
    half diagonal has 2^32 states."""
    import torch
    n = 33
    free, _ = torch.cuda.mem_get_info()
    if free < (1 << (n - 1)) + (1 << 30):
        pytest.skip("not enough device memory")
    cl = inst.instance(n, 3, 70, 8)
    assert np.any(np.abs(cl) == n)
    c = q.build_cost_diagonal_z2(cl, n)
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.integers(0, 1 << (n - 1), 3000, dtype=np.uint64),
                         np.arange((1 << (n - 1)) - 64, 1 << (n - 1), dtype=np.uint64)])
    got = c[torch.from_numpy(xs.astype(np.int64)).cuda()].cpu().numpy().astype(np.int64)
    assert np.array_equal(got, oracle.cost_at(cl, n, xs))
    del c
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [15, 16, 19, 22])
@pytest.mark.parametrize("p", [0, 1, 2, 5])
def test_half_run_matches_oracle(q, n, p):
    import torch
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 31 * n + p)
    rng = np.random.default_rng(n * 10 + p)
    g, b = rng.uniform(0, np.pi, p), rng.uniform(0, np.pi, p)  # both butterfly forms
    c = q.build_cost_diagonal_z2(cl, n)
    st = torch.empty(1 << (n - 1), dtype=torch.complex64, device="cuda")
    got = q.qaoa_run_z2(c, n, m, g, b, state=st)
    cost = oracle.cost(cl, n)
    check(got, oracle.qaoa(cost, n, g, b), f"n={n} p={p}")
    psi = oracle.state(cost, n, g, b)
    assert np.max(np.abs(st.cpu().numpy() - psi[: 1 << (n - 1)])) <= 1e-5
    again = q.qaoa_run_z2(c, n, m, g, b)
    assert tuple(again) == tuple(got)


@pytest.mark.parametrize("tb", [12, 13, 14])
@pytest.mark.parametrize("n", [17, 21, 25])
def test_half_run_tile_shapes(q, tb, n):
    ctx = q.Context()
    ctx.set_tune(n, {"tile_bits": tb, "low_run_bits": 4 + (n % 2), "page_bit": 18 if n > 20 else 64})
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 600 + n)
    rng = np.random.default_rng(tb + n)
    g, b = rng.uniform(0, np.pi, 3), rng.uniform(0, np.pi, 3)
    c = q.build_cost_diagonal_z2(cl, n, ctx=ctx)
    check(q.qaoa_run_z2(c, n, m, g, b, ctx=ctx), oracle.qaoa(oracle.cost(cl, n), n, g, b), f"tb={tb} n={n}")
    ctx.close()


@pytest.mark.parametrize("tb", [12, 13])
@pytest.mark.parametrize("split", [1, 2, 3])
def test_half_run_group_splits(q, tb, split):
    """n = 25 (three qubit groups): every split of the low index bits between
    the second and third group, on the half state, against the oracle."""
    n = 25
    ctx = q.Context()
    ctx.set_tune(n, {"tile_bits": tb, "low_run_bits": 4, "page_bit": 18, "split": split})
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 650)
    rng = np.random.default_rng(split + 10 * tb)
    g, b = rng.uniform(0, np.pi, 3), rng.uniform(0, np.pi, 3)
    c = q.build_cost_diagonal_z2(cl, n, ctx=ctx)
    check(q.qaoa_run_z2(c, n, m, g, b, ctx=ctx), oracle.qaoa(oracle.cost(cl, n), n, g, b), f"tb={tb} split={split}")
    ctx.close()


def test_half_uint16_and_k5(q):
    n, m = 17, 300
    cl = inst.instance(n, 5, m, 2)
    g, b = [0.3, -0.8, 1.9], [0.4, 2.2, -0.7]
    c = q.build_cost_diagonal_z2(cl, n)
    assert c.dtype.itemsize == 2
    check(q.qaoa_run_z2(c, n, m, g, b), oracle.qaoa(oracle.cost(cl, n), n, g, b))


@pytest.mark.parametrize("name", ["nae3_n24_p10", "nae3_n28_p10", "nae3_n30_p10"])
def test_half_workloads(q, golden, name):
    rec = golden[name]
    n, m = rec["n"], rec["m"]
    cl = inst.instance(n, 3, m, rec["seed"])
    g, b = inst.ramp_angles(rec["p"])
    c = q.build_cost_diagonal_z2(cl, n)
    for recipe, bb in (("ramp", b), ("ramp_min", -b)):
        got = q.qaoa_run_z2(c, n, m, g, bb)
        ref = rec["results"][recipe]
        assert abs(got.p_success - ref["p_success"]) <= 1e-5
        assert abs(got.expected_cost - ref["expected_cost"]) <= 1e-5 * ref["expected_cost"]
        if ref["p_success"] > 1e-3:
            assert abs(got.p_success - ref["p_success"]) <= 1e-4 * ref["p_success"]


def test_half_rejects_small_n(q):
    c = q.build_cost_diagonal_z2(inst.instance(14, 3, 29, 0), 14)
    with pytest.raises(q.QNAEError, match="n > 14"):
        q.qaoa_run_z2(c, 14, 29, [0.1], [0.2])
