"""Batched path (many instances per launch) against the single-instance path
and the FP64 oracle, through the C ABI."""
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


def ragged(count, seed, n_lo=3, n_hi=20):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        k = int(rng.integers(1, min(n, 5) + 1))
        m = int(rng.integers(0, 4 * n))
        if i % 7 == 3:
            m = 300 + n  # uint16 costs
        cl = inst.instance(n, k, m, 1000 * seed + i).reshape(m, k)
        p = int(rng.integers(0, 6))
        g, b = rng.uniform(-3, 3, p), rng.uniform(-3, 3, p)
        out.append((n, k, m, cl, g, b))
    return out


def test_batched_cost_matches_single(q):
    jobs = ragged(40, 1)
    costs, sols = q.build_cost_diagonals([j[3] for j in jobs], [j[0] for j in jobs], count_solutions=True)
    for (n, k, m, cl, g, b), c, s in zip(jobs, costs, sols):
        ref = oracle.cost(cl, n)
        assert np.array_equal(c.cpu().numpy().astype(np.int64), ref), (n, k, m)
        assert s == int((ref == 0).sum())


def test_batched_run_matches_single_and_oracle(q):
    jobs = ragged(48, 2)
    costs = q.build_cost_diagonals([j[3] for j in jobs], [j[0] for j in jobs])
    res = q.qaoa_run_batched(costs, [j[0] for j in jobs], [j[2] for j in jobs], [j[4] for j in jobs],
                             [j[5] for j in jobs])
    for (n, k, m, cl, g, b), c, r in zip(jobs, costs, res):
        alone = q.qaoa_run(c, n, m, g, b)
        assert np.allclose(r, alone, rtol=1e-12, atol=1e-15), (n, m, len(g), r, alone)
        ref = oracle.qaoa(oracle.cost(cl, n), n, g, b)
        assert abs(r.p_success - ref[0]) <= 1e-5
        assert abs(r.expected_cost - ref[1]) <= 1e-5 * max(ref[1], 1e-12) + 1e-9
        assert abs(r.norm - 1) <= 1e-5


def test_batched_states(q):
    import torch
    jobs = ragged(12, 3, n_lo=8, n_hi=19)
    costs = q.build_cost_diagonals([j[3] for j in jobs], [j[0] for j in jobs])
    states = [torch.empty(1 << j[0], dtype=torch.complex64, device="cuda") for j in jobs]
    q.qaoa_run_batched(costs, [j[0] for j in jobs], [j[2] for j in jobs], [j[4] for j in jobs],
                       [j[5] for j in jobs], states=states)
    for (n, k, m, cl, g, b), c, st in zip(jobs, costs, states):
        ref = torch.empty_like(st)
        q.qaoa_run(c, n, m, g, b, state=ref)
        assert torch.equal(st, ref), n


def test_batched_workload_512(q):
    """The 512-instance ragged batch (large enough that its clause records,
    tables and plans are built on the host thread pool): every result equals
    the single-instance path; costs and solution counts of a sample equal the
    single builds and the oracle; a sample is checked against the oracle."""
    import torch
    batch = inst.batched_workload(count=512)
    costs, sols = q.build_cost_diagonals([x["clauses"] for x in batch], [x["n"] for x in batch],
                                         count_solutions=True)
    for i in range(0, 512, 17):
        x = batch[i]
        c1, s1 = q.build_cost_diagonal(x["clauses"], x["n"], count_solutions=True)
        assert torch.equal(c1, costs[i]) and s1 == sols[i], i
    for i in range(0, 512, 101):
        x = batch[i]
        assert sols[i] == oracle.count_solutions(x["clauses"], x["n"]), i
    res = q.qaoa_run_batched(costs, [x["n"] for x in batch], [x["m"] for x in batch],
                             [x["gammas"] for x in batch], [x["betas"] for x in batch])
    for x, c, r in zip(batch, costs, res):
        alone = q.qaoa_run(c, x["n"], x["m"], x["gammas"], x["betas"])
        assert np.allclose(r, alone, rtol=1e-12, atol=1e-15)
    for i in range(0, 512, 37):
        x = batch[i]
        ref = oracle.qaoa(oracle.cost(x["clauses"], x["n"]), x["n"], x["gammas"], x["betas"])
        assert abs(res[i].p_success - ref[0]) <= 1e-5
        assert abs(res[i].expected_cost - ref[1]) <= 1e-5 * ref[1]


def test_graph_replay_matches_eager(q, monkeypatch):
    """A batch shape seen again replays a captured launch graph; every replay
    (with new angles, and eager work in between) equals the eager result."""
    import torch
    batch = inst.batched_workload(count=64, seed=5)
    ns = [x["n"] for x in batch]
    ms = [x["m"] for x in batch]
    costs = q.build_cost_diagonals([x["clauses"] for x in batch], ns)
    monkeypatch.setenv("QNAE_GRAPHS", "0")
    eager = q.Context()
    monkeypatch.setenv("QNAE_GRAPHS", "1")
    graph = q.Context()
    rng = np.random.default_rng(9)
    for rep in range(4):
        g = [rng.uniform(0, np.pi, 5) for _ in batch]
        b = [rng.uniform(0, np.pi, 5) for _ in batch]
        ref = q.qaoa_run_batched(costs, ns, ms, g, b, ctx=eager)
        got = q.qaoa_run_batched(costs, ns, ms, g, b, ctx=graph)
        assert got == ref, rep
        q.qaoa_run(costs[rep], ns[rep], ms[rep], g[rep], b[rep], ctx=eager)
        torch.cuda.synchronize()
    eager.close()
    graph.close()


def test_batched_half_state_instances(q):
    """Half-state instances (n > 14) next to full ones in one batch: each
    equals qaoa_run_z2 (or qaoa_run) alone; half cost jobs equal
    build_cost_diagonal_z2; a sample against the oracle."""
    import torch
    batch = inst.batched_workload(count=48, seed=3)
    ns = [x["n"] for x in batch]
    ms = [x["m"] for x in batch]
    cls = [x["clauses"] for x in batch]
    half = [x["n"] > 14 and i % 3 != 0 for i, x in enumerate(batch)]
    costs, sols = q.build_cost_diagonals(cls, ns, half=half, count_solutions=True)
    states = [torch.empty(1 << (n - (1 if h else 0)), dtype=torch.complex64, device="cuda") for n, h in zip(ns, half)]
    gs = [x["gammas"] for x in batch]
    bs = [x["betas"] for x in batch]
    res = q.qaoa_run_batched(costs, ns, ms, gs, bs, half=half, states=states)
    again = q.qaoa_run_batched(costs, ns, ms, gs, bs, half=half)  # graph replay of the same shape
    assert again == res
    for i, x in enumerate(batch):
        n, m = x["n"], x["m"]
        if half[i]:
            c1, s1 = q.build_cost_diagonal_z2(cls[i], n, count_solutions=True)
            assert torch.equal(c1, costs[i]) and s1 == sols[i]
            st = torch.empty(1 << (n - 1), dtype=torch.complex64, device="cuda")
            alone = q.qaoa_run_z2(c1, n, m, gs[i], bs[i], state=st)
        else:
            c1 = q.build_cost_diagonal(cls[i], n)
            assert torch.equal(c1, costs[i])
            st = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
            alone = q.qaoa_run(c1, n, m, gs[i], bs[i], state=st)
        assert np.allclose(res[i], alone, rtol=1e-12, atol=1e-15), (i, n, half[i])
        assert torch.equal(st, states[i])
    for i in range(0, 48, 5):
        x = batch[i]
        ref = oracle.qaoa(oracle.cost(x["clauses"], x["n"]), x["n"], x["gammas"], x["betas"])
        assert abs(res[i].p_success - ref[0]) <= 1e-5
        assert abs(res[i].expected_cost - ref[1]) <= 1e-5 * ref[1]
    with pytest.raises(q.QNAEError, match="half-state"):
        small = [k for k, x in enumerate(batch) if x["n"] <= 14][0]
        q.qaoa_run_batched([costs[small][: 1 << (ns[small] - 1)]], [ns[small]], [ms[small]], [gs[small]], [bs[small]],
                           half=True)


def test_empty_batches(q):
    """Zero instances: every batched entry point returns empty results and
    the context still serves the next call."""
    assert q.build_cost_diagonals([], []) == []
    costs, sols = q.build_cost_diagonals([], [], count_solutions=True)
    assert costs == [] and len(sols) == 0
    assert q.qaoa_run_batched([], [], [], [], []) == []
    dgs, dbs, res = q.qaoa_grad_batched([], [], [], [], [])
    assert dgs == [] and dbs == [] and res == []
    cl = inst.instance(9, 3, 19, 3)
    c = q.build_cost_diagonal(cl, 9)
    g, b = inst.ramp_angles(3)
    got = q.qaoa_run_batched([c], [9], [19], [g], [-b])
    assert np.allclose(got[0], q.qaoa_run(c, 9, 19, g, -b), rtol=1e-12, atol=1e-15)


SHAPES = [{"tile_bits": tb, "low_run_bits": low, "page_bit": page}
          for tb in (12, 13, 14) for low in (4, 5) for page in (18, 64)]


def test_batched_under_every_tile_shape(q):
    """Every tile shape the autotuners may keep, set for the batch's sizes:
    each batched result equals the single-instance path under the same
    shape (same plan, same rounding), and a sample matches the oracle."""
    jobs = [j for j in ragged(60, 6, n_lo=12, n_hi=20)]
    ns = [j[0] for j in jobs]
    costs = q.build_cost_diagonals([j[3] for j in jobs], ns)
    classes = {(n, "u16" if c.dtype.itemsize == 2 else "u8") for n, c in zip(ns, costs) if n > 14}
    for shape in SHAPES:
        ctx = q.Context()
        for n, dt in classes:
            ctx.set_tune(n, shape, cost_dtype=dt)
        res = q.qaoa_run_batched(costs, ns, [j[2] for j in jobs], [j[4] for j in jobs], [j[5] for j in jobs],
                                 ctx=ctx)
        for (n, k, m, cl, g, b), c, r in zip(jobs, costs, res):
            alone = q.qaoa_run(c, n, m, g, b, ctx=ctx)
            assert np.allclose(r, alone, rtol=1e-12, atol=1e-15), (shape, n, m, r, alone)
        for i in range(0, len(jobs), 13):
            n, k, m, cl, g, b = jobs[i]
            ref = oracle.qaoa(oracle.cost(cl, n), n, g, b)
            assert abs(res[i].p_success - ref[0]) <= 1e-5 and abs(res[i].norm - 1) <= 1e-5, shape
            assert abs(res[i].expected_cost - ref[1]) <= 1e-5 * max(ref[1], 1e-12) + 1e-9, shape
        ctx.close()


@pytest.mark.parametrize("split", [1, 2, 3])
def test_batched_group_splits(q, split):
    """Instances at n = 23..25 (three qubit groups at 13-bit tiles) with a
    group split set: the batched results equal the single-instance path under
    the same shape, which the oracle checks on one instance."""
    jobs = []
    for i, n in enumerate((23, 24, 25, 24)):
        m = inst.clause_count(n, 2.1)
        cl = inst.instance(n, 3, m, 700 + i)
        rng = np.random.default_rng(split * 10 + i)
        jobs.append((n, m, cl, rng.uniform(0, np.pi, 2), rng.uniform(0, np.pi, 2)))
    ns = [j[0] for j in jobs]
    ctx = q.Context()
    for n in set(ns):
        ctx.set_tune(n, {"tile_bits": 13, "low_run_bits": 4, "page_bit": 18, "split": split})
    costs = q.build_cost_diagonals([j[2] for j in jobs], ns, ctx=ctx)
    res = q.qaoa_run_batched(costs, ns, [j[1] for j in jobs], [j[3] for j in jobs], [j[4] for j in jobs], ctx=ctx)
    for (n, m, cl, g, b), c, r in zip(jobs, costs, res):
        assert np.allclose(r, q.qaoa_run(c, n, m, g, b, ctx=ctx), rtol=1e-12, atol=1e-15), (split, n)
    n, m, cl, g, b = jobs[0]
    ref = oracle.qaoa(oracle.cost(cl, n), n, g, b)
    assert abs(res[0].p_success - ref[0]) <= 1e-5 and abs(res[0].expected_cost - ref[1]) <= 1e-5 * ref[1]
    del costs
    ctx.close()


def test_autotune_batched_keeps_a_candidate(q):
    """The batch-level tuner keeps one of the candidate shapes for every
    (n, cost type) of the batch's tiled instances; afterwards batched and
    single runs on that context agree."""
    batch = inst.batched_workload(count=96, seed=3)
    ns = [x["n"] for x in batch]
    ms = [x["m"] for x in batch]
    gs = [x["gammas"] for x in batch]
    bs = [x["betas"] for x in batch]
    costs = q.build_cost_diagonals([x["clauses"] for x in batch], ns)
    ctx = q.Context()
    best = q.autotune_batched(costs, ns, ms, gs, bs, reps=1, ctx=ctx)
    assert {k: best[k] for k in ("tile_bits", "low_run_bits", "page_bit")} in SHAPES
    assert best["split"] in (0, 1, 2, 3)
    assert best["ms_per_layer"] > 0
    for n in sorted({n for n in ns if n > 14}):
        got = ctx.get_tune(n)
        assert (got["tile_bits"], got["low_run_bits"], got["page_bit"]) == \
            (best["tile_bits"], best["low_run_bits"], best["page_bit"]), n
    res = q.qaoa_run_batched(costs, ns, ms, gs, bs, ctx=ctx)
    for x, c, r in zip(batch, costs, res):
        assert np.allclose(r, q.qaoa_run(c, x["n"], x["m"], x["gammas"], x["betas"], ctx=ctx), rtol=1e-12,
                           atol=1e-15)
    small = [i for i, n in enumerate(ns) if n <= 14]
    assert q.autotune_batched([costs[i] for i in small], [ns[i] for i in small], [ms[i] for i in small],
                              [gs[i] for i in small], [bs[i] for i in small], ctx=ctx) == {}
    ctx.close()


def test_cached_plan_with_kept_states_and_changing_flips(q, monkeypatch):
    """A repeated batch shape reuses its plan and its captured launches while
    the angles change, including whether each final state must be reversed
    (an odd number of cot-form layers): every replay's results and kept
    states equal an eager context's."""
    import torch
    jobs = ragged(24, 7, n_lo=15, n_hi=19)
    ns = [j[0] for j in jobs]
    ms = [j[2] for j in jobs]
    costs = q.build_cost_diagonals([j[3] for j in jobs], ns)
    monkeypatch.setenv("QNAE_GRAPHS", "0")
    eager = q.Context()
    monkeypatch.setenv("QNAE_GRAPHS", "1")
    graph = q.Context()
    se = [torch.empty(1 << n, dtype=torch.complex64, device="cuda") for n in ns]
    sg = [torch.empty(1 << n, dtype=torch.complex64, device="cuda") for n in ns]
    rng = np.random.default_rng(17)
    for rep in range(6):
        # rep 0, 2, 4: every beta in the tan form; 1, 3, 5: one cot-form layer each
        g = [rng.uniform(-2, 2, 3) for _ in jobs]
        b = [rng.uniform(-0.6, 0.6, 3) for _ in jobs]
        if rep % 2:
            for bb in b:
                bb[1] = rng.uniform(1.0, 2.0)
        ref = q.qaoa_run_batched(costs, ns, ms, g, b, states=se, ctx=eager)
        got = q.qaoa_run_batched(costs, ns, ms, g, b, states=sg, ctx=graph)
        assert got == ref, rep
        for a, c in zip(sg, se):
            assert torch.equal(a, c), rep
    eager.close()
    graph.close()


def test_prepared_batch_and_cost_build_match(q):
    """Prepared cost builds and batches (arguments marshalled once) give the
    same diagonals, solution counts and results as the per-call functions,
    with angles as per-instance lists or as one [count, p] array, run after
    run with new angles."""
    import torch
    batch = inst.batched_workload(count=80, seed=11)
    ns = [x["n"] for x in batch]
    ms = [x["m"] for x in batch]
    cls = [x["clauses"] for x in batch]
    ref_costs, ref_sols = q.build_cost_diagonals(cls, ns, count_solutions=True)
    cb = q.PreparedCostBuild(cls, ns)
    for _ in range(2):
        costs, sols = cb.build(count_solutions=True)
        assert sols == ref_sols
        assert all(torch.equal(a, b) for a, b in zip(costs, ref_costs))
    pb = q.PreparedBatch(costs, ns, ms, [5] * len(batch))
    rng = np.random.default_rng(2)
    for rep in range(3):
        g = rng.uniform(0, np.pi, (len(batch), 5))
        b = rng.uniform(0, np.pi, (len(batch), 5))
        ref = np.array(q.qaoa_run_batched(costs, ns, ms, list(g), list(b)))
        assert np.array_equal(pb.run(g, b), ref), rep
        assert np.array_equal(pb.run(list(g), list(b)), ref), rep
