"""Sweep tile shapes: every shape the planner accepts gives the oracle's
result, and the autotuner keeps one of them."""
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


def check(got, ref):
    assert abs(got.p_success - ref[0]) <= 1e-5
    assert abs(got.expected_cost - ref[1]) <= 1e-5 * ref[1]
    assert abs(got.norm - 1.0) <= 1e-5


@pytest.mark.parametrize("n", [17, 23])
def test_every_shape_matches_oracle(q, n):
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 60 + n)
    rng = np.random.default_rng(n)
    g, b = rng.uniform(0, np.pi, 3), rng.uniform(0, np.pi, 3)
    ref = oracle.qaoa(oracle.cost(cl, n), n, g, b)
    ctx = q.Context()
    c = q.build_cost_diagonal(cl, n, ctx=ctx)
    for tb in (12, 13, 14):
        for low in (4, 5, 6):
            for page in (18, 64):
                ctx.set_tune(n, {"tile_bits": tb, "low_run_bits": low, "page_bit": page})
                assert ctx.get_tune(n)["tile_bits"] == tb
                check(q.qaoa_run(c, n, m, g, b, ctx=ctx), ref)
    ctx.close()


def test_autotune_keeps_a_candidate(q, tmp_path):
    from paper_2401_02852_amd import tuning
    ctx = q.Context()
    assert ctx.autotune(12) == {}
    shapes = tuning.autotune(ctx, [18, 20], ("u8", "u16"), reps=2)
    for (n, dt), t in shapes.items():
        assert t["tile_bits"] in (12, 13, 14) and t["low_run_bits"] in (4, 5) and t["page_bit"] in (18, 64)
        assert t["split"] in (0, 1, 2, 3)
        assert t["ms_per_layer"] > 0
        assert ctx.get_tune(n, dt)["tile_bits"] == t["tile_bits"]
    path = str(tmp_path / "tune.json")
    tuning.save(path, ctx, shapes)
    fresh = q.Context()
    assert tuning.load(path, fresh) == 4
    assert fresh.get_tune(20, "u16") == ctx.get_tune(20, "u16")
    n = 20
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 3)
    c = q.build_cost_diagonal(cl, n, ctx=fresh)
    check(q.qaoa_run(c, n, m, [0.3, 0.8], [0.6, 0.1], ctx=fresh), oracle.qaoa(oracle.cost(cl, n), n, [0.3, 0.8], [0.6, 0.1]))
    ctx.set_tune(n, None)
    assert ctx.get_tune(n)["ms_per_layer"] == 0.0
    with pytest.raises(q.QNAEError, match="tile_bits"):
        ctx.set_tune(n, {"tile_bits": 15, "low_run_bits": 4, "page_bit": 18})
    with pytest.raises(q.QNAEError, match="n=14"):
        ctx.set_tune(14, {"tile_bits": 13, "low_run_bits": 4, "page_bit": 18})
    with pytest.raises(q.QNAEError, match="split=4"):
        ctx.set_tune(n, {"tile_bits": 13, "low_run_bits": 4, "page_bit": 18, "split": 4})
    ctx.close()
    fresh.close()
