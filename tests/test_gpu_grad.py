"""Adjoint gradient on the GPU (through the C ABI) against the FP64 oracle's
adjoint and central finite differences of the oracle.

Tolerance: gradient of the p_succ part within 1e-5 absolute, of the E[C] part
within 1e-4 relative to the largest component (complex64 states, FP32 sums per
tile, FP64 across tiles)."""
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


def check(dg, db, rg, rb, w):
    """The p_succ part within 1e-5 absolute and within 1e-3 of the largest
    reference component (whichever is tighter: small gradients are held to
    the relative bound), the E[C] part within 1e-4 of the largest."""
    scale = max(np.max(np.abs(rg)), np.max(np.abs(rb)), 1e-12)
    tol = abs(w[0]) * min(1e-5, 1e-3 * scale + 1e-10) + 1e-4 * scale * (abs(w[1]) > 0)
    assert np.max(np.abs(dg - rg)) <= tol, (dg, rg)
    assert np.max(np.abs(db - rb)) <= tol, (db, rb)


def check_readout(r, ro):
    """p_succ within 1e-5 absolute and 1e-4 relative (whichever is tighter),
    E[C] within 1e-5 relative."""
    assert abs(r.p_success - ro[0]) <= min(1e-5, 1e-4 * ro[0] + 1e-12), (r, ro)
    assert abs(r.expected_cost - ro[1]) <= 1e-5 * ro[1], (r, ro)


@pytest.mark.parametrize("n", [4, 9, 13, 14, 16, 19])
@pytest.mark.parametrize("w", [(1.0, 0.0), (0.0, 1.0), (0.5, -0.3)])
def test_grad_vs_oracle_adjoint(q, n, w):
    rng = np.random.default_rng(n)
    p = 5
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 40 + n)
    g, b = rng.uniform(0, 1.5, p), rng.uniform(-1, 1, p)
    c = q.build_cost_diagonal(cl, n)
    dg, db, r = q.qaoa_grad(c, n, m, g, b, w_psucc=w[0], w_energy=w[1], checkpoint_every=2)
    rg, rb, ro = oracle.qaoa_grad(oracle.cost(cl, n), n, g, b, *w)
    check(dg, db, rg, rb, w)
    check_readout(r, ro)


@pytest.mark.parametrize("n", [7, 15])
def test_grad_vs_finite_differences(q, n):
    rng = np.random.default_rng(3)
    p = 3
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 7)
    g, b = rng.uniform(0, 1.5, p), rng.uniform(-1, 1, p)
    c = q.build_cost_diagonal(cl, n)
    for w in [(1.0, 0.0), (0.0, 1.0)]:
        dg, db, _ = q.qaoa_grad(c, n, m, g, b, w_psucc=w[0], w_energy=w[1])
        fg, fb = oracle.finite_difference_grad(oracle.cost(cl, n), n, g, b, *w, h=1e-4)
        check(dg, db, fg, fb, w)


@pytest.mark.parametrize("every", [1, 3, 4, 0, 2**31 - 1])
@pytest.mark.parametrize("p", [1, 4, 7])
def test_checkpoint_intervals(q, every, p):
    n = 17
    rng = np.random.default_rng(p)
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 11)
    g, b = rng.uniform(0, np.pi, p), rng.uniform(0, np.pi, p)  # exercises both butterfly forms
    c = q.build_cost_diagonal(cl, n)
    dg, db, _ = q.qaoa_grad(c, n, m, g, b, w_psucc=0.7, w_energy=0.2, checkpoint_every=every)
    rg, rb, _ = oracle.qaoa_grad(oracle.cost(cl, n), n, g, b, 0.7, 0.2)
    check(dg, db, rg, rb, (0.7, 0.2))


@pytest.mark.parametrize("n", [10, 18])
def test_grad_special_cases(q, n):
    """beta = 0: every dF/dgamma is 0; gamma = 0: every dF/dbeta is 0. The
    exact zeros come out as FP32 rounding of sums whose real parts are of
    order |F| = w_psucc + w_energy m, hence the tolerance 1e-5 |F|."""
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 5)
    c = q.build_cost_diagonal(cl, n)
    tol = 1e-5 * (1.0 + 0.5 * m)
    dg, _, _ = q.qaoa_grad(c, n, m, [0.3, 0.5, 0.9], [0.0, 0.0, 0.0], w_psucc=1.0, w_energy=0.5)
    assert np.max(np.abs(dg)) < tol
    _, db, _ = q.qaoa_grad(c, n, m, [0.0, 0.0, 0.0], [0.3, 0.5, 0.9], w_psucc=1.0, w_energy=0.5)
    assert np.max(np.abs(db)) < tol


def test_grad_three_groups_n23(q):
    """n = 23 is the smallest size whose layers take three qubit groups at
    13-bit tiles, so the reverse pass runs every adjoint kind, including the
    inverse mixer alone in the middle of a layer; satisfiable instance (seed
    124, 2 solutions), checkpoints every 2 of 3 layers, against the oracle's
    adjoint."""
    import torch
    n, p = 23, 3
    rng = np.random.default_rng(23)
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 124)
    g, b = rng.uniform(0, 1.5, p), rng.uniform(-1, 1, p)
    c = q.build_cost_diagonal(cl, n)
    cost = oracle.cost(cl, n)
    assert int((cost == 0).sum()) == 2
    for w in [(1.0, 0.0), (0.0, 1.0)]:
        dg, db, r = q.qaoa_grad(c, n, m, g, b, w_psucc=w[0], w_energy=w[1], checkpoint_every=2)
        rg, rb, ro = oracle.qaoa_grad(cost, n, g, b, *w)
        check(dg, db, rg, rb, w)
        check_readout(r, ro)
    del c
    torch.cuda.empty_cache()


def test_grad_extreme_mixer_angles(q):
    """Mixer angles at and near +-pi/2 (cotangent forms, t = 0 and small t),
    next to pi/4 (|t| about 1) and past pi/2, checkpoints every 1, 2 and 4
    layers, so reverse segments start with lam relabelled against the
    restored psi; against the oracle's adjoint."""
    n, p = 20, 6
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 13)  # 6 solutions
    g = np.array([0.4, 0.9, 0.2, 1.3, 0.6, 0.8])
    b = np.array([np.pi / 2, -np.pi / 4, 1.5707, np.pi / 4 + 1e-3, -1.56, 2.9])
    c = q.build_cost_diagonal(cl, n)
    cost = oracle.cost(cl, n)
    assert int((cost == 0).sum()) == 6
    w = (0.6, 0.3)
    rg, rb, ro = oracle.qaoa_grad(cost, n, g, b, *w)
    for every in (1, 2, 4):
        dg, db, r = q.qaoa_grad(c, n, m, g, b, w_psucc=w[0], w_energy=w[1], checkpoint_every=every)
        check(dg, db, rg, rb, w)
        check_readout(r, ro)


@pytest.mark.parametrize("n", [12, 17])
def test_grad_u16_costs(q, n):
    """m = 300 clauses: 16-bit cost values through the weighing, checkpointing,
    phase-carrying and resident kinds; mixer angles on both butterfly forms;
    against the oracle's adjoint."""
    rng = np.random.default_rng(100 + n)
    m, p = 300, 5
    cl = inst.instance(n, 3, m, 3)
    c = q.build_cost_diagonal(cl, n)
    assert str(c.dtype) == "torch.uint16"
    g, b = rng.uniform(0, 0.2, p), rng.uniform(0, np.pi, p)
    cost = oracle.cost(cl, n)
    for w in [(1.0, 0.0), (0.0, 1.0)]:
        dg, db, r = q.qaoa_grad(c, n, m, g, b, w_psucc=w[0], w_energy=w[1], checkpoint_every=2)
        rg, rb, ro = oracle.qaoa_grad(cost, n, g, b, *w)
        check(dg, db, rg, rb, w)
        assert abs(r.expected_cost - ro[1]) <= 1e-5 * ro[1], (r, ro)


def test_grad_n24_streaming(q):
    """n = 24: the reverse sweeps stream their states with nontemporal accesses
    (the two states exceed the last-level cache); both butterfly forms,
    checkpoints every 2 of 3 layers, satisfiable instance (seed 4, 96
    solutions), against the oracle's adjoint."""
    import torch
    n, p = 24, 3
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 4)
    rng = np.random.default_rng(24)
    g, b = rng.uniform(0, 1.5, p), rng.uniform(0, np.pi, p)
    c = q.build_cost_diagonal(cl, n)
    cost = oracle.cost(cl, n)
    w = (0.5, 0.2)
    dg, db, r = q.qaoa_grad(c, n, m, g, b, w_psucc=w[0], w_energy=w[1], checkpoint_every=2)
    rg, rb, ro = oracle.qaoa_grad(cost, n, g, b, *w)
    check(dg, db, rg, rb, w)
    check_readout(r, ro)
    del c
    torch.cuda.empty_cache()


def test_grad_u16_streaming(q):
    """n = 24 with m = 300: 16-bit cost values in the nontemporal reverse
    kinds (weighing, boundary, end) and the checkpointing forward sweeps,
    checkpoints every layer, both butterfly forms, against the oracle's
    adjoint."""
    import torch
    n, m, p = 24, 300, 2
    cl = inst.instance(n, 3, m, 5)
    rng = np.random.default_rng(2400)
    g, b = rng.uniform(0, 0.1, p), np.array([0.3, 1.4])
    c = q.build_cost_diagonal(cl, n)
    assert str(c.dtype) == "torch.uint16"
    cost = oracle.cost(cl, n)
    w = (0.3, 0.4)
    dg, db, r = q.qaoa_grad(c, n, m, g, b, w_psucc=w[0], w_energy=w[1], checkpoint_every=1)
    rg, rb, ro = oracle.qaoa_grad(cost, n, g, b, *w)
    check(dg, db, rg, rb, w)
    assert abs(r.expected_cost - ro[1]) <= 1e-5 * ro[1], (r, ro)
    del c
    torch.cuda.empty_cache()


def test_grad_workload_n22_p12(q, golden):
    """The differentiation workload: n = 22, m = 46, p = 12 from the linear
    ramp (beta negated), checkpoints every 4 layers, against the oracle's
    adjoint."""
    rec = golden["nae3_n22_p12"]
    n, m, p = rec["n"], rec["m"], rec["p"]
    cl = inst.instance(n, 3, m, rec["seed"])
    g, b = inst.ramp_angles(p)
    b = -b
    c = q.build_cost_diagonal(cl, n)
    cost = oracle.cost(cl, n)
    for w in [(1.0, 0.0), (0.0, 1.0)]:
        dg, db, r = q.qaoa_grad(c, n, m, g, b, w_psucc=w[0], w_energy=w[1], checkpoint_every=4)
        rg, rb, ro = oracle.qaoa_grad(cost, n, g, b, *w)
        check(dg, db, rg, rb, w)
        assert abs(r.p_success - rec["results"]["ramp_min"]["p_success"]) <= 1e-5


def test_autograd_function(q):
    import torch
    n, p = 16, 3
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 21)
    c = q.build_cost_diagonal(cl, n)
    g = torch.tensor([0.2, 0.5, 0.7], dtype=torch.float64, requires_grad=True)
    b = torch.tensor([-0.4, -0.3, -0.1], dtype=torch.float64, requires_grad=True)
    ps, e = q.QAOAFunction.apply(g, b, c, n, m)
    (3.0 * ps - 0.1 * e).backward()
    rg, rb, ro = oracle.qaoa_grad(oracle.cost(cl, n), n, g.detach().numpy(), b.detach().numpy(), 3.0, -0.1)
    check(g.grad.numpy(), b.grad.numpy(), rg, rb, (3.0, -0.1))
    assert abs(ps.item() - ro[0]) <= 1e-5


def test_adam_steps_raise_success_probability(q):
    import torch
    n, p = 14, 4
    m = inst.clause_count(n, 2.1)
    cl = inst.instance(n, 3, m, 2)
    c = q.build_cost_diagonal(cl, n)
    g = torch.full((p,), 0.01, dtype=torch.float64, requires_grad=True)
    b = torch.full((p,), -0.01, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([g, b], lr=0.05)
    first = None
    for _ in range(20):
        opt.zero_grad()
        ps, _ = q.QAOAFunction.apply(g, b, c, n, m)
        (-ps).backward()
        opt.step()
        first = ps.item() if first is None else first
    assert ps.item() > 2 * first
