"""Batched gradients and the fixed-angle pretraining / evaluation protocol
(Section 3.3, 4.1, 4.2) on the GPU, against the FP64 oracle."""
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


def check(dg, db, rg, rb, w, ec2=0.0):
    """p_succ part: 1e-5 absolute. E[C] part: 1e-4 of the largest component,
    plus the state tolerance (1e-6 relative) times the size of the weighted
    sums, |w_E| E[C^2]: with m in the hundreds the complex64 state's rounding,
    not the sum, bounds the error."""
    scale = max(np.max(np.abs(rg), initial=0), np.max(np.abs(rb), initial=0), 1e-12)
    tol = 1e-5 * abs(w[0]) + (1e-4 * scale + 1e-6 * abs(w[1]) * ec2) * (abs(w[1]) > 0)
    assert np.max(np.abs(dg - rg), initial=0) <= tol
    assert np.max(np.abs(db - rb), initial=0) <= tol


def test_grad_batched_matches_single_and_oracle(q):
    rng = np.random.default_rng(0)
    jobs = []
    for i in range(30):
        n = int(rng.integers(3, 17))
        k = int(rng.integers(2, min(n, 5) + 1))
        m = 260 + n if i % 7 == 2 else int(rng.integers(0, 3 * n))
        cl = inst.instance(n, k, m, 90 + i).reshape(m, k)
        p = int(rng.integers(0, 6))
        jobs.append((n, m, cl, rng.uniform(-2, 2, p), rng.uniform(-2, 2, p)))
    costs = q.build_cost_diagonals([j[2] for j in jobs], [j[0] for j in jobs])
    w = (0.7, 0.05)
    dgs, dbs, res = q.qaoa_grad_batched(costs, [j[0] for j in jobs], [j[1] for j in jobs], [j[3] for j in jobs],
                                        [j[4] for j in jobs], w_psucc=w[0], w_energy=w[1], checkpoint_every=2)
    for (n, m, cl, g, b), c, dg, db, r in zip(jobs, costs, dgs, dbs, res):
        sg, sb, sr = q.qaoa_grad(c, n, m, g, b, w_psucc=w[0], w_energy=w[1], checkpoint_every=2)
        assert np.allclose(dg, sg, rtol=1e-12, atol=1e-15) and np.allclose(db, sb, rtol=1e-12, atol=1e-15)
        assert np.allclose(tuple(r), tuple(sr), rtol=1e-12, atol=1e-15)
        cost = oracle.cost(cl, n)
        rg, rb, ro = oracle.qaoa_grad(cost, n, g, b, *w)
        ec2 = float((cost.astype(np.float64) ** 2 * np.abs(oracle.state(cost, n, g, b)) ** 2).sum())
        check(dg, db, rg, rb, w, ec2)
        assert abs(r.p_success - ro[0]) <= 1e-5


def test_pretrain_matches_oracle_gradient_adam(q):
    """Three epochs of the protocol on a small set; the same Adam run on the
    oracle's FP64 gradients lands on the same angles."""
    import torch
    from paper_2401_02852_amd import pretrain
    k, p, t, n = 3, 2, 12, 10
    out = pretrain.pretrain(k, p, t=t, n=n, epochs=3, lr=0.05, seed=4)
    costs = [oracle.cost(cl, n) for cl in out["instances"]]
    g = torch.full((p,), 0.01, dtype=torch.float64, requires_grad=True)
    b = torch.full((p,), 0.01, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([g, b], lr=0.05)
    hist = []
    for _ in range(3):
        dg_sum, db_sum, ps = np.zeros(p), np.zeros(p), 0.0
        for c in costs:
            dg, db, r = oracle.qaoa_grad(c, n, g.detach().numpy(), b.detach().numpy(), 1.0 / t, 0.0)
            dg_sum += dg
            db_sum += db
            ps += r[0] / t
        hist.append(ps)
        opt.zero_grad()
        g.grad = -torch.from_numpy(dg_sum)
        b.grad = -torch.from_numpy(db_sum)
        opt.step()
    assert np.allclose(out["history"], hist, rtol=0, atol=1e-5)
    assert np.allclose(out["gammas"], g.detach().numpy(), atol=1e-4)
    assert np.allclose(out["betas"], b.detach().numpy(), atol=1e-4)
    assert all(cl.shape[1] == k for cl in out["instances"])


def test_evaluate_small_ensemble(q):
    from paper_2401_02852_amd import pretrain
    g, b = np.array([0.2, 0.35]), np.array([-0.3, -0.15])
    ev = pretrain.evaluate(3, g, b, [10, 12], v=8, seed=3)
    for n, rec in ev.items():
        ens = pretrain.random_set(3, n, 8, 3 + 7919 * n, satisfiable=True)
        assert all(oracle.count_solutions(cl, n) > 0 for cl in ens)
        ref = [oracle.qaoa(oracle.cost(cl, n), n, g, b)[0] for cl in ens]
        assert abs(rec["mean_p_success"] - np.mean(ref)) <= 1e-5
        assert all(r >= 1 for r in rec["running_times"])
        assert rec["median_running_time"] == np.median(rec["running_times"])
    ex = pretrain.exponents(ev)
    assert np.isfinite(ex["C_hat"]) and np.isfinite(ex["C_tilde"])
