"""Fixed-angle pretraining and ensemble evaluation.

Section 3.3 selects fixed angles per (k, p) by maximising the mean success
probability (1/t) sum_i p_succ(sigma_i) over t = 100 random instances
CNF(n = 12, k, r_hat_k) with Adam for 100 epochs from beta = 0.01,
gamma = -0.01 in the paper's convention. The paper writes the mixer two ways:
exp(-i beta H_B) in Section 2.1 and exp(+i beta H_B) in Section 3.4 and
Appendix A.3/A.4. The start is read in the latter convention, because those
are the sections that describe the simulator the paper ran; this library
applies exp(-i beta H_B), so the paper's (gamma, beta) is this library's
(gamma, -beta), i.e. (-0.01, -0.01), which the global sign symmetry
(gamma, beta) -> (-gamma, -beta) maps to the default start (0.01, 0.01).
Under Section 2.1's convention the same start would be (0.01, -0.01) here;
`init` accepts either. Section 4.1
and 4.2 evaluate the angles on ensembles of satisfiable instances for a range
of n: the mean success probability and the median running time, and
Section 4.4 fits both to 2^(c n + d).

Every GPU step goes through the library: batched cost diagonals, batched
gradients, batched runs with kept states, and draws from those states. The
Adam update of the 2p angles runs in PyTorch on the host.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence

import numpy as np

from ._binding import Context, build_cost_diagonals, default_context, qaoa_grad_batched, qaoa_run_batched, sample


def running_time(sample_costs) -> int:
    """Instance running time (Section 4.2): draws until the first satisfying
    one (cost 0), counting it; 0 when none of the draws satisfies."""
    hit = np.flatnonzero(np.asarray(sample_costs) == 0)
    return int(hit[0]) + 1 if hit.size else 0


def r_hat(k: int) -> float:
    """Clause density near the NAE satisfiability threshold (Section 3.3,
    natural logarithm): (2^(k-1) - 1/2 - 1/(4 ln 2)) ln 2."""
    ln2 = math.log(2.0)
    return (2.0 ** (k - 1) - 0.5 - 1.0 / (4.0 * ln2)) * ln2


def random_set(k: int, n: int, count: int, seed: int, satisfiable: bool = False,
               ctx: Optional[Context] = None) -> List[np.ndarray]:
    """`count` instances of CNF(n, k, r_hat_k) (Poisson m, cnf_instance),
    instance j from PCG64(seed * 1_000_003 + j) for j = 0, 1, ...; with
    `satisfiable`, the ones without an NAE solution (counted on the GPU) are
    skipped."""
    from workloads.instances import cnf_instance  # the seeded generator (repository root)

    out: List[np.ndarray] = []
    j = 0
    r = r_hat(k)
    while len(out) < count:
        want = count - len(out)
        batch = [cnf_instance(n, k, r, seed * 1_000_003 + j + i) for i in range(want)]
        j += want
        if not satisfiable:
            out += batch
            continue
        _, sols = build_cost_diagonals(batch, [n] * want, count_solutions=True, ctx=ctx)
        out += [cl for cl, s in zip(batch, sols) if s > 0]
    return out


def pretrain(k: int, p: int, *, t: int = 100, n: int = 12, epochs: int = 100, lr: float = 0.01, seed: int = 0,
             init=(0.01, 0.01), checkpoint_every: int = 4, ctx: Optional[Context] = None) -> Dict:
    """Adam on the mean success probability over t training instances.
    Returns the angles, the objective before each epoch's step and the
    instances used."""
    import torch
    ctx = ctx or default_context()
    train = random_set(k, n, t, seed, ctx=ctx)
    ms = [cl.shape[0] for cl in train]
    costs = build_cost_diagonals(train, [n] * t, ctx=ctx)
    g = torch.full((p,), float(init[0]), dtype=torch.float64, requires_grad=True)
    b = torch.full((p,), float(init[1]), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([g, b], lr=lr)
    history = []
    for _ in range(epochs):
        gg = g.detach().numpy().copy()
        bb = b.detach().numpy().copy()
        dgs, dbs, res = qaoa_grad_batched(costs, [n] * t, ms, [gg] * t, [bb] * t, w_psucc=1.0 / t, w_energy=0.0,
                                          checkpoint_every=checkpoint_every, ctx=ctx)
        history.append(float(sum(r.p_success for r in res) / t))
        opt.zero_grad()
        g.grad = -torch.from_numpy(np.sum(dgs, axis=0))  # ascent on the objective
        b.grad = -torch.from_numpy(np.sum(dbs, axis=0))
        opt.step()
    return {"gammas": g.detach().numpy().copy(), "betas": b.detach().numpy().copy(), "history": history,
            "instances": train}


def evaluate(k: int, gammas, betas, ns: Sequence[int], *, v: int = 200, seed: int = 1, draw_block: int = 4096,
             max_draws: int = 1 << 22, ctx: Optional[Context] = None) -> Dict[int, Dict]:
    """For each n: v satisfiable instances of CNF(n, k, r_hat_k); the mean
    success probability (Section 4.1) and the median running time, draws from
    the final state until a satisfying one (Section 4.2; draws use NumPy
    PCG64(seed) uniforms). Running times past max_draws count as max_draws."""
    import torch
    ctx = ctx or default_context()
    rng = np.random.Generator(np.random.PCG64(seed))
    p = len(gammas)
    out = {}
    for n in ns:
        ens = random_set(k, n, v, seed + 7919 * n, satisfiable=True, ctx=ctx)
        costs = build_cost_diagonals(ens, [n] * v, ctx=ctx)
        states = [torch.empty(1 << n, dtype=torch.complex64, device="cuda") for _ in range(v)]
        res = qaoa_run_batched(costs, [n] * v, [cl.shape[0] for cl in ens], [gammas] * v, [betas] * v,
                               states=states, ctx=ctx)
        runs = []
        for st, c in zip(states, costs):
            drawn = 0
            rt = 0
            while rt == 0 and drawn < max_draws:
                _, sc = sample(st, n, rng.random(draw_block), cost=c, ctx=ctx)
                r = running_time(sc)
                if r:
                    rt = drawn + r
                drawn += draw_block
            runs.append(rt if rt else max_draws)
        out[n] = {"mean_p_success": float(np.mean([r.p_success for r in res])),
                  "median_running_time": float(np.median(runs)), "running_times": runs,
                  "p_success": [r.p_success for r in res], "p": p}
        del states
    return out


def fit_exponent(ns: Sequence[int], values: Sequence[float]):
    """Least-squares fit of values = 2^(c n + d) (Section 4.4): returns (c, d)."""
    x = np.asarray(ns, dtype=np.float64)
    y = np.log2(np.asarray(values, dtype=np.float64))
    A = np.stack([x, np.ones_like(x)], axis=1)
    (c, d), *_ = np.linalg.lstsq(A, y, rcond=None)
    return float(c), float(d)


def exponents(evaluation: Dict[int, Dict]):
    """C_hat from mean p_succ = 2^(-C_hat n + d), C_tilde from the median
    running time = 2^(C_tilde n + d), and their relative error."""
    ns = sorted(evaluation)
    c_hat = -fit_exponent(ns, [evaluation[n]["mean_p_success"] for n in ns])[0]
    c_tilde = fit_exponent(ns, [evaluation[n]["median_running_time"] for n in ns])[0]
    return {"C_hat": c_hat, "C_tilde": c_tilde, "relative_error": abs((c_hat - c_tilde) / c_hat)}
