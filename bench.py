#!/usr/bin/env python3
"""QAOA on random 3-NAE-SAT: amp-layer updates per second on one MI355X.

A step is the whole hot path on one instance: build the cost diagonal from the
clauses, run p layers of phase and mixer from |+>, and read out p_succ and
E[C]. The default workload is n = 30 variables, m = 63 clauses (r = 2.1),
p = 10 linear-ramp layers, complex64 state (8 GiB) and a uint8 cost diagonal.
The instance is the first satisfiable seed recorded in
tests/golden/workloads.json.

value = 2^n * p * steps / (time of the timed steps), inputs (the clause list)
already on the host and nothing else resident. Kernel times come from HIP
events recorded by the library on the stream it launches on.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def load_workload(name):
    """Instance and ramp angles of a named workload: m and seed from the
    stored oracle runs, or, for sizes beyond those, from the stored
    whole-diagonal digests."""
    from workloads import instances as inst
    with open(os.path.join(ROOT, "tests", "golden", "workloads.json")) as f:
        golden = json.load(f)
    if name in golden:
        rec = golden[name]
        n, k, r, p, _ = inst.SINGLE_WORKLOADS[name]
    else:  # "<digest workload>_p<layers>"
        base, layers = name.rsplit("_p", 1)
        with open(os.path.join(ROOT, "tests", "golden", "cost_digests.json")) as f:
            d = json.load(f)[base]
        n, k, p = d["n"], d["k"], int(layers)
        rec = {"n": n, "k": k, "m": d["m"], "seed": d["seed"], "p": p}
    cl = inst.instance(n, k, rec["m"], rec["seed"])
    g, b = inst.ramp_angles(p)
    return rec, cl, g, b


def cpu_baseline(sample_n: int, single_n: int = 22):
    """The FP64 oracle on a bounded sample of the same workload family: the
    whole path (cost, p = 10 ramp layers, readout) on one 3-NAE-SAT instance
    with sample_n variables and m = round(2.1 n), on all host threads; and the
    same at single_n variables on one thread."""
    import oracle
    from workloads import instances as inst

    def run(n):
        p = 10
        m = inst.clause_count(n, 2.1)
        cl = inst.instance(n, 3, m, 0)
        g, b = inst.ramp_angles(p)
        t0 = time.perf_counter()
        c = oracle.cost(cl, n)
        oracle.qaoa(c, n, g, b)
        dt = time.perf_counter() - t0
        return (2 ** n) * p / dt, dt, m

    threads = oracle.num_threads()  # loads the library before timing
    value, dt, m = run(sample_n)
    oracle.set_threads(1)
    v1, dt1, m1 = run(single_n)
    oracle.set_threads(threads)
    with open(os.path.join(ROOT, "tests", "golden", "workloads.json")) as f:
        n30 = json.load(f)["nae3_n30_p10"]
    return {"value": value, "unit": "amp-layer updates/s", "cores": threads, "host_ram_GiB": round(host_ram_gib(), 1),
            "kind": "oracle", "seconds": round(dt, 2),
            "sample": f"FP64 oracle, whole path (cost + 10 ramp layers + readout) on one random "
                      f"3-NAE-SAT instance, n={sample_n}, m={m}",
            "single_thread": {"value": v1, "seconds": round(dt1, 2), "cores": 1,
                              "sample": f"the same at n={single_n}, m={m1}"},
            # the headline size itself is too slow for this leg; its stored oracle run (cost diagonal
            # plus two p = 10 runs, ramp and ramp with beta negated) was timed when the golden
            # values were written, on another host
            "stored_n30_run": {"seconds": n30["oracle_seconds"], "cores": n30["oracle_threads"],
                               "value": 2 * (2 ** 30) * n30["p"] / n30["oracle_seconds"],
                               "sample": "nae3_n30_p10: cost diagonal + two 10-layer runs, FP64 oracle, "
                                         "timed by oracle/make_golden.py on an 8-thread host"}}


def parity_vs_oracle(q, ctx, rec, cost, n, m, p, g, b, res):
    """The headline step's readout against the FP64 oracle's stored values
    (tests/golden/workloads.json) for the workload's ramp and for the ramp
    with beta negated (one more, untimed run), with a verdict. Below the
    complex64 floor, num_solutions * n * p * (2^-24 * 2^(-n/2))^2 (FP32
    rounding of n * p butterflies on amplitudes of size 2^(-n/2), squared, on
    the solution states), p_succ is not resolved by the state's precision:
    only the absolute bound applies there."""
    floor = rec["num_solutions"] * n * p * (2.0 ** -24 * 2.0 ** (-n / 2)) ** 2
    out = {"reference": "tests/golden/workloads.json (FP64 oracle)",
           "tolerance": "|dp| <= 1e-5, relative dE <= 1e-5, |1 - norm| <= 1e-5, and relative dp <= 1e-4 when "
                        "p > 1e-3",
           "p_success_floor": floor}
    ok = True
    runs = (("ramp", res), ("ramp_min", q.qaoa_run(cost, n, m, g, -b, ctx=ctx)))
    for recipe, r in runs:
        ref = rec["results"][recipe]
        dp = abs(r.p_success - ref["p_success"])
        de = abs(r.expected_cost - ref["expected_cost"]) / abs(ref["expected_cost"])
        resolved = ref["p_success"] > floor
        good = dp <= 1e-5 and de <= 1e-5 and abs(r.norm - 1.0) <= 1e-5 and \
            (ref["p_success"] <= 1e-3 or dp <= 1e-4 * ref["p_success"])
        ok = ok and good
        out[recipe] = {"p_success": r.p_success, "oracle_p_success": ref["p_success"], "abs_dp": dp,
                       "rel_dp": dp / ref["p_success"] if resolved else None, "p_success_resolved": resolved,
                       "expected_cost": r.expected_cost, "oracle_expected_cost": ref["expected_cost"], "rel_dE": de,
                       "norm": r.norm, "pass": good}
    out["verdict"] = "pass" if ok else "FAIL"
    return out


def host_ram_gib():
    return os.sysconf("SC_PAGE_SIZE") * os.sysconf("SC_PHYS_PAGES") / 2 ** 30


def measured_traffic(stats):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary,
    weighted by this run's launches per sweep kind; None when the kernel
    sources changed since the counters were taken."""
    from paper_2401_02852_amd import profiling
    path = os.path.join(ROOT, "profiles", "sweep_n30_p10_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    per_kind, sha = profiling.read_traffic(path)
    if sha != profiling.kernel_source_hash():
        return None
    tot, launches = 0.0, 0
    for kind, (cnt, _ms, _b) in stats.items():
        if not kind.startswith("sweep_"):
            continue
        match = [v for k, v in per_kind.items() if k.endswith(" " + kind)]
        if not match:
            return None
        tot += cnt * (match[0][0] + match[0][1])
        launches += cnt
    return tot / launches if launches else None


def stream_ceilings(torch, gib=4, reps=5):
    """What the runtime's and torch's own streaming kernels reach on this
    device, as context for the roofline fraction (not an upper bound): a
    device-to-device copy (read + write, the sweeps' pattern), a fill (write
    only) and a sum (read only), over `gib` GiB, best of `reps`."""
    count = gib << 28  # float32 elements
    src = torch.ones(count, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)

    def best(fn, nbytes):
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return nbytes / (min(ms) * 1e-3) / 1e9

    size = count * 4
    out = {"bytes": size, "copy_GBps": best(lambda: dst.copy_(src), 2 * size),
           "fill_GBps": best(lambda: dst.fill_(1.0), size), "read_GBps": best(lambda: src.sum(), size)}
    del src, dst
    torch.cuda.empty_cache()
    return out


def scale_bench(q, ctx, names=("nae3_n24_p10", "nae3_n28_p10", "nae3_n33_p10"), steps=5, autotune=True):
    """The headline step (cost build + p = 10 ramp layers + readout) at other
    sizes of the same family: amp-layer updates/s and the sweeps' share of HBM
    peak. At n = 24 the 128 MiB state and 16 MiB cost fit the 256 MiB
    last-level cache, so its share of HBM peak is cache-inflated. n = 33
    holds a 64 GiB state and an 8 GiB cost (the instance whose whole cost
    diagonal the tests compare by digest; unsatisfiable, so p_succ is 0) on a
    context of its own, closed afterwards."""
    import torch
    out = {}
    main_ctx = ctx
    for name in names:
        rec, cl, g, b = load_workload(name)
        n, m, p = rec["n"], rec["m"], rec["p"]
        ctx = q.Context(0) if n > 32 else main_ctx
        shape = ctx.autotune(n, "u8", reps=2) if autotune else {}
        shape = shape or ctx.get_tune(n, "u8")
        cost = torch.empty(1 << n, dtype=torch.uint8, device="cuda")
        q.build_cost_diagonal(cl, n, out=cost, ctx=ctx)
        q.qaoa_run(cost, n, m, g, b, ctx=ctx)
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            q.build_cost_diagonal(cl, n, out=cost, ctx=ctx)
            res = q.qaoa_run(cost, n, m, g, b, ctx=ctx)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        ctx.profile(False)
        st = ctx.profile_read()
        sw = [v for k, v in st.items() if k.startswith("sweep_")]
        gbs = sum(v[2] for v in sw) / (sum(v[1] for v in sw) * 1e-3) / 1e9
        out[name] = {"n": n, "m": m, "p": p, "amp_layer_updates_per_s": (2 ** n) * p / dt,
                     "ms_per_step": dt * 1e3, "sweep_GBps": gbs, "sweep_frac_of_peak": gbs / HBM_PEAK_GBS,
                     "cache_resident": n <= 24, "p_success": res.p_success, "expected_cost": res.expected_cost,
                     "state_GiB": (8 << n) / 2 ** 30,
                     "tile_shape": {k: shape[k] for k in ("tile_bits", "low_run_bits", "page_bit", "split")}}
        del cost
        if ctx is not main_ctx:
            ctx.close()
            torch.cuda.empty_cache()
    return out


def batched_bench(q, ctx, reps=5, count=512):
    """512 ragged instances (k in {3, 5}, n in 10..20, p = 5, random angles):
    instance-layers/s of the batched path and of the plain path (one
    qnae_build_cost_diagonal + qnae_qaoa_run per instance) on the same GPU.
    The tile shape of the instances with n > 14 is tuned on this batch first
    (qnae_autotune_batched); both paths then run with it. The batched figure
    uses prepared calls (arguments marshalled once, everything else redone
    per call); the per-call figure marshals on every call."""
    import numpy as np
    import torch
    from workloads import instances as inst
    batch = inst.batched_workload(count=count)
    ns = [x["n"] for x in batch]
    ms = [x["m"] for x in batch]
    cls = [x["clauses"] for x in batch]
    gs = [x["gammas"] for x in batch]
    bs = [x["betas"] for x in batch]
    layers = sum(x["p"] for x in batch)
    costs = q.build_cost_diagonals(cls, ns, ctx=ctx)
    t0 = time.perf_counter()
    shape = q.autotune_batched(costs, ns, ms, gs, bs, reps=3, ctx=ctx)
    t_tune = time.perf_counter() - t0
    # the arguments marshalled once (the library still rebuilds clause
    # records, diagonals, phase tables and runs every kernel on each call)
    cb = q.PreparedCostBuild(cls, ns, outs=costs, ctx=ctx)
    pb = q.PreparedBatch(costs, ns, ms, [x["p"] for x in batch], ctx=ctx)
    G, B = np.stack(gs), np.stack(bs)
    cb.build()
    pb.run(G, B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        cb.build()
        pb.run(G, B)
    torch.cuda.synchronize()
    t_with = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        pb.run(G, B)
    torch.cuda.synchronize()
    t_without = (time.perf_counter() - t0) / reps
    # the same through the per-call functions (arguments marshalled every call)
    q.qaoa_run_batched(costs, ns, ms, gs, bs, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        q.build_cost_diagonals(cls, ns, outs=costs, ctx=ctx)
        q.qaoa_run_batched(costs, ns, ms, gs, bs, ctx=ctx)
    torch.cuda.synchronize()
    t_percall = (time.perf_counter() - t0) / reps
    # the same batch with half-state solves for n > 14 (NAE global-flip symmetry)
    half = [n > 14 for n in ns]
    hcosts = q.build_cost_diagonals(cls, ns, half=half, ctx=ctx)
    q.qaoa_run_batched(hcosts, ns, ms, gs, bs, half=half, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        q.build_cost_diagonals(cls, ns, outs=hcosts, half=half, ctx=ctx)
        q.qaoa_run_batched(hcosts, ns, ms, gs, bs, half=half, ctx=ctx)
    torch.cuda.synchronize()
    t_half = (time.perf_counter() - t0) / reps
    del hcosts
    for i in range(count):  # warm the plain path
        q.build_cost_diagonal(cls[i], ns[i], out=costs[i], ctx=ctx)
        q.qaoa_run(costs[i], ns[i], ms[i], gs[i], bs[i], ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(count):
        q.build_cost_diagonal(cls[i], ns[i], out=costs[i], ctx=ctx)
        q.qaoa_run(costs[i], ns[i], ms[i], gs[i], bs[i], ctx=ctx)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    for i in range(count):
        q.qaoa_run(costs[i], ns[i], ms[i], gs[i], bs[i], ctx=ctx)
    torch.cuda.synchronize()
    t_plain_nc = time.perf_counter() - t0
    return {"workload": f"{count} random k-NAE-SAT instances, k in {{3,5}}, n in 10..20, p=5, angles U(0,pi)",
            "instance_layers": layers,
            "instance_layers_per_s": layers / t_with,
            "instance_layers_per_s_cost_resident": layers / t_without,
            "instance_layers_per_s_per_call_marshalling": layers / t_percall,
            "prepared": "PreparedCostBuild + PreparedBatch (argument marshalling done once; every call rebuilds the "
                        "clause records, cost diagonals and phase tables and runs every kernel)",
            "plain_instance_layers_per_s": layers / t_plain,
            "plain_instance_layers_per_s_cost_resident": layers / t_plain_nc,
            "speedup_vs_plain": t_plain / t_with,
            "tile_shape": {k: shape.get(k) for k in ("tile_bits", "low_run_bits", "page_bit", "split")},
            "autotune_s": t_tune,
            "instance_layers_per_s_half_state": layers / t_half,
            "ms_per_batch": t_with * 1e3, "plain_ms": t_plain * 1e3}


def pretrain_bench(q, ctx, ks=(3, 9), p=8, v=200):
    """Fixed-angle pretraining (t = 100 instances of CNF(12, k, r_hat_k),
    Adam lr 0.01, 100 epochs, start (0.01, 0.01)) and evaluation on
    satisfiable ensembles (v per n): mean p_succ, median running time, and
    the fitted exponents C_hat, C_tilde with their relative error."""
    from paper_2401_02852_amd import pretrain
    out = {}
    for k in ks:
        t0 = time.perf_counter()
        tr = pretrain.pretrain(k, p, ctx=ctx)
        t1 = time.perf_counter()
        ns = list(range(12, 19 if k < 6 else 17))
        ev = pretrain.evaluate(k, tr["gammas"], tr["betas"], ns, v=v, ctx=ctx)
        t2 = time.perf_counter()
        out[f"k{k}"] = {"p": p, "train_s": t1 - t0, "epochs_per_s": 100 / (t1 - t0),
                        "train_objective": [tr["history"][0], tr["history"][-1]],
                        "gammas": [round(x, 5) for x in tr["gammas"]], "betas": [round(x, 5) for x in tr["betas"]],
                        "eval_s": t2 - t1, "ensemble": v,
                        "mean_p_success": {n: ev[n]["mean_p_success"] for n in ns},
                        "median_running_time": {n: ev[n]["median_running_time"] for n in ns},
                        **pretrain.exponents(ev)}
    return out


def z2_bench(q, ctx, steps=5):
    """The headline workload on the half-state path (NAE global-flip
    symmetry: state and cost for x < 2^(n-1)): the same step (half cost
    diagonal + p layers + readout), amp-layer updates of the full 2^n state
    per second, and the half sweeps' bandwidth."""
    import torch
    rec, cl, g, b = load_workload("nae3_n30_p10")
    n, m, p = rec["n"], rec["m"], rec["p"]
    cost = torch.empty(1 << (n - 1), dtype=torch.uint8, device="cuda")

    def step():
        q.build_cost_diagonal_z2(cl, n, out=cost, ctx=ctx)
        return q.qaoa_run_z2(cost, n, m, g, b, ctx=ctx)

    step()
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        res = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.profile(False)
    stats = ctx.profile_read()
    kinds = [k for k in stats if k.startswith("sweep_")]
    ms = sum(stats[k][1] for k in kinds)
    by = sum(stats[k][2] for k in kinds)
    achieved = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return {"workload": f"nae3_n30_p10 on the half state (2^{n - 1} stored amplitudes)",
            "amp_layer_updates_per_s": (2 ** n) * p * steps / dt, "ms_per_step": dt * 1e3 / steps,
            "sweep_GBps": achieved, "sweep_frac_of_peak": achieved / HBM_PEAK_GBS,
            "kernels": {k: {"launches": v[0], "avg_ms": v[1] / max(v[0], 1)} for k, v in stats.items()},
            "result": {"p_success": res.p_success, "expected_cost": res.expected_cost, "norm": res.norm}}


def sampling_bench(q, ctx, draws=100_000, ensemble=200):
    """Drawing bitstrings from the final state (Section 4.2). (1) Draws from
    the n = 30 workload's state (ramp with beta negated): draws/s and the
    tile-mass pass over the 8 GiB state. (2) Running times over an ensemble of
    satisfiable 3-NAE-SAT instances (n = 16, m = 34, p = 8, same ramp): median
    running time against 1/mean(p_succ)."""
    import numpy as np
    import torch
    from workloads import instances as inst
    rec, cl, g, b = load_workload("nae3_n30_p10")
    n, m = rec["n"], rec["m"]
    cost = q.build_cost_diagonal(cl, n, ctx=ctx)
    st = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    res = q.qaoa_run(cost, n, m, g, -b, state=st, ctx=ctx)
    u = np.random.default_rng(0).random(draws)
    q.sample(st, n, u, cost=cost, ctx=ctx)  # sizes the context's device and pinned buffers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, costs = q.sample(st, n, u, cost=cost, ctx=ctx)
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    q.sample(st, n, [], ctx=ctx)  # the two prefix passes alone
    dt0 = time.perf_counter() - t0
    del st, cost
    torch.cuda.empty_cache()
    out = {"workload": f"n={n} m={m} p=10 (seed {rec['seed']}), ramp with beta negated; {draws} draws",
           "draws_per_s": draws / dt, "ms": dt * 1e3, "prefix_pass_ms": dt0 * 1e3,
           "prefix_pass_GBps": 8 * 2 ** n / dt0 / 1e9,
           "share_satisfying": float((costs == 0).mean()), "p_success": res.p_success}
    # ensemble running times
    nn, pp = 16, 8
    mm = inst.clause_count(nn, 2.1)
    gg, bb = inst.ramp_angles(pp)
    rng = np.random.default_rng(1)
    runs, succ, seed = [], [], 0
    st = torch.empty(1 << nn, dtype=torch.complex64, device="cuda")
    t0 = time.perf_counter()
    while len(runs) < ensemble:
        c, sols = q.build_cost_diagonal(inst.instance(nn, 3, mm, seed), nn, count_solutions=True, ctx=ctx)
        seed += 1
        if sols == 0:
            continue
        r = q.qaoa_run(c, nn, mm, gg, -bb, state=st, ctx=ctx)
        rt, drawn = 0, 0
        while rt == 0 and drawn < 1 << 22:
            _, sc = q.sample(st, nn, rng.random(4096), cost=c, ctx=ctx)
            rt = q.running_time(sc)
            rt, drawn = (drawn + rt, drawn) if rt else (0, drawn + 4096)
        runs.append(rt)
        succ.append(r.p_success)
    out["ensemble"] = {"instances": ensemble, "n": nn, "m": mm, "p": pp, "median_running_time": float(np.median(runs)),
                       "inverse_mean_p_success": 1.0 / float(np.mean(succ)), "seconds": time.perf_counter() - t0}
    return out


def latency_bench(q, ctx, reps=200):
    """Launch-bound single solves: the n = 12, m = 25, p = 3 parity instance
    (linear ramp), one synchronous call at a time, with the cost diagonal
    resident and with its build included. Per-call wall time in microseconds."""
    import numpy as np
    import torch
    rec, cl, g, b = load_workload("nae3_n12_p3")
    n, m = rec["n"], rec["m"]
    cost = q.build_cost_diagonal(cl, n, ctx=ctx)
    torch.cuda.synchronize()

    def times(fn):
        for _ in range(10):
            fn()
        out = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            out.append((time.perf_counter() - t0) * 1e6)
        return np.percentile(out, 50), np.percentile(out, 99)

    run50, run99 = times(lambda: q.qaoa_run(cost, n, m, g, b, ctx=ctx))
    both50, both99 = times(lambda: q.qaoa_run(q.build_cost_diagonal(cl, n, out=cost, ctx=ctx), n, m, g, b, ctx=ctx))
    return {"workload": f"n={n} m={m} p=3 3-NAE-SAT (seed {rec['seed']}), linear ramp; {reps} calls",
            "run_p50_us": run50, "run_p99_us": run99, "build_and_run_p50_us": both50, "build_and_run_p99_us": both99}


def grad_bench(q, ctx, reps=20, adam_steps=200):
    """Differentiation workload: n = 22, m = 46, p = 12 from the linear ramp
    (beta negated), checkpoints every 4 layers. Time of one adjoint gradient
    against one forward run, then Adam (lr 0.01) maximising p_succ through
    QAOAFunction; the gradient/forward ratio also at n = 26 (same recipe).
    Parity of the gradient is the test suite's job."""
    import numpy as np
    import torch
    from workloads import instances as inst
    rec, cl, g0, b0 = load_workload("nae3_n22_p12")
    n, m, p = rec["n"], rec["m"], rec["p"]
    b0 = -b0
    cost = q.build_cost_diagonal(cl, n, ctx=ctx)
    torch.cuda.synchronize()

    def timed(fn):  # median of single synchronous calls
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    t_fwd = timed(lambda: q.qaoa_run(cost, n, m, g0, b0, ctx=ctx))
    t_grad = timed(lambda: q.qaoa_grad(cost, n, m, g0, b0, w_psucc=1.0, w_energy=0.0, checkpoint_every=4, ctx=ctx))
    g = torch.tensor(g0, dtype=torch.float64, requires_grad=True)
    b = torch.tensor(b0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([g, b], lr=0.01)
    start = None
    t0 = time.perf_counter()
    for _ in range(adam_steps):
        opt.zero_grad()
        ps, e = q.QAOAFunction.apply(g, b, cost, n, m, 4, ctx)
        (-ps).backward()
        opt.step()
        start = ps.item() if start is None else start
    dt = time.perf_counter() - t0
    # the same recipe at a size where a reverse sweep has many rounds of tiles
    n2 = 26
    m2 = inst.clause_count(n2, 2.1)
    cl2 = inst.instance(n2, 3, m2, 0)
    c2 = q.build_cost_diagonal(cl2, n2, ctx=ctx)
    t_fwd2 = timed(lambda: q.qaoa_run(c2, n2, m2, g0, b0, ctx=ctx))
    t_grad2 = timed(lambda: q.qaoa_grad(c2, n2, m2, g0, b0, w_psucc=1.0, w_energy=0.0, checkpoint_every=4, ctx=ctx))
    del c2
    return {"workload": f"n={n} m={m} p={p} 3-NAE-SAT (seed {rec['seed']}), linear ramp start, checkpoint every 4",
            "forward_ms": t_fwd * 1e3, "grad_ms": t_grad * 1e3, "grad_over_forward": t_grad / t_fwd,
            "adam_steps": adam_steps, "adam_steps_per_s": adam_steps / dt,
            "p_success_start": start, "p_success_end": ps.item(), "expected_cost_end": e.item(),
            f"n{n2}": {"workload": f"n={n2} m={m2} p={p} 3-NAE-SAT (seed 0), linear ramp start, checkpoint every 4",
                       "forward_ms": t_fwd2 * 1e3, "grad_ms": t_grad2 * 1e3, "grad_over_forward": t_grad2 / t_fwd2}}


def gradient_only(n, reps):
    """The gradient leg's recipe at one size (the stored n = 22 workload, or a
    random instance with m = round(2.1 n) for other n): one forward run, then
    `reps` gradients; prints the mean gradient time. For profiling runs."""
    import torch
    import paper_2401_02852_amd as q
    from workloads import instances as inst
    torch.cuda.set_device(0)
    ctx = q.Context(0)
    if n == 22:
        _, cl, g0, b0 = load_workload("nae3_n22_p12")
        m = len(cl)
    else:
        m = inst.clause_count(n, 2.1)
        cl = inst.instance(n, 3, m, 0)
        g0, b0 = inst.ramp_angles(12)
    b0 = -b0
    cost = q.build_cost_diagonal(cl, n, ctx=ctx)
    q.qaoa_run(cost, n, m, g0, b0, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        q.qaoa_grad(cost, n, m, g0, b0, w_psucc=1.0, w_energy=0.0, checkpoint_every=4, ctx=ctx)
    torch.cuda.synchronize()
    print(json.dumps({"gradient_only": {"n": n, "m": m, "p": len(g0), "reps": reps,
                                        "grad_ms": (time.perf_counter() - t0) * 1e3 / reps}}))


def serving_bench(q, ctx, count=2000, warm=100, rate=200.0, autotune=True):
    """Poisson request trace (n 14..26, p 2..20, k in {3, 5}) through the
    continuous-batching server and through the plain path one request at a
    time in arrival order (FIFO), at the trace's rate and at saturation (every
    arrival at t = 0). Latency is arrival to result in host memory; the first
    `warm` requests are excluded from the statistics."""
    import threading
    import numpy as np
    import torch
    from workloads import instances as inst
    trace = inst.serving_workload(count=count, rate=rate)
    layers = sum(r["p"] for r in trace[warm:])
    # the tile shape of every request size on the sweep path, for both paths
    tuned = {}
    if autotune:
        for n in sorted({r["n"] for r in trace if r["n"] > 14}):
            for dt in sorted({"u16" if r["m"] > 255 else "u8" for r in trace if r["n"] == n}):
                tuned[f"{n}/{dt}"] = ctx.autotune(n, dt, reps=2)
    pct = lambda a, x: float(np.percentile(np.asarray(a), x)) * 1e3

    def served(saturate):
        lat = [0.0] * count
        with q.Server(pool_bytes=64 << 30, max_slots=256, ctx=ctx) as srv:
            tickets = [None] * count
            lag = [0.0] * count
            ready = threading.Semaphore(0)

            def submitter():
                t0 = time.perf_counter()
                for i, r in enumerate(trace):
                    at = 0.0 if saturate else r["arrival_s"]
                    d = at - (time.perf_counter() - t0)
                    if d > 0:
                        time.sleep(d)
                    tickets[i] = srv.submit(r["clauses"], r["n"], r["gammas"], r["betas"])
                    lag[i] = max(0.0, time.perf_counter() - t0 - at)
                    ready.release()
            th = threading.Thread(target=submitter)
            th.start()
            t_first = None
            for i in range(count):
                ready.acquire()
                _, l = srv.wait(tickets[i])
                lat[i] = l + lag[i]
                if i == warm - 1:
                    t_first = time.perf_counter()
            t_end = time.perf_counter()
            th.join()
            st = srv.stats()
        return lat[warm:], t_end - t_first, st

    def plain(saturate):
        cost = {}
        lat = []
        t0 = time.perf_counter()
        t_first = None
        for i, r in enumerate(trace):
            at = 0.0 if saturate else r["arrival_s"]
            d = at - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            key = (r["n"], r["m"] > 255)
            if key not in cost:
                cost[key] = torch.empty(1 << r["n"], dtype=torch.uint16 if key[1] else torch.uint8, device="cuda")
            q.build_cost_diagonal(r["clauses"], r["n"], out=cost[key], ctx=ctx)
            q.qaoa_run(cost[key], r["n"], r["m"], r["gammas"], r["betas"], ctx=ctx)  # result on the host
            if i >= warm:
                lat.append(time.perf_counter() - t0 - at)
            if i == warm - 1:
                t_first = time.perf_counter()
        return lat, time.perf_counter() - t_first

    out = {"workload": f"{count} Poisson requests at {rate:g}/s (first {warm} warm-up), k in {{3,5}}, "
                       "n in 14..26, p in 2..20, angles U(0,pi)",
           "instance_layers": layers,
           "tile_shapes": {k: {f: v[f] for f in ("tile_bits", "low_run_bits", "page_bit", "split")}
                           for k, v in tuned.items() if v}}
    for mode, sat in (("rate", False), ("saturation", True)):
        lat, wall, st = served(sat)
        torch.cuda.synchronize()
        plat, pwall = plain(sat)
        out[mode] = {"served": {"p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "req_per_s": (count - warm) / wall,
                                "instance_layers_per_s": layers / wall, "ticks": st["ticks"],
                                "launches": st["launches"], "peak_pool_GiB": st["peak_pool_bytes"] / 2 ** 30},
                     "plain_fifo": {"p50_ms": pct(plat, 50), "p99_ms": pct(plat, 99),
                                    "req_per_s": (count - warm) / pwall, "instance_layers_per_s": layers / pwall}}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="nae3_n30_p10")
    ap.add_argument("--cpu-sample-n", type=int, default=28)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-scale", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-sampling", action="store_true")
    ap.add_argument("--no-z2", action="store_true")
    ap.add_argument("--no-pretrain", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the n=30 step (no other legs, no CPU baseline, no autotuning): for profiling")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile-shape", default="", metavar="TB,LOW,PAGE,SPLIT",
                    help="use this tile shape for the headline step instead of autotuning (e.g. the shape a "
                         "default run picked, for profiling runs that must time the same launches)")
    ap.add_argument("--no-ceilings", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run one plain device copy of MIB MiB (reference for HBM byte counters)")
    ap.add_argument("--gradient-only", type=int, default=0, metavar="N",
                    help="only run the gradient recipe (p = 12 linear ramp, checkpoints every 4) at n = N: "
                         "one forward run and --steps gradients, for profiling")
    args = ap.parse_args()
    if args.headline_only:
        for leg in ("cpu_baseline", "scale", "latency", "batched", "serving", "grad", "sampling", "z2", "pretrain",
                    "autotune", "ceilings"):
            setattr(args, "no_" + leg, True)
    if args.calibrate_copy:
        import torch
        src = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": args.calibrate_copy << 20}))
        return
    if args.gradient_only:
        gradient_only(args.gradient_only, max(args.steps, 1))
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(instances would shard by the top state bits across GPUs, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2401_02852_amd as q

    torch.cuda.set_device(0)
    rec, cl, g, b = load_workload(args.workload)
    n, m, p = rec["n"], rec["m"], rec["p"]
    ctx = q.Context(0)
    cost = torch.empty(1 << n, dtype=torch.uint8 if m <= 255 else torch.uint16, device="cuda")
    cdt = "u8" if m <= 255 else "u16"
    if args.tile_shape:
        tb, low, page, split = (int(x) for x in args.tile_shape.split(","))
        ctx.set_tune(n, {"tile_bits": tb, "low_run_bits": low, "page_bit": page, "split": split}, cdt)
        shape = ctx.get_tune(n, cdt)
    else:
        shape = {} if args.no_autotune else ctx.autotune(n, cdt, reps=3)
        shape = shape or ctx.get_tune(n, cdt)

    def step():
        q.build_cost_diagonal(cl, n, out=cost, ctx=ctx)
        return q.qaoa_run(cost, n, m, g, b, ctx=ctx)

    for _ in range(args.warmup):
        res = step()
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.profile(False)
    stats = ctx.profile_read()

    sweep_kinds = [k for k in stats if k.startswith("sweep_")]
    sw_launches = sum(stats[k][0] for k in sweep_kinds)
    sw_ms = sum(stats[k][1] for k in sweep_kinds)
    sw_bytes = sum(stats[k][2] for k in sweep_kinds)
    achieved = sw_bytes / (sw_ms * 1e-3) / 1e9 if sw_ms > 0 else 0.0
    layer_ms = sum(v[1] for k, v in stats.items() if k != "cost") / args.steps
    value = (2 ** n) * p * args.steps / dt

    out = {
        "metric": "QAOA amp-layer updates/s and % HBM peak at n=30",
        "value": value,
        "unit": "amp-layer updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "k": rec["k"], "m": m, "p": p,
                   "angles": "linear ramp", "seed": rec["seed"], "state": "complex64",
                   "cost": "uint8" if m <= 255 else "uint16",
                   "tile_shape": {k: shape[k] for k in ("tile_bits", "low_run_bits", "page_bit", "split")},
                   "autotuned": not args.no_autotune and not args.tile_shape},
        "roofline": {"bound": "hbm", "kernel": "sweep_kernel", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(stats),
                     "traffic_source": "profiles/sweep_n30_p10_hbm_traffic.txt: rocprofv3 FETCH_SIZE and WRITE_SIZE "
                                       "per sweep launch, scaled by a plain device copy, weighted by this run's "
                                       "launches per sweep kind (null when the kernel sources changed since)",
                     "launches": sw_launches, "avg_launch_ms": sw_ms / max(sw_launches, 1),
                     "algorithmic_bytes_per_launch": sw_bytes / max(sw_launches, 1),
                     # against the method's lower bound of one state read + write and one cost
                     # read per amp-layer (17 B), over the layer kernels' time
                     "frac_of_17B_lower_bound": 17.0 * (2 ** n) * p / (layer_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
                     if layer_ms > 0 else None},
        "kernels": {k: {"launches": v[0], "avg_ms": v[1] / max(v[0], 1),
                        "GBps": v[2] / (v[1] * 1e-3) / 1e9 if v[1] > 0 else None} for k, v in stats.items()},
        "layers_only_amp_layer_per_s": (2 ** n) * p / (layer_ms * 1e-3) if layer_ms > 0 else None,
        "result": {"p_success": res.p_success, "expected_cost": res.expected_cost, "norm": res.norm},
        "parity": parity_vs_oracle(q, ctx, rec, cost, n, m, p, g, b, res) if "results" in rec else
                  {"verdict": "no stored oracle readout for this workload (its diagonal digests are tested)"},
    }
    if not args.no_scale:
        out["scale"] = scale_bench(q, ctx, autotune=not args.no_autotune)
    if not args.no_latency:
        out["latency"] = latency_bench(q, ctx)
    if not args.no_batched:
        out["batched"] = batched_bench(q, ctx)
    if not args.no_grad:
        out["gradient"] = grad_bench(q, ctx)
    if not args.no_z2:
        out["z2_half_state"] = z2_bench(q, ctx)
    if not args.no_pretrain:
        out["pretraining"] = pretrain_bench(q, ctx)
    if not args.no_sampling:
        out["sampling"] = sampling_bench(q, ctx)
    if not args.no_serving:
        out["serving"] = serving_bench(q, ctx, count=args.serving_requests, autotune=not args.no_autotune)
    if not args.no_ceilings:  # last: its 8 GiB of torch buffers are freed again
        ceil = stream_ceilings(torch)
        ceil["sweeps_over_copy"] = achieved / ceil["copy_GBps"] if ceil["copy_GBps"] > 0 else None
        out["roofline"]["stream_ceilings"] = ceil
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
