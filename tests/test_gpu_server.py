"""Continuous-batching server (qnae_server_*) through the C ABI: every result
equals the single-instance path whatever else shares its launches (the
half-state path for n > 14, which the server uses for these NAE requests
unless QNAE_SERVER_HALF=0), against the FP64 oracle on a sample; pool limits
queue requests rather than fail them."""
import threading
import time

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


def requests(count, seed, n_lo=3, n_hi=20, p_hi=6):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        k = int(rng.integers(1, min(n, 5) + 1))
        m = int(rng.integers(0, 4 * n))
        if i % 9 == 4:
            m = 280 + n  # uint16 costs
        cl = inst.instance(n, k, m, 5000 * seed + i).reshape(m, k)
        p = int(rng.integers(0, p_hi + 1))
        g, b = rng.uniform(-3, 3, p), rng.uniform(-3, 3, p)
        out.append((n, k, m, cl, g, b))
    return out


def alone(q, r, half=True):
    n, k, m, cl, g, b = r
    if half and n > 14:
        return q.qaoa_run_z2(q.build_cost_diagonal_z2(cl, n), n, m, g, b)
    c = q.build_cost_diagonal(cl, n)
    return q.qaoa_run(c, n, m, g, b)


def close(a, b):
    return np.allclose(tuple(a), tuple(b), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("slots,tick_bytes,half", [(1, None, "1"), (5, None, "1"), (64, None, "1"), (7, "1", "1"),
                                                   (64, "3e7", "1"), (5, None, "0"), (64, "3e7", "0")])
def test_server_results_equal_single_path(q, slots, tick_bytes, half, monkeypatch):
    """tick_bytes 1: one sweep round per scheduler tick; 3e7: a few rounds;
    default: every round of a lightly loaded server in one tick. half 0: full
    states."""
    if tick_bytes:
        monkeypatch.setenv("QNAE_SERVER_TICK_BYTES", tick_bytes)
    monkeypatch.setenv("QNAE_SERVER_HALF", half)
    reqs = requests(40, slots)
    with q.Server(pool_bytes=1 << 28, max_slots=slots) as s:
        tickets = [s.submit(r[3], r[0], r[4], r[5]) for r in reqs]
        got = [s.wait(t, timeout_ms=60000) for t in tickets]
        st = s.stats()
    assert st["completed"] == len(reqs) and st["queued"] == 0 and st["active"] == 0
    assert st["peak_pool_bytes"] <= 1 << 28
    for r, (res, lat) in zip(reqs, got):
        assert lat > 0
        assert close(res, alone(q, r, half == "1")), (r[0], r[2], len(r[4]))
    for r, (res, _) in list(zip(reqs, got))[::7]:
        n, k, m, cl, g, b = r
        ref = oracle.qaoa(oracle.cost(cl, n), n, g, b)
        assert abs(res.p_success - ref[0]) <= 1e-5
        assert abs(res.expected_cost - ref[1]) <= 1e-5 * max(ref[1], 1e-12) + 1e-9


def test_server_admission_order_does_not_change_results(q):
    reqs = requests(24, 7, n_lo=12, n_hi=19)
    out = []
    for order in (np.arange(24), np.random.default_rng(1).permutation(24)):
        with q.Server(pool_bytes=1 << 26, max_slots=6) as s:
            t = {int(i): s.submit(reqs[i][3], reqs[i][0], reqs[i][4], reqs[i][5]) for i in order}
            out.append([s.wait(t[i])[0] for i in range(24)])
    for a, b in zip(*out):
        assert close(a, b)


def test_small_pool_queues_requests(q):
    """A 1 MiB pool holds one n = 17 request (half state: 512 KiB state +
    64 KiB costs + tables) at a time, so the others wait in the queue; n = 18
    can never fit."""
    reqs = requests(6, 11, n_lo=17, n_hi=17)
    with q.Server(pool_bytes=1 << 20, max_slots=8) as s:
        with pytest.raises(q.QNAEError, match="does not fit"):
            s.submit(inst.instance(18, 3, 30, 0), 18, [0.1], [0.2])
        tickets = [s.submit(r[3], r[0], r[4], r[5]) for r in reqs]
        got = [s.wait(t)[0] for t in tickets]
        assert s.stats()["peak_pool_bytes"] <= 1 << 20
    for r, res in zip(reqs, got):
        assert close(res, alone(q, r))


def test_server_ticket_errors_and_drain(q):
    reqs = requests(8, 3, n_lo=18, n_hi=20, p_hi=8)
    s = q.Server(pool_bytes=1 << 28, max_slots=2)
    tickets = [s.submit(r[3], r[0], r[4], r[5]) for r in reqs]
    with pytest.raises(q.QNAEError, match="unknown ticket"):
        s.wait(123456789)
    first, _ = s.wait(tickets[0])
    assert close(first, alone(q, reqs[0]))
    with pytest.raises(q.QNAEError, match="p="):
        s.submit(reqs[0][3], reqs[0][0], np.zeros(100001), np.zeros(100001))
    with pytest.raises(q.QNAEError, match="literal"):
        s.submit(np.array([[1, 40]], dtype=np.int32), 20, [0.1], [0.1])
    s.close()  # drains the rest without waiting for them
    with pytest.raises(Exception):
        s.wait(tickets[1])


def test_server_concurrent_submitters(q):
    reqs = requests(48, 5, n_lo=8, n_hi=18)
    results = [None] * len(reqs)
    with q.Server(pool_bytes=1 << 28, max_slots=16) as s:
        def worker(lo):
            for i in range(lo, len(reqs), 4):
                n, k, m, cl, g, b = reqs[i]
                results[i] = s.wait(s.submit(cl, n, g, b))[0]
                time.sleep(0.001)
        th = [threading.Thread(target=worker, args=(lo,)) for lo in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
    for r, res in zip(reqs, results):
        assert close(res, alone(q, r))


def test_serving_trace_sample(q):
    """The first requests of the Poisson serving trace (n 14..26, p 2..20,
    k in {3, 5}), submitted at their arrival times: a sample against the
    oracle, all against the single-instance path."""
    trace = inst.serving_workload(count=40)
    with q.Server(pool_bytes=8 << 30, max_slots=64) as s:
        t0 = time.perf_counter()
        tickets = []
        for r in trace:
            d = r["arrival_s"] - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            tickets.append(s.submit(r["clauses"], r["n"], r["gammas"], r["betas"]))
        got = [s.wait(t, timeout_ms=120000) for t in tickets]
    for r, (res, lat) in zip(trace, got):
        a = alone(q, (r["n"], r["k"], r["m"], r["clauses"], r["gammas"], r["betas"]))
        assert close(res, a), r["n"]
        assert 0 < lat < 60
    for r, (res, _) in zip(trace[:12], got[:12]):
        if r["n"] > 22:
            continue
        ref = oracle.qaoa(oracle.cost(r["clauses"], r["n"]), r["n"], r["gammas"], r["betas"])
        assert abs(res.p_success - ref[0]) <= 1e-5
        assert abs(res.expected_cost - ref[1]) <= 1e-5 * ref[1]


def test_cancel_queued_and_active(q, monkeypatch):
    """A queued request leaves the queue; an active one is dropped between
    ticks; both report QNAE_ECANCELED and free their pool blocks; the others
    complete unchanged."""
    monkeypatch.setenv("QNAE_SERVER_TICK_BYTES", "1")  # one sweep round per tick: long-lived requests
    big = requests(1, 21, n_lo=24, n_hi=24, p_hi=0)[0]
    g = np.linspace(0.1, 0.9, 80)
    reqs = requests(6, 22, n_lo=15, n_hi=18)
    with q.Server(pool_bytes=1 << 30, max_slots=1) as s:
        tb = s.submit(big[3], big[0], g, g[::-1])
        tickets = [s.submit(r[3], r[0], r[4], r[5]) for r in reqs]
        assert s.cancel(tickets[-1]) and s.cancel(tickets[-2])  # still queued behind the big one
        for _ in range(2000):
            if s.stats()["active"] == 1 and s.stats()["ticks"] > 2:
                break
            time.sleep(0.001)
        assert s.cancel(tb)  # active
        with pytest.raises(q.QNAEError, match="cancel"):
            s.wait(tb)
        for t in tickets[-2:]:
            with pytest.raises(q.QNAEError, match="cancel"):
                s.wait(t)
        got = [s.wait(t)[0] for t in tickets[:-2]]
        assert s.pool_in_use() == 0
        done = s.submit(reqs[0][3], reqs[0][0], reqs[0][4], reqs[0][5])
        s.wait(done)
        with pytest.raises(q.QNAEError, match="unknown ticket"):
            s.cancel(done)  # collected: forgotten
    for r, res in zip(reqs, got):
        assert close(res, alone(q, r))


def test_injected_fault_fails_cleanly(q, monkeypatch):
    """A device error at a scheduler tick (injected on the host before the tick
    launches anything) fails every request in flight or queued, frees the
    pool, and makes later submissions fail; the server still shuts down."""
    monkeypatch.setenv("QNAE_FAULT_INJECT", "server_tick:3")
    monkeypatch.setenv("QNAE_SERVER_TICK_BYTES", "1")
    reqs = requests(8, 23, n_lo=16, n_hi=20, p_hi=6)
    s = q.Server(pool_bytes=1 << 28, max_slots=3)
    tickets = [s.submit(r[3], r[0], r[4], r[5]) for r in reqs]
    outcomes = []
    for t in tickets:
        try:
            s.wait(t, timeout_ms=60000)
            outcomes.append("ok")
        except q.QNAEError as e:
            assert e.status == -3 and "injected" in str(e)
            outcomes.append("failed")
    assert "failed" in outcomes
    assert s.pool_in_use() == 0
    with pytest.raises(q.QNAEError, match="injected"):
        s.submit(reqs[0][3], reqs[0][0], reqs[0][4], reqs[0][5])
    s.close()


@pytest.mark.parametrize("tb", [12, 14])
def test_server_uses_the_tuned_tile_shape(q, tb, monkeypatch):
    """A server copies its context's tile shapes when made: requests of a
    tuned size run with that shape, and each result equals the single path
    on a context with the same shape (half and full states)."""
    for half in ("1", "0"):
        monkeypatch.setenv("QNAE_SERVER_HALF", half)
        ctx = q.Context()
        reqs = requests(24, 40 + tb, n_lo=15, n_hi=20)
        for n in range(15, 21):
            for dt in ("u8", "u16"):
                ctx.set_tune(n, {"tile_bits": tb, "low_run_bits": 5, "page_bit": 18}, cost_dtype=dt)
        with q.Server(pool_bytes=1 << 28, max_slots=8, ctx=ctx) as s:
            tickets = [s.submit(r[3], r[0], r[4], r[5]) for r in reqs]
            got = [s.wait(t, timeout_ms=60000)[0] for t in tickets]
        for r, res in zip(reqs, got):
            n, k, m, cl, g, b = r
            if half == "1":
                ref = q.qaoa_run_z2(q.build_cost_diagonal_z2(cl, n, ctx=ctx), n, m, g, b, ctx=ctx)
            else:
                ref = q.qaoa_run(q.build_cost_diagonal(cl, n, ctx=ctx), n, m, g, b, ctx=ctx)
            assert close(res, ref), (tb, half, n, m)
        ctx.close()
