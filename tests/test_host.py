"""CPU-side checks: the C ABI library loads and exports every declared symbol,
the input generators follow their recipe, and the benchmark refuses several
GPUs. No GPU compute here."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from workloads import instances as inst

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "qnae.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qnae_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["qnae_create", "qnae_destroy", "qnae_last_error", "qnae_build_cost_diagonal",
                     "qnae_qaoa_run"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2401_02852_amd import _binding
    path = _binding.library_path()
    if not os.path.exists(path):
        pytest.skip("libqnae.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in include/qnae.h but not exported"


def test_error_message_without_context():
    from paper_2401_02852_amd import _binding
    if not os.path.exists(_binding.library_path()):
        pytest.skip("libqnae.so not built")
    lib = _binding.load_library()
    # invalid arguments are rejected before any device work
    rc = lib.qnae_qaoa_run(None, None, 1, 0, 0, None, None, 0, None, None, None)
    assert rc == -1
    assert b"n=0" in lib.qnae_last_error(None)
    rc = lib.qnae_build_cost_diagonal(None, None, 0, 5, 3, None, 7, None, None)
    assert rc == -1
    assert b"cost_dtype" in lib.qnae_last_error(None)


def test_clause_count_rule():
    assert [inst.clause_count(n, 2.1) for n in (12, 15, 22, 24, 25, 28, 30)] == [25, 32, 46, 50, 53, 59, 63]
    assert inst.clause_count(20, 9.0) == 180


def test_random_clauses_distinct_variables_and_signs():
    cl = inst.instance(20, 5, 400, 3)
    assert cl.shape == (400, 5) and cl.dtype == np.int32
    assert np.all(np.abs(cl) >= 1) and np.all(np.abs(cl) <= 20)
    assert all(len(set(np.abs(r))) == 5 for r in cl)
    frac_neg = float((cl < 0).mean())
    assert 0.45 < frac_neg < 0.55
    assert np.array_equal(cl, inst.instance(20, 5, 400, 3))


def test_ramp_angles():
    g, b = inst.ramp_angles(3)
    assert np.allclose(g, [1 / 6, 1 / 3, 1 / 2]) and np.allclose(b, [1 / 3, 1 / 6, 0])


def test_batched_and_serving_recipes():
    batch = inst.batched_workload(count=40)
    assert all(10 <= x["n"] <= 20 and x["k"] in (3, 5) and x["p"] == 5 for x in batch)
    assert all(x["m"] == (inst.clause_count(x["n"], 2.1) if x["k"] == 3 else 9 * x["n"]) for x in batch)
    reqs = inst.serving_workload(count=200)
    t = np.array([r["arrival_s"] for r in reqs])
    assert np.all(np.diff(t) >= 0) and t[0] == 0.0
    assert 0.5 < (len(t) - 1) / t[-1] / 200 < 1.5
    assert all(14 <= r["n"] <= 26 and 2 <= r["p"] <= 20 for r in reqs)


def test_bench_refuses_multiple_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


class _NullCtx:
    """Context stand-in whose handle is NULL: the library validates the
    arguments, then rejects the call, so the binding's marshalling runs without
    a GPU."""
    handle = ctypes.c_void_p(None)
    device = 0


def _lib_or_skip():
    from paper_2401_02852_amd import _binding
    if not os.path.exists(_binding.library_path()):
        pytest.skip("libqnae.so not built")
    return _binding


def test_binding_marshalling_without_gpu():
    import torch
    b = _lib_or_skip()
    cl = inst.instance(8, 3, 10, 0)
    costs = [_fake_cuda(torch.zeros(256, dtype=torch.uint8)), _fake_cuda(torch.zeros(512, dtype=torch.uint8))]
    with pytest.raises(b.QNAEError, match="null context"):
        b.build_cost_diagonals([cl, cl], [8, 9], outs=costs, count_solutions=True, ctx=_NullCtx(), stream=0)
    with pytest.raises(b.QNAEError, match="null context"):
        b.qaoa_run_batched(costs, [8, 9], [10, 10], [[0.1, 0.2], []], [[0.3, 0.4], []], ctx=_NullCtx(), stream=0)
    with pytest.raises(b.QNAEError, match="instance 1"):
        b.qaoa_run_batched(costs, [8, 9], [10, 300], [[0.1], [0.2]], [[0.3], [0.4]], ctx=_NullCtx(), stream=0)
    with pytest.raises(b.QNAEError, match="null context"):
        b.qaoa_run(costs[0], 8, 10, [0.1], [0.2], ctx=_NullCtx(), stream=0)
    with pytest.raises(b.QNAEError, match="literal"):
        b.build_cost_diagonal(np.array([[1, 99]], dtype=np.int32), 8, out=costs[0], ctx=_NullCtx(), stream=0)
    with pytest.raises(b.QNAEError, match="null context"):
        b.build_cost_diagonal(cl, 8, out=costs[0], predicate="sat", ctx=_NullCtx(), stream=0)
    with pytest.raises(b.QNAEError, match="null context"):
        b.build_cost_diagonals([cl, cl], [8, 9], outs=costs, predicate=["sat", "nae"], ctx=_NullCtx(), stream=0)
    with pytest.raises(ValueError, match="predicate"):
        b.build_cost_diagonal(cl, 8, out=costs[0], predicate="xor", ctx=_NullCtx(), stream=0)
    lib = b.load_library()
    assert lib.qnae_build_cost_diagonal_pred(None, None, 0, 5, 3, 7, None, 1, None, None) == -1
    assert b"predicate=7" in lib.qnae_last_error(None)


def test_server_binding_without_gpu():
    b = _lib_or_skip()
    with pytest.raises(b.QNAEError, match="null context"):
        b.Server(pool_bytes=1 << 30, max_slots=4, ctx=_NullCtx())
    lib = b.load_library()
    assert lib.qnae_server_submit(None, None, 0, 4, 1, None, None, 0, None) == -1
    assert lib.qnae_server_destroy(None) == 0


def test_tune_binding_without_gpu():
    b = _lib_or_skip()
    lib = b.load_library()
    t = b._CTune(13, 4, 18, 0, 0.0)
    assert lib.qnae_set_tune(None, 20, 1, ctypes.byref(t)) == -1
    assert b"null context" in lib.qnae_last_error(None)
    assert lib.qnae_autotune(None, 20, 1, 0, ctypes.byref(t), None) == -1
    assert b"reps=0" in lib.qnae_last_error(None)
    assert lib.qnae_autotune(None, 40, 1, 1, ctypes.byref(t), None) == -1
    assert b"n=40" in lib.qnae_last_error(None)


def test_sample_validation_without_gpu():
    b = _lib_or_skip()
    lib = b.load_library()
    u = (ctypes.c_double * 2)(0.5, 1.0)
    out = (ctypes.c_uint64 * 2)()
    assert lib.qnae_sample(None, ctypes.c_void_p(0x1000), 10, None, 0, u, 2, out, None, None) == -1
    assert b"uniforms[1]=1" in lib.qnae_last_error(None)
    assert lib.qnae_sample(None, ctypes.c_void_p(0x1008), 10, None, 0, u, 1, out, None, None) == -1
    assert b"aligned" in lib.qnae_last_error(None)
    assert lib.qnae_sample(None, ctypes.c_void_p(0x1000), 10, None, 0, u, 1, out, None, None) == -1
    assert b"null context" in lib.qnae_last_error(None)


def test_pretrain_host_logic():
    from paper_2401_02852_amd import pretrain
    assert pretrain.running_time([3, 2, 0, 1, 0]) == 3 and pretrain.running_time([1, 1]) == 0
    assert abs(pretrain.r_hat(3) - 2.1760) < 1e-4 and abs(pretrain.r_hat(5) - 10.4938) < 1e-4
    ns = np.arange(12, 20)
    c, d = pretrain.fit_exponent(ns, 2.0 ** (-0.31 * ns + 1.7))
    assert abs(c + 0.31) < 1e-12 and abs(d - 1.7) < 1e-10
    ev = {n: {"mean_p_success": 2.0 ** (-0.2 * n), "median_running_time": 2.0 ** (0.25 * n)} for n in ns}
    ex = pretrain.exponents(ev)
    assert abs(ex["C_hat"] - 0.2) < 1e-12 and abs(ex["C_tilde"] - 0.25) < 1e-12
    assert abs(ex["relative_error"] - 0.25) < 1e-10


def test_cnf_instance_recipe():
    import time
    t0 = time.perf_counter()
    cls = [inst.cnf_instance(16, 9, 176.9, s) for s in range(20)]
    assert time.perf_counter() - t0 < 2.0
    ms = np.array([c.shape[0] for c in cls])
    assert abs(ms.mean() - 176.9 * 16) < 4 * np.sqrt(176.9 * 16 / 20)
    for c in cls:
        assert c.dtype == np.int32 and c.shape[1] == 9
        assert np.all(np.abs(c) >= 1) and np.all(np.abs(c) <= 16)
        assert all(len(set(np.abs(row))) == 9 for row in c[:200])
    allc = np.concatenate(cls)
    assert 0.48 < float((allc < 0).mean()) < 0.52
    counts = np.bincount(np.abs(allc).ravel(), minlength=17)[1:]
    assert counts.min() > 0.9 * counts.mean()
    assert np.array_equal(cls[3], inst.cnf_instance(16, 9, 176.9, 3))


def test_server_cancel_and_pool_without_gpu():
    b = _lib_or_skip()
    lib = b.load_library()
    assert lib.qnae_server_cancel(None, 1) == -1
    assert b"null server" in lib.qnae_last_error(None)
    assert lib.qnae_server_pool_in_use(None, None) == -1
    assert b._STATUS[-6] == "QNAE_ECANCELED"


class _Ctx:
    """Stands in for a Context: the binding's checks run before any call."""
    device = 0
    handle = None


def _fake_cuda(t, index=0):
    """A CPU tensor that reports itself as on cuda:index (the binding's
    checks read these attributes only; nothing reaches the library)."""
    import torch

    class FakeCuda(torch.Tensor):
        @property
        def is_cuda(self):
            return True

        @property
        def device(self):
            return torch.device("cuda", index)

    return torch.Tensor._make_subclass(FakeCuda, t)


def test_binding_rejects_bad_device_buffers():
    """Every wrapper checks a device buffer before the call: on the GPU, on
    the context's device, contiguous, of the right dtype and with exactly
    the entries the call reads or writes."""
    import torch
    from paper_2401_02852_amd import _binding as b
    ctx = _Ctx()
    n, m = 10, 5
    g, bb = [0.1, 0.2], [0.3, 0.4]
    good_cost = _fake_cuda(torch.zeros(1 << n, dtype=torch.uint8))
    cases = [
        (torch.zeros(1 << n, dtype=torch.uint8), "on the GPU"),
        (_fake_cuda(torch.zeros(1 << n, dtype=torch.uint8), index=1), "cuda:1"),
        (_fake_cuda(torch.zeros(1 << n, dtype=torch.int32)), "dtype"),
        (_fake_cuda(torch.zeros(1 << n, dtype=torch.float32)), "dtype"),
        (_fake_cuda(torch.zeros((1 << n) - 1, dtype=torch.uint8)), "entries"),
        (_fake_cuda(torch.zeros(2 << n, dtype=torch.uint8)[::2]), "contiguous"),
    ]
    for cost, msg in cases:
        with pytest.raises(ValueError, match=msg):
            b.qaoa_run(cost, n, m, g, bb, ctx=ctx)
        with pytest.raises(ValueError, match=msg):
            b.qaoa_grad(cost, n, m, g, bb, ctx=ctx)
        with pytest.raises(ValueError, match=msg):
            b.build_cost_diagonal(np.ones((m, 3), dtype=np.int32), n, out=cost, ctx=ctx)
        with pytest.raises(ValueError, match=msg):
            b.qaoa_run_batched([good_cost, cost], [n, n], [m, m], [g, g], [bb, bb], ctx=ctx)
        with pytest.raises(ValueError, match=msg):
            b.build_cost_diagonals([np.ones((m, 3), dtype=np.int32)] * 2, [n, n], outs=[good_cost, cost], ctx=ctx)
        with pytest.raises(ValueError, match=msg):
            b.qaoa_grad_batched([cost], [n], [m], [g], [bb], ctx=ctx)
    states = [
        (torch.zeros(1 << n, dtype=torch.complex64), "on the GPU"),
        (_fake_cuda(torch.zeros(1 << n, dtype=torch.complex128)), "dtype"),
        (_fake_cuda(torch.zeros(1 << (n - 1), dtype=torch.complex64)), "entries"),
        (_fake_cuda(torch.zeros(2 << n, dtype=torch.complex64)[1::2]), "contiguous"),
    ]
    for st, msg in states:
        with pytest.raises(ValueError, match=msg):
            b.qaoa_run(good_cost, n, m, g, bb, state=st, ctx=ctx)
        with pytest.raises(ValueError, match=msg):
            b.sample(st, n, [0.5], ctx=ctx)
        with pytest.raises(ValueError, match=msg):
            b.qaoa_run_batched([good_cost], [n], [m], [g], [bb], states=[st], ctx=ctx)
    half = _fake_cuda(torch.zeros(1 << (n - 1), dtype=torch.uint8))
    with pytest.raises(ValueError, match="entries"):
        b.qaoa_run_z2(good_cost, n, m, g, bb, ctx=ctx)
    with pytest.raises(ValueError, match="entries"):
        b.build_cost_diagonal_z2(np.ones((m, 3), dtype=np.int32), n, out=good_cost, ctx=ctx)
    with pytest.raises(ValueError, match="entries"):
        b.qaoa_run_z2(half, n, m, g, bb, state=_fake_cuda(torch.zeros(1 << n, dtype=torch.complex64)), ctx=ctx)
    with pytest.raises(ValueError, match="outside"):
        b.qaoa_run(good_cost, 40, m, g, bb, ctx=ctx)


def test_misaligned_device_buffers_rejected_without_gpu():
    """The sweeps and the cost kernel access state and cost with 16-byte
    loads and stores: every entry point rejects a misaligned buffer before
    it touches the device."""
    b = _lib_or_skip()
    lib = b.load_library()
    res = b._CResult()
    g = (ctypes.c_double * 1)(0.1)
    vp = ctypes.c_void_p
    assert lib.qnae_qaoa_run(None, vp(0x1000), 1, 20, 5, g, g, 1, vp(0x2008), ctypes.byref(res), None) == -1
    assert b"state_dev is not 16-byte aligned" in lib.qnae_last_error(None)
    assert lib.qnae_qaoa_run_z2(None, vp(0x1000), 1, 20, 5, g, g, 1, vp(0x2004), ctypes.byref(res), None) == -1
    assert b"state_dev is not 16-byte aligned" in lib.qnae_last_error(None)
    assert lib.qnae_qaoa_run(None, vp(0x1001), 1, 20, 5, g, g, 1, None, ctypes.byref(res), None) == -1
    assert b"cost_dev is not 16-byte aligned" in lib.qnae_last_error(None)
    cl = (ctypes.c_int32 * 3)(1, 2, 3)
    assert lib.qnae_build_cost_diagonal(None, cl, 1, 10, 3, vp(0x1008), 1, None, None) == -1
    assert b"cost_dev is not 16-byte aligned" in lib.qnae_last_error(None)
    job = b._CCostJob(cl, 1, 10, 3, 0x1004, 1, None, 0, 0)
    assert lib.qnae_build_cost_diagonal_batched(None, ctypes.byref(job), 1, None) == -1
    assert b"job 0: cost_dev is not 16-byte aligned" in lib.qnae_last_error(None)
    inst_ = b._CInstance(0x1000, 1, 20, 5, 1, g, g, 0x3008, 0)
    assert lib.qnae_qaoa_run_batched(None, ctypes.byref(inst_), 1, ctypes.byref(res), None) == -1
    assert b"instance 0: state_dev is not 16-byte aligned" in lib.qnae_last_error(None)


def test_noalloc_limits_without_gpu():
    """The entry point that allocates nothing refuses, before it touches the
    device, inputs beyond its static scratch: more than 4096 layers, phase
    tables above 2^18 entries, or no state buffer above n = 14."""
    b = _lib_or_skip()
    lib = b.load_library()
    res = b._CResult()
    g = (ctypes.c_double * 5000)()
    vp = ctypes.c_void_p
    assert lib.qnae_qaoa_run_noalloc(None, vp(0x1000), 1, 20, 5, g, g, 4097, vp(0x2000), ctypes.byref(res), None) == -1
    assert b"layers" in lib.qnae_last_error(None)
    assert lib.qnae_qaoa_run_noalloc(None, vp(0x1000), 1, 20, 255, g, g, 1100, vp(0x2000), ctypes.byref(res),
                                     None) == -1
    assert b"phase tables" in lib.qnae_last_error(None)
    assert lib.qnae_qaoa_run_noalloc(None, vp(0x1000), 1, 20, 5, g, g, 3, None, ctypes.byref(res), None) == -1
    assert b"state_dev is required" in lib.qnae_last_error(None)
    assert lib.qnae_qaoa_run_noalloc(None, vp(0x1000), 1, 20, 5, g, g, 3, vp(0x2008), ctypes.byref(res), None) == -1
    assert b"aligned" in lib.qnae_last_error(None)
    assert lib.qnae_qaoa_run_noalloc(None, vp(0x1000), 1, 20, 5, g, g, 3, vp(0x2000), ctypes.byref(res), None) == -1
    assert b"null context" in lib.qnae_last_error(None)


def test_prepared_batch_marshalling_without_gpu():
    """Prepared batches check their buffers once and marshal angles per run:
    a 2-D angle array must match every instance's p, lists are checked per
    instance; the call then reaches the library (which rejects the null
    context)."""
    import torch
    b = _lib_or_skip()
    ctx = _NullCtx()
    costs = [_fake_cuda(torch.zeros(1 << 10, dtype=torch.uint8)), _fake_cuda(torch.zeros(1 << 11, dtype=torch.uint8))]
    with pytest.raises(ValueError, match="entries"):
        b.PreparedBatch(costs, [10, 12], [5, 5], [2, 2], ctx=ctx)
    pb = b.PreparedBatch(costs, [10, 11], [5, 5], [2, 2], ctx=ctx)
    with pytest.raises(ValueError, match="shape"):
        pb.run(np.zeros((2, 3)), np.zeros((2, 3)))
    with pytest.raises(ValueError, match="prepared p"):
        pb.run([np.zeros(2), np.zeros(1)], [np.zeros(2), np.zeros(2)])
    with pytest.raises(b.QNAEError, match="null context"):
        pb.run(np.zeros((2, 2)), np.zeros((2, 2)), stream=0)
    with pytest.raises(b.QNAEError, match="null context"):
        pb.run([np.zeros(2), np.zeros(2)], [np.zeros(2), np.zeros(2)], stream=0)
    cl = inst.instance(10, 3, 5, 0)
    with pytest.raises(ValueError, match="entries"):
        b.PreparedCostBuild([cl, cl], [10, 12], outs=costs, ctx=ctx)
    cb = b.PreparedCostBuild([cl, inst.instance(11, 3, 5, 1)], [10, 11], outs=costs, ctx=ctx)
    with pytest.raises(b.QNAEError, match="null context"):
        cb.build(count_solutions=True, stream=0)


def test_profile_summaries_name_and_sum_kernel_variants(tmp_path):
    """Profile summaries: short kernel names for every template form the
    library launches, and one row per short name (the per-launch layout
    variants of a sweep kind summed, calls weighting the average)."""
    from paper_2401_02852_amd import profiling as pr
    ns = "void qnae::(anonymous namespace)::"
    assert pr.short_name(ns + "sweep_kernel<13, unsigned char, 2, false, false, 1>(qnae::SweepArgs)") == \
        "sweep_kernel<TB=13,uchar> sweep_boundary"
    assert pr.short_name(ns + "sweep_kernel<14, unsigned short, 3, true, false, 2>(qnae::SweepArgs)") == \
        "sweep_kernel<TB=14,ushort,half> sweep_final"
    assert pr.short_name(ns + "sweep_kernel<13, unsigned char, 2, false, true, 0>(qnae::SweepArgs)") == \
        "sweep_kernel<TB=13,uchar> sweep_boundary_ckpt"
    assert pr.short_name(ns + "adjoint_kernel<unsigned char, 1, false, true, true>(qnae::AdjointArgs)") == \
        "adjoint_kernel<uchar,stream,q1> adjoint_boundary"
    assert pr.short_name(ns + "adjoint_kernel<unsigned short, 0, true, false, false>(qnae::AdjointArgs)") == \
        "adjoint_kernel<ushort> adjoint_middle_weigh"
    stats = tmp_path / "p_kernel_stats.csv"
    stats.write_text(
        '"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs","StdDev"\n'
        f'"{ns}sweep_kernel<13, unsigned char, 1, false, false, 1>(qnae::SweepArgs)",3,9000,3000,60,2900,3100,1\n'
        f'"{ns}sweep_kernel<13, unsigned char, 1, false, false, 2>(qnae::SweepArgs)",1,1000,1000,40,1000,1000,0\n')
    out = tmp_path / "trace.txt"
    pr.trace(str(tmp_path), "p", str(out), "cmd")
    rows = [l for l in out.read_text().splitlines() if l.startswith("sweep_kernel")]
    assert len(rows) == 1
    f = rows[0].split()
    assert f[-5:] == ["4", "0.0025", "0.0010", "0.0031", "100.00"]
