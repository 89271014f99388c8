"""qnae_qaoa_run_noalloc (the entry point that allocates nothing: its device
scratch is the library's static array) against qnae_qaoa_run, both through
the C ABI, on the same inputs: the readout and the final state must be the
same (same kernels, same sweep plan, same summation order). The calls run
back to back with shrinking inputs, so each reuses the static scratch that
the previous, larger call left behind."""
import ctypes

import numpy as np
import pytest

from workloads import instances as inst

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2401_02852_amd as q
    q.load_library()
    return q


def noalloc(q, ctx, cost, n, m, g, b, state):
    """qnae_qaoa_run_noalloc called directly through ctypes."""
    from paper_2401_02852_amd import _binding as B
    import torch
    lib = q.load_library()
    g = np.ascontiguousarray(g, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    res = B._CResult()
    p = g.shape[0]
    f64 = ctypes.POINTER(ctypes.c_double)
    rc = lib.qnae_qaoa_run_noalloc(
        ctx.handle, ctypes.c_void_p(cost.data_ptr()), 1 if cost.dtype == torch.uint8 else 2, n, m,
        g.ctypes.data_as(f64) if p else None, b.ctypes.data_as(f64) if p else None, p,
        ctypes.c_void_p(state.data_ptr()) if state is not None else None, ctypes.byref(res),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, lib.qnae_last_error(ctx.handle)
    return (res.p_success, res.expected_cost, res.norm)


# n, k, m, p, seed: tiled runs (two and one high groups), a uint16 cost, the
# single-workgroup kernel; each call smaller than the one before
CASES = [(22, 3, 46, 6, 1), (17, 3, 36, 3, 2), (16, 5, 300, 2, 3), (12, 3, 25, 4, 4), (9, 3, 19, 2, 5)]


def test_noalloc_matches_qaoa_run(q):
    import torch
    ctx = q.Context()
    for keep in (True, False):
        for n, k, m, p, seed in CASES:
            if not keep and n > 14:
                continue  # above n = 14 the state buffer is required
            print(f"\n[noalloc] n={n} k={k} m={m} p={p} keep={keep}", flush=True)
            rng = np.random.default_rng(seed)
            cl = inst.instance(n, k, m, seed)
            # both butterfly forms: |tan beta| <= 1 and > 1 (the flipped relabelling)
            g = rng.uniform(-2, 2, p)
            b = np.where(np.arange(p) % 2 == 0, rng.uniform(-0.7, 0.7, p), rng.uniform(0.9, 2.2, p))
            cost = q.build_cost_diagonal(cl, n, ctx=ctx)
            ref_state = torch.empty(1 << n, dtype=torch.complex64, device="cuda") if keep else None
            got_state = torch.full((1 << n,), 7.0 + 7.0j, dtype=torch.complex64, device="cuda") if keep else None
            ref = tuple(q.qaoa_run(cost, n, m, g, b, state=ref_state, ctx=ctx))
            got = noalloc(q, ctx, cost, n, m, g, b, got_state)
            assert got == ref, (n, got, ref)
            if keep:
                assert torch.equal(got_state, ref_state)
            # and once more on the same scratch: the same again
            assert noalloc(q, ctx, cost, n, m, g, b, got_state) == ref
    ctx.close()


def test_noalloc_rejects_sizes_beyond_its_scratch(q):
    """Sizes beyond the static scratch are refused on the host before any
    device work: more than 2^18 tiles (n = 32 at 13-bit tiles), more than
    4096 layers, phase tables above 2^18 entries; a missing state above
    n = 14."""
    import torch
    from paper_2401_02852_amd import _binding as B
    lib = q.load_library()
    ctx = q.Context()
    cost = torch.zeros(1 << 10, dtype=torch.uint8, device="cuda")
    out = B._CResult()
    f64 = ctypes.POINTER(ctypes.c_double)
    g = np.zeros(5000)
    gp = g.ctypes.data_as(f64)
    vp = ctypes.c_void_p
    state = torch.zeros(16, dtype=torch.complex64, device="cuda")
    calls = [
        ((32, 10, 1, vp(state.data_ptr())), b"tile sums"),
        ((20, 10, 4097, vp(state.data_ptr())), b"layers"),
        ((20, 255, 1100, vp(state.data_ptr())), b"phase tables"),
        ((20, 10, 1, None), b"state_dev is required"),
    ]
    for (n, m, p, st), msg in calls:
        rc = lib.qnae_qaoa_run_noalloc(ctx.handle, vp(cost.data_ptr()), 1, n, m, gp, gp, p, st,
                                       ctypes.byref(out), None)
        assert rc == -1 and msg in lib.qnae_last_error(ctx.handle), (n, m, p)
    ctx.close()
