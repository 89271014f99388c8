"""Whole cost diagonals at full size against the oracle, bit for bit.

The oracle's diagonals (Section 3.2, eq. knaesatobj with the NAE predicate of
Appendix A.2, eq. demorgannae; the k-SAT predicate of Section 2.2) are stored
as SHA-256 digests of consecutive chunks of 2^24 states and of the whole
diagonal in natural index order (``tests/golden/cost_digests.json``, written
by ``oracle/make_digests.py`` from the oracle alone). Here the GPU's diagonal
is copied back chunk by chunk and hashed the same way: every entry of the
n = 24, 28 and 30 workloads, an n = 30 k-SAT diagonal, an n = 30 uint16
diagonal (m = 270) and an n = 33 diagonal (64-bit basis indices) is compared,
through the single, batched and half-diagonal builders.
"""
import hashlib
import json
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from workloads import instances as inst

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def q():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2401_02852_amd as q
    q.load_library()
    return q


@pytest.fixture(scope="module")
def digests():
    with open(os.path.join(ROOT, "tests", "golden", "cost_digests.json")) as f:
        return json.load(f)


def device_digests(cost, lg, count):
    """(chunk digests, whole SHA-256) of the first `count` chunks of 2^lg
    entries of a device cost diagonal, hashed as little-endian bytes."""
    per = 1 << lg
    group = max(1, (1 << 30) // (per * cost.element_size()))  # about 1 GiB per copy
    whole = hashlib.sha256()
    chunks = []
    with ThreadPoolExecutor(8) as pool:
        for g0 in range(0, count, group):
            g1 = min(count, g0 + group)
            host = cost[g0 * per:g1 * per].cpu().numpy()
            raw = host.astype(host.dtype.newbyteorder("<"), copy=False).tobytes()
            nb = per * host.dtype.itemsize
            parts = [raw[i * nb:(i + 1) * nb] for i in range(g1 - g0)]
            chunks += pool.map(lambda b: hashlib.sha256(b).hexdigest()[:16], parts)
            whole.update(raw)
            del host, raw, parts
    return chunks, whole.hexdigest()


def first_mismatch(got, want):
    bad = [i for i, (a, b) in enumerate(zip(got, want)) if a != b]
    return bad[0] if bad else None


def need_memory(nbytes):
    import torch
    free, _ = torch.cuda.mem_get_info()
    if free < nbytes + (1 << 30):
        pytest.skip("not enough device memory")


def workload(rec):
    return inst.instance(rec["n"], rec["k"], rec["m"], rec["seed"])


@pytest.mark.parametrize("name", ["nae3_n24_p10", "nae3_n28_p10", "nae3_n30_p10", "sat3_n30", "nae5_n30_u16",
                                  "nae3_n33"])
def test_whole_diagonal_matches_oracle(q, digests, name):
    import torch
    rec = digests[name]
    n, m, lg = rec["n"], rec["m"], rec["chunk_log2"]
    dtype = torch.uint8 if rec["dtype"] == "uint8" else torch.uint16
    need_memory((1 << n) * (1 if dtype == torch.uint8 else 2))
    print(f"\n[{name}] n={n} m={m} {rec['predicate']} {rec['dtype']}", flush=True)
    out = torch.empty(1 << n, dtype=dtype, device="cuda")
    c, sols = q.build_cost_diagonal(workload(rec), n, out=out, count_solutions=True, predicate=rec["predicate"])
    chunks, whole = device_digests(c, lg, len(rec["chunks"]))
    assert first_mismatch(chunks, rec["chunks"]) is None, \
        f"chunk {first_mismatch(chunks, rec['chunks'])} (states from {first_mismatch(chunks, rec['chunks']) << lg})"
    assert whole == rec["sha256"]
    assert sols == rec["num_zeros"]
    del out, c
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", ["nae3_n28_p10", "sat3_n30", "nae5_n30_u16"])
def test_whole_diagonal_batched_builder(q, digests, name):
    """The batched builder (a separate launch over several diagonals) gives
    the same diagonal, next to a small second job in the same launch."""
    import torch
    rec = digests[name]
    n, lg = rec["n"], rec["chunk_log2"]
    dtype = torch.uint8 if rec["dtype"] == "uint8" else torch.uint16
    need_memory((1 << n) * (1 if dtype == torch.uint8 else 2))
    print(f"\n[{name}] batched", flush=True)
    small = inst.instance(12, rec["k"], rec["m"], 1)
    outs = [torch.empty(1 << 12, dtype=dtype, device="cuda"), torch.empty(1 << n, dtype=dtype, device="cuda")]
    (c12, c), (s12, sols) = q.build_cost_diagonals([small, workload(rec)], [12, n], outs=outs, count_solutions=True,
                                                   predicate=rec["predicate"])
    chunks, whole = device_digests(c, lg, len(rec["chunks"]))
    assert first_mismatch(chunks, rec["chunks"]) is None
    assert whole == rec["sha256"] and sols == rec["num_zeros"]
    import oracle
    ref12 = oracle.cost(small, 12, predicate=rec["predicate"])
    assert np.array_equal(c12.cpu().numpy().astype(np.int64), ref12) and s12 == int((ref12 == 0).sum())
    del outs, c, c12
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", ["nae3_n28_p10", "nae3_n30_p10", "nae3_n33"])
def test_half_diagonal_matches_oracle(q, digests, name):
    """The half diagonal (x < 2^(n-1), NAE flip symmetry) is the first half
    of the whole one: its chunks equal the oracle's first half of chunks."""
    import torch
    rec = digests[name]
    n, lg = rec["n"], rec["chunk_log2"]
    need_memory(1 << (n - 1))
    print(f"\n[{name}] half", flush=True)
    c, sols = q.build_cost_diagonal_z2(workload(rec), n, count_solutions=True)
    half = len(rec["chunks"]) // 2
    chunks, _ = device_digests(c, lg, half)
    assert first_mismatch(chunks, rec["chunks"][:half]) is None
    assert sols == rec["num_zeros"]
    del c
    torch.cuda.empty_cache()
