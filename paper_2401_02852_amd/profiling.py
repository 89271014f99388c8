"""Summaries of rocprofv3 output for the sweep kernels.

    python -m paper_2401_02852_amd.profiling trace DIR PREFIX OUT.txt -- CMD...
    python -m paper_2401_02852_amd.profiling pmc FETCH_CSV WRITE_CSV \
        COPY_FETCH_CSV COPY_WRITE_CSV COPY_BYTES N OUT.txt -- CMD...

    python -m paper_2401_02852_amd.profiling counters OUT.txt CSV... -- CMD...

`trace` condenses a `--kernel-trace --stats --output-format csv` run into
per-kernel call counts and average durations. `pmc` turns two counter runs
(FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) into HBM bytes per launch of
each sweep kind. Each counter is scaled by what it reads for a plain device
copy of COPY_BYTES (the copy reads and writes COPY_BYTES), so the figures are
bytes, whatever the counter's own unit convention. The text after `--` is the
command that produced the input and is written into the summary. `counters`
averages any set of counters per launch of each kernel kind.

The summary records a hash of the kernel sources, so a reader (bench.py) can
tell whether the counters still describe the current kernels.
"""
from __future__ import annotations

import csv
import hashlib
import os
import re
import sys
from collections import OrderedDict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/sweep.hip", "csrc/tile.h", "csrc/cost.hip"]
ADJOINT_SOURCES = ["csrc/adjoint.hip", "csrc/tile.h"]

KIND_NAMES = {"0": "sweep_first", "1": "sweep_middle", "2": "sweep_boundary", "3": "sweep_final", "4": "sweep_p0"}


def kernel_source_hash(sources=None) -> str:
    """Hash of the forward kernels' sources (the headline traffic figure is
    tied to it), or of the given sources."""
    h = hashlib.sha256()
    for rel in sources or KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _hash_lines():
    return [f"kernel_sources_sha256_16: {kernel_source_hash()}",
            f"adjoint_sources_sha256_16: {kernel_source_hash(ADJOINT_SOURCES)}"]


def short_name(name: str) -> str:
    name = re.sub(r"qnae::\(anonymous namespace\)::", "", name)
    # (a sixth argument, whether the tiles pass through layout L1, is not
    # shown: both variants of a kind move the same bytes and are summed)
    m = re.match(r"void sweep_kernel<(\d+), ([a-z ]+), (\d)(?:, (true|false))?(?:, (true|false))?(?:, \d)?>", name)
    if m:
        half = ",half" if m.group(4) == "true" else ""
        ckpt = "_ckpt" if m.group(5) == "true" else ""
        return (f"sweep_kernel<TB={m.group(1)},{m.group(2).replace('unsigned ', 'u')}{half}> "
                f"{KIND_NAMES[m.group(3)]}{ckpt}")
    m = re.match(r"void adjoint_kernel<([a-z ]+), (\d)(?:, (true|false))?(?:, (true|false))?(?:, (true|false))?>", name)
    if m:
        kind = {"0": "middle", "1": "boundary", "2": "end"}[m.group(2)]
        weigh = "_weigh" if m.group(3) == "true" else ""
        stream = ",stream" if m.group(4) == "true" else ""
        q1 = ",q1" if m.group(5) == "true" else ""
        return f"adjoint_kernel<{m.group(1).replace('unsigned ', 'u')}{stream}{q1}> adjoint_{kind}{weigh}"
    return name.split("(")[0].replace("void ", "")


def trace(dirpath, prefix, out, cmd):
    rows = list(csv.DictReader(open(os.path.join(dirpath, f"{prefix}_kernel_stats.csv"))))
    lines = [f"# rocprofv3 kernel trace summary", f"command: {cmd}", *_hash_lines(), "",
             f"{'kernel':62s} {'calls':>6s} {'avg_ms':>9s} {'min_ms':>9s} {'max_ms':>9s} {'pct':>6s}"]
    agg = OrderedDict()  # rows of one short name summed
    for r in rows:
        a = agg.setdefault(short_name(r["Name"]), [0, 0.0, float("inf"), 0.0, 0.0])
        a[0] += int(r["Calls"])
        a[1] += float(r["AverageNs"]) * int(r["Calls"])
        a[2] = min(a[2], float(r["MinNs"]))
        a[3] = max(a[3], float(r["MaxNs"]))
        a[4] += float(r["Percentage"])
    for k, (calls, tot, lo, hi, pct) in sorted(agg.items(), key=lambda kv: -kv[1][4]):
        lines.append(f"{k:62s} {calls:6d} {tot / calls / 1e6:9.4f} {lo / 1e6:9.4f} {hi / 1e6:9.4f} {pct:6.2f}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _counter_rows(path):
    return [(short_name(r["Kernel_Name"]), float(r["Counter_Value"])) for r in csv.DictReader(open(path))]


def _copy_value(path):
    vals = [v for k, v in _counter_rows(path) if "copyBuffer" in k]
    return max(vals)


def pmc(fetch_csv, write_csv, cfetch_csv, cwrite_csv, copy_bytes, n, out, cmd):
    copy_bytes = int(copy_bytes)
    n = int(n)
    fscale = copy_bytes / (_copy_value(cfetch_csv) * 1024.0)
    wscale = copy_bytes / (_copy_value(cwrite_csv) * 1024.0)
    fetch = _counter_rows(fetch_csv)
    write = _counter_rows(write_csv)
    agg = OrderedDict()
    for (k, fv), (k2, wv) in zip(fetch, write):
        assert k == k2, (k, k2)
        a = agg.setdefault(k, [0, 0.0, 0.0])
        a[0] += 1
        a[1] += fv * 1024.0 * fscale
        a[2] += wv * 1024.0 * wscale
    amps = float(2 ** n)
    lines = ["# HBM traffic per launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (separate runs)",
             f"command: {cmd}",
             *_hash_lines(),
             f"copy_calibration: plain device copy of {copy_bytes} bytes; FETCH_SIZE scale {fscale:.4f}, "
             f"WRITE_SIZE scale {wscale:.4f} (bytes per counter KiB / 1024)",
             f"state_amplitudes: {int(amps)}", "",
             f"{'kernel':62s} {'calls':>6s} {'fetch_B':>14s} {'write_B':>14s} {'fetch_B/amp':>11s} {'write_B/amp':>11s}"]
    for k, (c, fb, wb) in agg.items():
        lines.append(f"{k:62s} {c:6d} {fb / c:14.0f} {wb / c:14.0f} {fb / c / amps:11.3f} {wb / c / amps:11.3f}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def counters(out, cmd, csvs):
    """Per kernel kind, the average per launch of every counter in the given
    `--pmc ... --output-format csv` counter_collection files."""
    agg = OrderedDict()
    names = []
    for path in csvs:
        for r in csv.DictReader(open(path)):
            k, c = short_name(r["Kernel_Name"]), r["Counter_Name"]
            if c not in names:
                names.append(c)
            a = agg.setdefault(k, {}).setdefault(c, [0, 0.0])
            a[0] += 1
            a[1] += float(r["Counter_Value"])
    lines = ["# rocprofv3 counters per launch (average over launches of each kernel kind)", f"command: {cmd}",
             *_hash_lines(), "",
             f"{'kernel':62s} " + " ".join(f"{c:>34s}" for c in names)]
    for k, per in agg.items():
        lines.append(f"{k:62s} " + " ".join(f"{per[c][1] / per[c][0]:34.1f}" if c in per else f"{'-':>34s}"
                                            for c in names))
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def read_traffic(path):
    """{kernel short name: (fetch bytes, write bytes) per launch} and the
    source hash recorded in a pmc summary."""
    out, sha = {}, None
    with open(path) as f:
        for line in f:
            if line.startswith("kernel_sources_sha256_16:"):
                sha = line.split(":", 1)[1].strip()
            m = re.match(r"^(\S.*?)\s+(\d+)\s+(\d+)\s+(\d+)\s+[\d.]+\s+[\d.]+$", line.rstrip())
            if m and not line.startswith("kernel"):
                out[m.group(1)] = (float(m.group(3)), float(m.group(4)))
    return out, sha


if __name__ == "__main__":
    argv = sys.argv[1:]
    cmd = ""
    if "--" in argv:
        i = argv.index("--")
        cmd = " ".join(argv[i + 1:])
        argv = argv[:i]
    if argv[0] == "trace":
        trace(*argv[1:4], cmd)
    elif argv[0] == "pmc":
        pmc(*argv[1:8], cmd)
    elif argv[0] == "counters":
        counters(argv[1], cmd, argv[2:])
    else:
        sys.exit(__doc__)
