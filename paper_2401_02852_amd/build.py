"""Build libqnae.so (HIP, gfx950) in-tree, next to this file.

    python -m paper_2401_02852_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqnae.so")
SOURCES = ["runtime.cpp", "qnae.cpp", "batch.cpp", "grad.cpp", "server.cpp", "tune.cpp", "sample.cpp", "cost.hip", "sweep.hip", "adjoint.hip", "sample.hip"]
ARCH = os.environ.get("QNAE_OFFLOAD_ARCH", "gfx950")


def build(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    cmds, objs = [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, src + ".o")
        cmd = [hipcc, "-c", "-fPIC", "-O3", "-std=c++17", "-Wall", "-Wno-unused-result",
               f"--offload-arch={ARCH}"]
        if src.endswith(".hip"):
            # Keep the compiler from forming packed FP32 instructions.
            cmd += ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
        cmd += ["-o", obj, path]
        cmds.append(cmd)
        objs.append(obj)

    def compile_one(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    jobs = max(1, min(len(cmds), os.cpu_count() or 1, int(os.environ.get("MAX_JOBS", "16"))))
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        futures = [pool.submit(compile_one, c) for c in cmds]
        # every compile ends before a failure is raised, so none is left
        # writing temporaries behind the caller's back
        errors = [f.exception() for f in futures]
    if any(errors):
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
        raise next(e for e in errors if e)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
