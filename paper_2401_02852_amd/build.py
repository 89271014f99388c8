"""Build libqnae.so (HIP, gfx950) in-tree, next to this file.

    python -m paper_2401_02852_amd.build

A .hip file is compiled in two passes: the device pass (gfx950 code object,
bundled) carries the device-only code generation flags, and the host pass
embeds that bundle. The packed-FP32 guard below is a gfx950 target feature,
so it never reaches the x86 host compiler.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqnae.so")
SOURCES = ["runtime.cpp", "qnae.cpp", "batch.cpp", "grad.cpp", "server.cpp", "tune.cpp", "sample.cpp", "noalloc.hip",
           "cost.hip", "sweep.hip", "adjoint.hip", "sample.hip"]
ARCH = os.environ.get("QNAE_OFFLOAD_ARCH", "gfx950")
COMMON = ["-fPIC", "-O3", "-std=c++17", "-Wall", "-Wno-unused-result"]
# Keep the device compiler from forming packed FP32 instructions
# (v_pk_add/mul/fma_f32); hipcc -O3 otherwise forms them from plain float code.
DEVICE_ONLY = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    return os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


def compile_steps(src: str, obj: str):
    """Commands that turn one source into one object file."""
    path = os.path.join(CSRC, src)
    if not src.endswith(".hip"):
        return [[hipcc(), "-c", *COMMON, f"--offload-arch={ARCH}", "-o", obj, path]]
    bundle = obj + ".hipfb"
    return [
        [hipcc(), "-c", *COMMON, f"--offload-arch={ARCH}", "--cuda-device-only", *DEVICE_ONLY, "-o", bundle, path],
        [hipcc(), "-c", *COMMON, f"--offload-arch={ARCH}", "--cuda-host-only",
         "-Xclang", "-fcuda-include-gpubinary", "-Xclang", bundle, "-o", obj, path],
    ]


def build(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor
    steps, objs, temps = [], [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, src + ".o")
        steps.append(compile_steps(src, obj))
        objs.append(obj)
        if src.endswith(".hip"):
            temps.append(obj + ".hipfb")

    def compile_one(cmds):
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)

    def cleanup(paths):
        for o in paths:
            if os.path.exists(o):
                os.remove(o)

    jobs = max(1, min(len(steps), os.cpu_count() or 1, int(os.environ.get("MAX_JOBS", "16"))))
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        futures = [pool.submit(compile_one, c) for c in steps]
        # every compile ends before a failure is raised, so none is left
        # writing temporaries behind the caller's back
        errors = [f.exception() for f in futures]
    if any(errors):
        cleanup(objs + temps)
        raise next(e for e in errors if e)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    cleanup(objs + temps)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
