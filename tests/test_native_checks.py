"""Host code under AddressSanitizer and UBSan (no GPU): the oracle's entry
points, and the sweep planner and clause records of the library's runtime."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    run(["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", "-o", exe, os.path.join(NATIVE, "oracle_check.c"),
         os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    out = run([exe], env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1"})
    assert "oracle checks ok" in out


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc not available")
def test_planner_under_sanitizers(tmp_path):
    exe = str(tmp_path / "planner_check")
    csrc = os.path.join(ROOT, "paper_2401_02852_amd", "csrc")
    run(["/opt/rocm/bin/hipcc", "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         "-Xarch_host", "-fno-omit-frame-pointer", "-o", exe, os.path.join(NATIVE, "planner_check.cpp"),
         os.path.join(csrc, "runtime.cpp")])
    out = run([exe], env={**os.environ, "ASAN_OPTIONS": "detect_leaks=0"})
    assert "planner and clause records ok" in out
