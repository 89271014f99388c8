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


def _gfx950_code_objects(lib_path):
    """The gfx950 code objects of a built HIP shared library: its
    .hip_fatbin section holds one offload bundle per translation unit."""
    import struct
    import tempfile
    objcopy = "/opt/rocm/llvm/bin/llvm-objcopy"
    with tempfile.TemporaryDirectory() as d:
        sec = os.path.join(d, "fatbin")
        run([objcopy, f"--dump-section=.hip_fatbin={sec}", lib_path, os.path.join(d, "stripped")])
        data = open(sec, "rb").read()
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    out, at = [], data.find(magic)
    while at >= 0:
        (entries,) = struct.unpack_from("<Q", data, at + len(magic))
        p = at + len(magic) + 8
        for _ in range(entries):
            off, size, tlen = struct.unpack_from("<QQQ", data, p)
            triple = data[p + 24:p + 24 + tlen].decode()
            p += 24 + tlen
            if triple.endswith("gfx950"):
                out.append(data[at + off:at + off + size])
        at = data.find(magic, at + 1)
    return out


@pytest.mark.skipif(not os.path.exists("/opt/rocm/llvm/bin/llvm-objdump"), reason="ROCm LLVM tools not available")
def test_no_packed_fp32_in_device_code(tmp_path):
    """The build keeps the device compiler from forming packed FP32
    instructions: none appears in the library's gfx950 code."""
    from paper_2401_02852_amd import _binding
    path = _binding.library_path()
    if not os.path.exists(path):
        pytest.skip("libqnae.so not built")
    cos = _gfx950_code_objects(path)
    assert len(cos) >= 4  # cost, sweep, adjoint, sample
    packed = scalar = 0
    for i, co in enumerate(cos):
        f = tmp_path / f"co{i}.o"
        f.write_bytes(co)
        asm = run(["/opt/rocm/llvm/bin/llvm-objdump", "-d", str(f)])
        scalar += sum(asm.count(op) for op in ("v_fma_f32", "v_fmac_f32", "v_add_f32", "v_mul_f32"))
        packed += sum(asm.count(op) for op in ("v_pk_add_f32", "v_pk_mul_f32", "v_pk_fma_f32"))
    assert scalar > 1000  # the butterflies are there, as unpacked FP32 operations
    assert packed == 0
