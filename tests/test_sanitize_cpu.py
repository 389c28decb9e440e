"""AddressSanitizer and UndefinedBehaviorSanitizer builds on the CPU: the C
oracle under a driver that calls every entry point on two small lattices,
and the host side of the HIP library (device code built as usual, host code
instrumented) under a driver of its C-ABI paths that need no GPU
(validation, null and invalid arguments, a context request without a usable
device).  Any sanitizer report fails the test."""
import concurrent.futures
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
REPORTS = ("ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:")


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert not any(k in out for k in REPORTS), out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["gcc", "-std=gnu11", "-fopenmp", *SAN, os.path.join(ROOT, "oracle", "wdr_oracle.c"),
                           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm", "-o", exe])
    out = _run(exe)
    assert "cgne" in out


def test_host_runtime_under_sanitizers(tmp_path):
    hipcc, clang = "/opt/rocm/bin/hipcc", "/opt/rocm/llvm/bin/clang"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not found")
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_1112_1243_amd", "csrc", "*.hip")))
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f] if f.startswith("-fsan") or f.startswith("-fno-san") else [f]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cmd = [hipcc, "--offload-arch=gfx950", "-fPIC", "-std=c++17", *host_san, "-Xclang", "-target-feature",
               "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with concurrent.futures.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    drv = str(tmp_path / "runtime_driver.o")
    subprocess.check_call([clang, *SAN, "-I", os.path.join(ROOT, "include"), "-c",
                           os.path.join(ROOT, "tests", "sanitize", "runtime_driver.c"), "-o", drv])
    exe = str(tmp_path / "runtime_driver")
    subprocess.check_call([clang + "++", "-fsanitize=address,undefined", "-o", exe, drv, *objs, "-L/opt/rocm/lib",
                           "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    out = _run(exe)
    assert "0 failures" in out
