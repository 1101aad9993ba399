"""The library's host code built with AddressSanitizer and UndefinedBehaviorSanitizer (the device
code is not instrumented), driven by tests/abi_host_check.c through the C ABI's argument
validation, default tables and error strings: calls that return before any HIP call, so no GPU
is needed."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)


def test_host_code_under_asan_ubsan(tmp_path):
    from paper_2407_09848_amd import build as B
    try:
        hipcc = B._hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    clang = "/opt/rocm/lib/llvm/bin/clang"
    if not os.path.exists(clang):
        clang = shutil.which("clang")
    if clang is None:
        pytest.skip("clang not available")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f"--offload-arch={B.ARCH}", "-O1", "-g", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", B.CSRC, *san]

    def compile_one(src):
        obj = str(tmp_path / src.replace(".hip", ".o"))
        r = subprocess.run([hipcc, *flags, "-c", os.path.join(B.CSRC, src), "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, B.SOURCES))
    lib = str(tmp_path / "libamgpoly_san.so")
    r = subprocess.run([hipcc, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *san, "-o", lib, *objs],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    exe = str(tmp_path / "abi_host_check")
    r = subprocess.run([clang, "-g", "-fsanitize=address,undefined", "-I", os.path.join(ROOT, "include"),
                        os.path.join(HERE, "abi_host_check.c"), str(lib), f"-Wl,-rpath,{tmp_path}", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0 and "host ABI checks passed" in r.stdout, r.stdout + r.stderr[-3000:]
