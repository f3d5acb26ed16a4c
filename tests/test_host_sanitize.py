"""The host runtime (C ABI validation, workspace carving, configuration and
tuning-file handling in csrc/api.cpp) under AddressSanitizer and
UndefinedBehaviorSanitizer.

api.cpp is host code only, so gcc builds it with ``-fsanitize=address,undefined``;
it is linked with the kernels' objects from the regular build into a separate
library, and the CPU boundary tests (tests/test_abi_cpu.py) run against that
library in a child process with the sanitizer runtimes preloaded.  No kernel is
launched: every call there returns before any work is enqueued.
"""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_0706_3060_amd")
CSRC = os.path.join(PKG, "csrc")
KERNEL_OBJECTS = ["forward.o", "batched.o", "adjoint.o", "jerk.o", "probe.o", "noalloc.o", "symmetric.o", "bsym.o", "bsym_adj.o", "symjerk.o"]
ROCM_INCLUDE = "/opt/rocm/include"
ROCM_LIB = "/opt/rocm/lib"


def _gcc_runtime(name):
    r = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_host_runtime_clean_under_asan_ubsan(tmp_path):
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if shutil.which("g++") is None or not asan or not ubsan:
        pytest.skip("g++ with AddressSanitizer/UndefinedBehaviorSanitizer is not available")
    if not os.path.isdir(ROCM_INCLUDE) or not os.path.isdir(ROCM_LIB):
        pytest.skip("ROCm headers and runtime are not installed")
    build_dir = os.path.join(PKG, "_build")
    if not all(os.path.exists(os.path.join(build_dir, o)) for o in KERNEL_OBJECTS):
        sys.path.insert(0, ROOT)
        from paper_0706_3060_amd import build
        build.build(verbose=False)
    api_obj = tmp_path / "api_sanitized.o"
    cc = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fPIC",
                         "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                         "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INCLUDE,
                         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
                         "-c", os.path.join(CSRC, "api.cpp"), "-o", str(api_obj)],
                        capture_output=True, text=True)
    assert cc.returncode == 0, cc.stderr
    lib = tmp_path / "libnbody_sanitized.so"
    ld = subprocess.run(["g++", "-shared", "-fsanitize=address,undefined", "-o", str(lib), str(api_obj)]
                        + [os.path.join(build_dir, o) for o in KERNEL_OBJECTS]
                        + ["-L" + ROCM_LIB, "-lamdhip64"], capture_output=True, text=True)
    assert ld.returncode == 0, ld.stderr
    env = dict(os.environ)
    env["NBODY_TEST_LIB"] = str(lib)
    env["LD_PRELOAD"] = asan + ":" + ubsan
    # the interpreter and torch are not built with the sanitizer: leaks and
    # allocator-pairing reports from them are not this library's
    env["ASAN_OPTIONS"] = "detect_leaks=0:alloc_dealloc_mismatch=0:detect_odr_violation=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    run = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_abi_cpu.py"),
                          "-q", "-x", "-p", "no:cacheprovider"],
                         capture_output=True, text=True, env=env, cwd=str(tmp_path), timeout=600)
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
