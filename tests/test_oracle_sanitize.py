"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/oracle.c is compiled with gcc together with ``oracle_sanitize_driver.c``
(which calls every exported oracle function on ragged small inputs into
exactly sized buffers, and checks thread-count independence and the refusal
of invalid sizes) with ``-fsanitize=address,undefined``; any out-of-bounds
access, use after free, leak, or undefined operation aborts the run.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE_SRC = os.path.join(ROOT, "oracle", "oracle.c")
DRIVER_SRC = os.path.join(HERE, "oracle_sanitize_driver.c")

FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-Wall"]


def _sanitizer_available(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text("int main(void) { return 0; }\n")
    r = subprocess.run(["gcc", "-fsanitize=address,undefined", "-o", str(tmp_path / "probe"),
                        str(src)], capture_output=True, text=True)
    return r.returncode == 0


def test_oracle_clean_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None or not _sanitizer_available(tmp_path):
        pytest.skip("gcc with AddressSanitizer/UndefinedBehaviorSanitizer is not available")
    exe = tmp_path / "oracle_sanitized"
    build = subprocess.run(["gcc", *FLAGS, "-o", str(exe), ORACLE_SRC, DRIVER_SRC, "-lm"],
                           capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "4"
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.strip() == "ok"
    assert "runtime error" not in run.stderr
