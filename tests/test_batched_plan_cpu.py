"""The batched planner and workspace layouts of the host runtime, on the CPU.

A fault of the persistent batched launch once came from a unit table sized for
fewer units than the planner could admit (the upload ran into the next region).
This test builds tests/batched_plan_driver.cpp, which compiles csrc/api.cpp
itself into the driver, so the functions under test are the ones the entry
points call.  It plans the 256-system ensemble of the batched workload (sizes
U{500..5000}, seed 4) and uneven, empty, tiny and huge ensembles for chip sizes
of 80, 256 and 304 CUs, 1 to 16 resident blocks per CU, blocks of 64 to 256
threads and 1, 2 or 4 rows per lane, and checks every unit, slot and table
against its region (see the driver).  No GPU is used.
"""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

from paper_0706_3060_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_0706_3060_amd")
CSRC = os.path.join(PKG, "csrc")
KERNEL_OBJECTS = ["forward.o", "batched.o", "adjoint.o", "jerk.o", "probe.o", "noalloc.o", "symmetric.o", "bsym.o", "bsym_adj.o", "symjerk.o"]
ROCM_INCLUDE = "/opt/rocm/include"
ROCM_LIB = "/opt/rocm/lib"


def _offsets(sizes):
    return np.concatenate([[0], np.cumsum(np.asarray(sizes, dtype=np.int64))]).astype(np.int64)


def test_batched_plans_stay_inside_their_regions(tmp_path):
    if shutil.which("g++") is None or not os.path.isdir(ROCM_INCLUDE):
        pytest.skip("g++ and the ROCm headers are needed")
    build_dir = os.path.join(PKG, "_build")
    if not all(os.path.exists(os.path.join(build_dir, o)) for o in KERNEL_OBJECTS):
        sys.path.insert(0, ROOT)
        from paper_0706_3060_amd import build
        build.build(verbose=False)
    exe = tmp_path / "plan_driver"
    cc = subprocess.run(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INCLUDE,
                         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
                         os.path.join(HERE, "batched_plan_driver.cpp"), "-o", str(exe)]
                        + [os.path.join(build_dir, o) for o in KERNEL_OBJECTS]
                        + ["-L" + ROCM_LIB, "-lamdhip64", "-Wl,-rpath," + ROCM_LIB],
                        capture_output=True, text=True)
    assert cc.returncode == 0, cc.stderr[-4000:]
    rng = np.random.default_rng(7)
    ensembles = {
        "ensemble256_seed4": W.ensemble_sizes(256, 4),
        "uneven": [0, 1, 0, 2, 63, 64, 65, 20000, 1, 0, 5000, 129, 3, 4097],
        "tiny4096": rng.integers(0, 41, 4096),
        "huge": [200000],
        "empty": [],
        "random24": rng.integers(0, 401, 24),
        "wide": rng.integers(500, 50001, 64),
    }
    files = []
    for name, sizes in ensembles.items():
        f = tmp_path / (name + ".i64")
        _offsets(sizes).tofile(str(f))
        files.append(str(f))
    run = subprocess.run([str(exe)] + files, capture_output=True, text=True, timeout=600)
    assert run.returncode == 0, (run.stdout + run.stderr)[-4000:]
    lines = [l for l in run.stdout.splitlines() if "violations=0" in l]
    assert len(lines) == len(files), run.stdout
