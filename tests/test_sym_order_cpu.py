"""The tile order of the symmetric all-pairs launch, on the CPU.

tests/sym_order_driver.cpp includes csrc/kernels.h, whose sym_tile_of maps each
workgroup of a launch to its tile (the kernels call the same functions).  For
block counts from 1 to 2048, including every remainder modulo the strip height
and the XCD count, the tiles must be the upper triangle of the block grid, each
exactly once, with fewer than 8 idle workgroups; the order index must invert;
the shares of 1, 2, 3, 8 and 13 equal parts (nbody_forces_share) must cover the
triangle exactly once; and the tiles that one XCD runs at a time must share
their blocks (at most 25 distinct blocks in any 96 consecutive workgroups of an
XCD, against about 97 for a row-major order).
"""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_0706_3060_amd", "csrc")
ROCM_INCLUDE = "/opt/rocm/include"


def test_symmetric_tile_order_shares_and_windows(tmp_path):
    if shutil.which("g++") is None or not os.path.isdir(ROCM_INCLUDE):
        pytest.skip("g++ and the ROCm headers are needed")
    exe = tmp_path / "sym_order"
    cc = subprocess.run(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INCLUDE,
                         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
                         os.path.join(HERE, "sym_order_driver.cpp"), "-o", str(exe)],
                        capture_output=True, text=True)
    assert cc.returncode == 0, cc.stderr[-4000:]
    sizes = list(range(1, 41)) + [63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1000, 2048]
    run = subprocess.run([str(exe)] + [str(s) for s in sizes], capture_output=True, text=True, timeout=300)
    assert run.returncode == 0, (run.stdout + run.stderr)[-4000:]
    lines = [l for l in run.stdout.splitlines() if l.endswith(" ok")]
    assert len(lines) == len(sizes), run.stdout
    for l in lines:
        nblk = int(re.search(r"nblk=(\d+)", l).group(1))
        worst = int(re.search(r"window_blocks_max=(\d+)", l).group(1))
        if nblk >= 64:
            assert worst <= 25, l
