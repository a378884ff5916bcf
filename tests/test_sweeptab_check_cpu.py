"""Runs tests/sweeptab_check.cpp: the segment records and low-pattern rows
of the default-shape sweep kernels (paper_2603_03019_amd/csrc/hq_sweeptab.h)
checked on the CPU against positions recomputed as layer start + colex rank,
for every layer, segment and lane, with FP64 and FP32 element offsets."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("st") / "sweeptab_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "paper_2603_03019_amd", "csrc"),
                    os.path.join(ROOT, "tests", "sweeptab_check.cpp"), "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("N", [10, 11, 13, 16, 17])
def test_sweep_tables(checker, N):
    r = subprocess.run([checker, str(N)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
