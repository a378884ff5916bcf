"""Runs tests/layout_check.cpp: the C++ index helpers that the layer kernels
use (paper_2603_03019_amd/csrc/hq_layout.h), exercised on the CPU with
bounds-checked tables for every (N, b) up to N = 14."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("lc") / "layout_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "paper_2603_03019_amd", "csrc"),
                    os.path.join(ROOT, "tests", "layout_check.cpp"), "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("N", list(range(1, 15)))
def test_layout_indices(checker, N):
    for b in range(1, min(N, 12) + 1):
        if N - b > 26:
            continue
        r = subprocess.run([checker, str(N), str(b)], capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr
