"""Runs tests/tables_check.cpp: the per-tile dispatch tables the sweep reads
(paper_2603_03019_amd/csrc/hq_tables.h), rebuilt into coefficients on the
CPU and compared with the oracle's Algorithm 3, for several deployments and
tile widths (bounds-checked, with the sanitizers)."""
import os
import subprocess

import numpy as np
import pytest

from oracle import cpu
from paper_2603_03019_amd.instances import config_instance

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("tc") / "tables_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-pthread", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "paper_2603_03019_amd", "csrc"),
                    os.path.join(ROOT, "tests", "tables_check.cpp"), "-o", exe], check=True)
    return exe


def _write(path, inst, b, states, expect):
    with open(path, "wb") as f:
        np.array([inst.N, inst.J, b, len(states)], dtype="<i4").tofile(f)
        np.asarray(inst.lam, dtype="<f8").tofile(f)
        np.asarray(inst.nu, dtype="<f8").tofile(f)
        np.asarray(inst.pref, dtype="<i4").reshape(-1).tofile(f)
        np.asarray(states, dtype="<u4").tofile(f)
        np.asarray(expect, dtype="<f8").reshape(-1).tofile(f)


@pytest.mark.parametrize("cfg,idx,N,J", [(1, 0, 10, 40), (2, 1, 14, 200), (3, 2, 16, 300), (4, 3, 12, 100)])
def test_tables_rebuild_algorithm3(checker, tmp_path, cfg, idx, N, J):
    inst = config_instance(cfg, idx, N=N, J=J)
    rng = np.random.default_rng(idx)
    states = np.unique(np.r_[rng.integers(0, 1 << N, 400), [0, (1 << N) - 1, 1, (1 << N) - 2]]).astype(np.uint32)
    expect = np.array([cpu.up_coefficients(inst, int(m)) for m in states])
    for b in sorted({1, 4, min(10, N), N - 2, N}):
        path = str(tmp_path / f"case_{b}.bin")
        _write(path, inst, b, states, expect)
        r = subprocess.run([checker, path], capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr
