"""The residual-check schedule and the stall rule of the outer loop
(csrc/hq_schedule.h), run on the CPU through tests/schedule_check.cpp
against model residuals: a geometric decay reaches tol with few checks; a
residual stuck at a rounding floor above tol, or a growing one, ends the
solve early as not converged instead of running to max_iters; a slow but
steady decay is not taken for a stall."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sc") / "schedule_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "paper_2603_03019_amd", "csrc"),
                    os.path.join(ROOT, "tests", "schedule_check.cpp"), "-o", exe], check=True)
    return exe


def run(checker, tol, max_iters, fixed, r0, rate, floor, noise=0.0):
    r = subprocess.run([checker], input=f"{tol} {max_iters} {fixed} {r0} {rate} {floor} {noise}\n",
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    what, k, checks = r.stdout.split()
    return what, int(k), int(checks)


def test_geometric_decay_reaches_tol_with_few_checks(checker):
    # rate 0.95 per iteration from 1: 1e-8 is crossed at k = 360
    what, k, checks = run(checker, 1e-8, 100000, 0, 1.0, 0.95, 0.0)
    assert what == "ok"
    assert 360 <= k <= 360 + 64
    assert checks <= 12


def test_fixed_cadence(checker):
    what, k, checks = run(checker, 1e-8, 100000, 1, 1.0, 0.95, 0.0)
    assert (what, k, checks) == ("ok", 360, 360)


def test_floor_above_tol_stalls_early(checker):
    # FP64 rounding floor at 1e-16, tol 1e-18: stop soon after the floor
    what, k, checks = run(checker, 1e-18, 100000, 0, 1.0, 0.9, 1e-16)
    assert what == "stalled"
    assert k < 500 and checks < 40


@pytest.mark.parametrize("noise", [0.3, 0.9])
def test_noisy_floor_stalls_early(checker, noise):
    # at the floor the residual fluctuates; fluctuations downwards must not
    # keep the solve alive
    what, k, checks = run(checker, 1e-18, 100000, 0, 1.0, 0.9, 1e-16, noise)
    assert what == "stalled"
    assert k < 1000 and checks < 80


def test_noisy_decay_still_converges(checker):
    what, k, _ = run(checker, 1e-8, 100000, 0, 1.0, 0.95, 0.0, 0.3)
    assert what == "ok" and k <= 400


def test_divergence_stalls_early(checker):
    what, k, _ = run(checker, 1e-8, 100000, 0, 1e-3, 1.01, 0.0)
    assert what == "stalled" and k < 200


def test_slow_steady_decay_is_not_a_stall(checker):
    # 0.9995 per iteration (4600 iterations a decade) still counts as progress
    what, k, _ = run(checker, 1e-3, 100000, 0, 1.0, 0.9995, 0.0)
    assert what == "ok" and k <= 13816 + 64


def test_max_iters_without_stall(checker):
    what, k, _ = run(checker, 1e-8, 500, 0, 1.0, 0.99, 0.0)
    assert (what, k) == ("max_iters", 500)
