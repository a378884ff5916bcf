"""The work plan of a batched solve (csrc/hq_batchplan.h), run on the CPU
through tests/batchplan_check.cpp: every instance gets 1..kmax ranks, about
its share of the states, as consecutive queue entries; and a simulation of
the work queue (work-groups take entries in order; the members of an
instance wait for each other at its barriers) never leaves a group waiting
forever when at least kmax work-groups run at once."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KMAX = 16


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("bp") / "batchplan_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "paper_2603_03019_amd", "csrc"),
                    os.path.join(ROOT, "tests", "batchplan_check.cpp"), "-o", exe], check=True)
    return exe


def plan(checker, sizes, cus, kmax=KMAX):
    text = f"{len(sizes)} {cus} {kmax}\n" + " ".join(f"{float(s):.17g}" for s in sizes) + "\n"
    r = subprocess.run([checker], input=text, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return [tuple(int(v) for v in line.split()) for line in r.stdout.splitlines()]


def simulate(entries, sizes, workers):
    """Event simulation of the queue; returns True if every instance finishes."""
    k_of = {}
    for item, rank, k in entries:
        k_of[item] = k
    pos, t = 0, 0.0
    held = {}          # item -> number of ranks taken
    running = []       # (finish time, item)
    free = workers
    done = set()
    while len(done) < len(k_of):
        # free work-groups take entries in queue order
        while free > 0 and pos < len(entries):
            item = entries[pos][0]
            held[item] = held.get(item, 0) + 1
            pos += 1
            free -= 1
            if held[item] == k_of[item]:  # the group is complete: it runs
                running.append((t + sizes[item] / k_of[item], item))
        if not running:
            return False  # every free slot is held by a group still waiting for members
        running.sort()
        t, item = running.pop(0)
        done.add(item)
        free += k_of[item]
    return True


@pytest.mark.parametrize("seed", range(6))
def test_plan_shape(checker, seed):
    rng = np.random.default_rng(seed)
    count = int(rng.integers(1, 400))
    ns = np.sort(rng.integers(1, 21, count))[::-1]
    sizes = 2.0 ** ns
    cus = int(rng.choice([8, 64, 256]))
    entries = plan(checker, sizes, cus)
    share = sizes.sum() / cus
    seen = {}
    for i, (item, rank, k) in enumerate(entries):
        assert 1 <= k <= KMAX and 0 <= rank < k
        seen.setdefault(item, []).append((i, rank, k))
    assert sorted(seen) == list(range(count))
    for item, rows in seen.items():
        idx = [r[0] for r in rows]
        assert idx == list(range(idx[0], idx[0] + len(idx)))       # consecutive entries
        assert [r[1] for r in rows] == list(range(len(rows)))     # ranks 0..k-1 in order
        k = rows[0][2]
        assert len(rows) == k
        assert k == min(KMAX, max(1, int(np.floor(sizes[item] / share + 0.5))))
    # queue order follows the instance order
    assert [e[0] for e in entries] == sorted(e[0] for e in entries)


@pytest.mark.parametrize("seed", range(8))
def test_queue_never_deadlocks(checker, seed):
    rng = np.random.default_rng(100 + seed)
    count = int(rng.integers(1, 300))
    sizes = 2.0 ** np.sort(rng.integers(4, 21, count))[::-1]
    cus = int(rng.choice([4, 16, 256]))
    entries = plan(checker, sizes, cus)
    for workers in (KMAX, KMAX + 1, 64, 512):
        assert simulate(entries, sizes, workers), (count, cus, workers)


def test_simulation_catches_interleaved_ranks(checker):
    # planted mistake: the same plan with the ranks of different instances
    # interleaved can leave every work-group waiting for a missing member
    sizes = np.array([2.0 ** 18] * 4)
    entries = plan(checker, sizes, 64)
    assert all(e[2] == KMAX for e in entries)
    interleaved = sorted(entries, key=lambda e: (e[1], e[0]))
    assert simulate(entries, sizes, KMAX)
    assert not simulate(interleaved, sizes, KMAX)
