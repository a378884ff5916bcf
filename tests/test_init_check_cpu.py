"""Calibration of the product-form starting iterate (csrc/hq_init.h), run
on the CPU through tests/init_check.cpp: the utilisations of the start it
builds, assembled here by enumerating every state (product form inside each
layer, birth-death layer law of (10) with the start's own mu(n), waiting
states of Proposition 2 above layer N), must equal the targets whenever
some start has them."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("ic") / "init_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "paper_2603_03019_amd", "csrc"),
                    os.path.join(ROOT, "tests", "init_check.cpp"), "-o", exe], check=True)
    return exe


def start_utilisation(x, nu, Lam, C):
    """Busy probabilities of the start with weights x, by enumeration."""
    N = len(x)
    m = np.arange(1 << N)
    bits = ((m[:, None] >> np.arange(N)) & 1).astype(bool)
    w = np.where(bits, x[None, :], 1.0).prod(axis=1)
    size = bits.sum(axis=1)
    busy_n = np.zeros((N + 1, N))
    mu_n = np.zeros(N + 1)
    for n in range(N + 1):
        sel = size == n
        p = w[sel] / w[sel].sum()
        busy_n[n] = p @ bits[sel]
        mu_n[n] = p @ (bits[sel] @ nu)
    g = np.ones(N + 1)
    for n in range(1, N + 1):
        g[n] = g[n - 1] * Lam / mu_n[n]
    a = Lam / nu.sum()
    tail = 0.0 if C == 0 else (a / (1 - a) if C < 0 else sum(a ** c for c in range(1, C + 1)))
    wait = g[N] * tail
    return (g @ busy_n + wait) / (g.sum() + wait)


def run(checker, nu, Lam, C, target):
    N = len(nu)
    fmt = lambda a: " ".join(f"{float(v):.17g}" for v in a)
    text = f"{N} {C} {float(Lam):.17g}\n{fmt(nu)}\n{fmt(target)}\n"
    r = subprocess.run([checker], input=text, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    v = np.array([float(s) for s in r.stdout.split()])
    return v[:N], v[N]


@pytest.mark.parametrize("N,C,seed", [(1, 0, 0), (2, 0, 1), (5, 0, 2), (8, 0, 3), (10, 3, 4), (9, -1, 5),
                                      (12, 0, 6)])
def test_reachable_targets_are_met(checker, N, C, seed):
    rng = np.random.default_rng(seed)
    nu = rng.uniform(0.5, 1.5, N)
    Lam = rng.uniform(0.3, 0.9) * nu.sum()
    xstar = np.exp(rng.normal(0.0, 0.8, N))
    target = start_utilisation(xstar, nu, Lam, C)
    x, err = run(checker, nu, Lam, C, target)
    got = start_utilisation(x, nu, Lam, C)
    assert np.abs(got - target).max() <= 1e-10
    assert err == pytest.approx(np.abs(got - target).max(), abs=1e-12)
    # the weights are fixed up to a common factor by the utilisations
    np.testing.assert_allclose(x / x.sum(), xstar / xstar.sum(), rtol=1e-7)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_unreachable_targets_keep_the_closest_start(checker, seed):
    rng = np.random.default_rng(100 + seed)
    N = 7
    nu = rng.uniform(0.5, 1.5, N)
    Lam = 0.6 * nu.sum()
    target = rng.uniform(0.05, 0.95, N)  # need not balance flows
    x, err = run(checker, nu, Lam, 0, target)
    assert np.all(np.isfinite(x)) and np.all(x > 0)
    got = start_utilisation(x, nu, Lam, 0)
    assert err == pytest.approx(np.abs(got - target).max(), abs=1e-12)
    odds = target / (1 - target)  # the first iterate; the result is no worse
    assert err <= np.abs(start_utilisation(odds, nu, Lam, 0) - target).max() + 1e-15
