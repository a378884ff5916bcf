"""What the trained network gains: the shipped warm-start network
(paper_2603_03019_amd/weights/warm_mlp.npy, trained on solves at N = 16..20)
on deployments it has not seen, against the cold start of Algorithm 1
(p_n = 1 / C(N, n)).  Every answer is checked against the FP64 oracle, and
the learned start must need fewer outer iterations on average.

* N = 18, J = 500 uniform demand, loads from the evaluation pool's
  generator (U[0.5, 0.9)): full oracle solves, L1 <= 1e-10;
* N = 24, J = 500 (the evaluation pool's own size): the oracle's balance
  residual of (1), with its own Algorithm-3 coefficients, on the GPU's
  answer <= 2e-8 (the solve stops at 1e-8).
"""
import sys

import numpy as np
import pytest

from oracle import cpu
from paper_2603_03019_amd import hq, warmstart
from paper_2603_03019_amd.instances import config_instance

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def net():
    m = warmstart.load_network()
    yield m
    hq.hq_mlp_destroy(m)


def _solve(inst, tol, **kw):
    ctx = hq.create_from_instance(inst, inner=hq.HQ_INNER_ONE, **kw)
    info = hq.hq_solve(ctx, tol)
    P = hq.hq_state(ctx)
    hq.hq_destroy(ctx)
    return info, P


def test_learned_start_needs_fewer_iterations_and_matches_oracle(net):
    cold_it, warm_it = [], []
    for idx in range(60000, 60004):
        inst = config_instance(6, idx, N=18)
        say(f"case warm gain N=18 idx={idx} load={inst.load:.3f}")
        ic, Pc = _solve(inst, 1e-12)
        iw, Pw = _solve(inst, 1e-12, mlp=net)
        ref = cpu.solve(inst, tol=1e-12, inner="one", check_every=10)
        lc, lw = float(np.abs(Pc - ref.P).sum()), float(np.abs(Pw - ref.P).sum())
        say(f"  iterations cold {ic['iterations']} learned {iw['iterations']} (kept {iw['warm_used']}); "
            f"L1 vs oracle {lc:.2e} / {lw:.2e}")
        assert lc <= 1e-10 and lw <= 1e-10
        cold_it.append(ic["iterations"])
        warm_it.append(iw["iterations"])
    say(f"  mean iterations cold {np.mean(cold_it):.1f} learned {np.mean(warm_it):.1f}")
    assert np.mean(warm_it) < 0.97 * np.mean(cold_it)


def test_learned_start_answers_at_evaluation_size_pass_the_oracle_residual(net):
    for idx in (50000, 50001):
        inst = config_instance(6, idx)  # N = 24, J = 500
        say(f"case warm N=24 idx={idx}")
        ic, _ = _solve(inst, 1e-8)
        iw, Pw = _solve(inst, 1e-8, mlp=net)
        r = cpu.residual(inst, Pw)
        say(f"  iterations cold {ic['iterations']} learned {iw['iterations']}; GPU residual "
            f"{iw['residual']:.3e}, oracle residual {r:.3e}")
        assert r <= 2e-8
