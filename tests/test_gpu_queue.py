"""Waiting room (Section 2.2, Proposition 2 and the remark after it) on the
GPU: unit-state distribution, marginals and waiting measures against the
oracle's assembly of the buffered birth-death marginal."""
import sys

import numpy as np
import pytest

from oracle import cpu
from paper_2603_03019_amd import hq
from paper_2603_03019_amd.instances import config_instance

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle(inst, C):
    res = cpu.solve(inst, tol=1e-13)
    P, tail, summ = cpu.buffered_state(res, inst, C)
    rho, pn = cpu.marginals(inst.N, P)
    return P, tail, summ, rho + summ[1], pn


@pytest.mark.parametrize("N,C,load", [(10, 3, 0.5), (10, hq.HQ_BUFFER_UNLIMITED, 0.8), (12, 40, 1.3),
                                      (17, 2, 0.7)])
def test_buffered_solve_matches_oracle(N, C, load):
    inst = config_instance(1, 5, N=N, J=60, load=load)
    say(f"case queue N={N} C={C} load={load}")
    ctx = hq.create_from_instance(inst, buffer=C)
    hq.hq_solve(ctx, 1e-12)
    P, tail, summ, rho, pn = _oracle(inst, C)
    Pg = hq.hq_state(ctx)
    assert np.abs(Pg - P).sum() <= 1e-10
    rg, png = hq.hq_marginals(ctx)
    np.testing.assert_allclose(rg, rho, rtol=1e-9)
    want_pn = pn.copy()
    want_pn[N] += summ[1]
    np.testing.assert_allclose(png, want_pn, rtol=1e-9, atol=1e-300)
    k = 8
    sg, tg = hq.hq_queue(ctx, k)
    np.testing.assert_allclose(sg, summ, rtol=1e-9, atol=1e-300)
    if C > 0:
        want_t = np.zeros(k)
        want_t[:min(k, C)] = tail[:k]
        np.testing.assert_allclose(tg, want_t, rtol=1e-9, atol=1e-300)
        assert Pg.sum() + tail.sum() == pytest.approx(1.0, abs=1e-12)
    # every unit is busy in the waiting states: they add to each rho_u
    assert np.all(rg >= summ[1])


def test_loss_system_has_no_waiting():
    inst = config_instance(1, 6)
    ctx = hq.create_from_instance(inst)
    hq.hq_solve(ctx, 1e-12)
    sg, tg = hq.hq_queue(ctx, 4)
    rho, pn = hq.hq_marginals(ctx)
    assert sg[1] == 0.0 and sg[2] == 0.0 and np.all(tg == 0.0)
    assert sg[0] == pytest.approx(pn[-1], rel=1e-12)
    assert sg[3] == pytest.approx(pn[-1], rel=1e-12)  # arrivals at the full state are lost


def test_batched_buffered_contexts():
    insts = [config_instance(4, 60 + i, N=n) for i, n in enumerate([12, 13, 14])]
    say("case queue batch")
    cs = [hq.create_from_instance(inst, buffer=5) for inst in insts]
    hq.hq_solve_batch(cs, 1e-11)
    for inst, c in zip(insts, cs):
        P, tail, summ, rho, pn = _oracle(inst, 5)
        assert np.abs(hq.hq_state(c) - P).sum() <= 1e-9
        sg, tg = hq.hq_queue(c, 5)
        np.testing.assert_allclose(sg, summ, rtol=1e-8)
        np.testing.assert_allclose(tg, tail, rtol=1e-8)
