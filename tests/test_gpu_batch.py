"""Batched solve (one persistent launch for many instances) against the CPU
oracle and against single-instance solves.  Bars: FP64 L1 <= 1e-10 per
instance, FP32 L1 <= 1e-6."""
import sys

import numpy as np
import pytest

from oracle import cpu
from paper_2603_03019_amd import hq
from paper_2603_03019_amd.instances import Instance, config_instance, make_instance

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _mixed_instances():
    insts = [config_instance(4, i, N=n, J=j) for i, (n, j) in
             enumerate([(12, 100), (6, 20), (13, 60), (9, 40), (10, 100), (14, 100), (11, 7)])]
    insts.append(Instance(1, 2, np.array([0.4, 0.6]), np.array([1.5]), np.array([[0], [0]], np.int32),
                          np.zeros((1, 2)), np.zeros((2, 2)), 1.0))
    z = config_instance(1, 3)
    z.lam = np.zeros_like(z.lam)
    insts.append(z)
    return insts


@pytest.mark.parametrize("inner", ["one", "closed"])
def test_batch_fp64_matches_oracle(inner):
    insts = _mixed_instances()
    say(f"case batch fp64 inner={inner} sizes={[i.N for i in insts]}")
    ctxs = [hq.create_from_instance(i, inner=hq.HQ_INNER_ONE if inner == "one" else hq.HQ_INNER_CLOSED)
            for i in insts]
    st, infos = hq.hq_solve_batch(ctxs, 1e-12)
    assert st == hq.HQ_OK
    for inst, ctx, info in zip(insts, ctxs, infos):
        P = hq.hq_state(ctx)
        ref = cpu.solve(inst, tol=1e-12, inner=inner)
        l1 = np.abs(P - ref.P).sum()
        assert l1 <= 1e-10, (inst.N, l1)
        if inst.Lambda > 0:
            assert info["residual"] <= 1e-12
            assert abs(info["iterations"] - ref.iterations) <= 8


def test_batch_matches_single_solves_and_repeats():
    insts = [config_instance(4, 20 + i) for i in range(5)]  # N ~ U{12..18}, J = 100
    say(f"case batch vs single sizes={[i.N for i in insts]}")
    a = [hq.create_from_instance(i) for i in insts]
    b = [hq.create_from_instance(i) for i in insts]
    hq.hq_solve_batch(a, 1e-11)
    first = [hq.hq_state(c) for c in a]
    hq.hq_solve_batch(a, 1e-11)  # the captured graph is reused: same answer
    for c, P in zip(a, first):
        assert np.array_equal(hq.hq_state(c), P)
    for c in b:
        hq.hq_solve(c, 1e-11)
    for ca, cb in zip(a, b):
        assert np.abs(hq.hq_state(ca) - hq.hq_state(cb)).sum() <= 1e-9
        ra, pa = hq.hq_marginals(ca)
        rb, pb = hq.hq_marginals(cb)
        np.testing.assert_allclose(ra, rb, atol=1e-9)


def test_batch_fp32_error():
    insts = [config_instance(4, 40 + i, N=n) for i, n in enumerate([12, 15, 16])]
    say("case batch fp32")
    ctxs = [hq.create_from_instance(i, precision=hq.HQ_FP32) for i in insts]
    st, infos = hq.hq_solve_batch(ctxs, 1e-10, allow_not_converged=True)
    for inst, ctx in zip(insts, ctxs):
        ref = cpu.solve(inst, tol=1e-12)
        assert np.abs(hq.hq_state(ctx) - ref.P).sum() <= 1e-6


def test_batch_rejects_polish_contexts():
    inst = config_instance(1, 0)
    say("case batch invalid")
    c = hq.create_from_instance(inst, precision=hq.HQ_FP32_POLISH64)
    with pytest.raises(hq.HQError) as e:
        hq.hq_solve_batch([c], 1e-8)
    assert e.value.status == hq.HQ_ERR_INVALID_ARG


def test_batch_product_start_matches_oracle():
    # product-form starts fitted to the exact utilisations, in a batch whose
    # largest instance is shared by several work-groups
    insts = [config_instance(4, 70 + i, N=n) for i, n in enumerate([16, 12, 13, 11])]
    say(f"case batch product start sizes={[i.N for i in insts]}")
    refs = [cpu.solve(inst, tol=1e-12) for inst in insts]
    ctxs = [hq.create_from_instance(inst, init_rho=cpu.marginals(inst.N, ref.P)[0])
            for inst, ref in zip(insts, refs)]
    cold = [hq.create_from_instance(inst) for inst in insts]
    st, infos = hq.hq_solve_batch(ctxs, 1e-11)
    assert st == hq.HQ_OK
    _, cold_infos = hq.hq_solve_batch(cold, 1e-11)
    for inst, ref, ctx, info, ci in zip(insts, refs, ctxs, infos, cold_infos):
        assert np.abs(hq.hq_state(ctx) - ref.P).sum() <= 1e-9, inst.N
        assert info["iterations"] <= ci["iterations"]


def test_full_benchmark_batch_answers_pass_the_oracle():
    """The bench's batched workload in full: 256 deployments with N ~
    U{12..18}, J = 100, in one batched solve to 1e-12.  Every answer's
    balance residual of (1), recomputed by the oracle with its own
    Algorithm-3 coefficients, is <= 2e-12; one deployment of each size is
    also compared state by state with the oracle's solve (L1 <= 1e-10)."""
    insts = [config_instance(4, i) for i in range(256)]
    say(f"case full batch: 256 deployments, N {min(i.N for i in insts)}..{max(i.N for i in insts)}")
    ctxs = [hq.create_from_instance(i, inner=hq.HQ_INNER_ONE) for i in insts]
    st, infos = hq.hq_solve_batch(ctxs, 1e-12)
    assert st == hq.HQ_OK
    assert hq.hq_batch_last_block() in (256, 512, 1024)
    worst, seen = 0.0, set()
    for k, (inst, ctx, info) in enumerate(zip(insts, ctxs, infos)):
        assert info["residual"] <= 1e-12, (k, info["residual"])
        P = hq.hq_state(ctx)
        r = cpu.residual(inst, P)
        worst = max(worst, r)
        assert r <= 2e-12, (k, inst.N, r)
        if inst.N not in seen:
            seen.add(inst.N)
            ref = cpu.solve(inst, tol=1e-12, inner="one")
            l1 = np.abs(P - ref.P).sum()
            say(f"  N={inst.N} (deployment {k}): L1 vs oracle {l1:.2e}")
            assert l1 <= 1e-10, (k, inst.N, l1)
        hq.hq_destroy(ctx)
    say(f"  largest oracle residual over the 256 answers: {worst:.3e}")
