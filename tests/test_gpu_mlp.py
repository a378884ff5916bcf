"""Warm-start network on the GPU: BF16 MFMA forward and backward against the
CPU reference (oracle/mlp.py, float64 with the same BF16 rounding points),
training, and a learned-start solve that still matches the oracle."""
import sys

import numpy as np
import pytest

from oracle import cpu
from oracle import mlp as ref
from paper_2603_03019_amd import hq
from paper_2603_03019_amd.instances import config_instance

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _data(rows, seed):
    rng = np.random.default_rng(seed)
    X = np.zeros((rows, ref.IN), dtype=np.float32)
    X[:, :16] = rng.random((rows, 16))
    t = (0.2 + 0.6 / (1.0 + np.exp(-(X[:, 0] - X[:, 3] + 0.5 * X[:, 7])))).astype(np.float32)
    return X, t


def test_forward_matches_reference():
    m = hq.hq_mlp_create(seed=3)
    p = hq.hq_mlp_get_params(m)
    X, _ = _data(77, 0)  # not a multiple of 32: exercises the padding
    say("case mlp forward")
    y = hq.hq_mlp_forward(m, X)
    yr, _ = ref.forward(p, X, bf=True)
    np.testing.assert_allclose(y, yr, rtol=2e-3, atol=2e-4)


def test_gradient_matches_reference():
    m = hq.hq_mlp_create(seed=5)
    p = hq.hq_mlp_get_params(m)
    X, t = _data(96, 1)
    say("case mlp gradient")
    g, loss = hq.hq_mlp_gradient(m, X, t)
    lr, gr = ref.loss_and_grad(p, X, t, bf=True)
    assert loss == pytest.approx(lr, rel=1e-4)
    cos = float(g @ gr / (np.linalg.norm(g) * np.linalg.norm(gr)))
    rel = float(np.linalg.norm(g - gr) / np.linalg.norm(gr))
    say(f"  cos {cos:.6f} rel {rel:.2e}")
    assert cos > 0.9999 and rel < 1e-2
    for a, b in [(ref.OFF_W1, ref.OFF_B1), (ref.OFF_W2, ref.OFF_B2), (ref.OFF_W3, ref.OFF_B3)]:
        blk = np.linalg.norm(g[a:b] - gr[a:b]) / np.linalg.norm(gr[a:b])
        assert blk < 2e-2


def test_training_reduces_loss_and_params_roundtrip():
    m = hq.hq_mlp_create(seed=7)
    X, t = _data(4096, 2)
    say("case mlp training")
    losses = hq.hq_mlp_train(m, X, t, epochs=30, batch=256, lr=2e-3, seed=1)
    say(f"  loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 0.2 * losses[0]
    p = hq.hq_mlp_get_params(m)
    m2 = hq.hq_mlp_create(seed=99)
    hq.hq_mlp_set_params(m2, p)
    np.testing.assert_array_equal(hq.hq_mlp_forward(m2, X[:64]), hq.hq_mlp_forward(m, X[:64]))


def test_learned_start_solves_to_the_same_answer():
    """The network only changes the initial iterate: the answer is the
    oracle's, whether the warm start is kept or the cold start wins."""
    train = [config_instance(5, 1000 + i, N=12, J=80) for i in range(6)]
    X, t = [], []
    for inst in train:
        r = cpu.solve(inst, tol=1e-10)
        rho, _ = cpu.marginals(inst.N, r.P)
        X.append(hq.hq_mlp_features(inst.N, inst.J, inst.lam, inst.nu, inst.pref))
        t.append(rho)
    m = hq.hq_mlp_create(seed=11)
    hq.hq_mlp_train(m, np.concatenate(X), np.concatenate(t).astype(np.float32), epochs=200, batch=32, lr=2e-3)
    inst = config_instance(5, 2000, N=13, J=80)
    say("case learned start")
    ctx = hq.create_from_instance(inst, mlp=m)
    info = hq.hq_solve(ctx, 1e-12)
    ref_r = cpu.solve(inst, tol=1e-12)
    assert np.abs(hq.hq_state(ctx) - ref_r.P).sum() <= 1e-10
    assert info["warm_used"] in (0, 1)
    # an explicit product-form start with the exact utilisations beats the cold start
    rho, _ = cpu.marginals(inst.N, ref_r.P)
    warm = hq.create_from_instance(inst, init_rho=rho)
    wi = hq.hq_solve(warm, 1e-12)
    cold = hq.hq_solve(hq.create_from_instance(inst), 1e-12)
    say(f"  iterations: exact-rho product start {wi['iterations']} (kept {wi['warm_used']}), cold {cold['iterations']}")
    assert np.abs(hq.hq_state(warm) - ref_r.P).sum() <= 1e-10
    assert wi["warm_used"] == 1 and wi["iterations"] < cold["iterations"]


@pytest.mark.parametrize("C", [0, 3])
def test_product_start_has_the_target_utilisations(C):
    # targets that some product-form start meets: those of weights xstar
    from test_init_check_cpu import start_utilisation
    inst = config_instance(1, 7, N=9, J=30)
    rng = np.random.default_rng(5)
    xstar = np.exp(rng.normal(0.0, 0.7, inst.N))
    target = start_utilisation(xstar, inst.nu, inst.lam.sum(), C)
    say(f"case product start C={C}")
    ctx = hq.create_from_instance(inst, init_rho=target, buffer=C)
    hq.hq_iterate(ctx, 0)  # the start only
    rho, _ = hq.hq_marginals(ctx)
    np.testing.assert_allclose(rho, target, rtol=0, atol=1e-10)
    # and inside each layer it is the product form of xstar
    pc = hq.hq_conditional(ctx)
    m = np.arange(1 << inst.N)
    bits = ((m[:, None] >> np.arange(inst.N)) & 1).astype(bool)
    w = np.where(bits, xstar[None, :], 1.0).prod(axis=1)
    size = bits.sum(axis=1)
    for n in range(inst.N + 1):
        sel = size == n
        np.testing.assert_allclose(pc[sel] / pc[sel].sum(), w[sel] / w[sel].sum(), rtol=1e-9)
