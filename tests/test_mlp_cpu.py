"""CPU checks of the warm-start network pieces that need no GPU: the float64
reference gradient (oracle/mlp.py) against central finite differences, and
the library's native feature extraction against an independent numpy
computation of the same definitions."""
import numpy as np
import pytest

from oracle import mlp as ref
from paper_2603_03019_amd import hq
from paper_2603_03019_amd.instances import config_instance


def _params(seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, scale, ref.NPARAM) / np.sqrt(np.r_[np.full(ref.OFF_B1, ref.IN),
                                                          np.ones(ref.OFF_W2 - ref.OFF_B1),
                                                          np.full(ref.OFF_B2 - ref.OFF_W2, ref.HID),
                                                          np.ones(ref.OFF_W3 - ref.OFF_B2),
                                                          np.full(ref.OFF_B3 - ref.OFF_W3, ref.HID), [1.0]])
    return p


def test_reference_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = _params()
    X = rng.random((24, ref.IN))
    t = rng.random(24)
    _, g = ref.loss_and_grad(p, X, t, bf=False)
    idx = np.r_[rng.choice(ref.OFF_B1, 40, replace=False), ref.OFF_B1 + rng.choice(256, 20, replace=False),
                ref.OFF_W2 + rng.choice(256 * 256, 60, replace=False), ref.OFF_B2 + rng.choice(256, 20, replace=False),
                ref.OFF_W3 + rng.choice(256, 20, replace=False), [ref.OFF_B3]]
    h = 1e-6
    for i in idx:
        e = np.zeros(ref.NPARAM)
        e[i] = h
        fd = (ref.loss_and_grad(p + e, X, t, bf=False)[0] - ref.loss_and_grad(p - e, X, t, bf=False)[0]) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-10), i


def test_bf16_rounding_is_nearest_even():
    vals = np.array([1.0, 1.00390625, 1.0078125, 1.005859375, 3.14159, -2.5e-3, 65504.0])
    got = ref.bf16(vals)
    # bfloat16 keeps 8 significant bits: the rounding error is at most half an ulp
    ulp = 2.0 ** (np.floor(np.log2(np.abs(vals))) - 7)
    assert np.all(np.abs(got - vals) <= ulp / 2 + 1e-12)
    assert got[1] == 1.0  # tie 1 + 2^-8 rounds to even (1.0)
    assert got[3] == 1.0078125  # 1 + 1.5 * 2^-8 rounds up


def _features_numpy(inst):
    N, lam, nu, pref = inst.N, inst.lam, inst.nu, inst.pref
    Lam, M = lam.sum(), nu.sum()
    load = Lam / M
    share = np.zeros((N, 9))
    expo = np.zeros(N)
    for j in range(inst.J):
        w = lam[j] / Lam
        for h in range(N):
            share[pref[j, h], min(h, 8)] += w
            expo[pref[j, h]] += w * load ** h
    f = np.zeros((N, 32))
    f[:, 0] = nu / (M / N)
    f[:, 1:10] = share
    f[:, 10] = load
    f[:, 11] = expo
    f[:, 12] = N / 32.0
    f[:, 13] = nu / nu.max()
    f[:, 14] = N * share[:, 0]
    f[:, 15] = 1.0
    # independence approximation of the utilisations: unit u receives the
    # calls whose earlier-ranked units are all busy (busy independently with
    # probabilities rho), and is busy with probability r_u / (r_u + nu_u)
    rho = np.full(N, min(load, 0.99))
    for _ in range(60):
        before = np.concatenate([np.ones((inst.J, 1)), rho[pref[:, :-1]]], axis=1)
        reach = np.cumprod(before, axis=1)
        r = np.zeros(N)
        np.add.at(r, pref, lam[:, None] * reach)
        rho = r / (r + nu)
    f[:, 16] = rho
    f[:, 17] = r / Lam
    f[:, 18] = np.clip(np.log(rho / (1.0 - rho)), -8.0, 8.0) / 8.0
    return f


@pytest.mark.parametrize("cfg,idx", [(5, 1000), (6, 50000), (1, 0)])
def test_native_features_match_definition(cfg, idx):
    inst = config_instance(cfg, idx)
    got = hq.hq_mlp_features(inst.N, inst.J, inst.lam, inst.nu, inst.pref)
    np.testing.assert_allclose(got, _features_numpy(inst), rtol=2e-6, atol=1e-7)
