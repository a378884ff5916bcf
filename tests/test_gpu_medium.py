"""The medium workload on the GPU against the FP64 oracle: N = 20 units,
J = 200 uniform demand nodes, at loads 0.3, 0.6 and 0.9, and a homogeneous
variant (every service rate 1, load 0.6).

* FP32 state (per-layer scales, FP64 sums): iterated to its rounding
  floor; L1 distance to the oracle's P <= 1e-6.
* FP32 state with the FP64 hand-over, and the FP64 state, solved to a
  balance residual of 1e-12: L1 <= 1e-10.
* Homogeneous rates: with mu(n) = n nu for every layer, the number-busy
  marginal is the Erlang loss law, whatever the preference lists
  (Section 3.2, homogeneous case; eq. (10)).

Each case also prints the paper's maximum percentage relative error,
eq. (15), of P against the oracle.
"""
import sys

import numpy as np
import pytest

from oracle import cpu, exact
from paper_2603_03019_amd import hq
from paper_2603_03019_amd.instances import config_instance

pytestmark = pytest.mark.gpu

VARIANTS = {"load0.3": dict(load=0.3), "load0.6": dict(load=0.6), "load0.9": dict(load=0.9),
            "homogeneous": dict(load=0.6, homogeneous=True)}
_ORACLE = {}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def mpre(P, ref):
    """Maximum percentage relative error, eq. (15), over the states."""
    mask = ref > 0
    return 100.0 * float(np.max(np.abs(P[mask] - ref[mask]) / ref[mask]))


def _case(name):
    inst = config_instance(2, 0, **VARIANTS[name])
    if name not in _ORACLE:
        say(f"case N=20 {name}: oracle to 1e-12")
        ref = cpu.solve(inst, tol=1e-12, inner="one", check_every=20)
        assert ref.converged and ref.residual <= 1e-12
        _ORACLE[name] = ref
    return inst, _ORACLE[name]


@pytest.fixture(scope="module", autouse=True)
def _built():
    cpu.build(force=False)
    hq.load()


@pytest.mark.parametrize("name", list(VARIANTS))
def test_fp32_state_at_its_floor(name):
    inst, ref = _case(name)
    say(f"case N=20 {name} FP32")
    ctx = hq.create_from_instance(inst, precision=hq.HQ_FP32)
    info = hq.hq_solve(ctx, 1e-12, allow_not_converged=True)
    P = hq.hq_state(ctx)
    l1 = float(np.abs(P - ref.P).sum())
    say(f"  FP32: {info['iterations']} iterations, residual floor {info['residual']:.2e}, "
        f"L1 vs oracle {l1:.2e}, MPRE {mpre(P, ref.P):.2e} %")
    assert info["residual"] <= 1e-6
    assert l1 <= 1e-6
    hq.hq_destroy(ctx)


@pytest.mark.parametrize("name", list(VARIANTS))
@pytest.mark.parametrize("prec", ["polish", "fp64"])
def test_fp64_results_match_oracle(name, prec):
    inst, ref = _case(name)
    say(f"case N=20 {name} {prec}")
    p = hq.HQ_FP32_POLISH64 if prec == "polish" else hq.HQ_FP64
    ctx = hq.create_from_instance(inst, precision=p)
    info = hq.hq_solve(ctx, 1e-12)
    P = hq.hq_state(ctx)
    l1 = float(np.abs(P - ref.P).sum())
    say(f"  {prec}: {info['iterations']} iterations ({info['fp64_iterations']} in FP64), residual "
        f"{info['residual']:.2e}, L1 vs oracle {l1:.2e}, MPRE {mpre(P, ref.P):.2e} %")
    assert info["residual"] <= 1e-12
    assert l1 <= 1e-10
    hq.hq_destroy(ctx)


@pytest.mark.parametrize("prec,bar", [("fp32", 1e-6), ("polish", 1e-12)])
def test_homogeneous_marginal_is_erlang(prec, bar):
    inst, _ = _case("homogeneous")
    a = inst.Lambda / 1.0
    want = exact.erlang_marginal(inst.N, a)
    p = hq.HQ_FP32 if prec == "fp32" else hq.HQ_FP32_POLISH64
    ctx = hq.create_from_instance(inst, precision=p)
    hq.hq_solve(ctx, 1e-12, allow_not_converged=(prec == "fp32"))
    _, pn = hq.hq_marginals(ctx)
    err = float(np.abs(pn - want).max())
    say(f"case N=20 homogeneous {prec}: max |p(n) - Erlang| {err:.2e}")
    assert err <= bar
    hq.hq_destroy(ctx)
