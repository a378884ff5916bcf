"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle.

Bars (written per test): FP64 state — L1 <= 1e-10 on converged P and
relative 1e-11 per entry at a fixed iteration count; FP32 state — L1 <= 1e-6.
"""
import sys

import numpy as np
import pytest

from oracle import cpu, exact
from paper_2603_03019_amd import hq
from paper_2603_03019_amd.instances import Instance, config_instance, make_instance

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _built():
    cpu.build(force=False)
    hq.load()


def _gpu(inst, **kw):
    return hq.create_from_instance(inst, **kw)


def _rel_close(a, b, rtol):
    scale = np.maximum(np.abs(a), np.abs(b))
    bad = np.abs(a - b) > rtol * scale + 1e-300
    return int(bad.sum())


@pytest.mark.parametrize("idx", [0, 1, 2, 3])
def test_small_fp64_converged_matches_oracle_and_dense(idx):
    inst = config_instance(1, idx)  # N=10, J=40, load 0.5
    say(f"case C1 idx={idx}")
    ctx = _gpu(inst)
    info = hq.hq_solve(ctx, 1e-12)
    P = hq.hq_state(ctx)
    ref = cpu.solve(inst, tol=1e-12)
    assert info["residual"] <= 1e-12
    assert np.abs(P - ref.P).sum() <= 1e-10
    assert np.abs(P - exact.dense_solve(inst)).sum() <= 1e-10
    assert abs(info["iterations"] - ref.iterations) <= 1


INNER = {"closed": hq.HQ_INNER_CLOSED, "one": hq.HQ_INNER_ONE, "literal": hq.HQ_INNER_LITERAL}


@pytest.mark.parametrize("inner", ["closed", "one", "literal"])
@pytest.mark.parametrize("N,J,b,cfg", [(10, 40, 0, 1), (12, 60, 4, 2), (14, 120, 6, 3), (15, 90, 10, 2),
                                       (13, 50, 12, 2), (16, 200, 8, 3), (16, 60, 0, 3), (17, 100, 0, 2)])
def test_iteration_path_matches_oracle(N, J, b, cfg, inner):
    """Same iterate after k outer iterations (Gauss-Seidel across layers,
    the same inner reading), entry by entry, for several tile widths.  The
    literal inner loop uses delta = 1e-6, where it takes a few inner steps."""
    inst = config_instance(cfg, 11, N=N, J=J)
    say(f"case path N={N} J={J} b={b} inner={inner}")
    ctx = _gpu(inst, inner=INNER[inner], tile_bits=b, delta=1e-6)
    done = 0
    for k in (1, 2, 5):
        hq.hq_iterate(ctx, k - done)
        done = k
        got = hq.hq_conditional(ctx)
        ref = cpu.solve(inst, tol=0.0, max_iters=k, inner=inner, delta=1e-6)
        assert _rel_close(got, ref.pcond, 1e-11) == 0, f"k={k}"
        sc = hq.hq_layer_scalars(ctx)
        np.testing.assert_allclose(sc[:, 0], ref.lam_n, rtol=1e-12)
        np.testing.assert_allclose(sc[:, 1], ref.mu_n, rtol=1e-12)
    hq.hq_destroy(ctx)


@pytest.mark.parametrize("load", [0.3, 0.9])
@pytest.mark.parametrize("inner", ["one", "closed"])
def test_medium_fp64_converged(load, inner):
    inst = config_instance(2, 1, N=16, J=200, load=load)
    say(f"case N=16 load={load} inner={inner}")
    ctx = _gpu(inst, inner=hq.HQ_INNER_ONE if inner == "one" else hq.HQ_INNER_CLOSED)
    info = hq.hq_solve(ctx, 1e-12)
    ref = cpu.solve(inst, tol=1e-12)
    P = hq.hq_state(ctx)
    assert np.abs(P - ref.P).sum() <= 1e-10
    rho, pn = hq.hq_marginals(ctx)
    rr, rp = cpu.marginals(inst.N, ref.P)
    np.testing.assert_allclose(rho, rr, rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(pn, rp, rtol=1e-9, atol=1e-15)
    if inner == "closed":
        # Lemma 1 (2): with the exact inner limit every layer keeps sum 1
        assert abs(info["mass_error"]) < 1e-9
    # (one inner update lets each layer sum drift by its own factor c_n;
    # the assembly (10) is invariant to that, P above already matched)


def test_edge_sizes():
    # N = 1: P(busy) = Lambda / (Lambda + nu)
    inst = Instance(1, 2, np.array([0.4, 0.6]), np.array([1.5]), np.array([[0], [0]], np.int32),
                    np.zeros((1, 2)), np.zeros((2, 2)), 1.0)
    say("case N=1")
    ctx = _gpu(inst)
    hq.hq_solve(ctx, 1e-14)
    P = hq.hq_state(ctx)
    assert P[1] == pytest.approx(1.0 / 2.5, abs=1e-15)
    # N = 2 hand example
    inst2 = Instance(2, 2, np.array([1.0, 2.0]), np.array([1.0, 3.0]), np.array([[0, 1], [1, 0]], np.int32),
                     np.zeros((2, 2)), np.zeros((2, 2)), 0.75)
    say("case N=2")
    ctx2 = _gpu(inst2)
    hq.hq_solve(ctx2, 1e-14)
    np.testing.assert_allclose(hq.hq_state(ctx2), np.array([30, 39, 17, 42]) / 128.0, atol=1e-14)
    # single demand node, ordered hunting with equal rates
    inst3 = make_instance(9, 1, config=901, index=0, load=0.8, homogeneous=True)
    say("case J=1")
    ctx3 = _gpu(inst3)
    hq.hq_solve(ctx3, 1e-13)
    rho, _ = hq.hq_marginals(ctx3)
    np.testing.assert_allclose(rho, exact.ordered_hunting_rho(inst3.pref[0], 9, inst3.Lambda), rtol=1e-9)


def test_zero_arrivals():
    inst = config_instance(1, 0)
    inst.lam = np.zeros_like(inst.lam)
    say("case Lambda=0")
    ctx = _gpu(inst)
    info = hq.hq_solve(ctx, 1e-10)
    P = hq.hq_state(ctx)
    assert P[0] == 1.0 and P[1:].sum() == 0.0 and info["iterations"] == 0


def test_homogeneous_erlang_on_gpu():
    inst = config_instance(2, 0, N=16, J=100, homogeneous=True, load=0.6)
    say("case Erlang N=16")
    ctx = _gpu(inst)
    hq.hq_solve(ctx, 1e-12)
    _, pn = hq.hq_marginals(ctx)
    np.testing.assert_allclose(pn, exact.erlang_marginal(16, inst.Lambda), rtol=1e-9, atol=1e-15)


def test_fp32_form_error_against_oracle():
    inst = config_instance(2, 2, N=18, J=200, load=0.6)
    ref = cpu.solve(inst, tol=1e-12)
    say("case FP32 N=18")
    # iterate the FP32 form to its storage floor (it stops when the residual stalls)
    ctx = _gpu(inst, precision=hq.HQ_FP32, max_iters=4000)
    info = hq.hq_solve(ctx, 1e-10, allow_not_converged=True)
    P = hq.hq_state(ctx)
    l1 = np.abs(P - ref.P).sum()
    say(f"  FP32 residual {info['residual']:.3e} L1 {l1:.3e}")
    assert l1 <= 1e-6
    say("case FP32+polish N=18")
    ctx2 = _gpu(inst, precision=hq.HQ_FP32_POLISH64)
    info2 = hq.hq_solve(ctx2, 1e-12)
    assert info2["fp64_iterations"] > 0
    assert np.abs(hq.hq_state(ctx2) - ref.P).sum() <= 1e-10


def test_not_converged_and_resume():
    inst = config_instance(2, 3, N=14, J=100)
    say("case max_iters / resume")
    ctx = _gpu(inst, max_iters=3, check_every=1)
    with pytest.raises(hq.HQError) as e:
        hq.hq_solve(ctx, 1e-12)
    assert e.value.status == hq.HQ_ERR_NOT_CONVERGED
    snap = hq.hq_conditional(ctx)  # iterate stays readable
    # resuming from the exported iterate reproduces the uninterrupted run bitwise
    a = _gpu(inst)
    hq.hq_iterate(a, 3 + 4)
    b = _gpu(inst, init_state=snap)
    hq.hq_iterate(b, 4)
    assert np.array_equal(hq.hq_conditional(a), hq.hq_conditional(b))


def test_deterministic_results():
    inst = config_instance(3, 4, N=16, J=300)
    say("case determinism")
    ctx = _gpu(inst)
    hq.hq_solve(ctx, 1e-10)
    P1 = hq.hq_state(ctx)
    hq.hq_solve(ctx, 1e-10)
    P2 = hq.hq_state(ctx)
    assert np.array_equal(P1, P2)


def test_paper_delta_stop_on_gpu():
    inst = config_instance(1, 5)
    say("case delta stop")
    ctx = _gpu(inst, stop=hq.HQ_STOP_DELTA)
    info = hq.hq_solve(ctx, 1e-12)
    ref = cpu.solve(inst, tol=1e-12, stop="delta")
    assert abs(info["iterations"] - ref.iterations) <= 1
    assert np.abs(hq.hq_state(ctx) - ref.P).sum() <= 1e-9


def test_state_device_export_to_torch():
    import torch

    inst = config_instance(1, 6)
    say("case device export")
    ctx = _gpu(inst)
    hq.hq_solve(ctx, 1e-12)
    out = torch.empty(1 << inst.N, dtype=torch.float64, device="cuda")
    hq.hq_state_device(ctx, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), hq.hq_state(ctx))


@pytest.mark.parametrize("stored", [-1, 3, 13])
def test_stored_coefficient_layers(stored):
    """Top layers with precomputed coefficients give the same iterate as the
    on-the-fly dispatch walk (and as the oracle)."""
    inst = config_instance(3, 12, N=14, J=300)
    say(f"case stored_layers={stored}")
    ctx = _gpu(inst, stored_layers=stored, inner=hq.HQ_INNER_ONE)
    hq.hq_iterate(ctx, 4)
    ref = cpu.solve(inst, tol=0.0, max_iters=4, inner="one")
    assert _rel_close(hq.hq_conditional(ctx), ref.pcond, 1e-11) == 0
    assert hq.hq_residual(ctx) == pytest.approx(cpu.residual(inst, ref.P), rel=1e-9)


def test_literal_inner_loop_converges_to_the_same_law():
    # any inner tolerance keeps the fixed point (the stationary law)
    inst = config_instance(2, 12, N=14, J=100)
    say("case literal inner converged")
    ref = cpu.solve(inst, tol=1e-13)
    for delta in (1e-3, 1e-9):
        ctx = _gpu(inst, inner=hq.HQ_INNER_LITERAL, delta=delta)
        hq.hq_solve(ctx, 1e-12)
        assert np.abs(hq.hq_state(ctx) - ref.P).sum() <= 1e-10
    with pytest.raises(hq.HQError):
        hq.hq_solve_batch([_gpu(inst, inner=hq.HQ_INNER_LITERAL, delta=1e-6)], 1e-8)


def test_fp64_residual_floor_ends_the_solve_early():
    """A tolerance below what FP64 can reach: the residual stalls at its
    rounding floor and the solve returns NOT_CONVERGED within a few hundred
    iterations (not at max_iters = 100000), single and batched."""
    inst = config_instance(1, 0)
    say("case stall N=10 tol=1e-18")
    ctx = _gpu(inst)
    info = hq.hq_solve(ctx, 1e-18, allow_not_converged=True)
    assert info["status"] == hq.HQ_ERR_NOT_CONVERGED
    assert info["iterations"] < 2000 and info["residual"] < 1e-12
    assert "stopped decreasing" in hq.hq_last_error()
    ctxs = [_gpu(config_instance(1, i)) for i in range(3)]
    st, infos = hq.hq_solve_batch(ctxs, 1e-18, allow_not_converged=True)
    assert st == hq.HQ_ERR_NOT_CONVERGED
    for x in infos:
        assert x["status"] == hq.HQ_ERR_NOT_CONVERGED
        assert x["iterations"] < 2000 and x["residual"] < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("inner", ["one", "closed", "literal"])
def test_default_shape_sweep_matches_general_kernels(inner, prec, monkeypatch):
    """The default-shape sweep kernels (10-bit tiles, from N = 16) against
    the general layer kernels on the same instance: iterates after 1, 3 and
    6 outer iterations and the balance residual agree to rounding."""
    inst = config_instance(3, 7, N=18, J=300)
    say(f"case sweep kernels vs general N=18 inner={inner} {prec}")
    p = hq.HQ_FP32 if prec == "fp32" else hq.HQ_FP64
    kw = dict(inner=INNER[inner], precision=p, delta=1e-6)
    new = _gpu(inst, **kw)
    monkeypatch.setenv("HQ_LEGACY_SWEEP", "1")
    old = _gpu(inst, **kw)
    monkeypatch.delenv("HQ_LEGACY_SWEEP")
    done = 0
    tol = 1e-12 if prec == "fp64" else 2e-7
    for k in (1, 3, 6):
        hq.hq_iterate(new, k - done)
        hq.hq_iterate(old, k - done)
        done = k
        a, b = hq.hq_conditional(new), hq.hq_conditional(old)
        assert _rel_close(a, b, tol) == 0, f"k={k}"
        ra, rb = hq.hq_residual(new), hq.hq_residual(old)
        assert ra == pytest.approx(rb, rel=1e-9 if prec == "fp64" else 1e-5)
    hq.hq_destroy(new)
    hq.hq_destroy(old)


@pytest.mark.parametrize("inner", ["one", "closed", "literal"])
def test_graph_replays_match_eager_launches(inner, monkeypatch):
    """An outer iteration is captured once as a graph of kernel launches and
    replayed: after every replay, with exports, residual checks and
    synchronisations in between, the iterate is bitwise the one of eager
    launches."""
    inst = config_instance(3, 3, N=17, J=150)
    say(f"case graph replays inner={inner}")
    kw = dict(inner=INNER[inner], delta=1e-6)
    g = _gpu(inst, **kw)
    monkeypatch.setenv("HQ_NO_GRAPH", "1")
    e = _gpu(inst, **kw)
    monkeypatch.delenv("HQ_NO_GRAPH")
    for k in range(6):
        hq.hq_iterate(g, 1)
        hq.hq_iterate(e, 1)
        a, b = hq.hq_conditional(g), hq.hq_conditional(e)
        assert np.array_equal(a, b), f"replay {k}"
        assert hq.hq_residual(g) == hq.hq_residual(e)
    # a full solve through the graphs reaches the same answer
    ig, ie = hq.hq_solve(g, 1e-11), hq.hq_solve(e, 1e-11)
    assert ig["iterations"] == ie["iterations"]
    assert np.array_equal(hq.hq_state(g), hq.hq_state(e))
    hq.hq_destroy(g)
    hq.hq_destroy(e)


@pytest.mark.parametrize("case", ["one-sweep", "closed-sweep", "one-stored", "delta-track"])
def test_fused_layer_scalars_match_finalize_launches(case, monkeypatch):
    """Small layers form the previous layer's scalars in their own launch
    instead of a finalize launch after every layer: the iterate, the layer
    scalars and a full solve are bitwise those of one finalize launch per
    layer (sweep kernel and look-ahead sweep at N = 17, stored-coefficient
    layers at N = 16, the paper's delta stopping rule)."""
    if case == "one-stored":
        inst, kw = config_instance(2, 5, N=16, J=150), dict(inner=hq.HQ_INNER_ONE, stored_layers=15)
    elif case == "closed-sweep":
        inst, kw = config_instance(3, 4, N=17, J=150), dict(inner=hq.HQ_INNER_CLOSED)
    elif case == "delta-track":
        inst, kw = config_instance(3, 4, N=17, J=150), dict(inner=hq.HQ_INNER_ONE, stop=hq.HQ_STOP_DELTA)
    else:
        inst, kw = config_instance(3, 4, N=17, J=150), dict(inner=hq.HQ_INNER_ONE)
    say(f"case fused layer scalars {case}")
    f = _gpu(inst, **kw)
    monkeypatch.setenv("HQ_NO_FUSE", "1")
    u = _gpu(inst, **kw)
    monkeypatch.delenv("HQ_NO_FUSE")
    for k in range(5):
        hq.hq_iterate(f, 1)
        hq.hq_iterate(u, 1)
        assert np.array_equal(hq.hq_conditional(f), hq.hq_conditional(u)), f"iteration {k}"
        assert np.array_equal(hq.hq_layer_scalars(f), hq.hq_layer_scalars(u)), f"iteration {k}"
    tol = 1e-9 if case == "delta-track" else 1e-11
    a, b = hq.hq_solve(f, tol), hq.hq_solve(u, tol)
    assert a["iterations"] == b["iterations"]
    assert np.array_equal(hq.hq_state(f), hq.hq_state(u))
    hq.hq_destroy(f)
    hq.hq_destroy(u)


@pytest.mark.parametrize("stored", [-1, 4])
def test_lookahead_closed_form_matches_two_passes_and_oracle(stored, monkeypatch):
    """The closed inner form in one pass per layer: the sums behind alpha_n
    (sum U~ and sum mu D~ over layer n) are re-indexed over layers n - 1 and
    n + 1 and accumulated while those layers are written.  Same iterate as
    the two-pass form (to rounding) and as the oracle's closed-form path;
    with stored coefficient layers too."""
    inst = config_instance(2, 21, N=17, J=120)
    say(f"case look-ahead closed N=17 stored={stored}")
    la = _gpu(inst, inner=hq.HQ_INNER_CLOSED, stored_layers=stored)
    monkeypatch.setenv("HQ_NO_LOOKAHEAD", "1")
    two = _gpu(inst, inner=hq.HQ_INNER_CLOSED, stored_layers=stored)
    monkeypatch.delenv("HQ_NO_LOOKAHEAD")
    done = 0
    for k in (1, 2, 5):
        hq.hq_iterate(la, k - done)
        hq.hq_iterate(two, k - done)
        done = k
        a, b = hq.hq_conditional(la), hq.hq_conditional(two)
        assert _rel_close(a, b, 1e-12) == 0, f"k={k}"
        ref = cpu.solve(inst, tol=0.0, max_iters=k, inner="closed")
        assert _rel_close(a, ref.pcond, 1e-11) == 0, f"k={k} vs oracle"
    ia, ib = hq.hq_solve(la, 1e-11), hq.hq_solve(two, 1e-11)
    assert abs(ia["iterations"] - ib["iterations"]) <= 1
    assert np.abs(hq.hq_state(la) - hq.hq_state(two)).sum() <= 1e-12
    hq.hq_destroy(la)
    hq.hq_destroy(two)
