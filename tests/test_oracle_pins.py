"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: the references are a hand
derivation (tests/golden), exact rational arithmetic, independent direct
solves with the generator built per source state, the Erlang-loss and
ordered-hunting closed forms, the invariants of Lemma 1 and of the model,
and metamorphic relations.  The mutation tests plant plausible mistakes in a
copy of the oracle source and check that the pins catch them.
"""
import math
import os
import re
import shutil
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest

from oracle import cpu, exact
from paper_2603_03019_amd.instances import Instance, config_instance, make_instance

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _inst(N, J, lam, nu, pref):
    return Instance(N=N, J=J, lam=np.asarray(lam, float), nu=np.asarray(nu, float),
                    pref=np.asarray(pref, np.int32).reshape(J, N), unit_xy=np.zeros((N, 2)),
                    atom_xy=np.zeros((J, 2)), load=float(np.sum(lam) / np.sum(nu)))


def _read_golden(name):
    d = {"pref": []}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *v = line.split()
            if k == "pref":
                d["pref"].append([int(x) for x in v])
            else:
                d[k] = v
    return d


@pytest.fixture(scope="module", autouse=True)
def _built():
    cpu.build(force=False)


# ---------------------------------------------------------------- exact pins

def test_golden_hand_derived_n2():
    """Section 2.1 / eq. (1)-(3): a 2-unit system solved by hand."""
    g = _read_golden("n2_hand.txt")
    inst = _inst(int(g["N"][0]), int(g["J"][0]), [float(x) for x in g["lam"]],
                 [float(x) for x in g["nu"]], g["pref"])
    want = np.array([int(x) for x in g["P_num"]], float) / float(g["P_den"][0])
    r = cpu.solve(inst, tol=1e-15, max_iters=10000)
    assert r.converged
    np.testing.assert_allclose(r.P, want, rtol=0, atol=1e-14)


def test_single_unit_closed_form():
    """N = 1: no layer is iterated; P(busy) = Lambda / (Lambda + nu)."""
    inst = _inst(1, 3, [0.3, 0.5, 0.2], [1.7], [[0], [0], [0]])
    r = cpu.solve(inst, tol=1e-15)
    assert r.P[1] == pytest.approx(1.0 / 2.7, abs=1e-15)
    assert r.P[0] == pytest.approx(1.7 / 2.7, abs=1e-15)


def _exact_rational(N, J, lam, nu, pref):
    """Stationary law by Gauss-Jordan elimination over the rationals, with
    the generator written out from the dispatch rule of Section 2.1."""
    S = 1 << N
    Q = [[Fraction(0)] * S for _ in range(S)]
    for l in range(S):
        for j in range(J):
            for u in pref[j]:
                if not (l >> u) & 1:
                    Q[l][l | (1 << u)] += lam[j]
                    break
        for u in range(N):
            if (l >> u) & 1:
                Q[l][l ^ (1 << u)] += nu[u]
        Q[l][l] = -sum(Q[l][c] for c in range(S) if c != l)
    # A x = b with A = Q^T, last row replaced by ones
    A = [[Q[c][r] for c in range(S)] for r in range(S)]
    A[-1] = [Fraction(1)] * S
    b = [Fraction(0)] * (S - 1) + [Fraction(1)]
    for col in range(S):
        piv = next(r for r in range(col, S) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        b[col], b[piv] = b[piv], b[col]
        inv = 1 / A[col][col]
        A[col] = [x * inv for x in A[col]]
        b[col] *= inv
        for r in range(S):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [x - f * y for x, y in zip(A[r], A[col])]
                b[r] -= f * b[col]
    return [float(x) for x in b]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_rational_tiny(seed):
    """N = 3: exact rational solve of (1)-(2) vs the oracle."""
    rng = np.random.default_rng(100 + seed)
    N, J = 3, 4
    lam = [Fraction(int(x), 4) for x in rng.integers(1, 9, J)]
    nu = [Fraction(int(x), 4) for x in rng.integers(2, 9, N)]
    pref = [list(rng.permutation(N)) for _ in range(J)]
    want = _exact_rational(N, J, lam, nu, pref)
    inst = _inst(N, J, [float(x) for x in lam], [float(x) for x in nu], pref)
    r = cpu.solve(inst, tol=1e-15, max_iters=20000)
    np.testing.assert_allclose(r.P, want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_dense_lu_pin_config_n10(idx):
    """N=10, J=40, load 0.5: oracle vs dense LU of (1)-(2), L1 <= 1e-10."""
    inst = config_instance(1, idx)
    Pd = exact.dense_solve(inst)
    r = cpu.solve(inst, tol=1e-12)
    assert r.converged and r.residual <= 1e-12
    assert np.abs(r.P - Pd).sum() <= 1e-10


@pytest.mark.parametrize("N,J,load,hom", [(2, 3, 0.4, False), (4, 6, 1.5, False), (5, 9, 0.2, False),
                                          (6, 12, 0.9, True), (7, 20, 3.0, False), (8, 30, 0.05, False)])
def test_dense_lu_pin_varied(N, J, load, hom):
    inst = make_instance(N, J, config=900, index=N, load=load, homogeneous=hom)
    Pd = exact.dense_solve(inst)
    r = cpu.solve(inst, tol=1e-13, max_iters=100000)
    assert np.abs(r.P - Pd).sum() <= 1e-10


def test_sparse_lu_pin_n13():
    """N=13 heterogeneous, clustered demand: oracle vs sparse LU."""
    inst = config_instance(3, 7, N=13, J=120)
    Ps = exact.sparse_solve(inst)
    r = cpu.solve(inst, tol=1e-13)
    assert np.abs(r.P - Ps).sum() <= 1e-10
    # both residual definitions agree on the oracle's answer
    assert exact.balance_residual(inst, r.P) == pytest.approx(r.residual, rel=1e-6, abs=1e-15)


# ------------------------------------------------------------ closed forms

def test_erlang_b_textbook_value():
    # B(10, 5) by the recursion B(k) = a B(k-1) / (k + a B(k-1))
    assert exact.erlang_b(10, 5.0) == pytest.approx(0.018384570336648, abs=1e-14)


def test_homogeneous_erlang_marginal_every_iteration():
    """nu_u = nu: mu(n) = n nu and lambda(n) = Lambda in every iteration, so
    (10) gives the truncated Poisson law regardless of the preference lists."""
    inst = config_instance(2, 0, N=12, J=60, homogeneous=True, load=0.6)
    a = inst.Lambda / 1.0
    want = exact.erlang_marginal(12, a)
    for iters in (1, 2, 5):
        r = cpu.solve(inst, tol=0.0, max_iters=iters)
        np.testing.assert_allclose(r.p_n, want, rtol=1e-12, atol=1e-15)
    r = cpu.solve(inst, tol=1e-13)
    _, pn = cpu.marginals(12, r.P)
    np.testing.assert_allclose(pn, want, rtol=1e-9, atol=1e-14)
    assert r.P[-1] == pytest.approx(exact.erlang_b(12, a), rel=1e-9)


def test_ordered_hunting_homogeneous():
    """All nodes share one list, equal rates: unit at rank h is busy with
    probability a (B(h-1, a) - B(h, a))."""
    N, J = 9, 5
    row = [4, 2, 7, 0, 8, 1, 3, 6, 5]
    inst = _inst(N, J, [0.7, 1.1, 0.4, 2.0, 0.9], [1.0] * N, [row] * J)
    r = cpu.solve(inst, tol=1e-13)
    rho, _ = cpu.marginals(N, r.P)
    np.testing.assert_allclose(rho, exact.ordered_hunting_rho(row, N, inst.Lambda), rtol=1e-9,
                               atol=1e-13)


def test_everyone_first_choice_unit_heterogeneous():
    """A unit that every node ranks first is idle-then-busy as an M/M/1/1
    queue: rho = Lambda / (Lambda + nu_u), whatever the other rates."""
    rng = np.random.default_rng(5)
    N, J = 7, 6
    pref = [[3] + list(rng.permutation([u for u in range(N) if u != 3])) for _ in range(J)]
    nu = rng.uniform(0.5, 1.5, N)
    lam = rng.uniform(0.1, 1.0, J)
    inst = _inst(N, J, lam, nu, pref)
    r = cpu.solve(inst, tol=1e-13)
    rho, _ = cpu.marginals(N, r.P)
    assert rho[3] == pytest.approx(lam.sum() / (lam.sum() + nu[3]), rel=1e-10)


def test_zero_arrivals():
    inst = _inst(3, 2, [0.0, 0.0], [1.0, 2.0, 3.0], [[0, 1, 2], [2, 1, 0]])
    r = cpu.solve(inst, tol=1e-12)
    assert r.P[0] == 1.0 and r.P[1:].sum() == 0.0


# -------------------------------------------------------------- invariants

def _dispatch(inst, m):
    """r(m, u): rate at which state m sends calls to idle unit u."""
    r = np.zeros(inst.N)
    for j in range(inst.J):
        f = exact.first_idle(m, inst.pref[j])
        if f >= 0:
            r[f] += inst.lam[j]
    return r


def test_up_rates_sum_to_lambda():
    """Proof of Lemma 1: sum over targets of lambda_{ml} = Lambda for every
    non-full m; with coefficients generated per target (Algorithm 3) that is
    sum_{u idle in l} a(l + u, u) = Lambda."""
    inst = config_instance(2, 3, N=11, J=80)
    rng = np.random.default_rng(0)
    for l in rng.integers(0, (1 << 11) - 1, 200):
        l = int(l)
        s = sum(cpu.up_coefficients(inst, l | (1 << u))[u] for u in range(11) if not (l >> u) & 1)
        assert s == pytest.approx(inst.Lambda, rel=1e-13)


def test_algorithm3_matches_per_source_dispatch():
    """a(m, u) generated per target equals r(m\\u, u) from the source side."""
    inst = config_instance(3, 1, N=12, J=150)
    rng = np.random.default_rng(1)
    for m in rng.integers(1, 1 << 12, 100):
        m = int(m)
        a = cpu.up_coefficients(inst, m)
        for u in range(12):
            if (m >> u) & 1:
                assert a[u] == pytest.approx(_dispatch(inst, m ^ (1 << u))[u], rel=1e-13, abs=1e-15)
            else:
                assert a[u] == 0.0


@pytest.fixture(scope="module")
def c1_solution():
    inst = config_instance(1, 4)
    return inst, cpu.solve(inst, tol=1e-13, want_layer_trace=True)


def test_probability_invariants(c1_solution):
    inst, r = c1_solution
    assert (r.P >= 0).all()
    assert r.P.sum() == pytest.approx(1.0, abs=1e-14)
    assert abs(r.mass_error) < 1e-12  # no renormalisation was needed
    assert r.residual <= 1e-13


def test_layer_normalisation_every_iteration(c1_solution):
    """Lemma 1 (2): sum_{C_n} p_n = 1 after every iteration (closed inner)."""
    _, r = c1_solution
    np.testing.assert_allclose(r.layer_trace, 1.0, rtol=0, atol=1e-12)


def test_flow_balance_per_unit(c1_solution):
    """Per unit: nu_u rho_u = sum_m P(m) r(m, u) (calls sent to u), and
    sum_u nu_u rho_u = Lambda (1 - P(full))."""
    inst, r = c1_solution
    N = inst.N
    rho, _ = cpu.marginals(N, r.P)
    sent = np.zeros(N)
    for m in range(1 << N):
        sent += r.P[m] * _dispatch(inst, m)
    np.testing.assert_allclose(inst.nu * rho, sent, rtol=1e-10)
    assert (inst.nu * rho).sum() == pytest.approx(inst.Lambda * (1 - r.P[-1]), rel=1e-11)


# ------------------------------------------------------------ metamorphic

def test_unit_relabelling_permutes_states():
    inst = config_instance(1, 6)
    N = inst.N
    perm = np.random.default_rng(3).permutation(N)  # old unit u -> new unit perm[u]
    inv = np.argsort(perm)
    relab = inst.copy()
    relab.nu = inst.nu[inv]
    relab.pref = perm[inst.pref].astype(np.int32)
    a = cpu.solve(inst, tol=1e-13).P
    b = cpu.solve(relab, tol=1e-13).P
    idx = np.zeros(1 << N, dtype=np.int64)
    for m in range(1 << N):
        mm = 0
        for u in range(N):
            if (m >> u) & 1:
                mm |= 1 << int(perm[u])
        idx[m] = mm
    np.testing.assert_allclose(b[idx], a, rtol=0, atol=1e-12)


def test_rate_scaling_invariance():
    inst = config_instance(1, 7)
    s = inst.copy()
    s.lam = inst.lam * 3.7
    s.nu = inst.nu * 3.7
    np.testing.assert_allclose(cpu.solve(s, tol=1e-13).P, cpu.solve(inst, tol=1e-13).P, atol=1e-12)


def test_merging_and_splitting_nodes():
    inst = config_instance(1, 8)
    # duplicate every node with half its rate, and merge identical lists
    split = inst.copy()
    split.J = 2 * inst.J
    split.lam = np.concatenate([inst.lam * 0.25, inst.lam * 0.75])
    split.pref = np.concatenate([inst.pref, inst.pref]).astype(np.int32)
    np.testing.assert_allclose(cpu.solve(split, tol=1e-13).P, cpu.solve(inst, tol=1e-13).P,
                               atol=1e-12)


def test_inner_modes_share_the_fixed_point():
    """The literal delta loop (delta -> 0), the closed-form limit and a single
    inner update all converge to the same stationary law; the literal loop
    tracks the closed form iteration by iteration."""
    inst = config_instance(1, 9)
    c = cpu.solve(inst, tol=0.0, max_iters=7, inner="closed")
    lit = cpu.solve(inst, tol=0.0, max_iters=7, inner="literal", delta=1e-16)
    np.testing.assert_allclose(lit.pcond, c.pcond, rtol=0, atol=1e-12)
    fin = [cpu.solve(inst, tol=1e-13, inner=m).P for m in ("closed", "literal", "one")]
    for P in fin[1:]:
        np.testing.assert_allclose(P, fin[0], atol=1e-11)


def test_paper_stopping_rule():
    inst = config_instance(1, 2)
    r = cpu.solve(inst, tol=1e-12, stop="delta")
    assert r.converged and r.max_delta <= 1e-12
    assert np.abs(r.P - exact.dense_solve(inst)).sum() < 1e-9


def test_layer_update_helpers_match_solver():
    """The sampled per-state update and the layer sums used at large N
    reproduce one closed-form layer step of the full solver."""
    inst = config_instance(1, 3)
    N = inst.N
    r1 = cpu.solve(inst, tol=0.0, max_iters=1)
    r2 = cpu.solve(inst, tol=0.0, max_iters=2)
    n = 4
    pl = r2.pcond  # layer n-1 from iteration 2
    pu = r1.pcond  # layer n+1 from iteration 1
    sums = cpu.layer_sums(inst, n, pl, pu)
    beta = r1.lam_n[n] / r1.mu_n[n + 1]
    Lprev = r2.lam_n[n - 1]
    alpha = cpu.closed_form_alpha(Lprev, beta, sums)
    states = np.array([m for m in range(1 << N) if bin(m).count("1") == n], dtype=np.uint32)
    got, _, _ = cpu.update_states(inst, states, pl, pu, alpha, beta)
    np.testing.assert_allclose(got, r2.pcond[states], rtol=1e-13, atol=1e-16)


# ------------------------------------------------------------------ mutants

_MUTANTS = {
    # only the most preferred busy unit is credited (misreading Algorithm 3)
    "walk_stops_early": ("a[u] += lam[j];\n        }", "a[u] += lam[j];\n            break;\n        }"),
    # the service-driven term of (12) uses the wrong unit's rate
    "wrong_service_rate": ("else dn += nu[u] * p[m | bit];", "else dn += nu[(u + 1) % N] * p[m | bit];"),
    # beta uses lambda(n+1) instead of lambda(n)
    "beta_index": ("const double beta = lamn[n] / mun[n + 1];", "const double beta = lamn[n + 1] / mun[n + 1];"),
    # p(n) product of (10) with an off-by-one in mu
    "pn_index": ("if (n > 0) g = g * lamn[n - 1] / mun[n];", "if (n > 0) g = g * lamn[n - 1] / mun[n > 1 ? n - 1 : 1];"),
}


@pytest.mark.parametrize("name", sorted(_MUTANTS))
def test_pins_catch_planted_mistakes(name, tmp_path):
    """Plant a plausible mistake in a copy of the oracle: the dense pin fails."""
    src = open(os.path.join(os.path.dirname(cpu.__file__), "hq_oracle.c")).read()
    old, new = _MUTANTS[name]
    assert src.count(old) >= 1, name
    mutated = src.replace(old, new)
    c = tmp_path / "m.c"
    so = tmp_path / "libm.so"
    c.write_text(mutated)
    subprocess.run(["gcc", "-O1", "-shared", "-fPIC", "-std=c99", "-D_POSIX_C_SOURCE=199309L",
                    str(c), "-o", str(so), "-lm"], check=True)
    import ctypes

    L = ctypes.CDLL(str(so))
    d = ctypes.POINTER(ctypes.c_double)
    i32 = ctypes.POINTER(ctypes.c_int32)
    L.orc_solve.restype = ctypes.c_int
    L.orc_solve.argtypes = [ctypes.c_int, ctypes.c_int, d, d, i32, ctypes.c_int, ctypes.c_double,
                            ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, d, d, d, d,
                            d, d, d]
    inst = config_instance(1, 0)
    lam = np.ascontiguousarray(inst.lam)
    nu = np.ascontiguousarray(inst.nu)
    pref = np.ascontiguousarray(inst.pref.reshape(-1))
    S = 1 << inst.N
    P, pc, lay, st = np.zeros(S), np.zeros(S), np.zeros(3 * (inst.N + 1)), np.zeros(8)
    dp = lambda a: a.ctypes.data_as(d)
    L.orc_solve(inst.N, inst.J, dp(lam), dp(nu), pref.ctypes.data_as(i32), 0, 0.0, 0, 1e-12, 3000, 1,
                None, dp(P), dp(pc), dp(lay), dp(st), None, None)
    err = np.abs(P - exact.dense_solve(inst)).sum()
    assert not (err <= 1e-6), f"mutant {name} escaped the dense pin (L1 {err:.2e})"


def test_balance_terms_match_generator():
    """Per-state balance terms (inflow - outflow) equal (P Q)_m with Q built
    per source state, for an arbitrary (not stationary) P."""
    inst = config_instance(3, 9, N=9, J=60)
    P = np.random.default_rng(4).random(1 << 9)
    Q = exact.generator_matrix(inst)
    states = np.arange(1 << 9, dtype=np.uint32)
    terms, out = cpu.balance_terms(inst, states, P)
    np.testing.assert_allclose(terms, P @ Q, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out, -np.diag(Q) * P, rtol=1e-13)


# ---------------------------------------------------------------------------
# Waiting room (Proposition 2 and the remark after it)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("N,C,idx", [(5, 1, 0), (6, 3, 1), (7, 2, 2)])
def test_buffered_marginal_matches_full_chain(N, C, idx):
    # the reformulation (loss-system layers + birth-death tail) against a
    # dense solve of the whole chain built per source, waiting states included
    inst = config_instance(1, idx, N=N, J=12)
    res = cpu.solve(inst, tol=1e-14)
    P, tail, summ = cpu.buffered_state(res, inst, C)
    Pd, tail_d = exact.buffered_dense_solve(inst, C)
    np.testing.assert_allclose(P, Pd, rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(tail, tail_d, rtol=1e-9)
    assert P.sum() + tail.sum() == pytest.approx(1.0, abs=1e-12)
    assert summ[1] == pytest.approx(tail_d.sum(), rel=1e-9)
    assert summ[3] == pytest.approx(tail_d[-1], rel=1e-9)  # arrivals find the room full
    assert summ[2] == pytest.approx(np.dot(np.arange(1, C + 1), tail_d), rel=1e-9)


def test_buffered_homogeneous_closed_form():
    # equal unit rates: the number in system is M/M/N/N+C whatever the lists
    N, C = 6, 4
    inst = config_instance(1, 3, N=N, J=20, homogeneous=True)
    a = float(np.sum(inst.lam)) / float(inst.nu[0])
    res = cpu.solve(inst, tol=1e-14)
    p, tail, summ = cpu.birth_death(res, inst, C)
    want = exact.buffered_erlang_marginal(N, a, C)
    np.testing.assert_allclose(np.r_[p, tail], want, rtol=1e-11)


def test_unlimited_room_erlang_c_and_limit():
    # unlimited room: P(wait) is Erlang C for equal rates, and a long finite
    # room converges to the geometric tail of the remark
    N = 6
    inst = config_instance(1, 4, N=N, J=20, homogeneous=True)
    inst = inst.__class__(**{**inst.__dict__, "lam": inst.lam * (4.5 / float(np.sum(inst.lam)))})
    a = 4.5 / float(inst.nu[0])
    res = cpu.solve(inst, tol=1e-14)
    p, _, summ = cpu.birth_death(res, inst, -1)
    assert summ[1] + p[N] == pytest.approx(exact.erlang_c(N, a), rel=1e-11)
    assert summ[3] == 0.0
    p2, tail2, summ2 = cpu.birth_death(res, inst, 400)
    np.testing.assert_allclose(p2, p, rtol=1e-12)
    assert summ2[2] == pytest.approx(summ[2], rel=1e-10)
    with pytest.raises(ValueError):
        over = inst.__class__(**{**inst.__dict__, "lam": inst.lam * 2.0})
        cpu.birth_death(cpu.solve(over, tol=1e-10), over, -1)


# ---------------------------------------------------------------------------
# Dispatch probabilities (unit workloads, response times)
# ---------------------------------------------------------------------------
def test_dispatch_flow_balance_against_dense_solve():
    # a unit's dispatch rate equals its completion rate nu_u rho_u, an exact
    # identity of the stationary law; P from LU, q from the brute-force oracle
    inst = config_instance(1, 7, N=8, J=25)
    P = exact.dense_solve(inst)
    q = cpu.dispatch(inst, P)
    full = P[-1]
    np.testing.assert_allclose(q.sum(axis=1), 1.0 - full, rtol=1e-12)
    rho = np.array([P[[m for m in range(1 << inst.N) if (m >> u) & 1]].sum() for u in range(inst.N)])
    np.testing.assert_allclose((inst.lam[:, None] * q).sum(axis=0), inst.nu * rho, rtol=1e-10)


def test_dispatch_ordered_hunting_closed_form():
    # one shared list, equal rates: the first h units form M/M/h/h, so the
    # (h+1)-th choice gets the calls that find h busy and it idle
    N = 7
    inst = config_instance(1, 8, N=N, J=5, homogeneous=True)
    row = inst.pref[0].copy()
    inst = inst.__class__(**{**inst.__dict__, "pref": np.tile(row, (inst.J, 1))})
    a = float(np.sum(inst.lam)) / float(inst.nu[0])
    P = exact.dense_solve(inst)
    q = cpu.dispatch(inst, P)
    B = [1.0] + [exact.erlang_b(h, a) for h in range(1, N + 1)]
    for h in range(N):
        np.testing.assert_allclose(q[:, row[h]], B[h] - B[h + 1], rtol=1e-10)


def test_golden_hand_derived_n2_dispatch_and_travel():
    """Dispatch rule of eq. (3) and the mean travel time, by hand on the
    2-unit system: per-node dispatch probabilities and a non-constant
    travel-time matrix (a weighting by q alone would give 452/172)."""
    g = _read_golden("n2_hand.txt")
    inst = _inst(int(g["N"][0]), int(g["J"][0]), [float(x) for x in g["lam"]],
                 [float(x) for x in g["nu"]], g["pref"])
    den = float(g["P_den"][0])
    P = np.array([int(x) for x in g["P_num"]], float) / den
    q = cpu.dispatch(inst, P)
    want_q = np.array([int(x) for x in g["q_num"]], float).reshape(2, 2) / den
    np.testing.assert_allclose(q, want_q, rtol=0, atol=1e-15)
    t = np.array([float(x) for x in g["travel"]]).reshape(2, 2)
    want = float(g["mean_travel_num"][0]) / float(g["mean_travel_den"][0])
    assert cpu.mean_travel(inst, q, t) == pytest.approx(want, rel=1e-14)


def test_mean_travel_unit_indicator_is_flow_share():
    """With t = 1 for unit u and 0 elsewhere, the mean travel time is the
    share of dispatched calls that unit u serves: nu_u rho_u over
    Lambda (1 - P(full)) (flow balance of unit u in the stationary law).
    A weighting by q alone, or by lambda alone, fails this."""
    inst = config_instance(1, 9, N=6, J=10)
    P = exact.dense_solve(inst)
    q = cpu.dispatch(inst, P)
    m = np.arange(1 << inst.N)
    Lam = float(np.sum(inst.lam))
    for u in range(inst.N):
        rho_u = P[(m >> u) & 1 == 1].sum()
        t = np.zeros((inst.J, inst.N))
        t[:, u] = 1.0
        want = inst.nu[u] * rho_u / (Lam * (1.0 - P[-1]))
        assert cpu.mean_travel(inst, q, t) == pytest.approx(want, rel=1e-10)


def test_mean_travel_definition():
    inst = config_instance(1, 9, N=6, J=10)
    P = exact.dense_solve(inst)
    q = cpu.dispatch(inst, P)
    t = np.ones((inst.J, inst.N)) * 3.5
    assert cpu.mean_travel(inst, q, t) == pytest.approx(3.5, rel=1e-14)
