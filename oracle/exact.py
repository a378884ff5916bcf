"""Independent exact solvers and closed forms — TEST INFRASTRUCTURE ONLY.

These pin the oracle of ``hq_oracle.c`` to something other than itself:

* ``generator_matrix`` builds the CTMC generator Q of Section 2.1 per
  SOURCE state: every demand node sends its calls to its first idle
  preferred unit (no call is sent when all units are busy, C = 0), and every
  busy unit completes service at its own rate.  The oracle builds its
  coefficients per TARGET state (Algorithm 3), so agreement also checks that
  reading of (3).
* ``dense_solve`` solves PQ = 0 with one balance equation replaced by
  sum(P) = 1, as (1)-(2) prescribe, by LU (numpy).  ``sparse_solve`` does the
  same with scipy's sparse LU for larger N.
* ``erlang_b`` / ``erlang_marginal``: with equal service rates nu the number
  of busy units is a truncated Poisson (Erlang loss) law for any preference
  lists — the birth-death form (10) with mu(n) = n nu and lambda(n) = Lambda.
* ``ordered_hunting_rho``: all nodes share one list and rates are equal: the
  first h units form an M/M/h/h system, so unit pi[h-1] is busy with
  probability a (B(h-1,a) - B(h,a)).
"""
from __future__ import annotations

import math

import numpy as np


def first_idle(m: int, row) -> int:
    """First unit in preference row that is idle in state m, or -1."""
    for u in row:
        if not (m >> int(u)) & 1:
            return int(u)
    return -1


def generator_matrix(inst, sparse: bool = False):
    """Q[l, m] = transition rate l -> m (l != m), Q[l, l] = -sum of row l."""
    N = inst.N
    S = 1 << N
    lam = np.asarray(inst.lam, dtype=np.float64)
    nu = np.asarray(inst.nu, dtype=np.float64)
    pref = np.asarray(inst.pref)
    rows, cols, vals = [], [], []
    # arrivals: group demand nodes by their first idle unit, state by state
    for l in range(S):
        busy = [(l >> u) & 1 for u in range(N)]
        acc = {}
        for j in range(inst.J):
            f = -1
            for u in pref[j]:
                if not busy[int(u)]:
                    f = int(u)
                    break
            if f >= 0:
                acc[f] = acc.get(f, 0.0) + lam[j]
        for f, r in acc.items():
            rows.append(l)
            cols.append(l | (1 << f))
            vals.append(r)
        for u in range(N):
            if busy[u]:
                rows.append(l)
                cols.append(l ^ (1 << u))
                vals.append(nu[u])
    rows = np.array(rows, dtype=np.int64)
    cols = np.array(cols, dtype=np.int64)
    vals = np.array(vals, dtype=np.float64)
    if sparse:
        import scipy.sparse as sp

        Q = sp.coo_matrix((vals, (rows, cols)), shape=(S, S)).tocsr()
        out = np.asarray(Q.sum(axis=1)).ravel()
        Q = Q - sp.diags(out)
        return Q.tocsc()
    Q = np.zeros((S, S))
    np.add.at(Q, (rows, cols), vals)
    Q[np.arange(S), np.arange(S)] -= Q.sum(axis=1)
    return Q


def dense_solve(inst) -> np.ndarray:
    """Stationary P of (1)-(2) by LU, one balance equation replaced by sum = 1."""
    Q = generator_matrix(inst)
    S = Q.shape[0]
    A = Q.T.copy()  # rows of A: balance equations (P Q)_m = 0
    A[-1, :] = 1.0
    b = np.zeros(S)
    b[-1] = 1.0
    return np.linalg.solve(A, b)


def sparse_solve(inst) -> np.ndarray:
    """Same system as dense_solve with scipy's sparse LU (N up to ~16)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl

    Q = generator_matrix(inst, sparse=True)
    S = Q.shape[0]
    A = Q.T.tolil()
    A[S - 1, :] = np.ones(S)
    b = np.zeros(S)
    b[-1] = 1.0
    return spl.spsolve(A.tocsc(), b)


def balance_residual(inst, P: np.ndarray) -> float:
    """sum |PQ| / sum P(m)(lambda_m + mu_m) with Q from generator_matrix."""
    Q = generator_matrix(inst, sparse=True)
    r = Q.T @ P
    out = -Q.diagonal() * P
    return float(np.abs(r).sum() / out.sum())


def erlang_b(n: int, a: float) -> float:
    """Erlang loss probability B(n, a) by the stable recursion B(k) = aB/(k+aB)."""
    b = 1.0
    for k in range(1, n + 1):
        b = a * b / (k + a * b)
    return b


def erlang_marginal(N: int, a: float) -> np.ndarray:
    """Truncated Poisson law p(n) proportional to a^n / n!, n = 0..N."""
    w = np.array([math.exp(n * math.log(a) - math.lgamma(n + 1)) for n in range(N + 1)])
    return w / w.sum()


def ordered_hunting_rho(pref_row, N: int, a: float) -> np.ndarray:
    """Busy probability of each unit when every call hunts the same list."""
    rho = np.zeros(N)
    for h in range(1, N + 1):
        rho[int(pref_row[h - 1])] = a * (erlang_b(h - 1, a) - erlang_b(h, a))
    return rho


def buffered_dense_solve(inst, C: int):
    """Stationary law of the chain with a waiting room of C calls, built
    from first principles (not from the reformulation): unit states
    0..2^N-1 as in generator_matrix, plus waiting states S-1+c, c = 1..C
    (all units busy, c calls waiting, first come first served).  From the
    full state an arrival moves to c = 1; from c an arrival moves to c + 1
    (lost when c = C); any completion at a waiting state hands the next call
    to the freed unit, so c drops by one.  Returns (P over unit states,
    P~ over waiting states)."""
    N = inst.N
    S = 1 << N
    full = S - 1
    lam_tot = float(np.sum(inst.lam))
    nu_tot = float(np.sum(inst.nu))
    T = S + C
    Q = np.zeros((T, T))
    Q[:S, :S] = generator_matrix(inst)
    # generator_matrix has no arrivals out of the full state; add them
    if C > 0:
        Q[full, S] += lam_tot
        Q[full, full] -= lam_tot
        for c in range(1, C + 1):
            i = S + c - 1
            if c < C:
                Q[i, i + 1] += lam_tot
            below = full if c == 1 else i - 1
            Q[i, below] += nu_tot
            Q[i, i] -= Q[i].sum() - Q[i, i]
    A = Q.T.copy()
    A[-1, :] = 1.0
    b = np.zeros(T)
    b[-1] = 1.0
    x = np.linalg.solve(A, b)
    return x[:S], x[S:]


def buffered_erlang_marginal(N: int, a: float, C: int) -> np.ndarray:
    """M/M/N/N+C law of the number in system, n = 0..N+C (homogeneous unit
    rates, a = Lambda / nu): a^n / n! up to N, then a^N / N! (a / N)^(n-N)."""
    w = [1.0]
    for n in range(1, N + C + 1):
        w.append(w[-1] * a / min(n, N))
    w = np.array(w)
    return w / w.sum()


def erlang_c(N: int, a: float) -> float:
    """Probability that an arrival waits in M/M/N with unlimited room, a < N."""
    B = erlang_b(N, a)
    return N * B / (N - a * (1.0 - B))
