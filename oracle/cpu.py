"""ctypes wrapper of the C oracle (``hq_oracle.c``) — TEST INFRASTRUCTURE ONLY.

Algorithm 1 of the paper in FP64 with the three inner-loop readings
(closed-form limit, literal delta loop, a single update), the balance
residual of (1), on-demand Algorithm-3 coefficients and per-layer update
checks used for sampled parity at large N.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hq_oracle.c")
_LIB = os.path.join(_HERE, "libhq_oracle.so")

INNER_CLOSED, INNER_LITERAL, INNER_ONE = 0, 1, 2
STOP_RESIDUAL, STOP_DELTA = 0, 1
_INNER = {"closed": INNER_CLOSED, "literal": INNER_LITERAL, "one": INNER_ONE}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over independent states)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
               "-D_POSIX_C_SOURCE=199309L", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        d = ctypes.POINTER(ctypes.c_double)
        i32 = ctypes.POINTER(ctypes.c_int32)
        u32 = ctypes.POINTER(ctypes.c_uint32)
        L.orc_solve.restype = ctypes.c_int
        L.orc_solve.argtypes = [ctypes.c_int, ctypes.c_int, d, d, i32, ctypes.c_int, ctypes.c_double,
                                ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, d, d, d, d,
                                d, d, d]
        L.orc_residual.restype = ctypes.c_double
        L.orc_residual.argtypes = [ctypes.c_int, ctypes.c_int, d, d, i32, d, d]
        L.orc_up_coefficients.restype = None
        L.orc_up_coefficients.argtypes = [ctypes.c_int, ctypes.c_int, d, i32, ctypes.c_uint32, d]
        L.orc_update_states.restype = None
        L.orc_update_states.argtypes = [ctypes.c_int, ctypes.c_int, d, d, i32, ctypes.c_longlong, u32,
                                        d, d, ctypes.c_double, ctypes.c_double, d, d, d]
        L.orc_layer_sums.restype = None
        L.orc_layer_sums.argtypes = [ctypes.c_int, ctypes.c_int, d, d, i32, ctypes.c_int, d, d, d]
        L.orc_marginals.restype = None
        L.orc_marginals.argtypes = [ctypes.c_int, d, d, d]
        L.orc_threads.restype = ctypes.c_int
        L.orc_birth_death.restype = ctypes.c_int
        L.orc_birth_death.argtypes = [ctypes.c_int, d, d, ctypes.c_double, ctypes.c_double, ctypes.c_int, d, d, d]
        L.orc_dispatch.restype = None
        L.orc_dispatch.argtypes = [ctypes.c_int, ctypes.c_int, i32, d, d]
        L.orc_time_sample.restype = ctypes.c_int
        L.orc_time_sample.argtypes = [ctypes.c_int, ctypes.c_int, d, d, i32, ctypes.c_int, ctypes.c_longlong,
                                      ctypes.c_longlong, ctypes.c_int, ctypes.c_int, d]
        L.orc_balance_terms.restype = None
        L.orc_balance_terms.argtypes = [ctypes.c_int, ctypes.c_int, d, d, i32, ctypes.c_longlong, u32, d, d, d]
        _lib = L
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _up(a: np.ndarray):
    assert a.dtype == np.uint32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def threads() -> int:
    return int(lib().orc_threads())


@dataclass
class OracleResult:
    P: np.ndarray  # [2^N] stationary distribution, bitmask order
    pcond: np.ndarray  # [2^N] conditional layer probabilities p_n(m)
    lam_n: np.ndarray  # [N+1] lambda(n)
    mu_n: np.ndarray  # [N+1] mu(n)
    p_n: np.ndarray  # [N+1] birth-death marginal p(n)
    iterations: int
    residual: float
    mass_error: float  # sum(P) - 1 before the final renormalisation
    drift: float  # max_n |sum p_n - 1|
    max_delta: float  # last max |p^k - p^(k-1)|
    coef_seconds: float
    iter_seconds: float
    threads: int
    converged: bool
    trace: Optional[np.ndarray] = None
    layer_trace: Optional[np.ndarray] = None


def _args(inst):
    lam = np.ascontiguousarray(inst.lam, dtype=np.float64)
    nu = np.ascontiguousarray(inst.nu, dtype=np.float64)
    pref = np.ascontiguousarray(inst.pref, dtype=np.int32).reshape(-1)
    return lam, nu, pref


def solve(inst, *, tol: float = 1e-12, inner: str = "closed", delta: float = 1e-15,
          stop: str = "residual", max_iters: int = 100000, check_every: int = 1,
          init_p: Optional[np.ndarray] = None, want_trace: bool = False,
          want_layer_trace: bool = False) -> OracleResult:
    """Algorithm 1 in FP64.  ``stop='residual'`` stops when the relative L1
    balance residual is <= tol (checked every ``check_every`` iterations);
    ``stop='delta'`` uses the paper's max |p^k - p^(k-1)| <= tol."""
    N, J = inst.N, inst.J
    lam, nu, pref = _args(inst)
    S = 1 << N
    P = np.zeros(S)
    pc = np.zeros(S)
    layer = np.zeros(3 * (N + 1))
    stats = np.zeros(8)
    trace = np.zeros(max_iters) if want_trace else None
    ltrace = np.zeros(max_iters * (N + 1)) if want_layer_trace else None
    ip = None if init_p is None else np.ascontiguousarray(init_p, dtype=np.float64)
    rc = lib().orc_solve(N, J, _dp(lam), _dp(nu), _ip(pref), _INNER[inner], delta,
                         STOP_DELTA if stop == "delta" else STOP_RESIDUAL, tol, max_iters,
                         check_every, _dp(ip), _dp(P), _dp(pc), _dp(layer), _dp(stats),
                         _dp(trace), _dp(ltrace))
    if rc < 0:
        raise ValueError("oracle rejected the input")
    it = int(stats[0])
    lay = layer.reshape(N + 1, 3)
    return OracleResult(
        P=P, pcond=pc, lam_n=lay[:, 0].copy(), mu_n=lay[:, 1].copy(), p_n=lay[:, 2].copy(),
        iterations=it, residual=float(stats[1]), mass_error=float(stats[2]), drift=float(stats[3]),
        max_delta=float(stats[4]), coef_seconds=float(stats[5]), iter_seconds=float(stats[6]),
        threads=int(stats[7]), converged=(rc == 0),
        trace=None if trace is None else trace[:it].copy(),
        layer_trace=None if ltrace is None else ltrace[: it * (N + 1)].reshape(it, N + 1).copy(),
    )


def time_sample(inst, n: int, first: int, count: int, reps: int, threads: int = 0) -> dict:
    """Time Algorithm 1 on `count` consecutive states of layer n: step 2's
    coefficient generation, then one outer-iteration update of those states
    (same code as ``solve``).  Returns seconds of each and the threads used."""
    lam, nu, pref = _args(inst)
    out = np.zeros(4)
    rc = lib().orc_time_sample(inst.N, inst.J, _dp(lam), _dp(nu), _ip(pref), int(n), int(first), int(count),
                               int(reps), int(threads), _dp(out))
    if rc != 0:
        raise ValueError("oracle rejected the timing sample")
    return {"coef_s": float(out[0]), "update_s": float(out[1]), "threads": int(out[2]),
            "checksum": float(out[3])}


def residual(inst, P: np.ndarray, want_terms: bool = False):
    """Relative L1 balance residual of P (bitmask order), eq. (1)."""
    lam, nu, pref = _args(inst)
    P = np.ascontiguousarray(P, dtype=np.float64)
    terms = np.zeros(1 << inst.N) if want_terms else None
    r = lib().orc_residual(inst.N, inst.J, _dp(lam), _dp(nu), _ip(pref), _dp(P), _dp(terms))
    return (float(r), terms) if want_terms else float(r)


def up_coefficients(inst, m: int) -> np.ndarray:
    """Algorithm 3 for one target state: a[u] = rate m\\{u} -> m (0 for idle u)."""
    lam, nu, pref = _args(inst)
    a = np.zeros(inst.N)
    lib().orc_up_coefficients(inst.N, inst.J, _dp(lam), _ip(pref), int(m), _dp(a))
    return a


def update_states(inst, states: np.ndarray, pl: np.ndarray, pu: np.ndarray, alpha: float,
                  beta: float):
    """(12) for sampled states of one layer with on-demand coefficients.
    Returns (p_new, U, D)."""
    lam, nu, pref = _args(inst)
    st = np.ascontiguousarray(states, dtype=np.uint32)
    n = len(st)
    out, U, D = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().orc_update_states(inst.N, inst.J, _dp(lam), _dp(nu), _ip(pref), n, _up(st),
                            _dp(np.ascontiguousarray(pl, dtype=np.float64)),
                            _dp(np.ascontiguousarray(pu, dtype=np.float64)), alpha, beta,
                            _dp(out), _dp(U), _dp(D))
    return out, U, D


def layer_sums(inst, n: int, pl: np.ndarray, pu: np.ndarray) -> np.ndarray:
    """[sum U, sum mu U, sum D, sum mu D] over layer n."""
    lam, nu, pref = _args(inst)
    out = np.zeros(4)
    lib().orc_layer_sums(inst.N, inst.J, _dp(lam), _dp(nu), _ip(pref), int(n),
                         _dp(np.ascontiguousarray(pl, dtype=np.float64)),
                         _dp(np.ascontiguousarray(pu, dtype=np.float64)), _dp(out))
    return out


def marginals(N: int, P: np.ndarray):
    """(rho_u, number-busy marginal) from P in bitmask order."""
    rho = np.zeros(N)
    pn = np.zeros(N + 1)
    lib().orc_marginals(N, _dp(np.ascontiguousarray(P, dtype=np.float64)), _dp(rho), _dp(pn))
    return rho, pn


def closed_form_alpha(Lprev: float, beta: float, sums: np.ndarray) -> float:
    """alpha_n = mu*(n) / lambda(n-1) for the closed-form inner limit:
    mu* = B / (1 - A), A = sum mu U / Lprev, B = beta sum mu D."""
    A = sums[1] / Lprev
    B = beta * sums[3]
    return (B / (1.0 - A)) / Lprev


def balance_terms(inst, states: np.ndarray, P: np.ndarray):
    """(inflow - outflow, outflow) of (1) at the sampled states."""
    lam, nu, pref = _args(inst)
    st = np.ascontiguousarray(states, dtype=np.uint32)
    out = np.zeros(len(st))
    of = np.zeros(len(st))
    lib().orc_balance_terms(inst.N, inst.J, _dp(lam), _dp(nu), _ip(pref), len(st), _up(st),
                            _dp(np.ascontiguousarray(P, dtype=np.float64)), _dp(out), _dp(of))
    return out, of


def birth_death(res: OracleResult, inst, C: int):
    """Marginal of the system with a waiting room of C calls (C < 0:
    unlimited), Proposition 2, from the lambda(n), mu(n) of a loss-system
    solve.  Returns (p[N+1], tail[C] or None, summary[4]) with summary =
    (P(all busy), P(wait), mean waiting, P(lost))."""
    N = inst.N
    p = np.zeros(N + 1)
    tail = np.zeros(C) if C > 0 else None
    summ = np.zeros(4)
    rc = lib().orc_birth_death(N, _dp(np.ascontiguousarray(res.lam_n)), _dp(np.ascontiguousarray(res.mu_n)),
                               float(np.sum(inst.lam)), float(np.sum(inst.nu)), int(C), _dp(p), _dp(tail),
                               _dp(summ))
    if rc != 0:
        raise ValueError("unlimited waiting room needs Lambda < sum of service rates")
    return p, tail, summ


def buffered_state(res: OracleResult, inst, C: int):
    """P over the 2^N unit states of the buffered system: the loss-system
    layers p_n(m) times the buffered p(n) (Proposition 2)."""
    p, tail, summ = birth_death(res, inst, C)
    scale = np.zeros(inst.N + 1)
    for n in range(inst.N + 1):
        scale[n] = p[n] / res.p_n[n] if res.p_n[n] > 0 else 0.0
    pop = np.array([bin(m).count("1") for m in range(1 << inst.N)])
    return res.P * scale[pop], tail, summ


def dispatch(inst, P: np.ndarray) -> np.ndarray:
    """q[j, u]: probability that a call from node j is sent to unit u
    (first idle unit of its list), from P in bitmask order."""
    _, _, pref = _args(inst)
    q = np.zeros(inst.J * inst.N)
    lib().orc_dispatch(inst.N, inst.J, _ip(pref), _dp(np.ascontiguousarray(P, dtype=np.float64)), _dp(q))
    return q.reshape(inst.J, inst.N)


def mean_travel(inst, q: np.ndarray, travel: np.ndarray) -> float:
    """Mean travel time of dispatched calls: sum_j lambda_j sum_u q_ju t_ju
    over sum_j lambda_j sum_u q_ju (travel[j, u] from unit u to node j)."""
    w = inst.lam[:, None] * q
    return float((w * travel).sum() / w.sum())
