"""Thin ctypes binding of libhq.so (include/hq.h) — argument marshalling only.

Every computation runs in the HIP library; this module converts numpy
arrays (or torch tensors) to pointers and status codes to exceptions.  It
fails loudly if the built library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhq.so")

HQ_MAX_N = 30
HQ_OK, HQ_ERR_INVALID_ARG, HQ_ERR_OUT_OF_MEMORY, HQ_ERR_DEVICE, HQ_ERR_NOT_CONVERGED, HQ_ERR_NUMERIC, \
    HQ_ERR_STATE = range(7)
HQ_FP64, HQ_FP32, HQ_FP32_POLISH64 = 0, 1, 2
HQ_INNER_CLOSED, HQ_INNER_ONE, HQ_INNER_LITERAL = 0, 1, 2
HQ_INIT_UNIFORM, HQ_INIT_PRODUCT, HQ_INIT_STATE, HQ_INIT_LEARNED = 0, 1, 2, 3
HQ_STOP_RESIDUAL, HQ_STOP_DELTA = 0, 1
HQ_BUFFER_UNLIMITED, HQ_BUFFER_MAX = -1, 65536

STATUS_NAMES = {0: "HQ_OK", 1: "HQ_ERR_INVALID_ARG", 2: "HQ_ERR_OUT_OF_MEMORY", 3: "HQ_ERR_DEVICE",
                4: "HQ_ERR_NOT_CONVERGED", 5: "HQ_ERR_NUMERIC", 6: "HQ_ERR_STATE"}

# every symbol include/hq.h declares
EXPORTED = ["hq_default_options", "hq_create", "hq_solve", "hq_marginals", "hq_queue", "hq_dispatch", "hq_state",
            "hq_solve_batch", "hq_solve_batch_noalloc", "hq_batch_last_block",
            "hq_destroy", "hq_last_error", "hq_iterate", "hq_reset", "hq_residual", "hq_conditional",
            "hq_layer_scalars", "hq_state_device", "hq_num_units", "hq_mlp_features", "hq_mlp_create",
            "hq_mlp_destroy", "hq_mlp_get_params", "hq_mlp_set_params", "hq_mlp_forward", "hq_mlp_gradient",
            "hq_mlp_train"]
HQ_MLP_IN, HQ_MLP_HIDDEN = 32, 256
HQ_MLP_PARAMS = HQ_MLP_IN * HQ_MLP_HIDDEN + HQ_MLP_HIDDEN + HQ_MLP_HIDDEN * HQ_MLP_HIDDEN + 2 * HQ_MLP_HIDDEN + 1


class HQError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class hq_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("inner", ctypes.c_int), ("init", ctypes.c_int),
                ("stop", ctypes.c_int), ("max_iters", ctypes.c_int), ("check_every", ctypes.c_int),
                ("tile_bits", ctypes.c_int), ("device", ctypes.c_int), ("stored_layers", ctypes.c_int),
                ("init_rho", ctypes.POINTER(ctypes.c_double)),
                ("init_state", ctypes.POINTER(ctypes.c_double)), ("stream", ctypes.c_void_p),
                ("mlp", ctypes.c_void_p), ("buffer", ctypes.c_int), ("delta", ctypes.c_double)]


class hq_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int), ("checks", ctypes.c_int),
                ("fp64_iterations", ctypes.c_int), ("residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("sweep_seconds", ctypes.c_double),
                ("state_updates_per_s", ctypes.c_double), ("mass_error", ctypes.c_double),
                ("max_layer_drift", ctypes.c_double), ("warm_used", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load libhq.so; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libhq.so not found at {path}: build it first (python __graft_entry__.py build)")
    L = ctypes.CDLL(path)
    c_int, c_double, vp = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    L.hq_default_options.argtypes = [ctypes.POINTER(hq_options)]
    L.hq_default_options.restype = None
    L.hq_create.argtypes = [c_int, c_int, dp, dp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(hq_options),
                            ctypes.POINTER(vp)]
    L.hq_create.restype = c_int
    L.hq_solve.argtypes = [vp, c_double, ctypes.POINTER(hq_info)]
    L.hq_solve.restype = c_int
    L.hq_marginals.argtypes = [vp, dp, dp]
    L.hq_marginals.restype = c_int
    L.hq_queue.argtypes = [vp, dp, dp, c_int]
    L.hq_queue.restype = c_int
    L.hq_dispatch.argtypes = [vp, dp, dp, dp]
    L.hq_dispatch.restype = c_int
    L.hq_state.argtypes = [vp, dp]
    L.hq_state.restype = c_int
    L.hq_solve_batch.argtypes = [ctypes.POINTER(vp), c_int, c_double, ctypes.POINTER(hq_info)]
    L.hq_solve_batch.restype = c_int
    L.hq_solve_batch_noalloc.argtypes = [ctypes.POINTER(vp), c_int, c_double, ctypes.POINTER(hq_info)]
    L.hq_solve_batch_noalloc.restype = c_int
    L.hq_batch_last_block.argtypes = []
    L.hq_batch_last_block.restype = c_int
    L.hq_destroy.argtypes = [vp]
    L.hq_destroy.restype = None
    L.hq_last_error.argtypes = []
    L.hq_last_error.restype = ctypes.c_char_p
    L.hq_iterate.argtypes = [vp, c_int]
    L.hq_iterate.restype = c_int
    L.hq_reset.argtypes = [vp]
    L.hq_reset.restype = c_int
    L.hq_residual.argtypes = [vp, dp]
    L.hq_residual.restype = c_int
    L.hq_conditional.argtypes = [vp, dp]
    L.hq_conditional.restype = c_int
    L.hq_layer_scalars.argtypes = [vp, dp]
    L.hq_layer_scalars.restype = c_int
    L.hq_state_device.argtypes = [vp, vp, vp]
    L.hq_state_device.restype = c_int
    L.hq_num_units.argtypes = [vp]
    L.hq_num_units.restype = c_int
    fp = ctypes.POINTER(ctypes.c_float)
    L.hq_mlp_features.argtypes = [c_int, c_int, dp, dp, ctypes.POINTER(ctypes.c_int32), fp]
    L.hq_mlp_features.restype = c_int
    L.hq_mlp_create.argtypes = [c_int, ctypes.c_ulonglong, ctypes.POINTER(vp)]
    L.hq_mlp_create.restype = c_int
    L.hq_mlp_destroy.argtypes = [vp]
    L.hq_mlp_destroy.restype = None
    L.hq_mlp_get_params.argtypes = [vp, fp]
    L.hq_mlp_get_params.restype = c_int
    L.hq_mlp_set_params.argtypes = [vp, fp]
    L.hq_mlp_set_params.restype = c_int
    L.hq_mlp_forward.argtypes = [vp, fp, c_int, fp]
    L.hq_mlp_forward.restype = c_int
    L.hq_mlp_gradient.argtypes = [vp, fp, fp, c_int, fp, fp]
    L.hq_mlp_gradient.restype = c_int
    L.hq_mlp_train.argtypes = [vp, fp, fp, c_int, c_int, c_int, ctypes.c_float, ctypes.c_ulonglong, fp]
    L.hq_mlp_train.restype = c_int
    _lib = L
    return L


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(status: int, allow=(HQ_OK,)):
    if status not in allow:
        raise HQError(status, hq_last_error())
    return status


def hq_last_error() -> str:
    return load().hq_last_error().decode()


def hq_default_options() -> hq_options:
    o = hq_options()
    load().hq_default_options(ctypes.byref(o))
    return o


class Context:
    """Owns an hq_ctx*; the arrays referenced by its options are kept alive."""

    def __init__(self, handle: ctypes.c_void_p, N: int, J: int = 0):
        self.handle = handle
        self.N = N
        self.J = J

    def __del__(self):
        try:
            hq_destroy(self)
        except Exception:
            pass


def hq_create(N: int, J: int, lambda_j, mu_i, pref_lists, opts: Optional[hq_options] = None,
              *, init_rho=None, init_state=None, stream=None, mlp=None, **fields) -> Context:
    """hq_create(N, J, lambda_j[J], mu_i[N], pref_lists[J*N], opts).  Keyword
    fields (precision=..., inner=..., ...) override entries of opts."""
    L = load()
    lam = np.ascontiguousarray(lambda_j, dtype=np.float64).reshape(-1)
    mu = np.ascontiguousarray(mu_i, dtype=np.float64).reshape(-1)
    pref = np.ascontiguousarray(pref_lists, dtype=np.int32).reshape(-1)
    if lam.size != J or mu.size != N or pref.size != J * N:
        raise HQError(HQ_ERR_INVALID_ARG, "array sizes do not match N and J")
    o = hq_default_options() if opts is None else opts
    for k, v in fields.items():
        setattr(o, k, v)
    keep = []
    if init_rho is not None:
        r = np.ascontiguousarray(init_rho, dtype=np.float64)
        keep.append(r)
        o.init_rho = _dptr(r)
        if "init" not in fields:
            o.init = HQ_INIT_PRODUCT
    if init_state is not None:
        s = np.ascontiguousarray(init_state, dtype=np.float64)
        keep.append(s)
        o.init_state = _dptr(s)
        if "init" not in fields:
            o.init = HQ_INIT_STATE
    if stream is not None:
        o.stream = ctypes.c_void_p(int(stream))
    if mlp is not None:
        o.mlp = mlp.handle
        if "init" not in fields:
            o.init = HQ_INIT_LEARNED
    h = ctypes.c_void_p()
    _check(L.hq_create(int(N), int(J), _dptr(lam), _dptr(mu), pref.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                       ctypes.byref(o), ctypes.byref(h)))
    return Context(h, int(N), int(J))


def hq_solve(ctx: Context, tol: float, *, allow_not_converged: bool = False) -> dict:
    info = hq_info()
    st = load().hq_solve(ctx.handle, float(tol), ctypes.byref(info))
    _check(st, (HQ_OK, HQ_ERR_NOT_CONVERGED) if allow_not_converged else (HQ_OK,))
    return info.as_dict()


def hq_marginals(ctx: Context):
    rho = np.zeros(ctx.N)
    pn = np.zeros(ctx.N + 1)
    _check(load().hq_marginals(ctx.handle, _dptr(rho), _dptr(pn)))
    return rho, pn


def hq_dispatch(ctx: Context, travel=None):
    """(q[J, N], mean travel time or None): q[j, i] = probability that a
    call from node j is sent to unit i; travel[j, i] = travel time from
    unit i to node j."""
    q = np.zeros(ctx.J * ctx.N)
    t = None if travel is None else np.ascontiguousarray(travel, dtype=np.float64).reshape(-1)
    if t is not None and t.size != ctx.J * ctx.N:
        raise HQError(HQ_ERR_INVALID_ARG, "travel must have J * N entries")
    mt = ctypes.c_double(0.0)
    _check(load().hq_dispatch(ctx.handle, _dptr(t), _dptr(q), ctypes.byref(mt) if t is not None else None))
    return q.reshape(ctx.J, ctx.N), (mt.value if t is not None else None)


def hq_queue(ctx: Context, length: int = 0):
    """Waiting-room measures: (summary[4], tail[length]) with summary =
    (P(all busy), P(a call waits), mean waiting, P(arrival lost)) and
    tail[c-1] = P~{c}."""
    summ = np.zeros(4)
    tail = np.zeros(length)
    _check(load().hq_queue(ctx.handle, _dptr(summ), _dptr(tail) if length else None, int(length)))
    return summ, tail


def hq_state(ctx: Context) -> np.ndarray:
    P = np.zeros(1 << ctx.N)
    _check(load().hq_state(ctx.handle, _dptr(P)))
    return P


def hq_state_device(ctx: Context, out, stream=None):
    """Export P into a float64 CUDA tensor `out` of 2^N elements."""
    ptr = out.data_ptr()
    s = ctypes.c_void_p(int(stream)) if stream is not None else None
    _check(load().hq_state_device(ctx.handle, ctypes.c_void_p(ptr), s))
    return out


def hq_solve_batch(ctxs: Sequence[Context], tol: float, *, allow_not_converged: bool = False):
    n = len(ctxs)
    arr = (ctypes.c_void_p * n)(*[c.handle for c in ctxs])
    infos = (hq_info * n)()
    st = load().hq_solve_batch(arr, n, float(tol), infos)
    _check(st, (HQ_OK, HQ_ERR_NOT_CONVERGED) if allow_not_converged else (HQ_OK,))
    return st, [infos[i].as_dict() for i in range(n)]


def hq_solve_batch_noalloc(ctxs: Sequence[Context], tol: float, *, allow_not_converged: bool = False):
    """hq_solve_batch with its scratch in the library's static device array
    (no device allocation during the call); at most 256 contexts."""
    n = len(ctxs)
    arr = (ctypes.c_void_p * max(n, 1))(*[c.handle for c in ctxs])
    infos = (hq_info * max(n, 1))()
    st = load().hq_solve_batch_noalloc(arr, n, float(tol), infos)
    _check(st, (HQ_OK, HQ_ERR_NOT_CONVERGED) if allow_not_converged else (HQ_OK,))
    return st, [infos[i].as_dict() for i in range(n)]


def hq_batch_last_block() -> int:
    """Work-group size of the most recent batched solve (0 before any)."""
    return int(load().hq_batch_last_block())


def hq_destroy(ctx: Context):
    if ctx is not None and ctx.handle:
        load().hq_destroy(ctx.handle)
        ctx.handle = None


def hq_iterate(ctx: Context, iters: int):
    _check(load().hq_iterate(ctx.handle, int(iters)))


def hq_reset(ctx: Context):
    _check(load().hq_reset(ctx.handle))


def hq_residual(ctx: Context) -> float:
    r = ctypes.c_double()
    _check(load().hq_residual(ctx.handle, ctypes.byref(r)))
    return r.value


def hq_conditional(ctx: Context) -> np.ndarray:
    p = np.zeros(1 << ctx.N)
    _check(load().hq_conditional(ctx.handle, _dptr(p)))
    return p


def hq_layer_scalars(ctx: Context) -> np.ndarray:
    """[N+1, 4]: lambda(n), mu(n), p(n), alpha_n."""
    out = np.zeros(4 * (ctx.N + 1))
    _check(load().hq_layer_scalars(ctx.handle, _dptr(out)))
    return out.reshape(ctx.N + 1, 4)


def hq_num_units(ctx: Context) -> int:
    return int(load().hq_num_units(ctx.handle))


def create_from_instance(inst, **kw) -> Context:
    """hq_create from a seeded instance (paper_2603_03019_amd.instances)."""
    return hq_create(inst.N, inst.J, inst.lam, inst.nu, inst.pref, **kw)


# ---------------------------------------------------------------- warm-start network

def _fptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class MLP:
    """Owns an hq_mlp* (the warm-start network)."""

    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        try:
            hq_mlp_destroy(self)
        except Exception:
            pass


def hq_mlp_create(device: int = -1, seed: int = 0) -> MLP:
    h = ctypes.c_void_p()
    _check(load().hq_mlp_create(int(device), int(seed), ctypes.byref(h)))
    return MLP(h)


def hq_mlp_destroy(m: MLP):
    if m is not None and m.handle:
        load().hq_mlp_destroy(m.handle)
        m.handle = None


def hq_mlp_features(N, J, lambda_j, mu_i, pref_lists) -> np.ndarray:
    lam = np.ascontiguousarray(lambda_j, dtype=np.float64).reshape(-1)
    mu = np.ascontiguousarray(mu_i, dtype=np.float64).reshape(-1)
    pref = np.ascontiguousarray(pref_lists, dtype=np.int32).reshape(-1)
    out = np.zeros((N, HQ_MLP_IN), dtype=np.float32)
    _check(load().hq_mlp_features(int(N), int(J), _dptr(lam), _dptr(mu),
                                  pref.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _fptr(out)))
    return out


def hq_mlp_get_params(m: MLP) -> np.ndarray:
    p = np.zeros(HQ_MLP_PARAMS, dtype=np.float32)
    _check(load().hq_mlp_get_params(m.handle, _fptr(p)))
    return p


def hq_mlp_set_params(m: MLP, params) -> None:
    p = np.ascontiguousarray(params, dtype=np.float32)
    assert p.size == HQ_MLP_PARAMS
    _check(load().hq_mlp_set_params(m.handle, _fptr(p)))


def hq_mlp_forward(m: MLP, X) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, HQ_MLP_IN)
    y = np.zeros(X.shape[0], dtype=np.float32)
    _check(load().hq_mlp_forward(m.handle, _fptr(X), X.shape[0], _fptr(y)))
    return y


def hq_mlp_gradient(m: MLP, X, t):
    X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, HQ_MLP_IN)
    t = np.ascontiguousarray(t, dtype=np.float32)
    g = np.zeros(HQ_MLP_PARAMS, dtype=np.float32)
    loss = ctypes.c_float()
    _check(load().hq_mlp_gradient(m.handle, _fptr(X), _fptr(t), X.shape[0], _fptr(g), ctypes.byref(loss)))
    return g, float(loss.value)


def hq_mlp_train(m: MLP, X, t, *, epochs: int, batch: int = 1024, lr: float = 1e-3, seed: int = 0):
    X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, HQ_MLP_IN)
    t = np.ascontiguousarray(t, dtype=np.float32)
    losses = np.zeros(max(epochs, 1), dtype=np.float32)
    _check(load().hq_mlp_train(m.handle, _fptr(X), _fptr(t), X.shape[0], int(epochs), int(batch), float(lr),
                               int(seed), _fptr(losses)))
    return losses[:epochs]
