"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol that include/hq.h declares, and rejects bad input before any
device work (status codes + hq_last_error)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2603_03019_amd import hq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "hq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hq_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = hq.load()
    names = _declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert sorted(hq.EXPORTED) == names


def test_batch_shape_report_before_any_batch():
    # no batched solve has run in this process (no device here)
    assert hq.hq_batch_last_block() == 0


def test_default_options():
    o = hq.hq_default_options()
    assert o.precision == hq.HQ_FP64 and o.inner == hq.HQ_INNER_ONE and o.init == hq.HQ_INIT_UNIFORM
    assert o.buffer == 0
    assert o.max_iters == 100000 and o.device == -1 and not o.stream


def _ok_args(N=4, J=3):
    lam = np.array([0.5, 0.2, 0.3])[:J]
    mu = np.ones(N)
    pref = np.array([np.roll(np.arange(N), j) for j in range(J)], dtype=np.int32)
    return N, J, lam, mu, pref


@pytest.mark.parametrize("case", ["N0", "Nbig", "J0", "neg_lambda", "nan_lambda", "zero_mu", "inf_mu",
                                  "not_perm", "out_of_range", "bad_precision", "bad_inner", "product_no_rho",
                                  "state_no_state", "bad_rho", "bad_tile", "bad_buffer", "big_buffer",
                                  "unstable_room", "literal_no_delta"])
def test_invalid_arguments_rejected_on_host(case):
    N, J, lam, mu, pref = _ok_args()
    kw = {}
    if case == "N0":
        N = 0
        mu = np.ones(0)
        pref = np.zeros((J, 0), np.int32)
    elif case == "Nbig":
        N = hq.HQ_MAX_N + 1
        mu = np.ones(N)
        pref = np.array([np.arange(N)] * J, dtype=np.int32)
    elif case == "J0":
        J = 0
        lam = np.zeros(0)
        pref = np.zeros((0, N), np.int32)
    elif case == "neg_lambda":
        lam = lam.copy()
        lam[1] = -0.1
    elif case == "nan_lambda":
        lam = lam.copy()
        lam[0] = np.nan
    elif case == "zero_mu":
        mu = mu.copy()
        mu[2] = 0.0
    elif case == "inf_mu":
        mu = mu.copy()
        mu[0] = np.inf
    elif case == "not_perm":
        pref = pref.copy()
        pref[1, 2] = pref[1, 3]
    elif case == "out_of_range":
        pref = pref.copy()
        pref[0, 0] = N
    elif case == "bad_precision":
        kw["precision"] = 7
    elif case == "bad_inner":
        kw["inner"] = 5
    elif case == "product_no_rho":
        kw["init"] = hq.HQ_INIT_PRODUCT
    elif case == "state_no_state":
        kw["init"] = hq.HQ_INIT_STATE
    elif case == "bad_rho":
        kw["init_rho"] = np.array([0.5, 1.5, 0.2, 0.1])
    elif case == "bad_tile":
        kw["tile_bits"] = 13
    elif case == "bad_buffer":
        kw["buffer"] = -2
    elif case == "big_buffer":
        kw["buffer"] = hq.HQ_BUFFER_MAX + 1
    elif case == "literal_no_delta":
        kw["inner"] = hq.HQ_INNER_LITERAL
    elif case == "unstable_room":
        kw["buffer"] = hq.HQ_BUFFER_UNLIMITED
        lam = lam * (4.0 / lam.sum())  # Lambda = sum of the service rates
    with pytest.raises(hq.HQError) as e:
        hq.hq_create(N, J, lam, mu, pref, **kw)
    assert e.value.status == hq.HQ_ERR_INVALID_ARG
    assert len(hq.hq_last_error()) > 0


def test_null_arguments():
    L = hq.load()
    assert L.hq_solve(None, 1e-8, None) == hq.HQ_ERR_INVALID_ARG
    assert L.hq_marginals(None, None, None) == hq.HQ_ERR_INVALID_ARG
    assert L.hq_queue(None, None, None, 0) == hq.HQ_ERR_INVALID_ARG
    assert L.hq_state(None, None) == hq.HQ_ERR_INVALID_ARG
    assert L.hq_iterate(None, 1) == hq.HQ_ERR_INVALID_ARG
    assert L.hq_num_units(None) == 0
    L.hq_destroy(None)  # NULL-safe
    # hq_create with a NULL out pointer
    N, J, lam, mu, pref = _ok_args()
    st = L.hq_create(N, J, lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     pref.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), None, None)
    assert st == hq.HQ_ERR_INVALID_ARG
    assert L.hq_solve_batch(None, 2, 1e-8, None) == hq.HQ_ERR_INVALID_ARG


def test_binding_fails_loudly_without_library(tmp_path):
    import importlib

    mod = importlib.import_module("paper_2603_03019_amd.hq")
    saved = mod._lib
    try:
        mod._lib = None
        with pytest.raises(RuntimeError, match="libhq.so not found"):
            mod.load(str(tmp_path / "missing.so"))
    finally:
        mod._lib = saved
