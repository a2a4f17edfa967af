"""The C ABI library loads, exports every declared symbol and rejects bad
arguments on the host (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "mps.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mps_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    from paper_2511_18296_amd import binding
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(binding.lib, n), n
    assert sorted(binding.EXPORTS) == names


def test_version_and_error_text():
    from paper_2511_18296_amd import binding
    assert binding.lib.mps_version() == 100
    n = C.c_int32(-1)
    st = binding.lib.mps_device_count(C.byref(n))
    if st == 0:
        pytest.skip("a GPU is visible")
    assert st == 3 and n.value == 0
    assert b"GPU" in binding.lib.mps_last_error()


def _params(**kw):
    from paper_2511_18296_amd import binding
    d = dict(nx=4, ny=4, nz=2, n_scen=8, n_periods=3, precedence=0, discount_rate=0.08,
             lam=0.5, pen_proc=100.0, pen_mine=100.0, proc_cap=1e6, mine_cap=1e6)
    d.update(kw)
    return binding.Params(**d)


@pytest.mark.parametrize("bad", [dict(nx=0), dict(n_scen=0), dict(n_scen=5000),
                                 dict(n_periods=0), dict(n_periods=127), dict(precedence=2),
                                 dict(discount_rate=-1.0), dict(lam=float("nan")),
                                 dict(pen_proc=-1.0), dict(mine_cap=float("inf"))])
def test_build_rejects_bad_params_before_any_device_work(bad):
    from paper_2511_18296_amd import binding
    h = C.c_void_p()
    prm = _params(**bad)
    st = binding.lib.mps_build_model(C.byref(prm), C.c_void_p(1), C.c_void_p(2),
                                     C.c_void_p(3), None, None, None, C.byref(h))
    assert st == 1, binding.lib.mps_last_error()
    assert h.value is None
    assert binding.lib.mps_last_error()


def test_null_arguments_rejected():
    from paper_2511_18296_amd import binding
    L = binding.lib
    h = C.c_void_p()
    prm = _params()
    assert L.mps_build_model(C.byref(prm), None, None, None, None, None, None, C.byref(h)) == 1
    assert L.mps_build_model(C.byref(prm), None, None, None, None, None, None, None) == 1
    assert L.mps_destroy_model(None) == 1
    assert L.mps_set_schedule(None, None, None) == 1
    assert L.mps_eval_moves(None, None, None, None, None, None, None, None) == 1
    assert L.mps_repair(None, None, None, None, 0, 0, None, None) == 1


def _lists(N, edges):
    """CSR predecessor lists from (block, predecessor) pairs."""
    import numpy as np
    ptr = np.zeros(N + 1, dtype=np.int32)
    idx = []
    for b in range(N):
        lst = [a for (c, a) in edges if c == b]
        idx += lst
        ptr[b + 1] = len(idx)
    return ptr, np.asarray(idx if idx else [0], dtype=np.int32)


@pytest.mark.parametrize("case", ["self", "range", "repeat", "indegree", "outdegree",
                                  "no_lists", "lists_without_csr"])
def test_build_rejects_bad_predecessor_lists(case):
    """Explicit predecessor lists (Eq. 15's sets) are validated on the host
    before any device work."""
    from paper_2511_18296_amd import binding
    N = 32
    csr = 1
    if case == "self":
        ptr, idx = _lists(N, [(5, 5)])
    elif case == "range":
        ptr, idx = _lists(N, [(5, 32)])
    elif case == "repeat":
        ptr, idx = _lists(N, [(5, 1), (5, 1)])
    elif case == "indegree":
        ptr, idx = _lists(N, [(20, a) for a in range(10)])
    elif case == "outdegree":
        ptr, idx = _lists(N, [(c, 0) for c in range(1, 11)])
    elif case == "no_lists":
        ptr = idx = None
    else:
        ptr, idx = _lists(N, [(5, 1)])
        csr = 0
    prm = _params(precedence=csr)
    h = C.c_void_p()
    lp = [None if a is None else a.ctypes.data_as(C.c_void_p) for a in (ptr, idx)]
    st = binding.lib.mps_build_model(C.byref(prm), C.c_void_p(1), C.c_void_p(2),
                                     C.c_void_p(3), lp[0], lp[1], None, C.byref(h))
    assert st == 1, binding.lib.mps_last_error()
    assert h.value is None


def test_valid_predecessor_lists_pass_the_host_checks():
    from paper_2511_18296_amd import binding
    N = 32
    ptr, idx = _lists(N, [(c, c - 16) for c in range(16, 32)] + [(17, 0), (17, 2)])
    prm = _params(precedence=1)
    h = C.c_void_p()
    st = binding.lib.mps_build_model(C.byref(prm), C.c_void_p(1), C.c_void_p(2),
                                     C.c_void_p(3), ptr.ctypes.data_as(C.c_void_p),
                                     idx.ctypes.data_as(C.c_void_p), None, C.byref(h))
    # past the list checks the call needs a GPU (MPS_E_DEVICE here) or
    # device pointers (MPS_E_INVALID_ARG for these fake ones)
    assert st in (1, 3) and b"predecessor" not in binding.lib.mps_last_error()


@pytest.mark.parametrize("n,k,ws", [(10, 0, 1 << 20), (10, 8193, 1 << 20), (-1, 4, 1 << 20),
                                    (1 << 31, 4, 1 << 20), (1000, 10, 16)])
def test_topk_argument_checks(n, k, ws):
    from paper_2511_18296_amd import binding
    L = binding.lib
    st = L.mps_topk(C.c_void_p(8), C.c_void_p(8), n, k, 1, 24, C.c_void_p(8), None,
                    C.c_void_p(8), C.c_void_p(8), ws, None)
    assert st == 1


def test_topk_ws_bytes_grows_with_n_and_k():
    from paper_2511_18296_amd import binding
    f = binding.lib.mps_topk_ws_bytes
    assert f(1000, 10) < f(100000, 10) and f(1000, 10) < f(1000, 4000)


def test_batch_argument_checks():
    """Batch entry points reject NULL handles and out-of-range k / counts on
    the host."""
    from paper_2511_18296_amd import binding
    L = binding.lib
    out = C.c_void_p()
    items = (binding.BatchItem * 1)()
    models = (C.c_void_p * 1)(None)
    assert L.mps_batch_create(None, items, 1, 4, 1, 24, C.byref(out)) == 1
    assert L.mps_batch_create(models, items, 1, 4, 1, 24, None) == 1
    assert L.mps_batch_create(models, items, 0, 4, 1, 24, C.byref(out)) == 1
    assert L.mps_batch_create(models, items, 1, 0, 1, 24, C.byref(out)) == 1
    assert L.mps_batch_create(models, items, 1, 1025, 1, 24, C.byref(out)) == 1
    assert L.mps_batch_create(models, items, 1, 4, 1, 24, C.byref(out)) == 1   # NULL model
    assert out.value is None
    t = binding.Tuning(1, 512, 8, 0)
    assert L.mps_batch_destroy(None) == 1
    assert L.mps_batch_set_tuning(None, -1, C.byref(t)) == 1
    assert L.mps_batch_get_tuning(None, 0, C.byref(t)) == 1
    assert L.mps_batch_set_workgroups(None, 0) == 1
    assert L.mps_batch_run(None, None) == 1
    assert L.mps_batch_graph_launch(None, None) == 1
    assert L.mps_batch_autotune(None, 3, None, None) == 1
