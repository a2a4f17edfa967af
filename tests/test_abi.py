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
    d = dict(nx=4, ny=4, nz=2, n_scen=8, n_periods=3, reserved=0, discount_rate=0.08,
             lam=0.5, pen_proc=100.0, pen_mine=100.0, proc_cap=1e6, mine_cap=1e6)
    d.update(kw)
    return binding.Params(**d)


@pytest.mark.parametrize("bad", [dict(nx=0), dict(n_scen=0), dict(n_scen=5000),
                                 dict(n_periods=0), dict(n_periods=127), dict(reserved=1),
                                 dict(discount_rate=-1.0), dict(lam=float("nan")),
                                 dict(pen_proc=-1.0), dict(mine_cap=float("inf"))])
def test_build_rejects_bad_params_before_any_device_work(bad):
    from paper_2511_18296_amd import binding
    h = C.c_void_p()
    prm = _params(**bad)
    st = binding.lib.mps_build_model(C.byref(prm), C.c_void_p(1), C.c_void_p(2),
                                     C.c_void_p(3), None, C.byref(h))
    assert st == 1, binding.lib.mps_last_error()
    assert h.value is None
    assert binding.lib.mps_last_error()


def test_null_arguments_rejected():
    from paper_2511_18296_amd import binding
    L = binding.lib
    h = C.c_void_p()
    prm = _params()
    assert L.mps_build_model(C.byref(prm), None, None, None, None, C.byref(h)) == 1
    assert L.mps_build_model(C.byref(prm), None, None, None, None, None) == 1
    assert L.mps_destroy_model(None) == 1
    assert L.mps_set_schedule(None, None, None) == 1
    assert L.mps_eval_moves(None, None, None, None, None, None, None, None) == 1
    assert L.mps_repair(None, None, None, None, 0, 0, None, None) == 1


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
