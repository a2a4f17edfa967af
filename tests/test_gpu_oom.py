"""Allocation failure during a model build: with the test allocation cap
(MPS_TEST_ALLOC_LIMIT, bytes) below what a model needs, mps_build_model
returns MPS_E_OUT_OF_MEMORY, hands out no handle and leaves no device memory
behind, whichever of its allocations is the one refused; a build without the
cap then succeeds."""
import ctypes as C

import numpy as np
import pytest
import torch

import mpsgen

pytestmark = pytest.mark.gpu


def _args(inst):
    from paper_2511_18296_amd.binding import Params
    v = torch.from_numpy(np.ascontiguousarray(inst.v)).cuda()
    words = mpsgen.ore_pack(inst.ore).view(np.int32)
    ore = torch.from_numpy(np.ascontiguousarray(words)).cuda()
    ton = torch.from_numpy(np.ascontiguousarray(inst.ton)).cuda()
    prm = Params(inst.nx, inst.ny, inst.nz, inst.S, inst.T, 0, inst.rate, inst.lam,
                 inst.pen_proc, inst.pen_mine, inst.pcap, inst.mcap)
    return prm, v, ore, ton


@pytest.mark.parametrize("limit", [1, 4096, 200_000, 2_000_000, 6_000_000])
def test_build_out_of_memory_leaves_nothing(limit, monkeypatch):
    from paper_2511_18296_amd.binding import lib, _ptr
    inst = mpsgen.make_instance(30, 30, 8, 64, 12, 3.0, 1500)
    prm, v, ore, ton = _args(inst)
    # one full build first: the library's code objects (and their static
    # device arrays) are loaded at first use, which is not what is measured
    h = C.c_void_p()
    assert lib.mps_build_model(C.byref(prm), _ptr(v), _ptr(ore), _ptr(ton), None, None, None,
                               C.byref(h)) == 0
    assert lib.mps_destroy_model(h) == 0
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    monkeypatch.setenv("MPS_TEST_ALLOC_LIMIT", str(limit))
    for _ in range(3):
        h = C.c_void_p()
        st = lib.mps_build_model(C.byref(prm), _ptr(v), _ptr(ore), _ptr(ton), None, None, None,
                                 C.byref(h))
        assert st == 2, lib.mps_last_error()
        assert h.value is None and b"limit" in lib.mps_last_error()
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    monkeypatch.delenv("MPS_TEST_ALLOC_LIMIT")
    h = C.c_void_p()
    assert lib.mps_build_model(C.byref(prm), _ptr(v), _ptr(ore), _ptr(ton), None, None, None,
                               C.byref(h)) == 0
    assert lib.mps_destroy_model(h) == 0
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
