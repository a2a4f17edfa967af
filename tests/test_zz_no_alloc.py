"""mps_topk_noalloc (the top-k selection with its workspace in a device array
the library owns) against mps_topk (caller workspace) on the same scores:
two calls in a row, the second on a smaller input with a smaller k, then an
empty input; results must be identical bit for bit.  Sizes beyond the
array's limit are refused before any work."""
import numpy as np
import pytest
import torch

import mpsgen
from gpu_common import gpu_model, instance, to_np

pytestmark = pytest.mark.gpu


def _both(score, flags, k):
    from paper_2511_18296_amd.binding import TopK, topk_noalloc
    t = TopK(score.shape[0], k)
    ri, rs, rc = t(score, flags)
    torch.cuda.synchronize()
    ref = (to_np(ri).copy(), to_np(rs).copy(), int(rc.item()))
    idx = torch.full((k,), -7, dtype=torch.int64, device="cuda")
    top = torch.full((k,), 7.0, dtype=torch.float32, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    topk_noalloc(score, flags, idx, top, cnt)
    torch.cuda.synchronize()
    got = (to_np(idx), to_np(top), int(cnt.item()))
    return ref, got


def _same(ref, got):
    np.testing.assert_array_equal(got[0], ref[0])
    np.testing.assert_array_equal(got[1], ref[1])
    assert got[2] == ref[2]


def test_noalloc_topk_matches_workspace_topk():
    from paper_2511_18296_amd.binding import MoveSet
    inst = instance("paper")
    m = gpu_model(inst)
    # first call: every move of the 32,000-block instance (512,000), k = 4,096
    sc, fl = m.eval_moves(MoveSet(True, True))
    ref, got = _both(sc, fl, 4096)
    assert ref[2] == 4096
    _same(ref, got)
    # second call: a smaller list (250,000 random moves), k = 1,000
    blk, per = mpsgen.random_moves(inst.N, inst.T, 250000, 1002)
    sc2, fl2 = m.eval_moves(MoveSet(False, True, torch.from_numpy(blk).cuda(),
                                    torch.from_numpy(per).cuda()))
    ref2, got2 = _both(sc2, fl2, 1000)
    assert ref2[2] == 1000
    _same(ref2, got2)
    # an empty input after them: count 0, every entry -1 / -inf
    e_sc = torch.empty(0, dtype=torch.float32, device="cuda")
    e_fl = torch.empty(0, dtype=torch.uint8, device="cuda")
    ref3, got3 = _both(e_sc, e_fl, 16)
    assert got3[2] == 0 and np.all(got3[0] == -1) and np.all(np.isneginf(got3[1]))
    _same(ref3, got3)


def test_noalloc_topk_refuses_sizes_beyond_its_array():
    from paper_2511_18296_amd.binding import lib, _ptr
    sc = torch.zeros(16, dtype=torch.float32, device="cuda")
    fl = torch.zeros(16, dtype=torch.uint8, device="cuda")
    idx = torch.zeros(16, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = lib.mps_topk_noalloc(_ptr(sc), _ptr(fl), (1 << 21) + 1, 16, 1, 0, _ptr(idx), None,
                              _ptr(cnt), None)
    assert st == 1 and b"exceeds" in lib.mps_last_error()
    st = lib.mps_topk_noalloc(_ptr(sc), _ptr(fl), 16, 8193, 1, 0, _ptr(idx), None,
                              _ptr(cnt), None)
    assert st == 1
