"""Cascading repair (Alg. 4 with its fallback) on the GPU against the
oracle: candidates are the best moves by score WITHOUT the precedence
requirement, so many of them need companion blocks; both sides walk the same
ordered list and must reach the same schedule with the same number of applied
(composite) moves, in soft and hard capacity mode and with small set limits."""
import numpy as np
import pytest

import oracle
from gpu_common import compare_scores, gpu_model, instance, to_np

pytestmark = pytest.mark.gpu

CASES = [("tiny", 300, False, 64), ("ragged", 200, False, 64), ("tight", 800, True, 64),
         ("tight", 800, False, 3), ("wide", 600, False, 64), ("one_period", 300, False, 64),
         ("max_periods", 1500, True, 32), ("paper", 2048, False, 64),
         ("largest", 4096, False, 256)]


@pytest.mark.parametrize("name,k,hard,max_set", CASES)
def test_cascade_matches_oracle(name, k, hard, max_set):
    from paper_2511_18296_amd.binding import MoveSet, NOOP, BAD, TopK
    inst = instance(name)
    m = gpu_model(inst)
    sc, fl = m.eval_moves()
    t = TopK(sc.numel(), k)
    idx, _, cnt = t(sc, fl, require=0, forbid=NOOP | BAD)
    cand = to_np(idx)[:int(cnt.item())]
    D = inst.T + 1
    applied = m.repair_cascade(MoveSet(), idx, cnt, hard=hard, max_set=max_set)
    p_gpu = to_np(m.get_schedule())
    o = oracle.Oracle(inst)
    q, a, J, acc, size = o.repair_cascade(inst.p0, cand // D, (cand % D).astype(np.int8),
                                          hard=hard, max_set=max_set)
    n_comp = int(np.count_nonzero(acc.astype(bool) & (size > 1)))
    print(f"{name}: applied {int(applied.item())} (oracle {a}, {n_comp} with companions) "
          f"of {len(cand)}; {int(np.count_nonzero(p_gpu != q))} blocks differ")
    assert int(applied.item()) == a
    np.testing.assert_array_equal(p_gpu, q)
    g = m.objective()
    ref = o.objective(q)
    assert g["J"] == pytest.approx(ref["J"], rel=1e-11)
    assert g["n_prec_viol"] == 0
    # the state after the walk evaluates like a fresh one
    sc2, fl2 = m.eval_moves()
    osc2, ofl2 = o.eval_moves(q, include_never=True)
    np.testing.assert_array_equal(to_np(fl2), ofl2)
    compare_scores(to_np(sc2), osc2, ofl2, ref["mu"], "after cascade")


def test_cascade_rejects_bad_arguments():
    import torch
    from paper_2511_18296_amd.binding import MoveSet, MpsError
    inst = instance("tiny")
    m = gpu_model(inst)
    idx = torch.zeros(4, dtype=torch.int64, device="cuda")
    cnt = torch.ones(1, dtype=torch.int32, device="cuda")
    for bad in (0, 257):
        with pytest.raises(MpsError):
            m.repair_cascade(MoveSet(), idx, cnt, max_set=bad)
