"""Pins of the oracle's cascading repair (Alg. 4 with its fallback: a
candidate that precedence forbids moves together with the blocks that
forbid it), on the CPU:
- special cases that reduce to the pinned plain repair: with sets limited to
  one block, or with candidates that need no companions, the decisions and
  the schedule equal or_repair's;
- brute force: every applied composite move raises J by exactly what
  re-scoring the whole schedule before and after it gives, and every result
  is precedence-feasible;
- a hand-worked column: moving the bottom of a four-block column to period 0
  takes the two blocks above it that are mined later, and no other;
- hard capacities hold for the period every applied set enters."""
import numpy as np
import pytest

import mpsgen
import oracle


def _candidates(inst, p, k, prec=False):
    o = oracle.Oracle(inst)
    sc, fl = o.eval_moves(p, include_never=True)
    req = oracle.PREC_OK if prec else 0
    idx, _ = oracle.topk(sc, fl, k, req=req, forbid=oracle.NOOP | oracle.BAD)
    D = inst.T + 1
    return (idx // D).astype(np.int32), (idx % D).astype(np.int8)


@pytest.mark.parametrize("hard", [False, True])
def test_single_block_sets_equal_plain_repair(hard):
    inst = mpsgen.make_instance(12, 10, 6, 40, 8, 2.0, 701)
    cb, ct = _candidates(inst, inst.p0, 600)
    o = oracle.Oracle(inst)
    q1, a1, J1, acc1 = o.repair(inst.p0, cb, ct, hard=hard)
    q2, a2, J2, acc2, size = o.repair_cascade(inst.p0, cb, ct, hard=hard, max_set=1)
    np.testing.assert_array_equal(q1, q2)
    np.testing.assert_array_equal(acc1, acc2)
    assert a1 == a2 and J1 == pytest.approx(J2, rel=1e-12)


def test_feasible_candidates_equal_plain_repair():
    inst = mpsgen.make_instance(10, 9, 5, 30, 6, 2.0, 702)
    cb, ct = _candidates(inst, inst.p0, 400, prec=True)
    o = oracle.Oracle(inst)
    q1, a1, J1, acc1 = o.repair(inst.p0, cb, ct)
    q2, a2, J2, acc2, size = o.repair_cascade(inst.p0, cb, ct, max_set=64)
    # the first candidate needs no companions; later ones may, once earlier
    # moves changed the schedule, so compare up to the first companion set
    first = np.flatnonzero(size > 1)
    stop = first[0] if len(first) else len(cb)
    np.testing.assert_array_equal(acc1[:stop], acc2[:stop])
    if stop == len(cb):
        np.testing.assert_array_equal(q1, q2)
        assert J1 == pytest.approx(J2, rel=1e-12)


@pytest.mark.parametrize("seed", [703, 704])
def test_each_applied_set_raises_j_by_its_rescored_change(seed):
    inst = mpsgen.make_instance(8, 7, 5, 25, 6, 2.0, seed)
    o = oracle.Oracle(inst)
    cb, ct = _candidates(inst, inst.p0, 300)
    p = inst.p0.copy()
    J = o.objective(p)["J"]
    n_sets = 0
    for b, t in zip(cb, ct):
        q, a, J2, acc, size = o.repair_cascade(p, [b], [t], max_set=64)
        if a:
            assert J2 > J, (b, t, J2, J)
            moved = np.flatnonzero(q != p)
            assert len(moved) == size[0] and np.all(q[moved] == t) and b in moved
            assert o.objective(q)["n_prec_viol"] == 0
            n_sets += size[0] > 1
        else:
            np.testing.assert_array_equal(q, p)
        p, J = q, o.objective(q)["J"]
    assert n_sets > 0, "no composite move was applied"


def test_column_hand_case():
    inst = mpsgen.make_instance(1, 1, 4, 3, 4, 1.0, 705)
    inst.lam = 0.0
    inst.pcap = inst.mcap = 1e300
    inst.v[:] = np.float32(1000.0)          # every block worth the same, positive
    inst.ore[:] = 1
    p = np.array([0, 1, 2, 3], dtype=np.int8)
    o = oracle.Oracle(inst)
    q, a, J, acc, size = o.repair_cascade(p, [3], [1], max_set=64)
    # moving block 3 to period 1 takes block 2 (period 2) but not block 1
    # (period 1) nor block 0 (period 0)
    assert a == 1 and size[0] == 2
    np.testing.assert_array_equal(q, [0, 1, 1, 1])
    d = o.discount()
    assert J - o.objective(p)["J"] == pytest.approx(1000.0 * (2 * d[1] - d[2] - d[3]),
                                                    rel=1e-12)
    # moving block 0 later (to never) takes every block below it
    q, a, J, acc, size = o.repair_cascade(p, [0], [4], max_set=64)
    assert size[0] == 4 and a == 0          # losing value: rejected
    np.testing.assert_array_equal(q, p)
    # a set larger than allowed is skipped
    q, a, J, acc, size = o.repair_cascade(p, [3], [0], max_set=2)
    assert size[0] == -1 and a == 0


def test_hard_capacity_holds_where_sets_enter():
    inst = mpsgen.make_instance(10, 10, 5, 30, 6, 2.0, 706)
    inst.pcap *= 0.9
    inst.mcap *= 0.85
    o = oracle.Oracle(inst)
    cb, ct = _candidates(inst, inst.p0, 500)
    q, a, J, acc, size = o.repair_cascade(inst.p0, cb, ct, hard=True, max_set=64)
    obj0 = o.objective(inst.p0, state=True)
    obj = o.objective(q, state=True)
    entered = {int(t) for t, ok in zip(ct, acc) if ok and t < inst.T}
    for t in entered:
        assert obj["M"][t] <= max(inst.mcap, obj0["M"][t])
    assert obj["n_prec_viol"] == 0 and a > 0
