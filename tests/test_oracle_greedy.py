"""Pins of the oracle's greedy initializer (Alg. 3 with the uncertainty
factors equal to 1), on the CPU:
- invariants: the result is precedence-feasible and meets both capacities
  hard, and no unplaced block has a period whose move the evaluator flags
  PREC_OK, MINE_OK and PROC_OK (the passes stop at a fixpoint);
- closed forms: on one bench (no precedence) with only a mining capacity of c
  blocks per period, the block of rank r (expected value descending, index
  ascending, computed here with numpy's stable sort) goes to period r // c,
  and blocks of rank >= c*T stay unplaced; with unbounded capacities a
  single column of blocks is mined entirely in period 0, in as many passes as
  the value order breaks the depth order, plus one."""
import numpy as np
import pytest

import mpsgen
import oracle


def _check_invariants(inst, p):
    o = oracle.Oracle(inst)
    T = inst.T
    obj = o.objective(p, state=True)
    assert obj["n_prec_viol"] == 0
    assert np.all(obj["M"] <= inst.mcap)
    assert np.all(obj["O"] <= inst.pcap)
    un = np.flatnonzero(p == T)
    if len(un):
        blk = np.repeat(un, T).astype(np.int32)
        per = np.tile(np.arange(T), len(un)).astype(np.int8)
        _, fl = o.eval_moves(p, block=blk, period=per)
        need = oracle.PREC_OK | oracle.MINE_OK | oracle.PROC_OK
        assert not np.any((fl & need) == need), "an unplaced block could be placed"
    return obj


@pytest.mark.parametrize("shape", [(10, 10, 5, 10, 5, 3.0, 1), (7, 5, 3, 37, 3, 1.5, 77),
                                   (12, 10, 6, 96, 8, 2.0, 80), (9, 7, 4, 50, 1, 2.0, 86)])
def test_greedy_result_is_feasible_and_a_fixpoint(shape):
    inst = mpsgen.make_instance(*shape)
    p, passes, placed = oracle.Oracle(inst).greedy_init()
    assert placed == int(np.count_nonzero(p < inst.T))
    assert passes >= 1
    _check_invariants(inst, p)


def test_greedy_tight_capacities():
    inst = mpsgen.make_instance(12, 10, 6, 96, 8, 2.0, 80)
    inst.pcap *= 0.85
    inst.mcap *= 0.8
    p, passes, placed = oracle.Oracle(inst).greedy_init()
    assert 0 < placed < inst.N
    _check_invariants(inst, p)


def test_greedy_one_bench_mining_capacity_only():
    inst = mpsgen.make_instance(9, 8, 1, 12, 6, 2.0, 611)
    c = 10
    inst.mcap = c * 15600.0
    inst.pcap = 1e300
    # equal expected values for a third of the blocks: the index decides
    inst.v[:, ::3] = np.float32(-46800.0)
    p, passes, placed = oracle.Oracle(inst).greedy_init()
    vd = inst.v.astype(np.float64).mean(axis=0)
    rank = np.empty(inst.N, dtype=np.int64)
    rank[np.argsort(-vd, kind="stable")] = np.arange(inst.N)
    want = np.where(rank < c * inst.T, rank // c, inst.T)
    np.testing.assert_array_equal(p, want.astype(np.int8))
    assert placed == min(inst.N, c * inst.T)
    assert passes == 2   # one pass places everything it can, the next nothing


def test_greedy_single_column_unbounded():
    nz = 7
    inst = mpsgen.make_instance(1, 1, nz, 5, 4, 1.0, 612)
    inst.mcap = 1e300
    inst.pcap = 1e300
    p, passes, placed = oracle.Oracle(inst).greedy_init()
    assert np.all(p == 0) and placed == nz
    vd = inst.v.astype(np.float64).mean(axis=0)
    rank = np.empty(nz, dtype=np.int64)
    rank[np.argsort(-vd, kind="stable")] = np.arange(nz)
    # block z is placed in the pass after its predecessor's when it ranks
    # before it, in the same pass otherwise
    pas = [1]
    for z in range(1, nz):
        pas.append(pas[-1] + (1 if rank[z] < rank[z - 1] else 0))
    assert passes == max(pas) + 1


def test_greedy_csr_lists_match_stencil():
    inst = mpsgen.make_instance(7, 6, 4, 23, 5, 1.5, 613)
    ptr, idx = mpsgen.stencil_precedence(inst.nx, inst.ny, inst.nz)
    a = oracle.Oracle(inst).greedy_init()
    b = oracle.Oracle(mpsgen.with_precedence(inst, ptr, idx)).greedy_init()
    np.testing.assert_array_equal(a[0], b[0])
    assert a[1:] == b[1:]
