"""GPU top-k and repair against the oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import mpsgen
import oracle
from gpu_common import compare_scores, gpu_model, instance, to_np

pytestmark = pytest.mark.gpu


def _flags_default():
    return oracle.PREC_OK, oracle.NOOP | oracle.BAD


@pytest.mark.parametrize("n,k,seed", [(0, 5, 0), (1, 1, 1), (1000, 1, 2), (5000, 300, 3),
                                      (70001, 4096, 4), (300000, 1024, 5),
                                      (1134000, 4096, 6), (20000, 8192, 7)])
def test_topk_exact_on_identical_scores(n, k, seed):
    """Same float32 scores on both sides: indices and scores bit-identical,
    including many exact ties (broken by the smaller index)."""
    from paper_2511_18296_amd.binding import TopK
    rng = np.random.default_rng(seed)
    score = np.round(rng.normal(size=n) * 50).astype(np.float32)  # heavy ties
    score[rng.random(n) < 0.01] = np.float32(0.0)
    flags = rng.integers(0, 32, size=n).astype(np.uint8)
    if n > 10:
        score[3] = np.nan
        flags[3] = oracle.PREC_OK
    t = TopK(max(n, 1), k)
    idx, sc, cnt = t(torch.from_numpy(score).cuda(), torch.from_numpy(flags).cuda(),
                     *_flags_default())
    c = int(cnt.item())
    ref_flags = np.where(np.isnan(score), 0, flags).astype(np.uint8)   # NaN never qualifies
    ref_i, ref_s = oracle.topk(score, ref_flags, k)
    assert c == len(ref_i)
    np.testing.assert_array_equal(to_np(idx)[:c], ref_i)
    np.testing.assert_array_equal(to_np(sc)[:c], ref_s.astype(np.float32))
    assert np.all(to_np(idx)[c:] == -1)


def test_topk_all_equal_scores():
    from paper_2511_18296_amd.binding import TopK
    n, k = 100000, 777
    score = np.full(n, 3.5, np.float32)
    flags = np.full(n, oracle.PREC_OK, np.uint8)
    t = TopK(n, k)
    idx, sc, cnt = t(torch.from_numpy(score).cuda(), torch.from_numpy(flags).cuda())
    assert int(cnt.item()) == k
    np.testing.assert_array_equal(to_np(idx), np.arange(k))


def test_topk_on_largest_moves_against_oracle_scores():
    """GPU top-4096 of GPU scores vs oracle top-4096 of FP64 scores: equal up
    to near-ties (items whose oracle scores differ by no more than the
    measured score error)."""
    from paper_2511_18296_amd.binding import TopK
    inst = instance("largest")
    m = gpu_model(inst)
    sc, fl = m.eval_moves()
    k = 4096
    t = TopK(sc.numel(), k)
    idx, tsc, cnt = t(sc, fl)
    o = oracle.Oracle(inst)
    osc, ofl = o.eval_moves(inst.p0, include_never=True)
    eps = compare_scores(to_np(sc), osc, ofl, o.objective(inst.p0)["mu"], "largest")
    ref_i, ref_s = oracle.topk(osc, ofl, k)
    c = int(cnt.item())
    assert c == len(ref_i) == k
    gi = to_np(idx)[:c]
    if not np.array_equal(gi, ref_i):
        # every disagreement must be a near-tie at the boundary or a swap
        kth = ref_s[-1]
        mism = set(gi) ^ set(ref_i)
        for i in mism:
            assert abs(osc[i] - kth) <= 2 * eps, (i, osc[i], kth)
        pos = {int(i): j for j, i in enumerate(gi)}
        for j, i in enumerate(ref_i):
            if int(i) in pos and pos[int(i)] != j:
                assert abs(osc[i] - osc[gi[j]]) <= 2 * eps
    print(f"top-4096 agreement: {len(set(gi) & set(ref_i))}/{k}, eps {eps:.3g}")


@pytest.mark.parametrize("name,k,hard", [("tiny", 400, False), ("tiny", 400, True),
                                         ("tight", 1000, False), ("ragged", 200, True),
                                         ("single", 150, False), ("flat", 300, False),
                                         ("wide", 600, False), ("wider", 500, True),
                                         ("one_period", 300, False),
                                         ("max_periods", 2000, True),
                                         ("largest", 4096, False)])
def test_repair_matches_oracle(name, k, hard):
    """Same ordered candidate list on both sides -> same accept decisions,
    same final schedule, same objective."""
    from paper_2511_18296_amd.binding import MoveSet, TopK
    inst = instance(name)
    m = gpu_model(inst)
    sc, fl = m.eval_moves()
    t = TopK(sc.numel(), k)
    idx, _, cnt = t(sc, fl)
    cand = to_np(idx)[:int(cnt.item())]
    D = inst.T + 1
    applied = m.repair(MoveSet(), idx, cnt, hard=hard)
    p_gpu = to_np(m.get_schedule())
    o = oracle.Oracle(inst)
    q, a, J, acc = o.repair(inst.p0, cand // D, (cand % D).astype(np.int8), hard=hard)
    assert int(applied.item()) == a
    np.testing.assert_array_equal(p_gpu, q)
    g = m.objective()
    ref = o.objective(q)
    assert g["J"] == pytest.approx(ref["J"], rel=1e-11)
    assert g["n_prec_viol"] == 0
    # the state after repair evaluates like a fresh one
    sc2, fl2 = m.eval_moves()
    osc2, ofl2 = o.eval_moves(q, include_never=True)
    np.testing.assert_array_equal(to_np(fl2), ofl2)
    compare_scores(to_np(sc2), osc2, ofl2, ref["mu"], "after repair")
    print(f"{name}: applied {a} of {len(cand)}")


def test_repair_list_moves_and_count_bound():
    from paper_2511_18296_amd.binding import MoveSet, TopK
    inst = instance("tiny")
    m = gpu_model(inst)
    o = oracle.Oracle(inst)
    rng = np.random.default_rng(9)
    blk = rng.integers(0, inst.N, size=3000).astype(np.int32)
    per = rng.integers(0, inst.T + 1, size=3000).astype(np.int8)
    mv = MoveSet(False, True, torch.from_numpy(blk).cuda(), torch.from_numpy(per).cuda())
    sc, fl = m.eval_moves(mv)
    t = TopK(3000, 500)
    idx, _, cnt = t(sc, fl)
    c = int(cnt.item())
    cand = to_np(idx)[:c]
    # only the first 100 candidates may be used
    applied = m.repair(mv, idx, cnt, max_cand=100)
    q, a, J, _ = o.repair(inst.p0, blk[cand[:100]], per[cand[:100]])
    assert int(applied.item()) == a
    np.testing.assert_array_equal(to_np(m.get_schedule()), q)


def test_state_save_restore_roundtrip():
    """A saved search state restores the schedule, objective and every move
    score bit for bit, after a repair has changed them."""
    from paper_2511_18296_amd.binding import MoveSet, TopK
    inst = instance("tight")
    m = gpu_model(inst)
    snap = m.save_state()
    sc0, fl0 = [t.clone() for t in m.eval_moves()]
    obj0 = m.objective()
    t = TopK(sc0.numel(), 500)
    idx, _, cnt = t(sc0, fl0)
    assert int(m.repair(MoveSet(), idx, cnt).item()) > 0
    assert m.objective()["J"] != obj0["J"]
    m.restore_state(snap)
    assert m.objective() == obj0
    sc1, fl1 = m.eval_moves()
    assert torch.equal(sc0, sc1) and torch.equal(fl0, fl1)
    np.testing.assert_array_equal(to_np(m.get_schedule()), inst.p0)


def test_repair_invalid_duplicate_and_repeated_calls():
    """Invalid entries (out-of-range ids, BAD moves) are skipped, repeated
    (block, period) pairs and repeated blocks follow the walk's rules, and a
    second call on the changed state (the per-block marks of the first call
    cleared) again equals the oracle walk."""
    from paper_2511_18296_amd.binding import MoveSet
    inst = instance("tight")
    m = gpu_model(inst)
    o = oracle.Oracle(inst)
    rng = np.random.default_rng(31)
    n_mv = 4000
    blk = rng.integers(0, inst.N, size=n_mv).astype(np.int32)
    per = rng.integers(0, inst.T + 1, size=n_mv).astype(np.int8)
    blk[5], per[6] = inst.N + 3, inst.T + 1          # two BAD moves
    blk[100:140] = blk[7]                            # one block, many periods
    blk[200:210], per[200:210] = blk[11], per[11]    # one move repeated
    mv = MoveSet(False, True, torch.from_numpy(blk).cuda(), torch.from_numpy(per).cuda())
    p = inst.p0.copy()
    for call in range(2):
        order = rng.permutation(n_mv).astype(np.int64)[:1500]
        order[:4] = [5, 6, -1, n_mv + 9]             # invalid ids first
        valid = (order >= 0) & (order < n_mv)
        ov = np.where(valid, order, 0)
        valid &= (blk[ov] < inst.N) & (per[ov] <= inst.T)
        idx = torch.from_numpy(order).cuda()
        cnt = torch.tensor([len(order)], dtype=torch.int32, device="cuda")
        applied = m.repair(mv, idx, cnt)
        q, a, _, _ = o.repair(p, blk[ov[valid]], per[ov[valid]])
        assert int(applied.item()) == a, call
        np.testing.assert_array_equal(to_np(m.get_schedule()), q)
        assert m.objective()["J"] == pytest.approx(o.objective(q)["J"], rel=1e-11)
        p = q


def test_repair_rejects_too_many_scenarios():
    from paper_2511_18296_amd.binding import MoveSet, MpsError
    inst = mpsgen.make_instance(4, 4, 2, 1100, 3, 1.5, 83)
    m = gpu_model(inst)
    idx = torch.zeros(4, dtype=torch.int64, device="cuda")
    cnt = torch.tensor([4], dtype=torch.int32, device="cuda")
    with pytest.raises(MpsError):
        m.repair(MoveSet(), idx, cnt)



@pytest.mark.parametrize("S,T,hard", [(256, 6, False), (257, 5, True), (1024, 4, False)])
def test_repair_scenario_chunk_edges(S, T, hard):
    """S at the edges of the walk's register chunks of 256 scenarios (one
    whole chunk, one scenario into the second, the largest S supported):
    same accept decisions, schedule and objective as the oracle walk."""
    from paper_2511_18296_amd.binding import MoveSet, TopK
    inst = mpsgen.make_instance(9, 8, 4, S, T, 2.0, 540 + S)
    m = gpu_model(inst)
    sc, fl = m.eval_moves()
    k = 300
    t = TopK(sc.numel(), k)
    idx, _, cnt = t(sc, fl)
    cand = to_np(idx)[:int(cnt.item())]
    D = inst.T + 1
    applied = m.repair(MoveSet(), idx, cnt, hard=hard)
    o = oracle.Oracle(inst)
    q, a, J, _ = o.repair(inst.p0, cand // D, (cand % D).astype(np.int8), hard=hard)
    assert int(applied.item()) == a
    np.testing.assert_array_equal(to_np(m.get_schedule()), q)
    assert m.objective()["J"] == pytest.approx(o.objective(q)["J"], rel=1e-11)
