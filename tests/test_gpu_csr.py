"""Explicit predecessor lists (MPS_PREC_CSR, Eq. 15's sets given as CSR
arrays) on the GPU:
- the 1-5 stencil written out as lists gives the grid mode's results bit for
  bit (objective, flags and scores, repair, greedy initializer);
- under the 1-9 cone: violation counts, flags bit for bit and scores within
  the contract against the oracle, repair and cascading repair decision for
  decision, the greedy initializer block for block, the relaxed objective and
  its adjoint, the gradient ranking and the LNS driver against the oracle."""
import numpy as np
import pytest
import torch

import mpsgen
import oracle
from gpu_common import compare_scores, gpu_model, to_np

pytestmark = pytest.mark.gpu

RELAX = (100.0 / (2 * 15600), 100.0 / (2 * 15600), 100.0 * 15600)


def _cone(nx, ny, nz, S, T, r, seed):
    inst = mpsgen.make_instance(nx, ny, nz, S, T, r, seed)
    ptr, idx = mpsgen.cone_precedence(nx, ny, nz)
    p0 = mpsgen.feasible_schedule_lists(inst.N, T, ptr, idx, seed + 50)
    return mpsgen.with_precedence(inst, ptr, idx, p0)


CONES = {"cone_small": (9, 8, 5, 24, 6, 2.0, 1201), "cone_mid": (24, 20, 8, 64, 10, 3.0, 1202),
         "cone_big": (40, 40, 10, 100, 12, 4.0, 1203)}


def test_stencil_lists_equal_grid_mode():
    from paper_2511_18296_amd.binding import MoveSet, TopK
    inst = mpsgen.make_instance(14, 12, 6, 40, 8, 2.0, 1200)
    ptr, idx = mpsgen.stencil_precedence(inst.nx, inst.ny, inst.nz)
    a = gpu_model(inst)
    b = gpu_model(mpsgen.with_precedence(inst, ptr, idx))
    assert a.objective() == b.objective()
    sa, fa = a.eval_moves()
    sb, fb = b.eval_moves()
    np.testing.assert_array_equal(to_np(fa), to_np(fb))
    np.testing.assert_array_equal(to_np(sa), to_np(sb))
    t = TopK(sa.numel(), 512)
    i, _, c = t(sa, fa)
    a.repair(MoveSet(), i, c)
    b.repair(MoveSet(), i, c)
    np.testing.assert_array_equal(to_np(a.get_schedule()), to_np(b.get_schedule()))
    assert a.greedy_init() == b.greedy_init()
    np.testing.assert_array_equal(to_np(a.get_schedule()), to_np(b.get_schedule()))


@pytest.mark.parametrize("name", list(CONES))
def test_cone_eval_and_objective(name):
    from paper_2511_18296_amd.binding import MoveSet
    inst = _cone(*CONES[name])
    m = gpu_model(inst)
    o = oracle.Oracle(inst)
    ref = o.objective(inst.p0)
    g = m.objective()
    assert g["n_prec_viol"] == ref["n_prec_viol"] == 0
    assert g["J"] == pytest.approx(ref["J"], rel=1e-11)
    sc, fl = m.eval_moves()
    osc, ofl = o.eval_moves(inst.p0, include_never=True)
    np.testing.assert_array_equal(to_np(fl), ofl)
    compare_scores(to_np(sc), osc, ofl, ref["mu"], name)
    # listed moves
    blk, per = mpsgen.random_moves(inst.N, inst.T, 20000, 1300)
    lsc, lfl = m.eval_moves(MoveSet(False, True, torch.from_numpy(blk).cuda(),
                                    torch.from_numpy(per).cuda()))
    lo, lof = o.eval_moves(inst.p0, block=blk, period=per)
    np.testing.assert_array_equal(to_np(lfl), lof)
    compare_scores(to_np(lsc), lo, lof, ref["mu"], name + " list")
    # an infeasible schedule: violation counts
    q = np.random.default_rng(5).integers(0, inst.T + 1, size=inst.N).astype(np.int8)
    m.set_schedule(torch.from_numpy(q).cuda())
    assert m.objective()["n_prec_viol"] == o.objective(q)["n_prec_viol"] > 0


@pytest.mark.parametrize("name", list(CONES))
def test_cone_repair_and_cascade(name):
    from paper_2511_18296_amd.binding import MoveSet, NOOP, BAD, TopK
    inst = _cone(*CONES[name])
    o = oracle.Oracle(inst)
    D = inst.T + 1
    m = gpu_model(inst)
    sc, fl = m.eval_moves()
    t = TopK(sc.numel(), 1024)
    idx, _, cnt = t(sc, fl)
    cand = to_np(idx)[:int(cnt.item())]
    applied = m.repair(MoveSet(), idx, cnt)
    q, a, J, acc = o.repair(inst.p0, cand // D, (cand % D).astype(np.int8))
    assert int(applied.item()) == a
    np.testing.assert_array_equal(to_np(m.get_schedule()), q)
    m2 = gpu_model(inst)
    idx2, _, cnt2 = t(sc, fl, require=0, forbid=NOOP | BAD)
    cand2 = to_np(idx2)[:int(cnt2.item())]
    applied2 = m2.repair_cascade(MoveSet(), idx2, cnt2, max_set=64)
    q2, a2, J2, acc2, size2 = o.repair_cascade(inst.p0, cand2 // D,
                                              (cand2 % D).astype(np.int8), max_set=64)
    assert int(applied2.item()) == a2
    np.testing.assert_array_equal(to_np(m2.get_schedule()), q2)
    print(f"{name}: repair applied {a}, cascade applied {a2} "
          f"({int(np.count_nonzero(acc2.astype(bool) & (size2 > 1)))} with companions)")


@pytest.mark.parametrize("name", list(CONES))
def test_cone_greedy_relaxed_rank(name):
    inst = _cone(*CONES[name])
    o = oracle.Oracle(inst)
    m = gpu_model(inst)
    # relaxed objective and adjoint at a random monotone plan
    x = mpsgen.random_monotone_x(inst.N, inst.T, 1400)
    xt = torch.from_numpy(x).cuda()
    saved = m.relaxed_saved()
    Jv = to_np(m.relaxed_fwd(xt, RELAX, saved))
    g = to_np(m.relaxed_bwd(xt, RELAX, saved))
    J_o, g_o = o.relaxed(x.astype(np.float64), *RELAX)
    assert abs(Jv[0] - J_o) <= 1e-5 * abs(Jv[1]), (Jv[0], J_o)
    assert np.abs(g - g_o).max() <= 1e-4 * np.abs(g_o).max()
    # gradient ranking at x(p)
    xi = torch.from_numpy(mpsgen.integer_x(inst.p0, inst.T)).cuda()
    m.relaxed_fwd(xi, RELAX, saved)
    gi = m.relaxed_bwd(xi, RELAX, saved)
    k = 512
    blk, per, gain, cnt = m.rank_moves(gi, k)
    D = inst.T + 1
    ab, at, ag = o.rank_moves(inst.p0, to_np(gi).astype(np.float64), inst.N * D)
    full = np.full(inst.N * D, -np.inf)
    full[ab.astype(np.int64) * D + at] = ag
    c = int(cnt.item())
    sel = to_np(blk)[:c].astype(np.int64) * D + to_np(per)[:c]
    assert c == min(k, len(ab)) and np.all(np.isfinite(full[sel]))
    kth = ag[c - 1]
    assert np.all(full[sel] >= kth - 2 * np.spacing(np.float32(abs(kth))))
    # greedy initializer
    passes, placed = m.greedy_init()
    q, passes_o, placed_o = o.greedy_init()
    np.testing.assert_array_equal(to_np(m.get_schedule()), q)
    assert (passes, placed) == (passes_o, placed_o)


def test_cone_lns_matches_oracle():
    inst = _cone(*CONES["cone_small"])
    n_iter, tile, k, rounds = 2, 3, 128, 6
    K = ((inst.nx + tile - 1) // tile) * ((inst.ny + tile - 1) // tile)
    u = np.random.default_rng(21).random(n_iter * K)
    m = gpu_model(inst)
    st, traj = m.lns_sa(n_iter, tile, k, rounds, 2e6, 1e6, 0.9, u)
    q, J, traj_o, st_o = oracle.Oracle(inst).lns_sa(inst.p0, n_iter, tile, k, rounds, 2e6, 1e6,
                                                    0.9, u)
    np.testing.assert_array_equal(traj[:, 3], traj_o[:, 3])
    np.testing.assert_array_equal(to_np(m.get_schedule()), q)
    assert st["applied"] == st_o["applied"]
