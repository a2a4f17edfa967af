"""Pins of the oracle's reading of explicit precedence lists (the sets
beta_b^Pred of Eq. 15 given as CSR arrays), on the CPU:
- the 1-5 stencil written out as lists gives bit-identical results to the
  grid reading (flags, scores, objective, repair, ranking, search), and the
  relaxed objective and gradient to FP64 rounding (another summation order);
- under the 1-9 cone the successor lists, precedence flags and violation
  counts equal brute force over the dense definition, move scores equal
  re-scoring of whole schedules, repair keeps every schedule feasible, and
  the exhaustive optimum of a 3x2x2 instance counts the feasible schedules
  that plain enumeration counts."""
import itertools

import numpy as np
import pytest

import mpsgen
import oracle

RELAX = (100.0 / (2 * 15600), 100.0 / (2 * 15600), 100.0 * 15600)


def _dense(N, ptr, idx):
    """pred[c][a] = a is a predecessor of c."""
    pred = np.zeros((N, N), dtype=bool)
    for c in range(N):
        pred[c, idx[ptr[c]:ptr[c + 1]]] = True
    return pred


def test_stencil_lists_equal_grid_reading():
    inst = mpsgen.make_instance(7, 6, 4, 23, 5, 1.5, 901)
    ptr, idx = mpsgen.stencil_precedence(inst.nx, inst.ny, inst.nz)
    g = oracle.Oracle(inst)
    c = oracle.Oracle(mpsgen.with_precedence(inst, ptr, idx))
    for b in range(inst.N):
        assert g.predecessors(b) == c.predecessors(b)
        assert g.successors(b) == c.successors(b)
    p = inst.p0
    assert g.objective(p) == c.objective(p)
    s1, f1 = g.eval_moves(p, include_never=True)
    s2, f2 = c.eval_moves(p, include_never=True)
    np.testing.assert_array_equal(f1, f2)
    np.testing.assert_array_equal(s1, s2)
    i, _ = oracle.topk(s1, f1, 150)
    D = inst.T + 1
    r1 = g.repair(p, (i // D).astype(np.int32), (i % D).astype(np.int8))
    r2 = c.repair(p, (i // D).astype(np.int32), (i % D).astype(np.int8))
    np.testing.assert_array_equal(r1[0], r2[0])
    assert r1[1:3] == r2[1:3]
    x = mpsgen.random_monotone_x(inst.N, inst.T, 17).astype(np.float64)
    J1, g1 = g.relaxed(x, *RELAX)
    J2, g2 = c.relaxed(x, *RELAX)
    # the precedence penalty sums the predecessors in list order (increasing
    # index) instead of the stencil's order: equal up to FP64 rounding
    assert J2 == pytest.approx(J1, rel=1e-13)
    np.testing.assert_allclose(g2, g1, rtol=0, atol=1e-12 * np.abs(g1).max())
    for a, b in zip(g.rank_moves(p, g1, 40), c.rank_moves(p, g1, 40)):
        np.testing.assert_array_equal(a, b)
    q1, J1, st1 = g.search(p, 0, 64)
    q2, J2, st2 = c.search(p, 0, 64)
    np.testing.assert_array_equal(q1, q2)
    assert J1 == J2 and st1 == st2


@pytest.fixture(scope="module")
def cone():
    inst = mpsgen.make_instance(6, 5, 4, 17, 6, 1.5, 902)
    ptr, idx = mpsgen.cone_precedence(inst.nx, inst.ny, inst.nz)
    p0 = mpsgen.feasible_schedule_lists(inst.N, inst.T, ptr, idx, 903)
    ci = mpsgen.with_precedence(inst, ptr, idx, p0)
    return ci, _dense(inst.N, ptr, idx)


def test_cone_lists_and_successors(cone):
    ci, pred = cone
    o = oracle.Oracle(ci)
    nx, ny = ci.nx, ci.ny
    for b in range(ci.N):
        x, y, z = b % nx, (b // nx) % ny, b // (nx * ny)
        want = sorted(xa + nx * (ya + ny * (z - 1))
                      for xa in range(x - 1, x + 2) for ya in range(y - 1, y + 2)
                      if z > 0 and 0 <= xa < nx and 0 <= ya < ny)
        assert o.predecessors(b) == want
        assert o.successors(b) == sorted(np.flatnonzero(pred[:, b]).tolist())
    # an interior block of an interior bench has nine of each
    b = 2 + nx * (2 + ny * 1)
    assert len(o.predecessors(b)) == 9 and len(o.successors(b)) == 9


def test_cone_flags_and_violations_by_brute_force(cone):
    ci, pred = cone
    o = oracle.Oracle(ci)
    rng = np.random.default_rng(904)
    T, D = ci.T, ci.T + 1
    for p in (ci.p0, rng.integers(0, T + 1, size=ci.N).astype(np.int8)):
        sc, fl = o.eval_moves(p, include_never=True)
        pp = p.astype(np.int64)
        for b in range(ci.N):
            preds = np.flatnonzero(pred[b])
            succs = np.flatnonzero(pred[:, b])
            for t in range(D):
                ok = np.all(pp[preds] <= t) and np.all(t <= pp[succs])
                assert bool(fl[b * D + t] & oracle.PREC_OK) == ok, (b, t)
        nv = int(sum(np.sum(pp[np.flatnonzero(pred[c])] > pp[c]) for c in range(ci.N)))
        assert o.objective(p)["n_prec_viol"] == nv


def test_cone_scores_equal_rescoring(cone):
    ci, pred = cone
    o = oracle.Oracle(ci)
    sc, fl = o.eval_moves(ci.p0, include_never=True)
    D = ci.T + 1
    rng = np.random.default_rng(905)
    for i in rng.choice(ci.N * D, size=60, replace=False):
        b, t = int(i // D), int(i % D)
        bf = o.eval_bruteforce(ci.p0, b, t)
        assert sc[i] == pytest.approx(bf, rel=1e-12, abs=1e-9 * abs(o.objective(ci.p0)["mu"]))


def test_cone_repair_keeps_feasibility(cone):
    ci, pred = cone
    o = oracle.Oracle(ci)
    sc, fl = o.eval_moves(ci.p0, include_never=True)
    idx, _ = oracle.topk(sc, fl, 200)
    D = ci.T + 1
    q, a, J, _ = o.repair(ci.p0, (idx // D).astype(np.int32), (idx % D).astype(np.int8))
    assert a > 0
    assert o.objective(q)["n_prec_viol"] == 0
    assert J > o.objective(ci.p0)["J"]
    qs, Js, _ = o.search(ci.p0, 0, 64)
    assert o.objective(qs)["n_prec_viol"] == 0
    s2, f2 = o.eval_moves(qs, include_never=True)
    ok = ((f2 & oracle.PREC_OK) != 0) & ((f2 & oracle.NOOP) == 0)
    assert s2[ok].max() <= 1e-6 * abs(o.objective(qs)["mu"])


def test_cone_exhaustive_optimum_counts_feasible_schedules():
    inst = mpsgen.make_instance(3, 2, 2, 4, 2, 1.0, 906)
    ptr, idx = mpsgen.cone_precedence(3, 2, 2)
    ci = mpsgen.with_precedence(inst, ptr, idx)
    o = oracle.Oracle(ci)
    J, best, cnt = o.optimum()
    # every schedule of the 12 blocks over {0, 1, 2}, feasibility checked on
    # the dense predecessor relation
    pred = _dense(ci.N, ptr, idx)
    pairs = np.argwhere(pred)          # (successor c, predecessor a)
    allp = np.array(list(itertools.product(range(3), repeat=ci.N)), dtype=np.int8)
    feas = np.all(allp[:, pairs[:, 1]] <= allp[:, pairs[:, 0]], axis=1)
    assert cnt == int(feas.sum())
    assert o.objective(best)["n_prec_viol"] == 0
    assert o.objective(best)["J"] == pytest.approx(J, rel=1e-12)
    # no precedence-feasible move improves the optimum
    sc, fl = o.eval_moves(best, include_never=True)
    ok = ((fl & oracle.PREC_OK) != 0) & ((fl & oracle.NOOP) == 0)
    assert sc[ok].max() <= 1e-9 * abs(o.objective(best)["mu"])
    # and J* is at least J of a sample of feasible schedules
    rng = np.random.default_rng(907)
    for row in rng.choice(np.flatnonzero(feas), size=200, replace=False):
        assert o.objective(allp[row])["J"] <= J + 1e-9 * abs(J)
