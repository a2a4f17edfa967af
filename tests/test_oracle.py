"""Pins of the FP64 oracle against facts fixed outside it: a hand-worked
example, closed forms, brute force on tiny inputs, invariants and library
routines.  CPU only."""
import itertools
import math
from types import SimpleNamespace

import numpy as np
import pytest

import mpsgen
import oracle
from conftest import golden_instance, load_golden


def small_instance(nx, ny, nz, S, T, seed, **kw):
    return mpsgen.make_instance(nx, ny, nz, S, T, 1.5, seed, **kw)


# --- discount, stencil -------------------------------------------------------

def test_discount_closed_form():
    inst = small_instance(2, 2, 2, 2, 12, 0)
    d = oracle.Oracle(inst).discount()
    for t in range(12):
        assert d[t] == pytest.approx(1.08 ** (-t), rel=1e-14)
    assert d[12] == 0.0


def test_stencil_matches_bruteforce_definition():
    inst = small_instance(5, 4, 3, 2, 3, 0)
    o = oracle.Oracle(inst)
    nx, ny, nz = 5, 4, 3
    coords = [(b % nx, (b // nx) % ny, b // (nx * ny)) for b in range(nx * ny * nz)]
    for b, (x, y, z) in enumerate(coords):
        pred = [a for a, (xa, ya, za) in enumerate(coords)
                if za == z - 1 and abs(xa - x) + abs(ya - y) <= 1]
        succ = [c for c, (xc, yc, zc) in enumerate(coords)
                if zc == z + 1 and abs(xc - x) + abs(yc - y) <= 1]
        assert o.predecessors(b) == pred
        assert o.successors(b) == succ


# --- hand-worked example -----------------------------------------------------

def test_hand_example_objective_and_moves():
    g = load_golden("hand_two_blocks.json")
    o = oracle.Oracle(golden_instance(g))
    p = np.array(g["schedule"], dtype=np.int8)
    obj = o.objective(p)
    for k, v in g["objective"].items():
        assert obj[k] == pytest.approx(v, abs=1e-9), k
    assert obj["n_prec_viol"] == 0
    sc, fl = o.eval_moves(p, include_never=True)
    ref = g["moves_exhaustive_with_never"]
    np.testing.assert_allclose(sc, ref["score"], atol=1e-9)
    np.testing.assert_array_equal(fl, ref["flags"])


def test_hand_example_relaxed():
    g = load_golden("hand_two_blocks.json")
    o = oracle.Oracle(golden_instance(g))
    r = g["relaxed"]
    x = np.array(r["x"], dtype=np.float64)
    J, grad = o.relaxed(x, r["mu_proc"], r["mu_mine"], r["mu_prec"])
    assert J == pytest.approx(r["J"], abs=1e-9)
    np.testing.assert_allclose(grad, r["grad"], atol=1e-9)


# --- objective against library routines -----------------------------------------

def test_objective_against_numpy(tiny):
    o = oracle.Oracle(tiny)
    p = tiny.p0
    obj = o.objective(p, state=True)
    d = 1.08 ** (-np.arange(tiny.T + 1, dtype=np.float64))
    d[tiny.T] = 0.0
    Ns = tiny.v.astype(np.float64) @ d[p.astype(np.int64)]
    np.testing.assert_allclose(obj["Ns"], Ns, rtol=1e-12)
    assert obj["mu"] == pytest.approx(np.mean(Ns), rel=1e-12)
    assert obj["sigma"] == pytest.approx(np.std(Ns), rel=1e-10)
    assert obj["n_prec_viol"] == 0


def test_infeasible_schedule_counted(tiny):
    o = oracle.Oracle(tiny)
    p = tiny.p0.copy()
    b = 3 + 10 * 4 + 100 * 2   # interior block on bench 2
    p[b - 100] = tiny.T        # its block above is never mined
    assert o.objective(p)["n_prec_viol"] >= 1


# --- move deltas -------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_delta_equals_full_rescoring(seed):
    inst = small_instance(4, 3, 3, 5, 4, seed)
    o = oracle.Oracle(inst)
    p = inst.p0
    sc, fl = o.eval_moves(p, include_never=True)
    D = inst.T + 1
    scale = abs(o.objective(p)["mu"])
    for i in range(inst.N * D):
        b, t = divmod(i, D)
        ref = o.eval_bruteforce(p, b, t)
        assert abs(sc[i] - ref) <= 1e-12 * scale, (b, t)


def test_noop_scores_exactly_zero(tiny):
    o = oracle.Oracle(tiny)
    sc, fl = o.eval_moves(tiny.p0, include_never=True)
    D = tiny.T + 1
    idx = np.arange(tiny.N) * D + tiny.p0.astype(np.int64)
    assert np.all(sc[idx] == 0.0)
    assert np.all(fl[idx] & oracle.NOOP)
    assert np.count_nonzero(fl & oracle.NOOP) == tiny.N


def test_single_scenario_has_no_risk_term():
    inst = small_instance(3, 3, 2, 1, 3, 5, pen_proc=0.0, pen_mine=0.0)
    o = oracle.Oracle(inst)
    sc, _, dR, dPp, dPm = o.eval_moves(inst.p0, include_never=True, components=True)
    d = o.discount()
    D = inst.T + 1
    for i in range(inst.N * D):
        b, t = divmod(i, D)
        expect = float(inst.v[0, b]) * (d[t] - d[inst.p0[b]])
        assert dR[i] == pytest.approx(expect, abs=1e-6)
    assert np.all(dPp == 0.0) and np.all(dPm == 0.0)


def test_risk_neutral_reduces_to_expectation(tiny):
    inst = SimpleNamespace(**{**vars(tiny), "lam": 0.0, "pen_proc": 0.0,
                              "pen_mine": 0.0})
    o = oracle.Oracle(inst)
    sc, _ = o.eval_moves(tiny.p0, include_never=True)
    d = o.discount()
    D = tiny.T + 1
    m = tiny.v.astype(np.float64).mean(axis=0)
    b = np.arange(tiny.N).repeat(D)
    t = np.tile(np.arange(D), tiny.N)
    expect = m[b] * (d[t] - d[tiny.p0[b]])
    np.testing.assert_allclose(sc, expect, rtol=1e-9, atol=1e-6)


def test_single_block_one_period_closed_form():
    inst = SimpleNamespace(nx=1, ny=1, nz=1, S=3, T=1, rate=0.08, lam=0.7,
                           pen_proc=5.0, pen_mine=7.0, pcap=1e9, mcap=1e9,
                           v=np.array([[10.0], [20.0], [60.0]], np.float32),
                           ore=np.ones((3, 1), np.uint8), ton=np.array([1.0]))
    o = oracle.Oracle(inst)
    sc, fl = o.eval_moves(np.array([1], np.int8), include_never=True)
    mu, sd = 30.0, math.sqrt(((10 - 30) ** 2 + (20 - 30) ** 2 + (60 - 30) ** 2) / 3)
    assert sc[0] == pytest.approx(mu - 0.7 * sd, rel=1e-14)
    assert sc[1] == 0.0
    assert fl[0] == oracle.PREC_OK | oracle.MINE_OK | oracle.PROC_OK


def test_capacity_flags_at_the_boundary():
    # one bench of two blocks, both ore; period 0 holds block 0 only.
    base = dict(nx=2, ny=1, nz=1, S=1, T=2, rate=0.0, lam=0.0, pen_proc=1.0,
                pen_mine=1.0, v=np.array([[5.0, 5.0]], np.float32),
                ore=np.ones((1, 2), np.uint8), ton=np.array([100.0, 100.0]))
    p = np.array([0, 1], np.int8)
    for cap, ok in [(200.0, True), (199.0, False)]:
        inst = SimpleNamespace(**base, pcap=cap, mcap=cap)
        sc, fl = oracle.Oracle(inst).eval_moves(p, block=np.array([1]),
                                                period=np.array([0], np.int8))
        assert bool(fl[0] & oracle.MINE_OK) == ok
        assert bool(fl[0] & oracle.PROC_OK) == ok
        # excess of 1 t in period 0, relief of nothing in period 1
        assert sc[0] == pytest.approx(0.0 if ok else -2.0, abs=1e-12)


def test_precedence_flags_hand_cases():
    # column of two blocks: b0 above b1
    inst = SimpleNamespace(nx=1, ny=1, nz=2, S=1, T=3, rate=0.0, lam=0.0,
                           pen_proc=0.0, pen_mine=0.0, pcap=1e9, mcap=1e9,
                           v=np.zeros((1, 2), np.float32),
                           ore=np.zeros((1, 2), np.uint8), ton=np.ones(2))
    o = oracle.Oracle(inst)
    p = np.array([1, 2], np.int8)
    blocks = np.array([1, 1, 1, 0, 0, 0, 0], np.int32)
    periods = np.array([1, 0, 3, 2, 3, 0, 1], np.int8)
    _, fl = o.eval_moves(p, block=blocks, period=periods)
    prec = (fl & oracle.PREC_OK) != 0
    # same period as predecessor ok; earlier than predecessor not; never ok for
    # the bottom block; top block after its successor not; top block never not
    # (successor still mined); earlier always ok for the top block; noop ok.
    assert prec.tolist() == [True, False, True, True, False, True, True]


def test_bad_moves_flagged(tiny):
    o = oracle.Oracle(tiny)
    blocks = np.array([-1, tiny.N, 0, 0], np.int32)
    periods = np.array([0, 0, -1, tiny.T + 1], np.int8)
    sc, fl = o.eval_moves(tiny.p0, block=blocks, period=periods)
    assert np.all(fl == oracle.BAD)
    assert np.all(sc == -np.finfo(np.float32).max)


# --- top-k ---------------------------------------------------------------------

def test_topk_against_python_sort():
    rng = np.random.default_rng(7)
    n = 5000
    score = np.round(rng.normal(size=n), 1)     # many exact ties
    flags = rng.integers(0, 32, size=n).astype(np.uint8)
    for k in (1, 17, 300, 5000):
        idx, sc = oracle.topk(score, flags, k)
        keep = [i for i in range(n) if (flags[i] & 1) and not (flags[i] & 24)]
        ref = sorted(keep, key=lambda i: (-score[i], i))[:k]
        assert idx.tolist() == ref
        np.testing.assert_array_equal(sc, score[ref])


# --- repair --------------------------------------------------------------------

def test_repair_invariants(tiny):
    o = oracle.Oracle(tiny)
    p = tiny.p0
    sc, fl = o.eval_moves(p, include_never=True)
    idx, _ = oracle.topk(sc, fl, 400)
    D = tiny.T + 1
    cb, ct = (idx // D).astype(np.int32), (idx % D).astype(np.int8)
    q, applied, J, acc = o.repair(p, cb, ct)
    assert applied == int(acc.sum()) > 0
    assert o.objective(q)["n_prec_viol"] == 0
    assert J == pytest.approx(o.objective(q)["J"], rel=1e-12)
    # replay: each accepted move is positive and PREC-feasible at its turn,
    # each rejected one is not (or its block already moved)
    cur = p.copy()
    moved = set()
    J0 = o.objective(p)["J"]
    total = 0.0
    for i in range(len(cb)):
        b, t = int(cb[i]), int(ct[i])
        if b in moved:
            assert acc[i] == 0
            continue
        s, f = o.eval_moves(cur, block=np.array([b]), period=np.array([t], np.int8))
        gain = o.eval_bruteforce(cur, b, t)
        assert s[0] == pytest.approx(gain, abs=1e-6)
        take = bool(f[0] & oracle.PREC_OK) and s[0] > 0
        assert bool(acc[i]) == take
        if take:
            cur[b] = t
            moved.add(b)
            total += gain
    np.testing.assert_array_equal(cur, q)
    assert J - J0 == pytest.approx(total, rel=1e-9)
    assert J > J0


def test_repair_hard_capacity_respects_capacities(tiny):
    o = oracle.Oracle(tiny)
    sc, fl = o.eval_moves(tiny.p0, include_never=True)
    idx, _ = oracle.topk(sc, fl, 400)
    D = tiny.T + 1
    q, applied, _, acc = o.repair(tiny.p0, idx // D, (idx % D).astype(np.int8),
                                  hard=True)
    st0 = o.objective(tiny.p0, state=True)
    st1 = o.objective(q, state=True)
    # no period that was within capacity is pushed over it
    for t in range(tiny.T):
        if st0["M"][t] <= tiny.mcap:
            assert st1["M"][t] <= tiny.mcap
        within = st0["O"][:, t] <= tiny.pcap
        assert np.all(st1["O"][within, t] <= tiny.pcap)


# --- tiny exhaustive optimum ------------------------------------------------------

def _count_feasible_3x3x2(T):
    """Transfer count over the two benches: every top-bench assignment times,
    per bottom block, the number of periods not earlier than its predecessors."""
    preds = []
    for y in range(3):
        for x in range(3):
            preds.append([xa + 3 * ya for xa, ya in
                          [(x, y), (x - 1, y), (x + 1, y), (x, y - 1), (x, y + 1)]
                          if 0 <= xa < 3 and 0 <= ya < 3])
    total = 0
    for top in itertools.product(range(T + 1), repeat=9):
        prod = 1
        for pr in preds:
            prod *= T + 1 - max(top[a] for a in pr)
        total += prod
    return total


def test_tiny_exhaustive_optimum():
    inst = mpsgen.make_instance(3, 3, 2, 4, 2, 1.0, 11)
    inst.pcap *= 0.8                      # make the capacities bind
    inst.mcap *= 0.8
    o = oracle.Oracle(inst)
    J_star, p_star, n_feas = o.optimum()
    assert n_feas == _count_feasible_3x3x2(2) == 651438
    assert o.objective(p_star)["J"] == pytest.approx(J_star, rel=1e-14)
    assert o.objective(p_star)["n_prec_viol"] == 0
    # no precedence-feasible move improves the optimum
    sc, fl = o.eval_moves(p_star, include_never=True)
    ok = (fl & oracle.PREC_OK) != 0
    assert sc[ok].max() <= 1e-9 * abs(J_star)
    # both search loops end at or below J*, from several starting schedules
    relax = (100.0 / (2 * 15600), 100.0 / (2 * 15600), 100.0 * 15600)
    for seed in range(4):
        p0 = mpsgen.make_instance(3, 3, 2, 4, 2, 1.0, 100 + seed).p0
        for mode in (0, 1):
            q, J, st = o.search(p0, mode, 8, relax)
            assert J <= J_star + 1e-9 * abs(J_star)
            assert o.objective(q)["n_prec_viol"] == 0


# --- relaxed objective -----------------------------------------------------------

def test_relaxed_at_integer_point_equals_objective(tiny):
    o = oracle.Oracle(tiny)
    x = mpsgen.integer_x(tiny.p0, tiny.T)
    J = o.relaxed(x.astype(np.float64), 0.0, 0.0, 1.0, grad=False)
    assert J == pytest.approx(o.objective(tiny.p0)["R"], rel=1e-12)


def test_relaxed_gradient_central_differences(tiny):
    o = oracle.Oracle(tiny)
    x = mpsgen.random_monotone_x(tiny.N, tiny.T, 2001).astype(np.float64)
    rp = (100.0 / (2 * 15600), 100.0 / (2 * 15600), 100.0 * 15600)
    J, g = o.relaxed(x, *rp)
    rng = np.random.default_rng(3001)
    h = 1e-6
    gscale = np.abs(g).max()
    for _ in range(60):
        b, t = int(rng.integers(tiny.N)), int(rng.integers(tiny.T))
        xp, xm = x.copy(), x.copy()
        xp[b, t] += h
        xm[b, t] -= h
        fd = (o.relaxed(xp, *rp, grad=False) - o.relaxed(xm, *rp, grad=False)) / (2 * h)
        assert abs(fd - g[b, t]) <= 1e-6 * gscale + 1e-5 * abs(fd), (b, t)


def test_rank_moves_is_directional_derivative(tiny):
    o = oracle.Oracle(tiny)
    p = tiny.p0
    x = mpsgen.integer_x(p, tiny.T).astype(np.float64)
    _, g = o.relaxed(x, 1e-4, 1e-4, 1e6)
    k = 200
    b, t, gain = o.rank_moves(p, g, k)
    assert len(b) == k
    for j in range(k):
        q = p.copy()
        q[b[j]] = t[j]
        dx = mpsgen.integer_x(q, tiny.T).astype(np.float64) - x
        assert gain[j] == pytest.approx(float((g * dx).sum()), rel=1e-9, abs=1e-6)
        assert t[j] != p[b[j]]
        # only precedence-feasible moves are ranked (brute force over Pred/Succ)
        assert all(p[a] <= t[j] for a in o.predecessors(int(b[j])))
        assert all(t[j] <= p[c] for c in o.successors(int(b[j])))
    D = tiny.T + 1
    key = [(-gain[j], int(b[j]) * D + int(t[j])) for j in range(k)]
    assert key == sorted(key)


def test_search_ends_at_local_optimum(tiny):
    o = oracle.Oracle(tiny)
    relax = (100.0 / (2 * 15600), 100.0 / (2 * 15600), 100.0 * 15600)
    J0 = o.objective(tiny.p0)["J"]
    for mode in (0, 1):
        q, J, st = o.search(tiny.p0, mode, 64, relax)
        assert J > J0 and st["applied"] > 0
        sc, fl = o.eval_moves(q, include_never=True)
        ok = ((fl & oracle.PREC_OK) != 0) & ((fl & oracle.NOOP) == 0)
        assert sc[ok].max() <= 0.0
