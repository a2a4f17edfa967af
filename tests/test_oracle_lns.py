"""Pins of the oracle's LNS + simulated-annealing driver (Alg. 2 without its
GA and RL parts), on the CPU:
- invariants: every schedule it returns is precedence-feasible, its J is the
  best J of the input and of every accepted candidate, and the same draws
  give the same run;
- special cases of the acceptance rule: at temperature 0 with eps = 0 a
  candidate is accepted exactly when it raises J; with a huge temperature
  every candidate is accepted; with eps larger than every penalty the
  penalties drop out and acceptance follows R alone."""
import numpy as np
import pytest

import mpsgen
import oracle


def _run(inst, n_iter=2, nb=4, k=128, rounds=6, eps=0.0, temp=0.0, cool=0.9, seed=1):
    o = oracle.Oracle(inst)
    K = ((inst.nx + nb - 1) // nb) * ((inst.ny + nb - 1) // nb)
    u = np.random.default_rng(seed).random(n_iter * K)
    return o, o.lns_sa(inst.p0, n_iter, nb, k, rounds, eps, temp, cool, u)


@pytest.fixture(scope="module")
def inst():
    return mpsgen.make_instance(12, 12, 6, 24, 8, 2.0, 1101)


def test_result_is_feasible_best_and_deterministic(inst):
    o, (q, J, traj, st) = _run(inst, temp=5e6, eps=2e6)
    ob = o.objective(q)
    assert ob["n_prec_viol"] == 0
    assert J == ob["J"]
    acc = traj[:, 3] == 1
    J0 = o.objective(inst.p0)["J"]
    assert J == max([J0] + list(traj[acc, 0]))
    assert st["accepted"] == int(acc.sum()) and st["steps"] == len(traj)
    o2, (q2, J2, traj2, st2) = _run(inst, temp=5e6, eps=2e6)
    np.testing.assert_array_equal(q, q2)
    np.testing.assert_array_equal(traj, traj2)


def test_zero_temperature_accepts_exactly_the_improvements(inst):
    o, (q, J, traj, st) = _run(inst, temp=0.0, eps=0.0)
    Jcur = o.objective(inst.p0)["J"]
    for Jc, R, P, a in traj:
        assert R - P == pytest.approx(Jc, rel=1e-12, abs=1e-6)
        assert bool(a) == (Jc > Jcur)
        if a:
            Jcur = Jc
    assert J == Jcur


def test_huge_temperature_accepts_everything(inst):
    o, (q, J, traj, st) = _run(inst, temp=1e30, eps=0.0)
    assert np.all(traj[:, 3] == 1)


def test_large_eps_ignores_penalties(inst):
    # eps above every penalty: f = R, so acceptance compares R, not J
    o, (q, J, traj, st) = _run(inst, temp=0.0, eps=1e30)
    Rcur = o.objective(inst.p0)["R"]
    seen_diff = False
    Jcur = o.objective(inst.p0)["J"]
    for Jc, R, P, a in traj:
        assert bool(a) == (R > Rcur)
        seen_diff |= (R > Rcur) != (Jc > Jcur)
        if a:
            Rcur, Jcur = R, Jc
    assert st["steps"] > 0


def test_eps_schedule_is_linear(inst):
    # temperature 0: every decision is f(cand) > f(cur) with the iteration's
    # eps = eps_max (1 - it / n_iter), the eps-relaxed fitness of Alg. 2
    n_iter, nb = 4, 4
    E = 3e6
    o, (q, J, traj, st) = _run(inst, n_iter=n_iter, nb=nb, temp=0.0, eps=E)
    K = ((inst.nx + nb - 1) // nb) * ((inst.ny + nb - 1) // nb)
    ob = o.objective(inst.p0)
    Rc, Pc = ob["R"], ob["Pp"] + ob["Pm"]
    for j, (Jc, R, P, a) in enumerate(traj):
        eps = E * (1.0 - (j // K) / n_iter)
        f = lambda r, p: r - max(0.0, p - eps)
        assert bool(a) == (f(R, P) > f(Rc, Pc)), j
        if a:
            Rc, Pc = R, P
