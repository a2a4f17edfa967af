"""Pins of the oracle's objective variants, on the CPU:
- the per-(s,t) value multiplier (Eq. 12's sigma(s,t)): all ones gives the
  base objective and scores bit for bit; a multiplier gamma_s that does not
  depend on the period scales each scenario NPV by gamma_s; move scores
  equal re-scoring of whole schedules;
- the CVaR risk measure: or_cvar equals the Rockafellar-Uryasev
  representation max_z [z - E(z - X)_+ / alpha] (lower tail) evaluated by
  brute force over z; alpha = 1 gives the mean and alpha <= 1/S the minimum;
  with lambda = 0 the objective is the base objective's; move scores equal
  re-scoring of whole schedules."""
import copy

import numpy as np
import pytest

import mpsgen
import oracle


def _variant(inst, mult=None, risk=0, alpha=0.1, lam=None):
    out = copy.copy(inst)
    out.mult = mult
    out.risk = risk
    out.alpha = alpha
    if lam is not None:
        out.lam = lam
    return out


def _rockafellar_uryasev(x, alpha):
    x = np.asarray(x, dtype=np.float64)
    best = -np.inf
    for z in x:
        best = max(best, z - np.maximum(0.0, z - x).sum() / (alpha * len(x)))
    return best


@pytest.mark.parametrize("n,alpha", [(10, 0.1), (200, 0.1), (37, 0.1), (37, 0.25), (5, 0.5),
                                     (13, 0.33), (7, 1.0), (1, 0.1), (50, 0.01)])
def test_cvar_equals_rockafellar_uryasev(n, alpha):
    x = np.random.default_rng(n * 7 + int(alpha * 100)).normal(1e6, 3e5, size=n)
    x[: n // 4] = x[0]   # ties
    assert oracle.cvar(x, alpha) == pytest.approx(_rockafellar_uryasev(x, alpha), rel=1e-12)


def test_cvar_limits():
    x = np.random.default_rng(3).normal(0, 1, size=64)
    assert oracle.cvar(x, 1.0) == pytest.approx(x.mean(), rel=1e-12)
    assert oracle.cvar(x, 1.0 / 64) == x.min()
    assert oracle.cvar(x, 0.001) == x.min()


def test_unit_multiplier_is_the_base_objective():
    inst = mpsgen.make_instance(8, 7, 4, 20, 5, 2.0, 801)
    base = oracle.Oracle(inst)
    var = oracle.Oracle(_variant(inst, mult=np.ones((inst.S, inst.T))))
    assert base.objective(inst.p0) == var.objective(inst.p0)
    s1, f1 = base.eval_moves(inst.p0)
    s2, f2 = var.eval_moves(inst.p0)
    np.testing.assert_array_equal(s1, s2)
    np.testing.assert_array_equal(f1, f2)


def test_scenario_multiplier_scales_each_npv():
    inst = mpsgen.make_instance(8, 7, 4, 20, 5, 2.0, 802)
    gamma = np.random.default_rng(5).uniform(0.5, 1.5, size=inst.S)
    mult = np.repeat(gamma[:, None], inst.T, axis=1)
    a = oracle.Oracle(inst).objective(inst.p0, state=True)
    b = oracle.Oracle(_variant(inst, mult=mult)).objective(inst.p0, state=True)
    np.testing.assert_allclose(b["Ns"], gamma * a["Ns"], rtol=1e-12)
    assert b["Pp"] == a["Pp"] and b["Pm"] == a["Pm"]


@pytest.mark.parametrize("risk,alpha", [(0, 0.1), (1, 0.1), (1, 0.3)])
def test_variant_scores_equal_rescoring(risk, alpha):
    inst = mpsgen.make_instance(6, 5, 4, 30, 5, 2.0, 803)
    mult = np.random.default_rng(6).uniform(0.6, 1.4, size=(inst.S, inst.T))
    o = oracle.Oracle(_variant(inst, mult=mult, risk=risk, alpha=alpha))
    sc, fl = o.eval_moves(inst.p0, include_never=True)
    D = inst.T + 1
    rng = np.random.default_rng(7)
    mu = abs(o.objective(inst.p0)["mu"])
    for i in rng.choice(inst.N * D, size=120, replace=False):
        bf = o.eval_bruteforce(inst.p0, i // D, i % D)
        assert sc[i] == pytest.approx(bf, rel=1e-9, abs=1e-9 * mu)


def test_cvar_with_zero_lambda_is_the_base_objective():
    inst = mpsgen.make_instance(6, 6, 3, 25, 4, 2.0, 804)
    a = oracle.Oracle(_variant(inst, lam=0.0)).objective(inst.p0)
    b = oracle.Oracle(_variant(inst, risk=1, alpha=0.1, lam=0.0)).objective(inst.p0)
    assert a["J"] == b["J"] and a["R"] == b["R"]


def test_cvar_objective_definition():
    inst = mpsgen.make_instance(6, 6, 3, 40, 4, 2.0, 805)
    o = oracle.Oracle(_variant(inst, risk=1, alpha=0.1))
    ob = o.objective(inst.p0, state=True)
    ns = ob["Ns"]
    want = ns.mean() - inst.lam * (ns.mean() - _rockafellar_uryasev(ns, 0.1))
    assert ob["R"] == pytest.approx(want, rel=1e-12)
