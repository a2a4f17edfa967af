"""The LNS + simulated-annealing driver (Alg. 2 without GA and RL) on the GPU
against the oracle's run with the same draws: the same trajectory step for
step (every candidate's J, R and penalty, every accept decision), the same
best schedule block for block, and the same counts of evaluated and applied
moves."""
import numpy as np
import pytest

import mpsgen
import oracle
from gpu_common import gpu_model, instance, to_np

pytestmark = pytest.mark.gpu

# (instance, iterations, tile, k, rounds, eps_max, temp0, cool, seed)
CASES = [("ragged", 2, 3, 64, 6, 1e6, 5e5, 0.9, 11),
         ("tight", 2, 4, 256, 8, 5e6, 2e6, 0.8, 12),
         ("lns_mid", 2, 5, 512, 8, 1e7, 1e6, 0.9, 13)]


def _inst(name):
    if name == "lns_mid":
        # 20 x 20 x 10 blocks, S = 50, T = 10: a mid-size instance of the
        # paper-scale shape family
        return mpsgen.make_instance(20, 20, 10, 50, 10, 3.0, 2)
    return instance(name)


@pytest.mark.parametrize("name,n_iter,tile,k,rounds,eps,temp,cool,seed", CASES)
def test_lns_matches_oracle(name, n_iter, tile, k, rounds, eps, temp, cool, seed):
    inst = _inst(name)
    K = ((inst.nx + tile - 1) // tile) * ((inst.ny + tile - 1) // tile)
    u = np.random.default_rng(seed).random(n_iter * K)
    m = gpu_model(inst)
    st, traj = m.lns_sa(n_iter, tile, k, rounds, eps, temp, cool, u)
    o = oracle.Oracle(inst)
    q, J, traj_o, st_o = o.lns_sa(inst.p0, n_iter, tile, k, rounds, eps, temp, cool, u)
    p = to_np(m.get_schedule())
    print(f"{name}: {st['steps']} steps, {st['accepted']} accepted "
          f"(oracle {st_o['accepted']}), J {inst_J(o, inst.p0):.6g} -> {st['J_best']:.8g} "
          f"(oracle {J:.8g}); {st['evaluations']} moves evaluated, {st['applied']} applied")
    np.testing.assert_array_equal(traj[:, 3], traj_o[:, 3])
    np.testing.assert_allclose(traj[:, :3], traj_o[:, :3], rtol=1e-9,
                               atol=1e-9 * abs(o.objective(inst.p0)["mu"]))
    assert (st["steps"], st["accepted"], st["evaluations"], st["applied"]) == \
        (st_o["steps"], st_o["accepted"], st_o["evaluations"], st_o["applied"])
    np.testing.assert_array_equal(p, q)
    assert st["J_best"] == pytest.approx(J, rel=1e-9)
    assert m.objective()["J"] == pytest.approx(J, rel=1e-9)


def inst_J(o, p):
    return o.objective(p)["J"]
