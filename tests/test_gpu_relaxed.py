"""Relaxed objective, its adjoint, gradient ranking and the search loops on
the GPU against the FP64 oracle (and FP64 central differences)."""
import numpy as np
import pytest
import torch

import mpsgen
import oracle
from gpu_common import gpu_model, instance, to_np

pytestmark = pytest.mark.gpu

RELAX = (100.0 / (2 * 15600), 100.0 / (2 * 15600), 100.0 * 15600)


@pytest.mark.parametrize("name", ["tiny", "ragged", "flat", "single", "one_period", "wider",
                                  "deep", "tall", "max_periods", "max_scen", "largest"])
def test_relaxed_forward_and_gradient_against_oracle(name):
    inst = instance(name)
    m = gpu_model(inst)
    x = mpsgen.random_monotone_x(inst.N, inst.T, 2000 + inst.seed)
    xt = torch.from_numpy(x).cuda()
    saved = m.relaxed_saved()
    Jv = to_np(m.relaxed_fwd(xt, RELAX, saved))
    g = to_np(m.relaxed_bwd(xt, RELAX, saved))
    o = oracle.Oracle(inst)
    J_o, g_o = o.relaxed(x.astype(np.float64), *RELAX)
    mu = abs(Jv[1])
    assert abs(Jv[0] - J_o) <= 1e-5 * mu, (Jv[0], J_o)
    err = np.abs(g - g_o).max()
    assert err <= 1e-4 * np.abs(g_o).max(), (err, np.abs(g_o).max())
    print(f"{name}: |J err| {abs(Jv[0] - J_o):.3g}, max |grad err| {err:.3g} "
          f"of {np.abs(g_o).max():.3g}")


FD_COORDS, FD_PARTS = 1000, 5


@pytest.fixture(scope="module")
def fd_case():
    """The GPU adjoint at a random monotone x on the 54,000-block instance,
    and 1,000 seeded coordinates to check it at."""
    inst = instance("largest")
    m = gpu_model(inst)
    x = mpsgen.random_monotone_x(inst.N, inst.T, 2005)
    xt = torch.from_numpy(x).cuda()
    saved = m.relaxed_saved()
    m.relaxed_fwd(xt, RELAX, saved)
    g = to_np(m.relaxed_bwd(xt, RELAX, saved))
    rng = np.random.default_rng(3005)
    coords = [(int(rng.integers(inst.N)), int(rng.integers(inst.T))) for _ in range(FD_COORDS)]
    return inst, x.astype(np.float64), g, coords


@pytest.mark.parametrize("part", range(FD_PARTS))
def test_gradient_against_fp64_central_differences(fd_case, part):
    """GPU adjoint vs FP64 central differences (h = 1e-6) of the oracle on
    1,000 random coordinates, in five parts of 200: each coordinate costs two
    full oracle passes over 54,000 blocks."""
    inst, x, g, coords = fd_case
    o = oracle.Oracle(inst)
    xd = x.copy()
    h = 1e-6
    gmax = np.abs(g).max()
    worst = 0.0
    n = FD_COORDS // FD_PARTS
    for b, t in coords[part * n:(part + 1) * n]:
        old = xd[b, t]
        xd[b, t] = old + h
        jp = o.relaxed(xd, *RELAX, grad=False)
        xd[b, t] = old - h
        jm = o.relaxed(xd, *RELAX, grad=False)
        xd[b, t] = old
        fd = (jp - jm) / (2 * h)
        worst = max(worst, abs(fd - g[b, t]) / gmax)
    assert worst <= 1e-4, worst
    print(f"part {part}: max |adjoint - FD| / max|grad| over {n} coordinates: {worst:.3g}")


def test_relaxed_integer_point_equals_objective():
    inst = instance("tiny")
    m = gpu_model(inst)
    x = torch.from_numpy(mpsgen.integer_x(inst.p0, inst.T)).cuda()
    Jv = to_np(m.relaxed_fwd(x, (0.0, 0.0, 1.0), m.relaxed_saved()))
    assert Jv[0] == pytest.approx(m.objective()["R"], rel=1e-6)


def test_autograd_function_matches_adjoint():
    from paper_2511_18296_amd.binding import RelaxedNPV
    inst = instance("ragged")
    m = gpu_model(inst)
    x = torch.from_numpy(mpsgen.random_monotone_x(inst.N, inst.T, 7)).cuda().requires_grad_()
    J = RelaxedNPV.apply(x, m, RELAX)
    (2.5 * J).backward()
    saved = m.relaxed_saved()
    m.relaxed_fwd(x.detach(), RELAX, saved)
    g = m.relaxed_bwd(x.detach(), RELAX, saved)
    torch.testing.assert_close(x.grad, 2.5 * g, rtol=1e-6, atol=0)


def test_rank_moves_against_oracle_ranking():
    inst = instance("largest")
    m = gpu_model(inst)
    x = torch.from_numpy(mpsgen.integer_x(inst.p0, inst.T)).cuda()
    saved = m.relaxed_saved()
    m.relaxed_fwd(x, RELAX, saved)
    g = m.relaxed_bwd(x, RELAX, saved)
    k = 4096
    blk, per, gain, cnt = m.rank_moves(g, k)
    assert int(cnt.item()) == k
    o = oracle.Oracle(inst)
    ob, ot, og = o.rank_moves(inst.p0, to_np(g).astype(np.float64), k)
    D = inst.T + 1
    gi = to_np(blk).astype(np.int64) * D + to_np(per)
    oi = ob.astype(np.int64) * D + ot
    np.testing.assert_allclose(to_np(gain), og, rtol=1e-6, atol=1e-6 * np.abs(og).max())
    if not np.array_equal(gi, oi):
        kth = og[-1]
        for i in set(gi) ^ set(oi):
            assert abs(float(og[np.searchsorted(-og, -kth)]) - kth) <= 1e-6 * abs(kth) + 1e-3
    assert len(set(gi) & set(oi)) >= k - 8


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("name", ["tight", "one_period", "max_periods"])
def test_search_reaches_oracle_quality(name, mode):
    inst = instance(name)
    m = gpu_model(inst)
    st = m.search(mode, 256, RELAX)
    o = oracle.Oracle(inst)
    q_o, J_o, st_o = o.search(inst.p0, mode, 256, RELAX)
    p = to_np(m.get_schedule())
    obj = o.objective(p)
    assert obj["n_prec_viol"] == 0
    assert st["J"] == pytest.approx(obj["J"], rel=1e-9)
    # a local optimum of the exact objective
    sc, fl = o.eval_moves(p, include_never=True)
    ok = ((fl & oracle.PREC_OK) != 0) & ((fl & oracle.NOOP) == 0)
    assert sc[ok].max() <= 1e-6 * abs(obj["mu"])
    # J can sit near zero when the penalties offset the NPV: measure the gap
    # on the scale of the larger of |J| and |mu|
    rel = abs(st["J"] - J_o) / max(abs(J_o), abs(obj["mu"]))
    print(f"{name} mode {mode}: GPU J {st['J']:.8g} vs oracle {J_o:.8g} (rel {rel:.2g}), "
          f"{st['iterations']} rounds, {st['evaluations']} evaluations")
    assert rel <= 1e-3
