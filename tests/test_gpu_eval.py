"""GPU parity of the state and move evaluation against the FP64 oracle,
through the C ABI.  Flags must match bit for bit; scores within the
contract 1e-5 * |mu| (and the measured error is printed)."""
import numpy as np
import pytest
import torch

import mpsgen
import oracle
from gpu_common import compare_scores, gpu_model, instance, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["tiny", "ragged", "flat", "single", "tight", "paper"])
def test_objective_parity(name):
    inst = instance(name)
    m = gpu_model(inst)
    g = m.objective()
    o = oracle.Oracle(inst).objective(inst.p0)
    for k in ("mu", "R", "Pp", "Pm", "J"):
        assert g[k] == pytest.approx(o[k], rel=1e-12, abs=1e-6), k
    assert g["sigma"] == pytest.approx(o["sigma"], rel=1e-9, abs=1e-6)
    assert g["n_prec_viol"] == o["n_prec_viol"] == 0


@pytest.mark.parametrize("name", ["tiny", "ragged", "flat", "single", "tight", "one_period",
                                  "max_periods", "max_scen", "many_jobs"])
@pytest.mark.parametrize("never", [False, True])
def test_eval_exhaustive_small(name, never):
    inst = instance(name)
    from paper_2511_18296_amd.binding import MoveSet
    m = gpu_model(inst)
    sc, fl, dR, dPp, dPm = m.eval_moves(MoveSet(True, never), components=True)
    torch.cuda.synchronize()
    o = oracle.Oracle(inst)
    osc, ofl, odR, odPp, odPm = o.eval_moves(inst.p0, include_never=never, components=True)
    np.testing.assert_array_equal(to_np(fl), ofl)
    mu = o.objective(inst.p0)["mu"]
    err = compare_scores(to_np(sc), osc, ofl, mu, name)
    # components too, and score = dR - dPp - dPm on the device
    for a, b in ((dR, odR), (dPp, odPp), (dPm, odPm)):
        assert np.abs(to_np(a) - b).max() <= 1e-5 * abs(mu)
    print(f"{name} never={never}: max score error {err:.3g} (|mu| = {abs(mu):.3g})")


def test_eval_list_paper_scale():
    """250,000 random moves on the 40x40x20, S=50, T=15 instance, plus BAD ones."""
    from paper_2511_18296_amd.binding import MoveSet
    inst = instance("paper")
    m = gpu_model(inst)
    blk, per = mpsgen.random_moves(inst.N, inst.T, 250000, 1002)
    blk[:4] = [-1, inst.N, 5, 7]
    per[:4] = [0, 0, -1, inst.T + 1]
    mv = MoveSet(False, True, torch.from_numpy(blk).cuda(), torch.from_numpy(per).cuda())
    sc, fl = m.eval_moves(mv)
    o = oracle.Oracle(inst)
    osc, ofl = o.eval_moves(inst.p0, block=blk, period=per)
    np.testing.assert_array_equal(to_np(fl), ofl)
    assert np.all(to_np(fl)[:4] == oracle.BAD)
    assert np.all(to_np(sc)[:4] == -np.finfo(np.float32).max)
    err = compare_scores(to_np(sc), osc, ofl, o.objective(inst.p0)["mu"], "paper list")
    print(f"paper-scale list: max score error {err:.3g}")


def test_eval_short_lists_on_disjoint_tiles():
    """Short lists (fewer than eight moves per 64-block tile) mark the tiles
    they touch and the block pass skips the rest: consecutive short lists on
    disjoint and overlapping tile sets of one model, each against the oracle,
    then a long list (all tiles) and a short one again."""
    from paper_2511_18296_amd.binding import MoveSet
    inst = instance("paper")
    m = gpu_model(inst)
    o = oracle.Oracle(inst)
    mu = o.objective(inst.p0)["mu"]
    rng = np.random.default_rng(31)
    tiles = (inst.N + 63) // 64
    cases = []
    for lo, hi, n in ((0, tiles // 3, 700), (tiles // 3, 2 * tiles // 3, 300),
                      (tiles // 4, tiles // 2, 1000), (0, tiles, 9 * tiles),
                      (2 * tiles // 3, tiles, 50)):
        blk = rng.integers(lo * 64, min(inst.N, hi * 64), n).astype(np.int32)
        per = rng.integers(0, inst.T + 1, n).astype(np.int8)
        cases.append((blk, per))
    for j, (blk, per) in enumerate(cases):
        mv = MoveSet(False, True, torch.from_numpy(blk).cuda(), torch.from_numpy(per).cuda())
        sc, fl = m.eval_moves(mv)
        osc, ofl = o.eval_moves(inst.p0, block=blk, period=per)
        np.testing.assert_array_equal(to_np(fl), ofl, err_msg=f"list {j}")
        compare_scores(to_np(sc), osc, ofl, mu, f"list {j}")


def test_eval_list_empty():
    from paper_2511_18296_amd.binding import MoveSet
    inst = instance("tiny")
    m = gpu_model(inst)
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    sc, fl = m.eval_moves(MoveSet(False, True, e, e.to(torch.int8)))
    assert sc.numel() == 0 and fl.numel() == 0


def test_eval_exhaustive_largest():
    """All 1,134,000 moves of the 60x60x15, S=200, T=20 instance."""
    inst = instance("largest")
    m = gpu_model(inst)
    sc, fl = m.eval_moves()
    o = oracle.Oracle(inst)
    osc, ofl = o.eval_moves(inst.p0, include_never=True)
    np.testing.assert_array_equal(to_np(fl), ofl)
    err = compare_scores(to_np(sc), osc, ofl, o.objective(inst.p0)["mu"], "largest")
    print(f"largest exhaustive: max score error {err:.3g}")


def test_eval_after_schedule_change_and_determinism():
    inst = instance("ragged")
    m = gpu_model(inst)
    rng = np.random.default_rng(5)
    # any schedule, also an infeasible one
    p = rng.integers(0, inst.T + 1, size=inst.N).astype(np.int8)
    m.set_schedule(torch.from_numpy(p).cuda())
    a = [t.clone() for t in m.eval_moves()]
    b = [t.clone() for t in m.eval_moves()]
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    o = oracle.Oracle(inst)
    osc, ofl = o.eval_moves(p, include_never=True)
    np.testing.assert_array_equal(to_np(a[1]), ofl)
    compare_scores(to_np(a[0]), osc, ofl, o.objective(p)["mu"], "random schedule")
    g = m.objective()
    assert g["n_prec_viol"] == o.objective(p)["n_prec_viol"]


def test_eval_rejects_tables_beyond_lds():
    """S = 4096 with T = 126 leaves one tile's period tables no room in LDS:
    an argument error before any launch, and the model stays usable."""
    from paper_2511_18296_amd.binding import MoveSet, MpsError
    inst = mpsgen.make_instance(2, 2, 2, 4096, 126, 2.0, 89)
    m = gpu_model(inst)
    for ms in (MoveSet(True, True), MoveSet(True, False)):
        with pytest.raises(MpsError, match="LDS"):
            m.eval_moves(ms)
    o = oracle.Oracle(inst).objective(inst.p0)
    assert m.objective()["J"] == pytest.approx(o["J"], rel=1e-12, abs=1e-6)
