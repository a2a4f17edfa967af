"""Seeded instance generator: distribution, reproducibility, feasibility."""
import math

import numpy as np

import mpsgen
import oracle


def test_grade_field_unit_variance_and_lognormal():
    rng = np.random.default_rng(0)
    g = mpsgen.grade_field(12, 12, 8, 64, 3.0, rng).astype(np.float64)
    z = (np.log(g) - math.log(mpsgen.GRADE_MEDIAN)) / mpsgen.GRADE_LOGSD
    # every block has unit variance across scenarios (sampling error ~ 1/sqrt(64))
    var = z.var(axis=0)
    assert abs(var.mean() - 1.0) < 0.05
    assert abs(z.mean()) < 0.1
    # median grade 0.8 g/t
    assert abs(np.median(g) - 0.8) < 0.05


def test_ore_fraction_and_values():
    inst = mpsgen.make_instance(20, 20, 6, 40, 5, 3.0, 5)
    frac = inst.ore.mean()
    # P(g > 20/54) for lognormal(ln 0.8, 0.6) = Phi((ln 0.8 - ln(20/54))/0.6) ~ 0.900
    assert abs(frac - 0.900) < 0.03
    waste = inst.ore == 0
    assert np.all(inst.v[waste] == np.float32(-15600.0 * 3.0))
    assert np.all(inst.v[~waste] > np.float32(-15600.0 * 3.0))


def test_schedule_feasible_and_seeded():
    a = mpsgen.make_instance(8, 7, 6, 3, 9, 2.0, 42)
    b = mpsgen.make_instance(8, 7, 6, 3, 9, 2.0, 42)
    np.testing.assert_array_equal(a.v, b.v)
    np.testing.assert_array_equal(a.p0, b.p0)
    assert oracle.Oracle(a).objective(a.p0)["n_prec_viol"] == 0
    assert a.p0.min() >= 0 and a.p0.max() <= a.T


def test_capacities_follow_recipe():
    inst = mpsgen.tiny_plain()
    ore_t = (inst.ore * inst.ton[None, :]).sum(axis=1).mean()
    assert inst.pcap == ore_t / inst.T
    assert abs(inst.mcap - 1.1 * inst.N * 15600.0 / inst.T) < 1e-6


def test_ore_pack_roundtrip():
    rng = np.random.default_rng(1)
    ore = (rng.random((70, 33)) < 0.9).astype(np.uint8)
    w = mpsgen.ore_pack(ore)
    assert w.shape == (3, 33) and w.dtype == np.uint32
    for s in range(70):
        np.testing.assert_array_equal((w[s // 32] >> (s % 32)) & 1, ore[s])


def test_random_moves_and_relaxed_x():
    b, t = mpsgen.random_moves(1000, 7, 5000, 9)
    assert b.min() >= 0 and b.max() < 1000 and t.min() >= 0 and t.max() <= 7
    x = mpsgen.random_monotone_x(50, 6, 3)
    assert np.all(np.diff(x, axis=1) >= 0) and x.min() >= 0 and x.max() < 1
