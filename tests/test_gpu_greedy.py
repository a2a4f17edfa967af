"""The greedy initializer (Alg. 3, uncertainty factors 1) on the GPU against
the oracle: the same schedule block for block, the same number of passes
and of placed blocks, and the model's objective equal to the oracle's
objective of that schedule."""
import numpy as np
import pytest

import oracle
from gpu_common import gpu_model, instance, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["tiny", "ragged", "flat", "single", "one_period", "tight",
                                  "wide", "max_periods", "paper", "largest"])
def test_greedy_init_matches_oracle(name):
    inst = instance(name)
    m = gpu_model(inst)
    passes, placed = m.greedy_init()
    p = to_np(m.get_schedule())
    q, passes_o, placed_o = oracle.Oracle(inst).greedy_init()
    print(f"{name}: {passes} passes, {placed} of {inst.N} blocks placed "
          f"({int(np.count_nonzero(p != q))} blocks differ)")
    np.testing.assert_array_equal(p, q)
    assert (passes, placed) == (passes_o, placed_o)
    obj = oracle.Oracle(inst).objective(q)
    assert m.objective()["J"] == pytest.approx(obj["J"], rel=1e-9)


def test_greedy_init_max_pass_stops_early():
    inst = instance("paper")
    m = gpu_model(inst)
    passes, placed = m.greedy_init(max_pass=2)
    q, passes_o, placed_o = oracle.Oracle(inst).greedy_init(max_pass=2)
    assert passes == passes_o == 2 and placed == placed_o
    np.testing.assert_array_equal(to_np(m.get_schedule()), q)
