"""Helpers shared by the GPU tests (instances, oracle runs, comparisons)."""
import functools

import numpy as np
import torch

import mpsgen
import oracle

# Contract: float deltas within 1e-5 of |expected NPV| of the schedule.
CONTRACT_REL = 1e-5


@functools.lru_cache(maxsize=None)
def instance(name):
    if name == "tiny":
        return mpsgen.tiny_plain()
    if name == "paper":
        return mpsgen.paper_scale()
    if name == "largest":
        return mpsgen.largest_plain()
    if name == "ragged":
        # N, S, T that fill no tile, word or wave evenly
        return mpsgen.make_instance(7, 5, 3, 37, 3, 1.5, 77)
    if name == "flat":
        # one bench: no precedence at all
        return mpsgen.make_instance(13, 11, 1, 65, 4, 2.0, 78)
    if name == "single":
        return mpsgen.make_instance(6, 6, 4, 1, 6, 2.0, 79)
    if name == "wide":
        # S in (256, 512]: two scenario chunks per lane in the repair walk
        return mpsgen.make_instance(10, 9, 5, 300, 7, 2.0, 81)
    if name == "wider":
        # S in (512, 1024], not a multiple of 4
        return mpsgen.make_instance(8, 8, 4, 701, 5, 2.0, 82)
    if name == "deep":
        # T = 40 (three period tiles), S + 1 rows in two scenario groups of the
        # relaxed forward, four scenario passes of its adjoint
        return mpsgen.make_instance(20, 15, 6, 400, 40, 2.0, 84)
    if name == "tall":
        # T = 120: 32-block pieces, three per chunk in the relaxed forward;
        # 64-block adjoint tiles with five scenario passes
        return mpsgen.make_instance(25, 20, 20, 150, 120, 2.0, 85)
    if name == "one_period":
        # T = 1: the only destinations are period 0 and "never"
        return mpsgen.make_instance(9, 7, 4, 50, 1, 2.0, 86)
    if name == "max_periods":
        # T = MPS_MAX_PERIODS = 126: the widest period range a period byte holds
        return mpsgen.make_instance(6, 5, 4, 37, 126, 2.0, 87)
    if name == "max_scen":
        # S = MPS_MAX_SCENARIOS = 4096 (128 ore words per block; beyond what
        # the repair walk takes)
        return mpsgen.make_instance(4, 4, 3, 4096, 8, 2.0, 88)
    if name == "many_jobs":
        # T x ceil(S/64) = 126 x 16 = 2,016 table jobs: more than one job count
        # per thread in the scan of the one-launch table rebuild
        inst = mpsgen.make_instance(3, 3, 2, 1000, 126, 2.0, 90)
        inst.pcap *= 8.0         # some periods near capacity, not all over it
        return inst
    if name == "tight":
        inst = mpsgen.make_instance(12, 10, 6, 96, 8, 2.0, 80)
        inst.pcap *= 0.85        # capacities bind in most periods
        inst.mcap *= 0.8
        return inst
    raise KeyError(name)


def gpu_model(inst):
    from paper_2511_18296_amd.binding import Model
    return Model.from_instance(inst, device="cuda")


def to_np(t):
    return t.detach().cpu().numpy()


def compare_scores(gpu_score, ora_score, flags, mu, label=""):
    """Max |gpu - oracle| over non-BAD moves; asserts the contract bound."""
    ok = (flags & oracle.BAD) == 0
    err = np.abs(gpu_score[ok].astype(np.float64) - ora_score[ok])
    mx = float(err.max()) if err.size else 0.0
    bound = CONTRACT_REL * abs(mu)
    assert mx <= bound, f"{label}: max |score err| {mx:.4g} > {bound:.4g}"
    return mx
