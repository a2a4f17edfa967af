"""Batched evaluation (three persistent launches, no waits between
workgroups) through the C ABI.  For every model of a mixed batch:
- flags against the oracle, bit-exact;
- scores against the oracle, within the contract;
- scores and flags against the single-model path, bit-identical (same
  arithmetic);
- the top k against the sort-based oracle selection of the same scores,
  bit-exact.
Every tuning, graph replays and the autotuner give the same results."""
import numpy as np
import pytest
import torch

import mpsgen
import oracle
from gpu_common import compare_scores, to_np
from test_gpu_batch import _batch_inputs, _outputs, _say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def phased():
    from paper_2511_18296_amd.binding import Batch, Model
    insts, moves = _batch_inputs()
    models = [Model.from_instance(i) for i in insts]
    dev = [(torch.from_numpy(b).cuda(), torch.from_numpy(p).cuda()) for b, p in moves]
    k = 256
    _say(f"creating a batch of {len(models)} models, k={k}")
    batch = Batch(models, dev, k)
    return insts, moves, models, dev, batch, k


def test_phased_batch_matches_oracle_and_single_path(phased):
    from paper_2511_18296_amd.binding import MoveSet, TopK
    insts, moves, models, dev, batch, k = phased
    _say("run")
    batch.run()
    out = _outputs(batch)
    _say("run finished")
    for i, inst in enumerate(insts):
        blk, per = moves[i]
        sc, fl, ti, ts, cnt = out[i]
        o = oracle.Oracle(inst)
        osc, ofl = o.eval_moves(inst.p0, block=blk, period=per)
        np.testing.assert_array_equal(fl, ofl, err_msg=f"model {i} flags")
        if len(blk):
            mu = o.objective(inst.p0)["mu"]
            compare_scores(sc, osc, fl, mu, f"model {i}")
        # single-model path: identical arithmetic, identical bits
        ssc, sfl = models[i].eval_moves(MoveSet(False, True, dev[i][0], dev[i][1]))
        np.testing.assert_array_equal(to_np(ssc), sc)
        np.testing.assert_array_equal(to_np(sfl), fl)
        # top k of these very scores: the sort-based selection, bit for bit
        ri, rs = oracle.topk(sc, fl, k)
        assert cnt == len(ri), (i, cnt, len(ri))
        np.testing.assert_array_equal(ti[:cnt], ri)
        np.testing.assert_array_equal(ts[:cnt], rs.astype(np.float32))
        assert np.all(ti[cnt:] == -1)
        assert np.all(np.isneginf(ts[cnt:]))
        if len(blk):
            t = TopK(len(blk), k)
            si, ss, sc_ = t(ssc, sfl)
            assert int(sc_.item()) == cnt
            np.testing.assert_array_equal(to_np(si)[:cnt], ti[:cnt])


@pytest.mark.parametrize("tiles,mpi,rows", [(1, 512, 8), (4, 16384, 16), (8, 2048, 32),
                                            (64, 65536, 8)])
def test_phased_tunings_agree(phased, tiles, mpi, rows):
    insts, moves, models, dev, batch, k = phased
    batch.set_tuning(2, 4096, 32)
    batch.run()
    ref = _outputs(batch)
    batch.set_tuning(tiles, mpi, rows)
    batch.set_workgroups(37)
    batch.run()
    got = _outputs(batch)
    batch.set_workgroups(0)
    for a, b in zip(ref, got):
        for x, y in zip(a[:4], b[:4]):
            np.testing.assert_array_equal(x, y)
        assert a[4] == b[4]


def test_phased_graph_replays(phased):
    """The captured graph replayed several times, with other device work and
    host synchronisation between replays: every replay equals the eager run."""
    from paper_2511_18296_amd.binding import MoveSet
    insts, moves, models, dev, batch, k = phased
    batch.run()
    ref = _outputs(batch)
    s = torch.cuda.Stream()
    for rep in range(4):
        for i in range(len(batch.models)):
            batch.score[i].fill_(np.nan)
            batch.flags[i].zero_()
            batch.top_idx[i].fill_(-7)
            batch.top_count[i].fill_(-1)
        models[0].eval_moves(MoveSet(False, True, dev[0][0], dev[0][1]))   # unrelated work
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            batch.graph_launch(s)
        s.synchronize()
        got = _outputs(batch)
        for a, b in zip(ref, got):
            for x, y in zip(a[:4], b[:4]):
                np.testing.assert_array_equal(x, y, err_msg=f"replay {rep}")
            assert a[4] == b[4]


def test_phased_autotune_keeps_results(phased):
    insts, moves, models, dev, batch, k = phased
    batch.set_tuning(2, 4096, 32)
    batch.run()
    ref = _outputs(batch)
    us = batch.autotune(reps=2)
    assert us > 0
    got = _outputs(batch)
    for i, (a, b) in enumerate(zip(ref, got)):
        for x, y in zip(a[:4], b[:4]):
            np.testing.assert_array_equal(x, y)
        t = batch.tuning(i)
        assert t["rows"] in (8, 16, 32) and 1 <= t["tiles_per_item"] <= 64
        assert t["moves_per_item"] % 512 == 0


def test_phased_k_extremes():
    from paper_2511_18296_amd.binding import Batch, Model, MAX_BATCH_TOPK
    inst = mpsgen.make_instance(14, 12, 6, 48, 9, 2.0, 520)
    blk, per = mpsgen.random_moves(inst.N, inst.T, 50000, 1520)
    m = Model.from_instance(inst)
    d = (torch.from_numpy(blk).cuda(), torch.from_numpy(per).cuda())
    for k in (1, 7, MAX_BATCH_TOPK):
        b = Batch([m], [d], k)
        b.run()
        torch.cuda.synchronize()
        sc, fl = to_np(b.score[0]), to_np(b.flags[0])
        ri, rs = oracle.topk(sc, fl, k)
        c = int(b.top_count[0].item())
        assert c == len(ri) == k
        np.testing.assert_array_equal(to_np(b.top_idx[0])[:c], ri)
        b.close()


def test_phased_rejects_bad_arguments():
    from paper_2511_18296_amd.binding import Batch, Model, MpsError
    inst = mpsgen.make_instance(6, 6, 3, 16, 4, 1.5, 521)
    m = Model.from_instance(inst)
    blk, per = mpsgen.random_moves(inst.N, inst.T, 100, 1521)
    d = (torch.from_numpy(blk).cuda(), torch.from_numpy(per).cuda())
    with pytest.raises(MpsError):
        Batch([m], [d], 0)
    with pytest.raises(MpsError):
        Batch([m], [d], 1025)
    b = Batch([m], [d], 4)
    with pytest.raises(MpsError):
        b.set_tuning(0, 4096, 8)
    with pytest.raises(MpsError):
        b.set_tuning(1, 1000, 8)
    with pytest.raises(MpsError):
        b.set_tuning(1, 4096, 12)
    with pytest.raises(MpsError):
        b.set_workgroups(-1)
    b.close()


@pytest.mark.parametrize("case", ["all_equal", "narrow", "mixed"])
def test_phased_topk_selection_paths(case):
    """The top-k phases take different routes by how the boundary keys
    spread: all scores equal (more than 1,024 keys share every score bit:
    the single-workgroup walk), scores in a narrow band (a level-1 pass),
    and a batch mixing both with an ordinary model.  Every route gives the
    sort-based selection of the same scores, bit for bit."""
    from paper_2511_18296_amd.binding import Batch, Model
    inst = mpsgen.make_instance(16, 14, 6, 40, 8, 2.0, 530)
    D = inst.T + 1
    osc, ofl = oracle.Oracle(inst).eval_moves(inst.p0, include_never=True)
    ok = ((ofl & oracle.PREC_OK) != 0) & ((ofl & (oracle.NOOP | oracle.BAD)) == 0)
    cand = np.flatnonzero(ok)
    assert len(cand) > 1000
    lists = []
    if case in ("all_equal", "mixed"):
        i = cand[len(cand) // 2]                      # one qualifying move, repeated
        lists.append((np.full(6000, i // D, np.int32), np.full(6000, i % D, np.int8)))
    if case in ("narrow", "mixed"):
        # the 150 best moves, 40 copies each: 2,280 keys share the top 12 key
        # bits of the boundary, at most 80 the top 23
        order = cand[np.argsort(-osc[cand], kind="stable")]
        sel = np.repeat(order[:150], 40)
        lists.append(((sel // D).astype(np.int32), (sel % D).astype(np.int8)))
    if case == "mixed":
        lists.append(mpsgen.random_moves(inst.N, inst.T, 20000, 532))
    models = [Model.from_instance(inst) for _ in lists]
    dev = [(torch.from_numpy(b).cuda(), torch.from_numpy(p).cuda()) for b, p in lists]
    for k in (256, 1024):
        b = Batch(models, dev, k)
        b.run()
        torch.cuda.synchronize()
        for i in range(len(lists)):
            sc, fl = to_np(b.score[i]), to_np(b.flags[i])
            ri, rs = oracle.topk(sc, fl, k)
            c = int(b.top_count[i].item())
            assert c == len(ri), (case, i, k, c, len(ri))
            np.testing.assert_array_equal(to_np(b.top_idx[i])[:c], ri)
            np.testing.assert_array_equal(to_np(b.top_score[i])[:c], rs.astype(np.float32))
        b.close()


def test_phased_lists_changed_after_create_stay_exact(phased):
    """The block order of the move lists is computed when the batch is built;
    lists that change afterwards (in place, same lengths) are still scored
    exactly, each move at its own position (only the locality is lost), and
    a retune recomputes the order with the same results."""
    from paper_2511_18296_amd.binding import MoveSet
    insts, moves, models, dev, batch, k = phased
    rng = np.random.default_rng(77)
    saved = [(b.clone(), p.clone()) for b, p in dev]
    try:
        for (b, p), inst in zip(dev, insts):
            n = b.shape[0]
            if n == 0:
                continue
            nb = rng.integers(0, inst.N, n).astype(np.int32)
            npd = rng.integers(0, inst.T + 1, n).astype(np.int8)
            b.copy_(torch.from_numpy(nb))
            p.copy_(torch.from_numpy(npd))
        torch.cuda.synchronize()
        for attempt in ("unchanged order", "after retune"):
            if attempt == "after retune":
                _retune_each(batch, len(models))
            _say(f"run with changed lists ({attempt})")
            batch.run()
            out = _outputs(batch)
            for i, inst in enumerate(insts):
                sc, fl, ti, ts, cnt = out[i]
                ssc, sfl = models[i].eval_moves(MoveSet(False, True, dev[i][0], dev[i][1]))
                np.testing.assert_array_equal(to_np(sfl), fl, err_msg=f"model {i} {attempt}")
                np.testing.assert_array_equal(to_np(ssc), sc, err_msg=f"model {i} {attempt}")
                ri, rs = oracle.topk(sc, fl, k)
                assert cnt == len(ri)
                np.testing.assert_array_equal(ti[:cnt], ri)
    finally:
        for (b, p), (b0, p0) in zip(dev, saved):
            b.copy_(b0)
            p.copy_(p0)
        torch.cuda.synchronize()
        _retune_each(batch, len(models))


def _retune_each(batch, n):
    # every model keeps its tuning; setting it recomputes its block order
    for i in range(n):
        t = batch.tuning(i)
        batch.set_tuning(t["tiles_per_item"], t["moves_per_item"], t["rows"], i=i)
