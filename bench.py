"""Benchmark of the candidate-move evaluation engine on one MI355X.

Workload: the 60x60x15 = 54,000-block grid, T = 20 periods, S = 200
scenarios (grade range 6 blocks, seed 3).  One step is the first iteration
of the exhaustive search from the seeded schedule: restore the seeded search
state (one device copy of the schedule and its derived state), evaluate all
1,134,000 moves (every block x 21 destinations, never-mined included),
select the top 4,096, repair greedily with them -- all on the device.  Every
step therefore does the same work.  Eight independent copies of the instance
are used round-robin so that consecutive steps do not find their block
values in the 256 MB Infinity Cache.

Prints ONE JSON line (rank 0).  `value` = move-scenario evaluations per
second of whole steps; `roofline` is that of the move-evaluation kernel,
timed with events on the stream it runs on over a burst of launches (its
per-step phase time, bracketed by events of its own, also times the event
markers).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the exhaustive evaluation kernel, measured with
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE and scaled by what the same
# counters read for a device copy of known size (profiles/ holds the
# summaries).  Keyed by the SHA-1 of the kernel's sources: a changed kernel
# reports null until it is measured again.
MEASURED_TRAFFIC = {
    # 60x60x15, S=200, T=20: FETCH_SIZE 22,824.9 KiB x 2.000 (a 256 MiB copy
    # reads 131,083.5 KiB) + WRITE_SIZE 5,537.1 KiB x 1.000 (the copy writes
    # 262,144.0 KiB)
    "fdee77ac0f29b426f623591fb04248986ace76c4": 22824.9 * 1024 * 2.000 + 5537.1 * 1024 * 1.000,
}
EVAL_SOURCES = ("eval.hip", "eval_dev.h", "internal.h")
RELAX_SOURCES = ("relaxed.hip", "internal.h")
# HBM bytes per call of the relaxed passes on the same instance, from the same
# counter runs and calibration (profiles/relaxed_fwd_bwd_60x60x15_S200_T20.md):
# forward = chunk + reduce + final kernels, adjoint = tile kernel.
MEASURED_RELAX_TRAFFIC = {
    "d18d02c3b153074d45b7b1849a363f2943255d81": {
        "relaxed_fwd": (26859.1 + 4021.0 + 9.5) * 1024 * 2.000 + (4000.6 + 226.5 + 4.7) * 1024 * 1.000,
        "relaxed_bwd": 29007.6 * 1024 * 2.000 + 4218.8 * 1024 * 1.000},
}


def source_sha(files):
    import hashlib
    h = hashlib.sha1()
    for f in files:
        with open(os.path.join(ROOT, "paper_2511_18296_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def eval_source_sha():
    return source_sha(EVAL_SOURCES)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def eval_bytes(N, S, T, D):
    """Algorithmic HBM bytes of one exhaustive evaluation: v (4SN), ore words
    (4*ceil(S/32)*N), per-block mean and variance (8N), tonnage (4N),
    schedule (N), score + flags (5*N*D)."""
    W = (S + 31) // 32
    return 4 * S * N + 4 * W * N + 8 * N + 4 * N + N + 5 * N * D


def cpu_model():
    """The host CPU as /proc/cpuinfo describes its first logical CPU: model
    name, then family/model/stepping, clock and cache size where given."""
    fields = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not line.strip():
                    break   # the first logical CPU only
                k, _, v = line.partition(":")
                fields[k.strip()] = v.strip()
    except OSError:
        return "unknown"
    name = fields.get("model name", "unknown")
    extra = [f"{k} {fields[k]}" for k in ("cpu family", "model", "stepping", "cpu MHz",
                                          "cache size") if k in fields]
    return name + (" (" + ", ".join(extra) + ")" if extra else "")


def cpu_baseline(inst, k, min_seconds=10.0, max_reps=200):
    """The FP64 oracle on the host: full steps of the same workload (all moves,
    top-k, repair from the seeded schedule), repeated until at least
    min_seconds of host time have passed, with every OpenMP thread of the
    process and then with one thread."""
    import numpy as np
    import oracle
    o = oracle.Oracle(inst)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    D = inst.T + 1
    n = inst.N * D

    def run(nt, secs):
        reps = 0
        t0 = time.perf_counter()
        while True:
            sc, fl = o.eval_moves(inst.p0, include_never=True, threads=nt)
            idx, _ = oracle.topk(sc, fl, k)
            o.repair(inst.p0, (idx // D).astype(np.int32), (idx % D).astype(np.int8))
            reps += 1
            dt = time.perf_counter() - t0
            if dt >= secs or reps >= max_reps:
                return reps, dt

    reps, dt = run(threads, min_seconds)
    reps1, dt1 = run(1, min_seconds)
    return {"value": reps * n * inst.S / dt, "unit": "move-scenario evals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{reps} full steps (each: eval of all {n:,} moves x {inst.S} scenarios, "
                      f"top-{k}, repair) of the same instance, {dt:.1f} s",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "single_thread": {"value": reps1 * n * inst.S / dt1, "cores": 1,
                              "sample": f"{reps1} full steps, {dt1:.1f} s"}}


def batch_bytes(insts, moves):
    """Algorithmic HBM bytes of one batched launch: per model v (4SN), ore
    words (4*ceil(S/32)*N), per-block scalars read once (p, ton32, ton64,
    m_b, V_b: 21N), the move list (5M) and scores + flags (5M)."""
    tot = 0
    for inst, (blk, _) in zip(insts, moves):
        W = (inst.S + 31) // 32
        tot += 4 * inst.S * inst.N + 4 * W * inst.N + 21 * inst.N + 10 * len(blk)
    return tot


def _gen_batch_member(spec):
    import mpsgen
    inst = mpsgen.make_instance(spec["nx"], spec["ny"], spec["nz"], spec["S"], spec["T"],
                                spec["r"], spec["seed"])
    blk, per = mpsgen.random_moves(inst.N, inst.T, spec["M"], spec["seed"] + 1000)
    return inst, (blk, per)


def batched_leg(steps, k=256):
    """64 models of mixed sizes with 10k-300k random moves each in one
    persistent launch (autotuned), replayed as a HIP graph."""
    import mpsgen
    import torch
    from concurrent.futures import ProcessPoolExecutor
    from paper_2511_18296_amd.binding import Batch, Model
    specs = mpsgen.batched_specs()
    workers = max(1, min(16, os.cpu_count() or 1))
    with ProcessPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(_gen_batch_member, specs))
    insts = [r[0] for r in res]
    moves = [r[1] for r in res]
    models = [Model.from_instance(i) for i in insts]
    dev = [(torch.from_numpy(b).cuda(), torch.from_numpy(p).cuda()) for b, p in moves]
    batch = Batch(models, dev, k)
    tuned_us = batch.autotune(reps=3)
    for _ in range(3):
        batch.graph_launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        batch.graph_launch()
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / steps * 1e-3
    B = batch_bytes(insts, moves)
    evals = sum(len(b) * i.S for i, (b, _) in zip(insts, moves))
    tun = {}
    for i, inst in enumerate(insts):
        tun.setdefault(f"S<={32 if inst.S <= 32 else 64 if inst.S <= 64 else 128 if inst.S <= 128 else 'max'}",
                       batch.tuning(i))
    return {"instances": len(insts), "blocks": int(sum(i.N for i in insts)),
            "moves": int(sum(len(b) for b, _ in moves)), "topk_per_instance": k,
            "us_per_launch": t * 1e6, "autotune_median_us": tuned_us,
            "move_scenario_evals_per_s": evals / t, "algorithmic_bytes": B,
            "achieved_GBs": B / t / 1e9, "frac_of_hbm_peak": B / t / 1e9 / HBM_PEAK_GBS,
            "graph_replays_timed": steps, "tuning": tun}


RELAX = (100.0 / (2 * 15600), 100.0 / (2 * 15600), 100.0 * 15600)


def burst_seconds(fn, n=20):
    """Seconds per call of fn(i), over n back-to-back calls between two HIP
    events on the current stream (after one untimed call)."""
    import torch
    fn(0)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for i in range(n):
        fn(i)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / n * 1e-3


def copy_peak_gbs(mib=256):
    """Device-to-device copy bandwidth (read + write bytes) of two rotating
    pairs of MIB MiB buffers."""
    import torch
    n = mib * (1 << 20) // 4
    bufs = [torch.ones(n, dtype=torch.float32, device="cuda") for _ in range(4)]
    t = burst_seconds(lambda i: bufs[2 * (i % 2) + 1].copy_(bufs[2 * (i % 2)]), 10)
    del bufs
    return 2 * n * 4 / t / 1e9


def kernel_legs(models, inst):
    """The other rows of the path on their own, each timed over a burst of
    back-to-back launches rotating over the copies of the 54,000-block
    instance: the relaxed forward and adjoint, the gradient ranking; and the
    list evaluation of the paper-scale configuration (32,000 blocks, S = 50,
    250,000 random moves), a latency-sized case."""
    import torch
    import mpsgen
    from paper_2511_18296_amd.binding import Model, MoveSet
    N, S, T = inst.N, inst.S, inst.T
    W = (S + 31) // 32
    x = torch.from_numpy(mpsgen.integer_x(inst.p0, T)).cuda()
    saved = [m.relaxed_saved() for m in models]
    J = [torch.empty(6, dtype=torch.float64, device="cuda") for _ in models]
    grads = [torch.empty_like(x) for _ in models]
    nm = len(models)
    t_fwd = burst_seconds(lambda i: models[i % nm].relaxed_fwd(x, RELAX, saved[i % nm], J[i % nm]))
    t_bwd = burst_seconds(
        lambda i: models[i % nm].relaxed_bwd(x, RELAX, saved[i % nm], None, grads[i % nm]))
    t_rank = burst_seconds(lambda i: models[i % nm].rank_moves(grads[i % nm], 4096))
    b_fwd = 4 * S * N + 4 * W * N + 4 * N * T
    b_bwd = 4 * S * N + 4 * W * N + 8 * N * T
    traffic = MEASURED_RELAX_TRAFFIC.get(source_sha(RELAX_SOURCES), {})
    out = {
        "relaxed_fwd": {"us": t_fwd * 1e6, "algorithmic_bytes": b_fwd,
                        "GBs": b_fwd / t_fwd / 1e9, "frac": b_fwd / t_fwd / 1e9 / HBM_PEAK_GBS,
                        "traffic": traffic.get("relaxed_fwd")},
        "relaxed_bwd": {"us": t_bwd * 1e6, "algorithmic_bytes": b_bwd,
                        "GBs": b_bwd / t_bwd / 1e9, "frac": b_bwd / t_bwd / 1e9 / HBM_PEAK_GBS,
                        "traffic": traffic.get("relaxed_bwd")},
        "rank_moves_top4096_us": t_rank * 1e6,
    }
    pinst = mpsgen.paper_scale()
    pm = Model.from_instance(pinst)
    blk, per = mpsgen.random_moves(pinst.N, pinst.T, 250000, 2 + 1000)
    mv = MoveSet(False, True, torch.from_numpy(blk).cuda(), torch.from_numpy(per).cuda())
    sc = torch.empty(250000, dtype=torch.float32, device="cuda")
    fl = torch.empty(250000, dtype=torch.uint8, device="cuda")
    t_list = burst_seconds(lambda i: pm.eval_moves(mv, out=[sc, fl]))
    out["list_eval_paper_scale"] = {"us": t_list * 1e6, "moves": 250000,
                                    "move_scenario_evals_per_s": 250000 * pinst.S / t_list}
    return out


def rows_leg(model, seed_state, inst, k):
    """The rows beyond the plain engine on the 54,000-block instance: the
    greedy initializer, cascading repair over the best moves without the
    precedence requirement, evaluation of all moves under the value
    multiplier and under CVaR10; and the LNS + SA driver on the paper-scale
    instance (32,000 blocks, S = 50, T = 15)."""
    import numpy as np
    import torch
    import mpsgen
    from paper_2511_18296_amd.binding import Model, MoveSet, TopK, NOOP, BAD
    out = {}
    D = inst.T + 1
    M = inst.N * D
    # greedy initializer (synchronising call: host wall time)
    model.restore_state(seed_state)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    passes, placed = model.greedy_init()
    out["greedy_init"] = {"ms": (time.perf_counter() - t0) * 1e3, "passes": passes,
                          "placed": placed, "J": model.objective()["J"]}
    # cascading repair: candidates without the precedence requirement
    model.restore_state(seed_state)
    ex = MoveSet(True, True)
    sc, fl = model.eval_moves(ex)
    tk = TopK(M, k)
    idx, _, cnt = tk(sc, fl, require=0, forbid=NOOP | BAD)
    applied = torch.zeros(1, dtype=torch.int32, device="cuda")

    def casc(i):
        model.restore_state(seed_state)
        model.repair_cascade(ex, idx, cnt, max_set=64, applied=applied)

    t_c = burst_seconds(casc, 3)
    out["cascade_repair"] = {"us": t_c * 1e6, "candidates": k,
                             "applied": int(applied.item()), "max_set": 64}
    # objective variants: all 1,134,000 moves
    model.restore_state(seed_state)
    mult = np.random.default_rng(7).uniform(0.6, 1.4, size=(inst.S, inst.T))
    score = torch.empty(M, dtype=torch.float32, device="cuda")
    flags = torch.empty(M, dtype=torch.uint8, device="cuda")
    for name, mu, risk in (("multiplier", mult, 0), ("cvar10", None, 1),
                           ("multiplier_cvar10", mult, 1)):
        model.set_objective_variant(mu, risk, 0.1)
        t = burst_seconds(lambda i: model.eval_moves(ex, out=[score, flags]), 5)
        out[f"eval_{name}"] = {"us": t * 1e6, "move_scenario_evals_per_s": M * inst.S / t}
    model.set_objective_variant(None, 0)
    model.restore_state(seed_state)
    # LNS + SA on the paper-scale instance
    pinst = mpsgen.paper_scale()
    pm = Model.from_instance(pinst)
    n_iter, tile = 1, 10
    K = ((pinst.nx + tile - 1) // tile) * ((pinst.ny + tile - 1) // tile)
    u = np.random.default_rng(4).random(n_iter * K)
    J0 = pm.objective()["J"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, traj = pm.lns_sa(n_iter, tile, 1024, 8, 1e7, 1e6, 0.9, u)
    dt = time.perf_counter() - t0
    out["lns_sa_paper_scale"] = {"seconds": dt, "steps": st["steps"],
                                 "accepted": st["accepted"],
                                 "moves_evaluated": st["evaluations"],
                                 "moves_per_s": st["evaluations"] / dt,
                                 "applied": st["applied"], "J_start": J0,
                                 "J_best": st["J_best"], "tile": tile, "k": 1024, "rounds": 8}
    return out


def search_leg(model, seed_state, k):
    """Gradient-ranked search vs exhaustive search from the same seeded schedule."""
    import torch
    out = {}
    for name, mode in (("exhaustive", 0), ("gradient_ranked", 1)):
        model.restore_state(seed_state)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = model.search(mode, k, RELAX, max_iter=10000)
        dt = time.perf_counter() - t0
        out[name] = {"J": st["J"], "iterations": int(st["iterations"]),
                     "exact_evaluations": int(st["evaluations"]),
                     "applied": int(st["applied"]), "seconds": dt}
    JE, JG = out["exhaustive"]["J"], out["gradient_ranked"]["J"]
    out["rel_diff"] = abs(JG - JE) / abs(JE)
    # Both loops stop at a schedule that an exhaustive round cannot improve,
    # i.e. at a local optimum of the same neighbourhood; which one depends on
    # the order of the applied moves.  The exhaustive loop alone, run with a
    # different list length, shows how far apart such end points lie.
    spread = {}
    for kk in (k // 2, 2 * k):
        model.restore_state(seed_state)
        st = model.search(0, kk, RELAX, max_iter=10000)
        spread[str(kk)] = {"J": st["J"], "rel_diff_to_exhaustive": abs(st["J"] - JE) / abs(JE),
                           "iterations": int(st["iterations"])}
    out["exhaustive_other_k"] = spread
    out["relax_weights"] = list(RELAX)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--no-rows", action="store_true", help="skip the next-row legs")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--copies", type=int, default=8)
    ap.add_argument("--k", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-search", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before the steps, copy a device buffer of MIB MiB three times "
                         "(the reference kernel for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the engine runs on a single MI355X; multi-GPU sharding is not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import mpsgen
    from paper_2511_18296_amd.binding import Model, MoveSet, TopK

    torch.cuda.set_device(0)
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {args.copy_calibration} MiB")
        del src, dst
    log("generating the 54,000-block instance ...")
    inst = mpsgen.largest_plain()
    N, S, T = inst.N, inst.S, inst.T
    D = T + 1
    M = N * D
    models = [Model.from_instance(inst) for _ in range(args.copies)]
    seeds = [m.save_state() for m in models]
    score = torch.empty(M, dtype=torch.float32, device="cuda")
    flags = torch.empty(M, dtype=torch.uint8, device="cuda")
    tk = TopK(M, args.k)
    applied = torch.zeros(args.copies, dtype=torch.int32, device="cuda")
    ex = MoveSet(True, True)

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)]
          for _ in range(args.steps)]

    def step(i, events=None):
        r = i % args.copies
        m = models[r]
        if events:
            events[4].record()
        m.restore_state(seeds[r])
        if events:
            events[0].record()
        m.eval_moves(ex, out=[score, flags])
        if events:
            events[1].record()
        tk(score, flags)
        if events:
            events[2].record()
        m.repair(ex, tk.idx, tk.count, applied=applied[r:r + 1])
        if events:
            events[3].record()

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps); {args.steps} eager steps with phase events")
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i, ev[i])
    torch.cuda.synchronize()
    wall_eager = time.perf_counter() - t0
    # every copy's eager result (a step restores its copy's seed, so one
    # more step of each copy gives it, also for copies the timed steps missed)
    for r in range(args.copies):
        step(r)
    torch.cuda.synchronize()
    eager_J = [m.objective()["J"] for m in models]

    t_rest = sum(e[4].elapsed_time(e[0]) for e in ev) / args.steps * 1e-3
    t_eval = sum(e[0].elapsed_time(e[1]) for e in ev) / args.steps * 1e-3
    t_topk = sum(e[1].elapsed_time(e[2]) for e in ev) / args.steps * 1e-3
    t_rep = sum(e[2].elapsed_time(e[3]) for e in ev) / args.steps * 1e-3

    # The timed steps: each step captured once per instance copy as a HIP
    # graph (restore, evaluation, top-k, repair) and replayed; every replay
    # must end at the eager result.
    graphs = []
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        for r in range(args.copies):
            step(r)   # warm the capture stream
    torch.cuda.current_stream().wait_stream(cap)
    torch.cuda.synchronize()
    for r in range(args.copies):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=cap):
            step(r)
        graphs.append(g)
    for r in range(args.copies):
        graphs[r].replay()
    torch.cuda.synchronize()
    for r, m in enumerate(models):
        assert m.objective()["J"] == eager_J[r], "graph replay differs from the eager step"
    log(f"timing {args.steps} graph-replayed steps")
    gev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        gev[i][0].record()
        graphs[i % args.copies].replay()
        gev[i][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for r, m in enumerate(models):
        assert m.objective()["J"] == eager_J[r], "graph replay differs from the eager step"
    per_step = sorted(a.elapsed_time(b) * 1e-3 for a, b in gev)

    def pct(xs, q):
        return xs[min(len(xs) - 1, int(round(q * (len(xs) - 1))))]

    ms = wall / args.steps * 1e3
    value = M * S * args.steps / wall
    B = eval_bytes(N, S, T, D)
    # The evaluation kernel's duration for the roofline: a burst of
    # back-to-back launches (rotating over the copies) between two events on
    # the launch stream.  An event pair around a single launch also times the
    # two event markers, about 5 us.
    burst = 20
    ea = torch.cuda.Event(enable_timing=True)
    eb = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ea.record()
    for i in range(burst):
        models[i % args.copies].eval_moves(ex, out=[score, flags])
    eb.record()
    torch.cuda.synchronize()
    t_eval_kernel = ea.elapsed_time(eb) / burst * 1e-3
    achieved = B / t_eval_kernel / 1e9
    objs = [m.objective() for m in models]
    n_applied = [int(a) for a in applied.cpu().tolist()]
    copy_gbs = copy_peak_gbs()
    legs = kernel_legs(models, inst)
    log(f"legs: {json.dumps(legs)}")
    log(f"restore {t_rest*1e6:.1f} us, eval {t_eval*1e6:.1f} us, topk {t_topk*1e6:.1f} us, "
        f"repair {t_rep*1e6:.1f} us, "
        f"step {ms:.3f} ms; eval kernel {t_eval_kernel*1e6:.1f} us in a burst of {burst}")

    out = {
        "metric": "move-scenario evals/s at 54k blocks,S=200; HBM GB/s; "
                  "grad-ranked vs exhaustive",
        "value": value,
        "unit": "move-scenario evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "largest plain: 60x60x15 = 54,000 blocks, T=20, S=200, "
                               "exhaustive 1,134,000 moves, top-4096, greedy repair "
                               "(first search iteration from the seeded schedule)",
                   "blocks": N, "scenarios": S, "periods": T, "moves": M, "topk": args.k,
                   "copies_rotated": args.copies},
        "roofline": {"kernel": "k_eval_exh", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": MEASURED_TRAFFIC.get(eval_source_sha()),
                     "bytes_per_launch": B, "launch_us": t_eval_kernel * 1e6,
                     "timing": f"{burst} back-to-back launches between two HIP events",
                     "measured_copy_GBs": copy_gbs, "frac_of_measured_copy": achieved / copy_gbs,
                     "source_sha1": eval_source_sha()},
        "timing": {"value": f"{args.steps} graph-replayed steps between two host "
                            "synchronisations (wall clock)",
                   "step_us_median": pct(per_step, 0.5) * 1e6,
                   "step_us_p10": pct(per_step, 0.1) * 1e6,
                   "step_us_p90": pct(per_step, 0.9) * 1e6,
                   "per_step_events": f"event pair around each of the {args.steps} replays",
                   "eager_ms_per_step": wall_eager / args.steps * 1e3},
        "phases_us": {"restore": t_rest * 1e6, "eval": t_eval * 1e6, "topk": t_topk * 1e6,
                      "repair": t_rep * 1e6,
                      "method": "eager steps, events between the phases (each includes "
                                "its event markers)"},
        "eval_move_scenario_evals_per_s": M * S / t_eval_kernel,
        "repair": {"applied_per_step": n_applied[0],
                   "us_per_applied_move": t_rep * 1e6 / max(1, n_applied[0]),
                   "us_per_candidate": t_rep * 1e6 / args.k},
        "legs": legs,
        "final_J": [o["J"] for o in objs],
    }
    if not args.no_rows:
        log("rows: greedy, cascade, variants, LNS ...")
        out["rows"] = rows_leg(models[0], seeds[0], inst, args.k)
        log(f"rows: {json.dumps(out['rows'])}")
    if not args.no_search:
        log("search comparison (exhaustive vs gradient-ranked) ...")
        out["search"] = search_leg(models[0], seeds[0], args.k)
        log(f"search: {json.dumps(out['search'])}")
    del models, seeds
    torch.cuda.empty_cache()
    if not args.no_batched:
        log("batched: generating 64 instances ...")
        out["batched"] = batched_leg(20)
        log(f"batched: {json.dumps(out['batched'])}")
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(inst, args.k)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
