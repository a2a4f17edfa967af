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
timed with events on the stream it runs on.
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def eval_bytes(N, S, T, D):
    """Algorithmic HBM bytes of one exhaustive evaluation: v (4SN), ore words
    (4*ceil(S/32)*N), per-block mean and variance (8N), tonnage (4N),
    schedule (N), score + flags (5*N*D)."""
    W = (S + 31) // 32
    return 4 * S * N + 4 * W * N + 8 * N + 4 * N + N + 5 * N * D


def cpu_baseline(inst, k):
    """The FP64 oracle on the host: one full step of the same workload."""
    import numpy as np
    import oracle
    o = oracle.Oracle(inst)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    D = inst.T + 1
    t0 = time.perf_counter()
    sc, fl = o.eval_moves(inst.p0, include_never=True, threads=threads)
    idx, _ = oracle.topk(sc, fl, k)
    o.repair(inst.p0, (idx // D).astype(np.int32), (idx % D).astype(np.int8))
    dt = time.perf_counter() - t0
    n = inst.N * D
    return {"value": n * inst.S / dt, "unit": "move-scenario evals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"one full step (eval of all {n:,} moves x {inst.S} scenarios, "
                      f"top-{k}, repair) of the same instance, {dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--copies", type=int, default=8)
    ap.add_argument("--k", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the engine runs on a single MI355X; see DESIGN.md for sharding)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import mpsgen
    from paper_2511_18296_amd.binding import Model, MoveSet, TopK

    torch.cuda.set_device(0)
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
    log(f"warmup done ({args.warmup} steps); timing {args.steps} steps")
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i, ev[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    t_rest = sum(e[4].elapsed_time(e[0]) for e in ev) / args.steps * 1e-3
    t_eval = sum(e[0].elapsed_time(e[1]) for e in ev) / args.steps * 1e-3
    t_topk = sum(e[1].elapsed_time(e[2]) for e in ev) / args.steps * 1e-3
    t_rep = sum(e[2].elapsed_time(e[3]) for e in ev) / args.steps * 1e-3
    ms = wall / args.steps * 1e3
    value = M * S * args.steps / wall
    B = eval_bytes(N, S, T, D)
    achieved = B / t_eval / 1e9
    objs = [m.objective() for m in models]
    log(f"restore {t_rest*1e6:.1f} us, eval {t_eval*1e6:.1f} us, topk {t_topk*1e6:.1f} us, "
        f"repair {t_rep*1e6:.1f} us, "
        f"step {ms:.3f} ms")

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
                     "traffic": None, "bytes_per_launch": B},
        "phases_us": {"restore": t_rest * 1e6, "eval": t_eval * 1e6, "topk": t_topk * 1e6,
                      "repair": t_rep * 1e6},
        "eval_move_scenario_evals_per_s": M * S / t_eval,
        "final_J": [o["J"] for o in objs],
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(inst, args.k)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
