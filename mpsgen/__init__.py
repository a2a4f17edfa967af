"""Seeded synthetic instances for the candidate-move evaluation engine.

This module produces INPUTS only: a 3-D block grid, per-scenario grades and
block values, ore indicators, tonnages, capacities, a precedence-feasible
starting schedule, random candidate moves and relaxed schedules.  It holds
none of the evaluation arithmetic (no discounting, no NPV, no risk measure,
no penalties, no move scoring); both the FP64 oracle and the HIP library
consume what it returns.

The workloads stand in for the paper's block models, whose source deposit
data is not available (Sec. 7; block size 20 x 20 x 15 m, 50-200+ geological
scenarios, lognormal grade shocks as in Sec. 7.1.3).  The recipe:

* grid nx x ny x nz, block index b = x + nx*(y + ny*z), z = 0 is the top bench;
* grade field per scenario: i.i.d. N(0,1) noise smoothed along x, y and z by
  the kernel w(k) = exp(-|k|/r), |k| <= floor(3r), zero padding, each axis
  pass divided by sqrt(sum of the in-bounds w(k)^2) so every block has unit
  variance; grade g = exp(ln 0.8 + 0.6 z) g/t, stored as float32;
* tonnage 15,600 t per block (20*20*15 m^3 at 2.6 t/m^3);
* block value (float32 arithmetic, evaluated left to right):
  margin = g*0.9*60 - 20 ($/t), v = max(ton*margin, 0) - ton*3, and
  ore = [margin > 0] (the block is processed iff its margin is positive);
* processing capacity = (mean over scenarios of the total ore tonnage) / T,
  mining capacity = 1.1 * (total tonnage) / T;
* starting schedule: u_b = min(T, floor(T*(z_b + xi_b)/(nz + 1))), xi ~ U[0,1),
  then top-down p_b = max(u_b, p of the five blocks of the bench above that
  sit directly over b or share a face with that block), which makes it
  precedence-feasible by construction.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.ndimage import correlate1d

TONNAGE = 15600.0
PRICE = 60.0        # $ per gram of metal
RECOVERY = 0.9
PROC_COST = 20.0    # $ per processed tonne
MINE_COST = 3.0     # $ per mined tonne
GRADE_MEDIAN = 0.8  # g/t
GRADE_LOGSD = 0.6


@dataclass
class Instance:
    nx: int
    ny: int
    nz: int
    S: int
    T: int
    grade: np.ndarray        # float32 [S][N]
    v: np.ndarray            # float32 [S][N]
    ore: np.ndarray          # uint8   [S][N] (0/1)
    ton: np.ndarray          # float64 [N]
    p0: np.ndarray           # int8    [N], 0..T (T = never mined)
    pcap: float
    mcap: float
    rate: float = 0.08
    lam: float = 0.5
    pen_proc: float = 100.0
    pen_mine: float = 100.0
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def W(self) -> int:
        return (self.S + 31) // 32


def _smooth_axis(a: np.ndarray, axis: int, r: float) -> np.ndarray:
    K = int(math.floor(3.0 * r))
    k = np.arange(-K, K + 1, dtype=np.float64)
    w = np.exp(-np.abs(k) / r)
    out = correlate1d(a, w, axis=axis, mode="constant", cval=0.0)
    n = a.shape[axis]
    ones = np.ones(n, dtype=np.float64)
    norm = np.sqrt(correlate1d(ones, w * w, mode="constant", cval=0.0))
    shape = [1] * a.ndim
    shape[axis] = n
    return out / norm.reshape(shape)


def grade_field(nx, ny, nz, S, r, rng) -> np.ndarray:
    """Unit-variance smoothed Gaussian field -> lognormal grades, float32 [S][N]."""
    z = rng.standard_normal((S, nz, ny, nx))
    for axis in (3, 2, 1):          # x, y, z
        z = _smooth_axis(z, axis, r)
    g = np.exp(math.log(GRADE_MEDIAN) + GRADE_LOGSD * z)
    return g.reshape(S, nx * ny * nz).astype(np.float32)


def block_values(grade: np.ndarray, ton: np.ndarray):
    """float32 block values and ore indicators from grades (input recipe)."""
    t32 = ton.astype(np.float32)[None, :]
    margin = grade * np.float32(RECOVERY) * np.float32(PRICE) - np.float32(PROC_COST)
    v = np.maximum(t32 * margin, np.float32(0.0)) - t32 * np.float32(MINE_COST)
    ore = (margin > np.float32(0.0)).astype(np.uint8)
    return v.astype(np.float32), ore


def feasible_schedule(nx, ny, nz, T, rng) -> np.ndarray:
    """Seeded precedence-feasible schedule (top-down max over the 1-5 stencil)."""
    xi = rng.random((nz, ny, nx))
    zz = np.arange(nz, dtype=np.float64)[:, None, None]
    u = np.minimum(T, np.floor(T * (zz + xi) / (nz + 1))).astype(np.int64)
    p = u.copy()
    for z in range(1, nz):
        above = p[z - 1]
        m = above.copy()
        m[:, 1:] = np.maximum(m[:, 1:], above[:, :-1])
        m[:, :-1] = np.maximum(m[:, :-1], above[:, 1:])
        m[1:, :] = np.maximum(m[1:, :], above[:-1, :])
        m[:-1, :] = np.maximum(m[:-1, :], above[1:, :])
        p[z] = np.maximum(p[z], m)
    return p.reshape(-1).astype(np.int8)


def make_instance(nx, ny, nz, S, T, r, seed, *, rate=0.08, lam=0.5,
                  pen_proc=100.0, pen_mine=100.0, ton=None) -> Instance:
    rng = np.random.default_rng(seed)
    N = nx * ny * nz
    grade = grade_field(nx, ny, nz, S, r, rng)
    if ton is None:
        ton = np.full(N, TONNAGE, dtype=np.float64)
    ton = np.asarray(ton, dtype=np.float64)
    v, ore = block_values(grade, ton)
    p0 = feasible_schedule(nx, ny, nz, T, rng)
    ore_tonnage = (ore.astype(np.float64) * ton[None, :]).sum(axis=1)   # per scenario
    pcap = float(ore_tonnage.mean() / T)
    mcap = float(1.1 * ton.sum() / T)
    return Instance(nx, ny, nz, S, T, grade, v, ore, ton, p0, pcap, mcap,
                    rate, lam, pen_proc, pen_mine, seed, {"r": r})


def ore_pack(ore: np.ndarray) -> np.ndarray:
    """Pack ore indicators [S][N] into uint32 words [ceil(S/32)][N];
    scenario s is bit (s % 32) of word s // 32."""
    S, N = ore.shape
    W = (S + 31) // 32
    out = np.zeros((W, N), dtype=np.uint64)
    for s in range(S):
        out[s // 32] |= ore[s].astype(np.uint64) << np.uint64(s % 32)
    return out.astype(np.uint32)


def random_moves(N, T, M, seed):
    """M uniform candidate moves: block in [0, N), destination in {0..T}."""
    rng = np.random.default_rng(seed)
    block = rng.integers(0, N, size=M, dtype=np.int64).astype(np.int32)
    period = rng.integers(0, T + 1, size=M, dtype=np.int64).astype(np.int8)
    return block, period


def random_monotone_x(N, T, seed) -> np.ndarray:
    """Relaxed cumulative schedule: per block, sorted U[0,1) draws (float32 [N][T])."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.random((N, T)), axis=1).astype(np.float32)


def integer_x(p: np.ndarray, T: int) -> np.ndarray:
    """x[b,t] = [t >= p_b] as float32 [N][T] (the integer point of a schedule)."""
    t = np.arange(T)[None, :]
    return (t >= p.astype(np.int64)[:, None]).astype(np.float32)


# --- the workloads -----------------------------------------------------------

def tiny_plain(seed=1):
    """10x10x5 = 500 blocks, T=5, S=10, range 3."""
    return make_instance(10, 10, 5, 10, 5, 3.0, seed)


def paper_scale(seed=2):
    """40x40x20 = 32,000 blocks, T=15, S=50, range 5 (+250,000 random moves)."""
    return make_instance(40, 40, 20, 50, 15, 5.0, seed)


def largest_plain(seed=3):
    """60x60x15 = 54,000 blocks, T=20, S=200, range 6 (exhaustive moves)."""
    return make_instance(60, 60, 15, 200, 20, 6.0, seed)


def batched_specs(n_inst=64, seed=4):
    """Sizes of the batched workload: N ~ U[2000, 54000], depth ~ U{5..15},
    nx = ny = round(sqrt(N/depth)), T ~ U{5..20}, S ~ U{20..200},
    moves ~ U[10k, 300k]; instance i is generated from seed 400 + i."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n_inst):
        N = int(rng.integers(2000, 54001))
        depth = int(rng.integers(5, 16))
        side = max(2, int(round(math.sqrt(N / depth))))
        T = int(rng.integers(5, 21))
        S = int(rng.integers(20, 201))
        M = int(rng.integers(10000, 300001))
        n_real = side * side * depth
        r = 3.0 + math.floor(3.0 * n_real / 54000.0)
        specs.append(dict(nx=side, ny=side, nz=depth, S=S, T=T, r=r, M=M,
                          seed=400 + i))
    return specs


def batch_member(spec):
    """One instance of the batched workload and its random move list
    (seed + 1000), from a spec as batched_specs() returns."""
    inst = make_instance(spec["nx"], spec["ny"], spec["nz"], spec["S"], spec["T"],
                         spec["r"], spec["seed"])
    blk, per = random_moves(inst.N, inst.T, spec["M"], spec["seed"] + 1000)
    return inst, (blk, per)


def batch_members(specs, workers=16):
    """batch_member of every spec, generated in a pool of worker processes."""
    import os
    from concurrent.futures import ProcessPoolExecutor
    workers = max(1, min(workers, os.cpu_count() or 1, len(specs)))
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(batch_member, specs))


def cone_precedence(nx, ny, nz, reach=1):
    """Explicit predecessor lists of a square slope cone: the predecessors of
    block (x, y, z) are the blocks (x + dx, y + dy, z - 1) with |dx|, |dy| <=
    reach inside the grid (reach 1: the 1-9 pattern).  Returns (pred_ptr
    int32 [N+1], pred_idx int32), each list in increasing block index."""
    N = nx * ny * nz
    ptr = np.zeros(N + 1, dtype=np.int32)
    idx = []
    for b in range(N):
        x, y, z = b % nx, (b // nx) % ny, b // (nx * ny)
        lst = []
        if z > 0:
            for dy in range(-reach, reach + 1):
                for dx in range(-reach, reach + 1):
                    xa, ya = x + dx, y + dy
                    if 0 <= xa < nx and 0 <= ya < ny:
                        lst.append(xa + nx * (ya + ny * (z - 1)))
        lst.sort()
        idx.extend(lst)
        ptr[b + 1] = len(idx)
    return ptr, np.asarray(idx, dtype=np.int32)


def stencil_precedence(nx, ny, nz):
    """The 1-5 slope stencil written out as explicit predecessor lists (the
    block right above and its four face neighbours, one bench up)."""
    N = nx * ny * nz
    ptr = np.zeros(N + 1, dtype=np.int32)
    idx = []
    for b in range(N):
        x, y, z = b % nx, (b // nx) % ny, b // (nx * ny)
        lst = []
        if z > 0:
            for dx, dy in ((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)):
                xa, ya = x + dx, y + dy
                if 0 <= xa < nx and 0 <= ya < ny:
                    lst.append(xa + nx * (ya + ny * (z - 1)))
        lst.sort()
        idx.extend(lst)
        ptr[b + 1] = len(idx)
    return ptr, np.asarray(idx, dtype=np.int32)


def feasible_schedule_lists(N, T, pred_ptr, pred_idx, seed):
    """Seeded schedule feasible under explicit predecessor lists whose
    predecessors all have smaller indices: u_b uniform on 0..T, then in index
    order p_b = max(u_b, p of every predecessor)."""
    rng = np.random.default_rng(seed)
    u = rng.integers(0, T + 1, size=N)
    p = np.zeros(N, dtype=np.int64)
    for b in range(N):
        lo = 0
        for k in range(pred_ptr[b], pred_ptr[b + 1]):
            a = pred_idx[k]
            assert a < b
            lo = max(lo, p[a])
        p[b] = max(u[b], lo)
    return p.astype(np.int8)


def with_precedence(inst, pred_ptr, pred_idx, p0=None):
    """The instance with explicit predecessor lists (and optionally another
    starting schedule)."""
    import copy
    out = copy.copy(inst)
    out.pred_ptr = np.asarray(pred_ptr, dtype=np.int32)
    out.pred_idx = np.asarray(pred_idx, dtype=np.int32)
    if p0 is not None:
        out.p0 = np.asarray(p0, dtype=np.int8)
    return out

