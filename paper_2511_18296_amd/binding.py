"""ctypes binding of libmps (include/mps.h): argument marshalling only.

Every computation runs in the HIP library; torch supplies device memory and
the current stream.  Importing this module loads libmps.so and raises if it
is missing, so a missing build can never fall back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmps.so")

PREC_OK, MINE_OK, PROC_OK, NOOP, BAD = 1, 2, 4, 8, 16
MAX_PERIODS, MAX_SCENARIOS, MAX_TOPK = 126, 4096, 8192
MAX_BATCH_TOPK, MAX_BATCH = 1024, 4096
MAX_REPAIR_SCENARIOS = 1024

STATUS = {0: "MPS_OK", 1: "MPS_E_INVALID_ARG", 2: "MPS_E_OUT_OF_MEMORY",
          3: "MPS_E_DEVICE", 4: "MPS_E_INFEASIBLE", 5: "MPS_E_NOT_CAPTURABLE",
          6: "MPS_E_INTERNAL"}


class MpsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("n_scen", C.c_int32), ("n_periods", C.c_int32),
                ("precedence", C.c_int32), ("discount_rate", C.c_double),
                ("lam", C.c_double), ("pen_proc", C.c_double),
                ("pen_mine", C.c_double), ("proc_cap", C.c_double),
                ("mine_cap", C.c_double)]


class Objective(C.Structure):
    _fields_ = [("mu", C.c_double), ("sigma", C.c_double), ("R", C.c_double),
                ("Pp", C.c_double), ("Pm", C.c_double), ("J", C.c_double),
                ("n_prec_viol", C.c_int64)]


class Moves(C.Structure):
    _fields_ = [("exhaustive", C.c_int32), ("include_never", C.c_int32),
                ("n", C.c_int64), ("block", C.c_void_p), ("period", C.c_void_p)]


class RelaxParams(C.Structure):
    _fields_ = [("mu_proc", C.c_double), ("mu_mine", C.c_double),
                ("mu_prec", C.c_double)]


class SearchStats(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("evaluations", C.c_int64),
                ("applied", C.c_int64), ("J", C.c_double)]


class LnsParams(C.Structure):
    _fields_ = [("n_iter", C.c_int32), ("tile", C.c_int32), ("k", C.c_int32),
                ("max_rounds", C.c_int32), ("eps_max", C.c_double), ("temp0", C.c_double),
                ("cool", C.c_double)]


class LnsStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("accepted", C.c_int64), ("evaluations", C.c_int64),
                ("applied", C.c_int64), ("J_best", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("tiles_per_item", C.c_int32), ("moves_per_item", C.c_int32),
                ("rows", C.c_int32), ("reserved", C.c_int32)]


class BatchItem(C.Structure):
    _fields_ = [("block", C.c_void_p), ("period", C.c_void_p), ("n", C.c_int64),
                ("score", C.c_void_p), ("flags", C.c_void_p), ("top_idx", C.c_void_p),
                ("top_score", C.c_void_p), ("top_count", C.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "or python paper_2511_18296_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, st = C.c_void_p, C.c_int32, C.c_int64, C.c_int
    sigs = {
        "mps_last_error": ([], C.c_char_p),
        "mps_version": ([], i32),
        "mps_device_count": ([vp], st),
        "mps_build_model": ([vp, vp, vp, vp, vp, vp, vp, vp], st),
        "mps_destroy_model": ([vp], st),
        "mps_model_dims": ([vp, vp, vp, vp], st),
        "mps_set_schedule": ([vp, vp, vp], st),
        "mps_get_schedule": ([vp, vp, vp], st),
        "mps_get_objective": ([vp, vp, vp], st),
        "mps_objective_async": ([vp, vp, vp], st),
        "mps_eval_moves": ([vp, vp, vp, vp, vp, vp, vp, vp], st),
        "mps_topk_ws_bytes": ([i64, i32], C.c_size_t),
        "mps_topk": ([vp, vp, i64, i32, C.c_uint8, C.c_uint8, vp, vp, vp, vp,
                      C.c_size_t, vp], st),
        "mps_topk_noalloc": ([vp, vp, i64, i32, C.c_uint8, C.c_uint8, vp, vp, vp, vp], st),
        "mps_repair": ([vp, vp, vp, vp, i32, i32, vp, vp], st),
        "mps_repair_cascade": ([vp, vp, vp, vp, i32, i32, i32, vp, vp], st),
        "mps_relaxed_saved_bytes": ([vp], C.c_size_t),
        "mps_relaxed_fwd": ([vp, vp, vp, vp, vp, vp], st),
        "mps_relaxed_bwd": ([vp, vp, vp, vp, vp, vp, vp], st),
        "mps_rank_ws_bytes": ([vp, i32], C.c_size_t),
        "mps_rank_moves": ([vp, vp, i32, vp, vp, vp, vp, vp, C.c_size_t, vp], st),
        "mps_search": ([vp, i32, i32, vp, i32, vp, vp], st),
        "mps_greedy_init": ([vp, i32, vp, vp, vp], st),
        "mps_lns_sa": ([vp, vp, vp, vp, vp, vp], st),
        "mps_set_objective_variant": ([vp, vp, i32, C.c_double, vp], st),
        "mps_state_bytes": ([vp], C.c_size_t),
        "mps_state_save": ([vp, vp, vp], st),
        "mps_state_restore": ([vp, vp, vp], st),
        "mps_batch_create": ([vp, vp, i32, i32, C.c_uint8, C.c_uint8, vp], st),
        "mps_batch_destroy": ([vp], st),
        "mps_batch_set_tuning": ([vp, i32, vp], st),
        "mps_batch_get_tuning": ([vp, i32, vp], st),
        "mps_batch_set_workgroups": ([vp, i32], st),
        "mps_batch_run": ([vp, vp], st),
        "mps_batch_graph_launch": ([vp, vp], st),
        "mps_batch_autotune": ([vp, i32, vp, vp], st),
    }
    for name, (args, res) in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


lib = _load()

# every symbol include/mps.h declares (checked by the CPU tests)
EXPORTS = ("mps_last_error", "mps_version", "mps_device_count", "mps_build_model",
           "mps_destroy_model", "mps_model_dims", "mps_set_schedule",
           "mps_get_schedule", "mps_get_objective", "mps_objective_async",
           "mps_eval_moves", "mps_topk_ws_bytes", "mps_topk", "mps_topk_noalloc", "mps_repair",
           "mps_repair_cascade",
           "mps_relaxed_saved_bytes", "mps_relaxed_fwd", "mps_relaxed_bwd",
           "mps_rank_ws_bytes", "mps_rank_moves", "mps_search", "mps_greedy_init",
           "mps_set_objective_variant", "mps_lns_sa",
           "mps_state_bytes",
           "mps_state_save", "mps_state_restore", "mps_batch_create", "mps_batch_destroy",
           "mps_batch_set_tuning", "mps_batch_get_tuning", "mps_batch_set_workgroups",
           "mps_batch_run", "mps_batch_graph_launch", "mps_batch_autotune")


def check(status: int):
    if status != 0:
        raise MpsError(status, lib.mps_last_error().decode())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t, dtype, shape=None, name="array"):
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def device_count() -> int:
    n = C.c_int32(0)
    lib.mps_device_count(C.byref(n))
    return n.value


@dataclass
class MoveSet:
    """Exhaustive (all b*D + t') or an explicit list of (block, period)."""
    exhaustive: bool = True
    include_never: bool = True
    block: torch.Tensor | None = None
    period: torch.Tensor | None = None

    def c(self) -> Moves:
        if self.exhaustive:
            return Moves(1, int(self.include_never), 0, None, None)
        n = int(self.block.shape[0])
        return Moves(0, int(self.include_never), n, self.block.data_ptr() if n else None,
                     self.period.data_ptr() if n else None)


class Model:
    """A block model on the GPU (mps_build_model) with its current schedule."""

    def __init__(self, nx, ny, nz, S, T, v, ore_words, ton, *, rate=0.08, lam=0.5,
                 pen_proc=100.0, pen_mine=100.0, proc_cap, mine_cap, pred_ptr=None,
                 pred_idx=None, stream=None):
        N = nx * ny * nz
        W = (S + 31) // 32
        _dev(v, torch.float32, (S, N), "v")
        _dev(ore_words, torch.int32, (W, N), "ore_words")
        _dev(ton, torch.float64, (N,), "ton")
        csr = pred_ptr is not None
        lists = [None, None]
        if csr:
            # host arrays, read during the build
            self._pred = (np.ascontiguousarray(pred_ptr, dtype=np.int32),
                          np.ascontiguousarray(pred_idx, dtype=np.int32))
            lists = [a.ctypes.data_as(C.c_void_p) for a in self._pred]
        self.prm = Params(nx, ny, nz, S, T, 1 if csr else 0, rate, lam, pen_proc, pen_mine,
                          proc_cap, mine_cap)
        self.N, self.S, self.T, self.W = N, S, T, W
        self.device = v.device
        h = C.c_void_p()
        check(lib.mps_build_model(C.byref(self.prm), _ptr(v), _ptr(ore_words),
                                  _ptr(ton), lists[0], lists[1], _stream(stream), C.byref(h)))
        self.h = h
        self._objbuf = torch.empty(8, dtype=torch.float64, device=self.device)

    @classmethod
    def from_instance(cls, inst, device="cuda", stream=None):
        """Build from a generated instance (numpy arrays copied to the GPU);
        explicit predecessor lists (pred_ptr, pred_idx) when it carries them."""
        import mpsgen
        v = torch.from_numpy(np.ascontiguousarray(inst.v)).to(device)
        words = mpsgen.ore_pack(inst.ore).view(np.int32)
        ore = torch.from_numpy(np.ascontiguousarray(words)).to(device)
        ton = torch.from_numpy(np.ascontiguousarray(inst.ton, dtype=np.float64)).to(device)
        m = cls(inst.nx, inst.ny, inst.nz, inst.S, inst.T, v, ore, ton, rate=inst.rate,
                lam=inst.lam, pen_proc=inst.pen_proc, pen_mine=inst.pen_mine,
                proc_cap=inst.pcap, mine_cap=inst.mcap,
                pred_ptr=getattr(inst, "pred_ptr", None),
                pred_idx=getattr(inst, "pred_idx", None), stream=stream)
        p = torch.from_numpy(np.ascontiguousarray(inst.p0, dtype=np.int8)).to(device)
        m.set_schedule(p, stream)
        return m

    def close(self):
        if getattr(self, "h", None):
            check(lib.mps_destroy_model(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def n_moves(self, moves: MoveSet) -> int:
        if moves.exhaustive:
            return self.N * (self.T + 1 if moves.include_never else self.T)
        return int(moves.block.shape[0])

    def set_schedule(self, p, stream=None):
        _dev(p, torch.int8, (self.N,), "p")
        check(lib.mps_set_schedule(self.h, _ptr(p), _stream(stream)))

    def get_schedule(self, out=None, stream=None):
        if out is None:
            out = torch.empty(self.N, dtype=torch.int8, device=self.device)
        check(lib.mps_get_schedule(self.h, _ptr(out), _stream(stream)))
        return out

    def save_state(self, buf=None, stream=None):
        """Checkpoint of the search state (device uint8 tensor)."""
        n = int(lib.mps_state_bytes(self.h))
        if buf is None:
            buf = torch.empty(n, dtype=torch.uint8, device=self.device)
        check(lib.mps_state_save(self.h, _ptr(buf), _stream(stream)))
        return buf

    def restore_state(self, buf, stream=None):
        check(lib.mps_state_restore(self.h, _ptr(buf), _stream(stream)))

    def objective(self, stream=None) -> dict:
        o = Objective()
        check(lib.mps_get_objective(self.h, C.byref(o), _stream(stream)))
        return dict(mu=o.mu, sigma=o.sigma, R=o.R, Pp=o.Pp, Pm=o.Pm, J=o.J,
                    n_prec_viol=int(o.n_prec_viol))

    def objective_async(self, out=None, stream=None):
        out = self._objbuf if out is None else out
        check(lib.mps_objective_async(self.h, _ptr(out), _stream(stream)))
        return out

    def eval_moves(self, moves: MoveSet | None = None, *, components=False, out=None,
                   stream=None):
        moves = moves or MoveSet()
        if not moves.exhaustive:
            _dev(moves.block, torch.int32, None, "block")
            _dev(moves.period, torch.int8, moves.block.shape, "period")
        n = self.n_moves(moves)
        if out is None:
            out = [torch.empty(n, dtype=torch.float32, device=self.device),
                   torch.empty(n, dtype=torch.uint8, device=self.device)]
            if components:
                out += [torch.empty(n, dtype=torch.float32, device=self.device)
                        for _ in range(3)]
        comp = out[2:5] if components else [None, None, None]
        mv = moves.c()
        check(lib.mps_eval_moves(self.h, C.byref(mv), _ptr(out[0]), _ptr(out[1]),
                                 *[_ptr(t) for t in comp], _stream(stream)))
        return tuple(out)

    def repair(self, moves: MoveSet, idx, count, max_cand=None, hard=False, applied=None,
               stream=None):
        max_cand = int(idx.shape[0]) if max_cand is None else max_cand
        if applied is None:
            applied = torch.zeros(1, dtype=torch.int32, device=self.device)
        mv = moves.c()
        check(lib.mps_repair(self.h, C.byref(mv), _ptr(idx), _ptr(count), int(max_cand),
                             int(bool(hard)), _ptr(applied), _stream(stream)))
        return applied

    def repair_cascade(self, moves: MoveSet, idx, count, max_cand=None, hard=False,
                       max_set=64, applied=None, stream=None):
        """Cascading repair (mps_repair_cascade) over the same kind of list."""
        max_cand = int(idx.shape[0]) if max_cand is None else max_cand
        if applied is None:
            applied = torch.zeros(1, dtype=torch.int32, device=self.device)
        mv = moves.c()
        check(lib.mps_repair_cascade(self.h, C.byref(mv), _ptr(idx), _ptr(count),
                                     int(max_cand), int(bool(hard)), int(max_set),
                                     _ptr(applied), _stream(stream)))
        return applied


    # ---- relaxed objective -------------------------------------------------
    def relaxed_saved(self):
        n = int(lib.mps_relaxed_saved_bytes(self.h))
        return torch.empty(n, dtype=torch.uint8, device=self.device)

    def relaxed_fwd(self, x, relax, saved, J_out=None, stream=None):
        _dev(x, torch.float32, (self.N, self.T), "x")
        rp = RelaxParams(*relax)
        if J_out is None:
            J_out = torch.empty(6, dtype=torch.float64, device=self.device)
        check(lib.mps_relaxed_fwd(self.h, _ptr(x), C.byref(rp), _ptr(J_out), _ptr(saved),
                                  _stream(stream)))
        return J_out

    def relaxed_bwd(self, x, relax, saved, dJ=None, grad=None, stream=None):
        _dev(x, torch.float32, (self.N, self.T), "x")
        rp = RelaxParams(*relax)
        if grad is None:
            grad = torch.empty_like(x)
        if dJ is not None:
            _dev(dJ, torch.float64, None, "dJ")
        check(lib.mps_relaxed_bwd(self.h, _ptr(x), C.byref(rp), _ptr(saved), _ptr(dJ),
                                  _ptr(grad), _stream(stream)))
        return grad

    def rank_moves(self, grad, k, stream=None):
        _dev(grad, torch.float32, (self.N, self.T), "grad")
        nb = int(lib.mps_rank_ws_bytes(self.h, int(k)))
        # zero-filled once; each call leaves it ready for the next
        cache = self.__dict__.setdefault("_rank_ws", {})
        ws = cache.get(nb)
        if ws is None:
            ws = cache[nb] = torch.zeros(nb, dtype=torch.uint8, device=self.device)
        blk = torch.empty(k, dtype=torch.int32, device=self.device)
        per = torch.empty(k, dtype=torch.int8, device=self.device)
        gain = torch.empty(k, dtype=torch.float32, device=self.device)
        cnt = torch.zeros(1, dtype=torch.int32, device=self.device)
        check(lib.mps_rank_moves(self.h, _ptr(grad), int(k), _ptr(blk), _ptr(per), _ptr(gain),
                                 _ptr(cnt), _ptr(ws), nb, _stream(stream)))
        return blk, per, gain, cnt

    def search(self, mode, k, relax=(0.0, 0.0, 0.0), max_iter=1000, stream=None) -> dict:
        rp = RelaxParams(*relax)
        st = SearchStats()
        check(lib.mps_search(self.h, int(mode), int(k), C.byref(rp), int(max_iter),
                             C.byref(st), _stream(stream)))
        return dict(iterations=st.iterations, evaluations=st.evaluations,
                    applied=st.applied, J=st.J)

    def set_objective_variant(self, mult=None, risk=0, alpha=0.1, stream=None):
        """Value multiplier sigma(s,t) (host array [S][T] or None) and risk
        measure (0: std, 1: CVaR of the lower alpha tail); re-derives the
        state (mps_set_objective_variant)."""
        ptr = None
        if mult is not None:
            mult = np.ascontiguousarray(mult, dtype=np.float64)
            if mult.shape != (self.S, self.T):
                raise ValueError(f"mult must have shape {(self.S, self.T)}")
            ptr = mult.ctypes.data_as(C.c_void_p)
        check(lib.mps_set_objective_variant(self.h, ptr, int(risk), float(alpha),
                                            _stream(stream)))

    def lns_sa(self, n_iter, tile, k, max_rounds, eps_max, temp0, cool, u, stream=None):
        """LNS + SA driver (mps_lns_sa); returns (stats dict, trajectory [steps][4])."""
        K = ((self.prm.nx + tile - 1) // tile) * ((self.prm.ny + tile - 1) // tile)
        u = np.ascontiguousarray(u, dtype=np.float64)
        if u.shape != (n_iter * K,):
            raise ValueError(f"u must hold n_iter * tiles = {n_iter * K} draws")
        traj = np.zeros((n_iter * K, 4))
        prm = LnsParams(int(n_iter), int(tile), int(k), int(max_rounds), float(eps_max),
                        float(temp0), float(cool))
        st = LnsStats()
        check(lib.mps_lns_sa(self.h, C.byref(prm), u.ctypes.data_as(C.c_void_p),
                             traj.ctypes.data_as(C.c_void_p), C.byref(st), _stream(stream)))
        return dict(steps=st.steps, accepted=st.accepted, evaluations=st.evaluations,
                    applied=st.applied, J_best=st.J_best), traj

    def greedy_init(self, max_pass=1000, stream=None):
        """Replace the schedule by the greedy initializer's (mps_greedy_init);
        returns (passes, placed)."""
        passes, placed = C.c_int32(0), C.c_int64(0)
        check(lib.mps_greedy_init(self.h, int(max_pass), C.byref(passes), C.byref(placed),
                                  _stream(stream)))
        return passes.value, placed.value


class RelaxedNPV(torch.autograd.Function):
    """J(x) of the relaxed schedule, with the hand-written adjoint as backward.

    J = RelaxedNPV.apply(x, model, (mu_proc, mu_mine, mu_prec)) returns a
    float64 scalar on the GPU; J.backward() fills x.grad through
    mps_relaxed_bwd on the current stream."""

    @staticmethod
    def forward(ctx, x, model, relax):
        saved = model.relaxed_saved()
        Jv = model.relaxed_fwd(x.detach(), relax, saved)
        ctx.model, ctx.relax = model, relax
        ctx.save_for_backward(x, saved)
        return Jv[0].clone()

    @staticmethod
    def backward(ctx, gJ):
        x, saved = ctx.saved_tensors
        dJ = gJ.detach().to(torch.float64).reshape(1).contiguous()
        g = ctx.model.relaxed_bwd(x.detach(), ctx.relax, saved, dJ=dJ)
        return g, None, None


class TopK:
    """Reusable top-k buffers (workspace, indices, scores, count)."""

    def __init__(self, n, k, device="cuda"):
        self.n, self.k = int(n), int(k)
        self.ws_bytes = int(lib.mps_topk_ws_bytes(self.n, self.k))
        # zero-filled before the first call; every call leaves it so
        self.ws = torch.zeros(self.ws_bytes, dtype=torch.uint8, device=device)
        self.idx = torch.empty(self.k, dtype=torch.int64, device=device)
        self.score = torch.empty(self.k, dtype=torch.float32, device=device)
        self.count = torch.zeros(1, dtype=torch.int32, device=device)

    def __call__(self, score, flags, require=PREC_OK, forbid=NOOP | BAD, stream=None):
        n = int(score.shape[0])
        if n > self.n:
            raise ValueError(f"{n} items exceed the {self.n} this TopK was sized for")
        _dev(score, torch.float32, None, "score")
        _dev(flags, torch.uint8, score.shape, "flags")
        check(lib.mps_topk(_ptr(score), _ptr(flags), n, self.k, require, forbid,
                           _ptr(self.idx), _ptr(self.score), _ptr(self.count),
                           _ptr(self.ws), self.ws_bytes, _stream(stream)))
        return self.idx, self.score, self.count


def topk_noalloc(score, flags, idx, top_score, count, require=PREC_OK, forbid=NOOP | BAD,
                 stream=None):
    """mps_topk with the library-owned workspace: writes the caller's idx
    (int64 [k]), top_score (float32 [k] or None) and count (int32 [1])."""
    _dev(score, torch.float32, None, "score")
    _dev(flags, torch.uint8, score.shape, "flags")
    _dev(idx, torch.int64, None, "idx")
    _dev(count, torch.int32, (1,), "count")
    if top_score is not None:
        _dev(top_score, torch.float32, idx.shape, "top_score")
    check(lib.mps_topk_noalloc(_ptr(score), _ptr(flags), int(score.shape[0]),
                               int(idx.shape[0]), require, forbid, _ptr(idx),
                               _ptr(top_score), _ptr(count), _stream(stream)))
    return idx, top_score, count


def topk(score, flags, k, require=PREC_OK, forbid=NOOP | BAD, stream=None):
    t = TopK(score.shape[0], k, score.device)
    idx, sc, cnt = t(score, flags, require, forbid, stream)
    c = int(cnt.item())
    return idx[:c].clone(), sc[:c].clone()


class Batch:
    """Many models with their own move lists, evaluated in one persistent
    launch that ends with each model's top k (mps_batch_*).

    moves[i] is (block int32 [n_i], period int8 [n_i]) on the GPU.  The
    batch owns the output tensors: score[i], flags[i], top_idx[i],
    top_score[i], top_count[i]."""

    def __init__(self, models, moves, k, require=PREC_OK, forbid=NOOP | BAD):
        if len(models) != len(moves):
            raise ValueError("one move list per model")
        self.models, self.k = list(models), int(k)
        dev = models[0].device
        self.block, self.period = [], []
        self.score, self.flags, self.top_idx, self.top_score, self.top_count = [], [], [], [], []
        items = (BatchItem * len(models))()
        for i, (blk, per) in enumerate(moves):
            _dev(blk, torch.int32, None, "block")
            _dev(per, torch.int8, blk.shape, "period")
            n = int(blk.shape[0])
            self.block.append(blk)
            self.period.append(per)
            self.score.append(torch.empty(n, dtype=torch.float32, device=dev))
            self.flags.append(torch.empty(n, dtype=torch.uint8, device=dev))
            self.top_idx.append(torch.empty(self.k, dtype=torch.int64, device=dev))
            self.top_score.append(torch.empty(self.k, dtype=torch.float32, device=dev))
            self.top_count.append(torch.zeros(1, dtype=torch.int32, device=dev))
            items[i] = BatchItem(blk.data_ptr() if n else None, per.data_ptr() if n else None, n,
                                 self.score[i].data_ptr() if n else None,
                                 self.flags[i].data_ptr() if n else None,
                                 self.top_idx[i].data_ptr(), self.top_score[i].data_ptr(),
                                 self.top_count[i].data_ptr())
        hs = (C.c_void_p * len(models))(*[m.h.value for m in models])
        h = C.c_void_p()
        check(lib.mps_batch_create(hs, items, len(models), self.k, require, forbid,
                                   C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            check(lib.mps_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, tiles_per_item, moves_per_item, rows, i=-1):
        t = Tuning(tiles_per_item, moves_per_item, rows, 0)
        check(lib.mps_batch_set_tuning(self.h, int(i), C.byref(t)))

    def tuning(self, i) -> dict:
        t = Tuning()
        check(lib.mps_batch_get_tuning(self.h, int(i), C.byref(t)))
        return dict(tiles_per_item=t.tiles_per_item, moves_per_item=t.moves_per_item,
                    rows=t.rows)

    def set_workgroups(self, n):
        check(lib.mps_batch_set_workgroups(self.h, int(n)))

    def run(self, stream=None):
        check(lib.mps_batch_run(self.h, _stream(stream)))

    def graph_launch(self, stream=None):
        check(lib.mps_batch_graph_launch(self.h, _stream(stream)))

    def autotune(self, reps=5, stream=None) -> float:
        us = C.c_double(0.0)
        check(lib.mps_batch_autotune(self.h, int(reps), C.byref(us), _stream(stream)))
        return us.value
