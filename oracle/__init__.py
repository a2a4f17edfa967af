"""Python access to the plain FP64 C oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product package never imports it.

Instances are duck-typed: any object with nx, ny, nz, S, T, rate, lam,
pen_proc, pen_mine, pcap, mcap, v (float32 [S][N]), ore (uint8 [S][N]) and
ton (float64 [N]) attributes (the seeded generator's Instance has them).  An
instance may also carry explicit predecessor lists (Eq. 15's sets) as
pred_ptr (int32 [N+1]) and pred_idx (int32 [pred_ptr[N]]); without them the
precedence is the grid's 1-5 slope stencil.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

PREC_OK, MINE_OK, PROC_OK, NOOP, BAD = 1, 2, 4, 8, 16


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain -O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-Wall", "-o", tmp,
               os.path.join(HERE, "oracle.c"), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Inst(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("S", C.c_int32), ("T", C.c_int32),
                ("rate", C.c_double), ("lam", C.c_double),
                ("pen_proc", C.c_double), ("pen_mine", C.c_double),
                ("pcap", C.c_double), ("mcap", C.c_double),
                ("v", C.c_void_p), ("ore", C.c_void_p), ("ton", C.c_void_p),
                ("pred_ptr", C.c_void_p), ("pred_idx", C.c_void_p),
                ("succ_ptr", C.c_void_p), ("succ_idx", C.c_void_p),
                ("mult", C.c_void_p), ("risk", C.c_int32), ("alpha", C.c_double)]

MAX_DEG = 9   # OR_MAX_DEG: predecessors (and successors) per block


class _Obj(C.Structure):
    _fields_ = [("mu", C.c_double), ("sigma", C.c_double), ("R", C.c_double),
                ("Pp", C.c_double), ("Pm", C.c_double), ("J", C.c_double),
                ("n_prec_viol", C.c_int64)]


class _Relax(C.Structure):
    _fields_ = [("mu_proc", C.c_double), ("mu_mine", C.c_double),
                ("mu_prec", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.or_discount.argtypes = [i32, dbl, vp]
        L.or_successor_csr.argtypes = [i64, vp, vp, vp, vp]
        L.or_predecessors.argtypes = [vp, i32, vp]
        L.or_predecessors.restype = i32
        L.or_successors.argtypes = [vp, i32, vp]
        L.or_successors.restype = i32
        L.or_objective.argtypes = [vp, vp, vp, vp, vp, vp]
        L.or_eval_moves.argtypes = [vp, vp, i32, i32, i64, vp, vp, vp, vp, vp,
                                    vp, vp, i32]
        L.or_eval_bruteforce.argtypes = [vp, vp, i32, i32]
        L.or_eval_bruteforce.restype = dbl
        L.or_topk.argtypes = [vp, vp, i64, i32, C.c_uint8, C.c_uint8, vp, vp]
        L.or_topk.restype = i32
        L.or_repair.argtypes = [vp, vp, i32, vp, vp, i32, vp, vp]
        L.or_repair.restype = i32
        L.or_relaxed_d.argtypes = [vp, vp, vp, vp]
        L.or_relaxed_d.restype = dbl
        L.or_relaxed.argtypes = [vp, vp, vp, vp]
        L.or_relaxed.restype = dbl
        L.or_rank_moves.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        L.or_rank_moves.restype = i32
        L.or_search.argtypes = [vp, vp, i32, i32, vp, i32, vp, i32]
        L.or_search.restype = dbl
        L.or_repair_cascade.argtypes = [vp, vp, i32, vp, vp, i32, i32, vp, vp, vp]
        L.or_repair_cascade.restype = i32
        L.or_cvar.argtypes = [vp, i32, dbl]
        L.or_cvar.restype = dbl
        L.or_lns_sa.argtypes = [vp, vp, i32, i32, i32, i32, dbl, dbl, dbl, vp, vp, vp, i32]
        L.or_lns_sa.restype = dbl
        L.or_greedy_init.argtypes = [vp, vp, i32, vp]
        L.or_greedy_init.restype = i32
        L.or_optimum.argtypes = [vp, vp, vp]
        L.or_optimum.restype = dbl
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Oracle:
    """One instance bound to the C oracle (keeps its arrays alive)."""

    def __init__(self, inst):
        self.inst = inst
        self.S, self.T = int(inst.S), int(inst.T)
        self.N = int(inst.nx) * int(inst.ny) * int(inst.nz)
        self.v = np.ascontiguousarray(inst.v, dtype=np.float32)
        self.ore = np.ascontiguousarray(inst.ore, dtype=np.uint8)
        self.ton = np.ascontiguousarray(inst.ton, dtype=np.float64)
        assert self.v.shape == (self.S, self.N) and self.ore.shape == (self.S, self.N)
        assert self.ton.shape == (self.N,)
        pp = getattr(inst, "pred_ptr", None)
        ptrs = [None] * 4
        if pp is not None:
            self.pred_ptr = np.ascontiguousarray(pp, dtype=np.int32)
            self.pred_idx = np.ascontiguousarray(inst.pred_idx, dtype=np.int32)
            N = self.N
            assert self.pred_ptr.shape == (N + 1,) and self.pred_ptr[0] == 0
            assert np.all(np.diff(self.pred_ptr) >= 0)
            assert np.all(np.diff(self.pred_ptr) <= MAX_DEG)
            assert self.pred_idx.shape == (int(self.pred_ptr[-1]),)
            assert np.all((self.pred_idx >= 0) & (self.pred_idx < N))
            self.succ_ptr = np.empty(N + 1, dtype=np.int32)
            self.succ_idx = np.empty(len(self.pred_idx), dtype=np.int32)
            lib().or_successor_csr(N, _ptr(self.pred_ptr), _ptr(self.pred_idx),
                                   _ptr(self.succ_ptr), _ptr(self.succ_idx))
            assert np.all(np.diff(self.succ_ptr) <= MAX_DEG)
            ptrs = [self.pred_ptr.ctypes.data, self.pred_idx.ctypes.data,
                    self.succ_ptr.ctypes.data, self.succ_idx.ctypes.data]
        mult = getattr(inst, "mult", None)
        self.mult = None
        if mult is not None:
            self.mult = np.ascontiguousarray(mult, dtype=np.float64)
            assert self.mult.shape == (self.S, self.T)
        risk = int(getattr(inst, "risk", 0))
        alpha = float(getattr(inst, "alpha", 0.1))
        assert risk in (0, 1) and 0.0 < alpha <= 1.0
        self.c = _Inst(int(inst.nx), int(inst.ny), int(inst.nz), self.S, self.T,
                       float(inst.rate), float(inst.lam), float(inst.pen_proc),
                       float(inst.pen_mine), float(inst.pcap), float(inst.mcap),
                       self.v.ctypes.data, self.ore.ctypes.data, self.ton.ctypes.data,
                       *ptrs, self.mult.ctypes.data if self.mult is not None else None,
                       risk, alpha)
        self.ref = C.byref(self.c)

    def _p(self, p):
        p = np.ascontiguousarray(p, dtype=np.int8)
        assert p.shape == (self.N,)
        return p

    def discount(self):
        d = np.empty(self.T + 1)
        lib().or_discount(self.T, float(self.inst.rate), _ptr(d))
        return d

    def predecessors(self, b):
        out = np.empty(MAX_DEG, dtype=np.int32)
        n = lib().or_predecessors(self.ref, int(b), _ptr(out))
        return sorted(out[:n].tolist())

    def successors(self, b):
        out = np.empty(MAX_DEG, dtype=np.int32)
        n = lib().or_successors(self.ref, int(b), _ptr(out))
        return sorted(out[:n].tolist())

    def objective(self, p, state=False):
        p = self._p(p)
        o = _Obj()
        Ns = np.empty(self.S)
        O = np.empty((self.S, self.T))
        M = np.empty(self.T)
        lib().or_objective(self.ref, _ptr(p), C.byref(o), _ptr(Ns), _ptr(O), _ptr(M))
        r = dict(mu=o.mu, sigma=o.sigma, R=o.R, Pp=o.Pp, Pm=o.Pm, J=o.J,
                 n_prec_viol=int(o.n_prec_viol))
        if state:
            r.update(Ns=Ns, O=O, M=M)
        return r

    def eval_moves(self, p, block=None, period=None, include_never=True,
                   threads=0, components=False):
        p = self._p(p)
        exhaustive = block is None
        if exhaustive:
            D = self.T + 1 if include_never else self.T
            n = self.N * D
            bptr = tptr = None
        else:
            block = np.ascontiguousarray(block, dtype=np.int32)
            period = np.ascontiguousarray(period, dtype=np.int8)
            n = block.shape[0]
            bptr, tptr = _ptr(block), _ptr(period)
        score = np.empty(n)
        flags = np.empty(n, dtype=np.uint8)
        comp = [np.empty(n) for _ in range(3)] if components else None
        cp = [_ptr(a) for a in comp] if components else [None] * 3
        lib().or_eval_moves(self.ref, _ptr(p), int(exhaustive), int(include_never),
                            n, bptr, tptr, _ptr(score), _ptr(flags), *cp, int(threads))
        if components:
            return score, flags, comp[0], comp[1], comp[2]
        return score, flags

    def eval_bruteforce(self, p, b, t):
        return lib().or_eval_bruteforce(self.ref, _ptr(self._p(p)), int(b), int(t))

    def repair(self, p, cand_block, cand_period, hard=False):
        q = self._p(p).copy()
        cb = np.ascontiguousarray(cand_block, dtype=np.int32)
        ct = np.ascontiguousarray(cand_period, dtype=np.int8)
        acc = np.zeros(cb.shape[0], dtype=np.uint8)
        J = C.c_double()
        a = lib().or_repair(self.ref, _ptr(q), cb.shape[0], _ptr(cb), _ptr(ct),
                            int(bool(hard)), C.byref(J), _ptr(acc))
        return q, int(a), J.value, acc

    def repair_cascade(self, p, cand_block, cand_period, hard=False, max_set=64):
        q = self._p(p).copy()
        cb = np.ascontiguousarray(cand_block, dtype=np.int32)
        ct = np.ascontiguousarray(cand_period, dtype=np.int8)
        acc = np.zeros(cb.shape[0], dtype=np.uint8)
        size = np.zeros(cb.shape[0], dtype=np.int32)
        J = C.c_double()
        a = lib().or_repair_cascade(self.ref, _ptr(q), cb.shape[0], _ptr(cb), _ptr(ct),
                                    int(bool(hard)), int(max_set), C.byref(J), _ptr(acc),
                                    _ptr(size))
        return q, int(a), J.value, acc, size

    def relaxed(self, x, mu_proc, mu_mine, mu_prec, grad=True):
        x = np.ascontiguousarray(x)
        assert x.shape == (self.N, self.T)
        rp = _Relax(mu_proc, mu_mine, mu_prec)
        g = np.empty((self.N, self.T)) if grad else None
        if x.dtype == np.float64:
            J = lib().or_relaxed_d(self.ref, _ptr(x), C.byref(rp),
                                   _ptr(g) if grad else None)
        else:
            x = x.astype(np.float32)
            J = lib().or_relaxed(self.ref, _ptr(x), C.byref(rp),
                                 _ptr(g) if grad else None)
        return (J, g) if grad else J

    def rank_moves(self, p, grad, k):
        p = self._p(p)
        grad = np.ascontiguousarray(grad, dtype=np.float64)
        b = np.empty(k, dtype=np.int32)
        t = np.empty(k, dtype=np.int8)
        gain = np.empty(k)
        c = lib().or_rank_moves(self.ref, _ptr(p), _ptr(grad), int(k), _ptr(b),
                                _ptr(t), _ptr(gain))
        return b[:c], t[:c], gain[:c]

    def search(self, p, mode, k, relax=(0.0, 0.0, 0.0), max_iter=1000, threads=0):
        q = self._p(p).copy()
        rp = _Relax(*relax)
        stats = np.zeros(3, dtype=np.int64)
        J = lib().or_search(self.ref, _ptr(q), int(mode), int(k), C.byref(rp),
                            int(max_iter), _ptr(stats), int(threads))
        return q, J, dict(iterations=int(stats[0]), evaluations=int(stats[1]),
                          applied=int(stats[2]))

    def greedy_init(self, max_pass=1000):
        p = np.empty(self.N, dtype=np.int8)
        placed = C.c_int64()
        passes = lib().or_greedy_init(self.ref, _ptr(p), int(max_pass), C.byref(placed))
        return p, int(passes), int(placed.value)

    def lns_sa(self, p, n_iter, nb, k, max_rounds, eps_max, temp0, cool, u, threads=0):
        """LNS + SA driver; returns (best schedule, J_best, trajectory, stats)."""
        q = self._p(p).copy()
        kx = (int(self.inst.nx) + nb - 1) // nb
        ky = (int(self.inst.ny) + nb - 1) // nb
        u = np.ascontiguousarray(u, dtype=np.float64)
        assert u.shape == (n_iter * kx * ky,)
        traj = np.zeros((n_iter * kx * ky, 4))
        stats = np.zeros(4, dtype=np.int64)
        J = lib().or_lns_sa(self.ref, _ptr(q), int(n_iter), int(nb), int(k), int(max_rounds),
                            float(eps_max), float(temp0), float(cool), _ptr(u), _ptr(traj),
                            _ptr(stats), int(threads))
        return q, J, traj, dict(steps=int(stats[0]), accepted=int(stats[1]),
                                evaluations=int(stats[2]), applied=int(stats[3]))

    def optimum(self):
        best = np.zeros(self.N, dtype=np.int8)
        cnt = C.c_int64()
        J = lib().or_optimum(self.ref, _ptr(best), C.byref(cnt))
        return J, best, int(cnt.value)


def cvar(x, alpha):
    """CVaR of the lower alpha tail of x (or_cvar)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().or_cvar(_ptr(x), x.shape[0], float(alpha))


def topk(score, flags, k, req=PREC_OK, forbid=NOOP | BAD):
    score = np.ascontiguousarray(score, dtype=np.float64)
    flags = np.ascontiguousarray(flags, dtype=np.uint8)
    n = score.shape[0]
    idx = np.empty(max(k, 1), dtype=np.int64)
    sc = np.empty(max(k, 1))
    c = lib().or_topk(_ptr(score), _ptr(flags), n, int(k), int(req), int(forbid),
                      _ptr(idx), _ptr(sc))
    return idx[:c], sc[:c]
