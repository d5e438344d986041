"""ctypes binding of the CPU oracle (oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg. The product library never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

TRACE_DTYPE = np.dtype([
    ("iter", np.int64), ("var", np.int32), ("kind", np.int32), ("x_old", np.float64),
    ("x_new", np.float64), ("score", np.float64), ("viol", np.int64), ("obj", np.float64),
])

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.cpp with g++ (IEEE FP64, no contraction, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    i32, i64, u64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [i32, i32, P, P, P, P, P, P, P, P, P, f64, i32]
    lib.orc_destroy.argtypes = [P]
    lib.orc_num_norm_rows.restype = i32
    lib.orc_num_norm_rows.argtypes = [P]
    lib.orc_norm_rows.argtypes = [P, P, P]
    lib.orc_bounds.argtypes = [P, P, P, P]
    lib.orc_residual.restype = i64
    lib.orc_residual.argtypes = [P, P, f64, P]
    lib.orc_best_shift.argtypes = [P, P, P, f64, P, i64, P, P]
    lib.orc_jump_values.argtypes = [P, P, P, f64, P, P]
    lib.orc_jump_values.restype = None
    lib.orc_weighted_violation.argtypes = [P, P, P, f64, i32, f64]
    lib.orc_weighted_violation.restype = f64
    lib.orc_start_point.argtypes = [P, u64, P]
    lib.orc_splitmix64.restype = u64
    lib.orc_splitmix64.argtypes = [u64, u64]
    lib.orc_set_threads.argtypes = [i32]
    lib.orc_set_threads.restype = None
    lib.orc_threads.argtypes = []
    lib.orc_threads.restype = i32
    lib.orc_set_threads(1)
    lib.orc_exact_sum.restype = f64
    lib.orc_exact_sum.argtypes = [P, i64]
    lib.orc_objective.restype = f64
    lib.orc_objective.argtypes = [P, P]
    lib.orc_tabu_run.restype = i64
    lib.orc_tabu_run.argtypes = [P, i64, i32, u64, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.orc_tabu_resume.restype = i64
    lib.orc_tabu_resume.argtypes = [P, i64, i32, P, P, P, i64, i32, f64, P, f64, P, P, P, P, P, P, P, P, P, P, P]
    lib.orc_learned_replay.restype = i64
    lib.orc_learned_replay.argtypes = [P, i64, i32, u64, P, i32, P, P, P, P, P, P, P, P, P, P, P, P, P]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def splitmix64(seed: int, index: int) -> int:
    return int(_load().orc_splitmix64(seed, index))


def set_threads(k: int) -> int:
    """Threads of the oracle's per-column and per-row loops (results do not
    depend on it); returns the count in effect."""
    lib = _load()
    lib.orc_set_threads(int(k))
    return int(lib.orc_threads())


def exact_sum(values) -> float:
    """The oracle's exactly rounded sum of a list of doubles."""
    v = np.ascontiguousarray(values, dtype=np.float64)
    return float(_load().orc_exact_sum(_p(v), v.shape[0]))


class OracleProblem:
    """The normalised problem held by the oracle."""

    def __init__(self, mip, eps: float = 1e-6, binary_as_general: bool = False):
        lib = _load()
        self._keep = [
            np.ascontiguousarray(mip.csr_row_ptr, dtype=np.int64),
            np.ascontiguousarray(mip.csr_col, dtype=np.int32),
            np.ascontiguousarray(mip.csr_val, dtype=np.float64),
            np.ascontiguousarray(mip.sense, dtype=np.uint8),
            np.ascontiguousarray(mip.rhs, dtype=np.float64),
            np.ascontiguousarray(mip.lb, dtype=np.float64),
            np.ascontiguousarray(mip.ub, dtype=np.float64),
            np.ascontiguousarray(mip.is_int, dtype=np.uint8),
            np.ascontiguousarray(mip.obj, dtype=np.float64),
        ]
        self.n = int(mip.n)
        self.eps = eps
        self.h = lib.orc_create(int(mip.n), int(mip.m), *[_p(a) for a in self._keep], float(eps),
                                int(bool(binary_as_general)))
        self.mp = int(lib.orc_num_norm_rows(self.h))
        self._lib = lib

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self._lib.orc_destroy(h)
            self.h = None

    def norm_rows(self):
        orig = np.empty(self.mp, dtype=np.int32)
        sign = np.empty(self.mp, dtype=np.int8)
        self._lib.orc_norm_rows(self.h, _p(orig), _p(sign))
        return orig, sign

    def bounds(self):
        lb = np.empty(self.n)
        ub = np.empty(self.n)
        isb = np.empty(self.n, dtype=np.uint8)
        self._lib.orc_bounds(self.h, _p(lb), _p(ub), _p(isb))
        return lb, ub, isb

    def residual(self, x, cutoff_rhs: float = float("inf")):
        x = np.ascontiguousarray(x, dtype=np.float64)
        r = np.empty(self.mp + 1)
        v = self._lib.orc_residual(self.h, _p(x), float(cutoff_rhs), _p(r))
        return r, int(v)

    def best_shift(self, x, w, cutoff_rhs: float = float("inf"), cols=None):
        x = np.ascontiguousarray(x, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.shape[0] == self.mp + 1
        if cols is None:
            xh = np.empty(self.n)
            s = np.empty(self.n)
            self._lib.orc_best_shift(self.h, _p(x), _p(w), float(cutoff_rhs), None, 0, _p(xh), _p(s))
        else:
            cols = np.ascontiguousarray(cols, dtype=np.int32)
            xh = np.empty(cols.shape[0])
            s = np.empty(cols.shape[0])
            self._lib.orc_best_shift(self.h, _p(x), _p(w), float(cutoff_rhs), _p(cols), cols.shape[0],
                                     _p(xh), _p(s))
        return xh, s

    def jump_values(self, x, w, cutoff_rhs: float = float("inf")):
        """Jump value and jump score of every column (weighted violation)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.shape[0] == self.mp + 1
        jv = np.empty(self.n)
        js = np.empty(self.n)
        self._lib.orc_jump_values(self.h, _p(x), _p(w), float(cutoff_rhs), _p(jv), _p(js))
        return jv, js

    def weighted_violation(self, x, w, j: int, t: float, cutoff_rhs: float = float("inf")) -> float:
        """V_j(t): the weighted violation of column j's rows with x_j = t."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float32)
        return float(self._lib.orc_weighted_violation(self.h, _p(x), _p(w), float(cutoff_rhs), int(j), float(t)))

    def objective(self, x) -> float:
        x = np.ascontiguousarray(x, dtype=np.float64)
        return float(self._lib.orc_objective(self.h, _p(x)))

    def start_point(self, seed: int):
        x = np.empty(self.n)
        self._lib.orc_start_point(self.h, int(seed), _p(x))
        return x

    def learned_replay(self, iters: int, tenure: int, seed: int, full_every: int, sets, set_offsets, x0=None):
        """The learned proposal form of the walk (orc_learned_replay): full
        evaluations by the block rule, the listed sets (original indices)
        everywhere else."""
        sets = np.ascontiguousarray(sets if sets is not None and len(sets) else np.zeros(1), dtype=np.int32)
        offs = np.ascontiguousarray(set_offsets, dtype=np.int64)
        assert offs.shape[0] == iters + 1
        return self._walk(iters, tenure, seed, x0, lambda *a: self._lib.orc_learned_replay(
            self.h, int(iters), int(tenure), int(seed), a[0], int(full_every), _p(sets), _p(offs), *a[1:]))

    def tabu_resume(self, iters: int, tenure: int, x, w, tabu_until, k0: int, best_obj: float = float("inf"),
                    best_x=None, cutoff_rhs: float = float("inf")):
        """The plain walk continued for `iters` iterations from its state at the
        start of iteration k0 (point x, weights w of m'+1 rows, last tabu
        iteration of every variable, best feasible objective and point, cutoff
        right-hand side); trace records k0 .. k0 + iters - 1."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float32)
        tb = np.ascontiguousarray(tabu_until, dtype=np.int64)
        has = best_x is not None and np.isfinite(best_obj)
        bx = np.ascontiguousarray(best_x if has else np.zeros(self.n), dtype=np.float64)
        assert x.shape[0] == self.n and w.shape[0] == self.mp + 1 and tb.shape[0] == self.n
        return self._walk(iters, tenure, 0, None, lambda *a: self._lib.orc_tabu_resume(
            self.h, int(iters), int(tenure), _p(x), _p(w), _p(tb), int(k0), int(has),
            float(best_obj) if has else 0.0, _p(bx), float(cutoff_rhs), *a[1:]))

    def tabu_run(self, iters: int, tenure: int, seed: int, x0=None):
        return self._walk(iters, tenure, seed, x0, lambda *a: self._lib.orc_tabu_run(
            self.h, int(iters), int(tenure), int(seed), *a))

    def _walk(self, iters, tenure, seed, x0, call):
        trace = np.zeros(max(iters, 1), dtype=TRACE_DTYPE)
        x = np.empty(self.n)
        r = np.empty(self.mp + 1)
        w = np.empty(self.mp + 1, dtype=np.float32)
        best_obj = ctypes.c_double()
        best_x = np.empty(self.n)
        has_best = ctypes.c_int32()
        bc = ctypes.c_double()
        x0p = None
        if x0 is not None:
            x0 = np.ascontiguousarray(x0, dtype=np.float64)
            x0p = _p(x0)
        inf_v = ctypes.c_int64()
        inf_k = ctypes.c_int64()
        inf_x = np.empty(self.n)
        call(x0p, _p(trace), _p(x), _p(r), _p(w), ctypes.byref(best_obj), _p(best_x), ctypes.byref(has_best),
             ctypes.byref(bc), ctypes.byref(inf_v), ctypes.byref(inf_k), _p(inf_x))
        return {
            "trace": trace[:iters], "x": x, "r": r, "w": w, "best_obj": best_obj.value,
            "best_x": best_x if has_best.value else None, "cutoff_rhs": bc.value,
            "inf_viol": inf_v.value, "inf_iter": inf_k.value, "inf_x": inf_x if inf_k.value != -2 else None,
        }


# ---- diversity-driven restarts of parallel walks --------------------------
# Section 3.1 "Parallel Tabu Search Instances" (a paragraph the compiled
# paper leaves out): the diversity of an instance is measured against the
# other active instances by the Hamming distance over the discrete variables,
# d(x, y) = #{i in I : x_i != y_i}, and instances too similar to others are
# restarted. Readings (design notes): walks run in segments of `every`
# iterations; at the end of each segment (before the last) walk w restarts
# when some walk w' < w on the same problem lies at distance < min_distance
# (all distances taken at the points before any restart of that boundary);
# a restart keeps the walk's iteration count, best feasible point and cutoff
# row, and starts again from the start point of seed walk_seed + c * GOLDEN
# (mod 2^64, c = the walk's restart count) with unit weights and an empty
# tabu list.

RESTART_SEED_STEP = 0x9E3779B97F4A7C15


def hamming_discrete(x, y, is_int) -> int:
    """d(x, y) over the integer (binary and general integer) variables."""
    return int(np.count_nonzero((np.asarray(x) != np.asarray(y)) & (np.asarray(is_int) == 1)))


def restart_seed(seed: int, count: int) -> int:
    return (int(seed) + int(count) * RESTART_SEED_STEP) % (1 << 64)


def batch_restarts(problems, walk_prob, walk_seed, iters: int, tenure: int, every: int, min_distance: int):
    """Independent walks with diversity-driven restarts. problems: list of
    (OracleProblem, MIP). Returns per walk a dict with the trace, final x, r,
    w, best objective and point, cutoff, and the iterations at which the
    walk restarted."""
    nw = len(walk_prob)
    st = []
    for w in range(nw):
        P, mip = problems[walk_prob[w]]
        st.append({"x": P.start_point(int(walk_seed[w])), "w": np.ones(P.mp + 1, dtype=np.float32),
                   "tabu": np.full(P.n, -1, dtype=np.int64), "best_obj": float("inf"), "best_x": None,
                   "cutoff": float("inf"), "traces": [], "restarts": [], "count": 0, "r": None})
    k0 = 0
    while k0 < iters:
        seg = min(every, iters - k0) if every > 0 else iters - k0
        for w in range(nw):
            P, mip = problems[walk_prob[w]]
            S = st[w]
            o = P.tabu_resume(seg, tenure, S["x"], S["w"], S["tabu"], k0, S["best_obj"], S["best_x"], S["cutoff"])
            tr = o["trace"]
            moved = tr["var"] >= 0
            for k, j in zip(tr["iter"][moved], tr["var"][moved]):
                S["tabu"][j] = k + tenure
            S.update(x=o["x"], w=o["w"], r=o["r"], best_obj=o["best_obj"], best_x=o["best_x"], cutoff=o["cutoff_rhs"])
            S["traces"].append(tr)
        k0 += seg
        if k0 >= iters or every <= 0:
            continue
        points = [st[w]["x"].copy() for w in range(nw)]
        for w in range(nw):
            P, mip = problems[walk_prob[w]]
            close = any(walk_prob[v] == walk_prob[w] and hamming_discrete(points[w], points[v], mip.is_int) < min_distance
                        for v in range(w))
            if not close:
                continue
            S = st[w]
            S["count"] += 1
            S["restarts"].append(k0)
            S["x"] = P.start_point(restart_seed(walk_seed[w], S["count"]))
            S["w"] = np.ones(P.mp + 1, dtype=np.float32)
            S["tabu"] = np.full(P.n, -1, dtype=np.int64)
    out = []
    for S in st:
        out.append({"trace": np.concatenate(S["traces"]) if S["traces"] else np.zeros(0, dtype=TRACE_DTYPE),
                    "x": S["x"], "r": S["r"], "w": S["w"], "best_obj": S["best_obj"], "best_x": S["best_x"],
                    "cutoff_rhs": S["cutoff"], "restarts": list(S["restarts"])})
    return out
