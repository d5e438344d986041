"""Python binding of libchap.so, the gfx950 tabu-search best-shift library.

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/chap.h. PyTorch provides device
memory and streams. There is no CPU fallback: importing the binding raises if
the library has not been built.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchap.so")

CHAP_OK = 0
ERRORS = {-1: "CHAP_EINVAL", -2: "CHAP_ENOMEM", -3: "CHAP_EHIP", -4: "CHAP_ESTATE", -5: "CHAP_ENOTBUILT"}

TRACE_DTYPE = np.dtype([
    ("iter", np.int64), ("var", np.int32), ("kind", np.int32), ("x_old", np.float64),
    ("x_new", np.float64), ("score", np.float64), ("viol", np.int64), ("obj", np.float64),
])


class ChapOptions(ctypes.Structure):
    _fields_ = [("feas_tol", ctypes.c_double), ("graph_iters", ctypes.c_int32), ("short_max", ctypes.c_int32),
                ("chunk_min", ctypes.c_int32), ("chunk_len", ctypes.c_int32), ("row_stage", ctypes.c_int32),
                ("rescore_cap", ctypes.c_int32)]


class LearnedOptions(ctypes.Structure):
    _fields_ = [("topk", ctypes.c_int32), ("full_every", ctypes.c_int32), ("train_steps", ctypes.c_int32),
                ("train_pairs", ctypes.c_int32), ("lr", ctypes.c_float), ("log_sets", ctypes.c_int32),
                ("log_pairs", ctypes.c_int64), ("train_seed", ctypes.c_uint64),
                ("refresh_every", ctypes.c_int32)]


class ChapError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load_library():
    """Load libchap.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2605_05086_amd/build.py (hipcc, gfx950)")
    # PyTorch carries its own HIP runtime beside the system one the library
    # links; PyTorch's must reach the device first (the other order leaves
    # PyTorch without a visible GPU), so it is initialised before the library
    # can make its first HIP call
    try:
        import torch

        torch.cuda.is_available()
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, u64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    lib.chap_options_default.argtypes = [ctypes.POINTER(ChapOptions)]
    lib.chap_options_default.restype = None
    lib.chap_last_error.restype = ctypes.c_char_p
    lib.chap_problem_create.argtypes = [ctypes.POINTER(P), i32, i32, P, P, P, P, P, P, P, P, P, P, P, P,
                                        ctypes.POINTER(ChapOptions)]
    lib.chap_problem_create.restype = ctypes.c_int
    lib.chap_problem_destroy.argtypes = [P]
    lib.chap_problem_destroy.restype = None
    lib.chap_problem_num_norm_rows.argtypes = [P]
    lib.chap_problem_num_norm_rows.restype = i32
    lib.chap_problem_norm_row_map.argtypes = [P, P, P]
    lib.chap_problem_norm_row_map.restype = ctypes.c_int
    lib.chap_best_shift.argtypes = [P, P, P, f64, P, P, P]
    lib.chap_best_shift.restype = ctypes.c_int
    lib.chap_best_shift_noalloc.argtypes = [P, P, P, f64, P, P, P]
    lib.chap_best_shift_noalloc.restype = ctypes.c_int
    lib.chap_best_shift_noalloc_max_bytes.argtypes = []
    lib.chap_best_shift_noalloc_max_bytes.restype = ctypes.c_size_t
    lib.chap_best_shift_pass_ms.argtypes = [P, ctypes.POINTER(f64)]
    lib.chap_best_shift_pass_ms.restype = ctypes.c_int
    lib.chap_tabu_run.argtypes = [P, i64, i32, u64, P, ctypes.POINTER(P), P]
    lib.chap_tabu_run.restype = ctypes.c_int
    lib.chap_batch_run.argtypes = [P, i32, P, P, P, i32, i64, i32, P, P]
    lib.chap_batch_run.restype = ctypes.c_int
    lib.chap_run_trace.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(i64)]
    lib.chap_run_trace.restype = ctypes.c_int
    lib.chap_run_state.argtypes = [P, P, P, P, ctypes.POINTER(f64), P, ctypes.POINTER(f64)]
    lib.chap_run_state.restype = ctypes.c_int
    lib.chap_run_best_infeasible.argtypes = [P, P, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.chap_run_best_infeasible.restype = ctypes.c_int
    lib.chap_run_elapsed_ms.argtypes = [P]
    lib.chap_run_elapsed_ms.restype = f64
    lib.chap_run_destroy.argtypes = [P]
    lib.chap_run_destroy.restype = None
    lib.chap_model_create.argtypes = [ctypes.POINTER(P), u64]
    lib.chap_model_create.restype = ctypes.c_int
    lib.chap_model_destroy.argtypes = [P]
    lib.chap_model_destroy.restype = None
    lib.chap_model_get_params.argtypes = [P, P]
    lib.chap_model_get_params.restype = ctypes.c_int
    lib.chap_model_set_params.argtypes = [P, P]
    lib.chap_model_set_params.restype = ctypes.c_int
    lib.chap_model_forward.argtypes = [P, P, i64, P, P]
    lib.chap_model_forward.restype = ctypes.c_int
    lib.chap_model_grad.argtypes = [P, P, P, i64, P, P]
    lib.chap_model_grad.restype = ctypes.c_int
    lib.chap_model_train.argtypes = [P, P, P, i64, i32, i32, ctypes.c_float, u64, P]
    lib.chap_model_train.restype = ctypes.c_int
    lib.chap_autotune.argtypes = [P, P, i32, i64, ctypes.POINTER(ChapOptions), P]
    lib.chap_autotune.restype = ctypes.c_int
    lib.chap_learned_options_default.argtypes = [ctypes.POINTER(LearnedOptions)]
    lib.chap_learned_options_default.restype = None
    lib.chap_learned_run.argtypes = [P, P, ctypes.POINTER(LearnedOptions), i64, i32, u64, P, ctypes.POINTER(P), P]
    lib.chap_learned_run.restype = ctypes.c_int
    lib.chap_run_learned_stats.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.chap_run_learned_stats.restype = ctypes.c_int
    lib.chap_jump_values.argtypes = [P, P, P, ctypes.c_double, P, P, P]
    lib.chap_jump_values.restype = ctypes.c_int
    lib.chap_jump_values_ms.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
    lib.chap_jump_values_ms.restype = ctypes.c_int
    lib.chap_batch_restarts.argtypes = [P, ctypes.c_int32, P, P, ctypes.c_int32, i64, ctypes.c_int32, i64, i64, P, P]
    lib.chap_batch_restarts.restype = ctypes.c_int
    lib.chap_run_restarts.argtypes = [P, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(i64)]
    lib.chap_run_restarts.restype = ctypes.c_int
    lib.chap_run_rescored.argtypes = [P, ctypes.POINTER(i64)]
    lib.chap_run_rescored.restype = ctypes.c_int
    lib.chap_run_proposals.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(i64)]
    lib.chap_run_proposals.restype = ctypes.c_int
    lib.chap_run_pairs.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(i64)]
    lib.chap_run_pairs.restype = ctypes.c_int
    lib.chap_features.argtypes = [P, P, P, f64, P, P, P, P, i64, i64, P, P]
    lib.chap_features.restype = ctypes.c_int
    _lib = lib
    return lib


def _release(fn: str, handle, _mod=__import__("sys").modules[__name__]) -> None:
    """Destroys a handle; a no-op while the interpreter shuts down (module
    globals may already be gone then)."""
    lib = getattr(_mod, "_lib", None)
    if lib is not None:
        f = getattr(lib, fn, None)
        if f is not None:
            f(handle)


def _check(rc: int):
    if rc != CHAP_OK:
        raise ChapError(rc, load_library().chap_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def default_options() -> ChapOptions:
    o = ChapOptions()
    load_library().chap_options_default(ctypes.byref(o))
    return o


class Run:
    """Result of a walk: the trace, the best objective and cutoff, and the
    final state (x, resid, w, best_x: host arrays, read from the library on
    first access)."""

    def __init__(self, handle, n: int, mp: int):
        lib = load_library()
        self._h = handle
        self._n, self._mp = n, mp
        self._state = None
        rec = ctypes.c_void_p()
        cnt = ctypes.c_int64()
        _check(lib.chap_run_trace(handle, ctypes.byref(rec), ctypes.byref(cnt)))
        if cnt.value > 0:
            buf = (ctypes.c_char * (cnt.value * TRACE_DTYPE.itemsize)).from_address(rec.value)
            self.trace = np.frombuffer(bytes(buf), dtype=TRACE_DTYPE).copy()
        else:
            self.trace = np.zeros(0, dtype=TRACE_DTYPE)
        best_obj = ctypes.c_double()
        cut = ctypes.c_double()
        _check(lib.chap_run_state(handle, None, None, None, ctypes.byref(best_obj), None, ctypes.byref(cut)))
        self.best_obj = best_obj.value
        self.cutoff_rhs = cut.value
        self.elapsed_ms = lib.chap_run_elapsed_ms(handle)
        ev, hi, st = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.chap_run_learned_stats(handle, ctypes.byref(ev), ctypes.byref(hi), ctypes.byref(st)))
        self.evals, self.hits, self.stalls = ev.value, hi.value, st.value
        rs = ctypes.c_int64()
        _check(lib.chap_run_rescored(handle, ctypes.byref(rs)))
        self.rescored = rs.value
        rp, rc_ = ctypes.c_void_p(), ctypes.c_int64()
        _check(lib.chap_run_restarts(handle, ctypes.byref(rp), ctypes.byref(rc_)))
        self.restarts = (list(np.ctypeslib.as_array((ctypes.c_int64 * rc_.value).from_address(rp.value)))
                         if rc_.value > 0 else [])
        sets, offs, iters = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int64()
        _check(lib.chap_run_proposals(handle, ctypes.byref(sets), ctypes.byref(offs), ctypes.byref(iters)))
        self.set_offsets = None
        self.sets = None
        if iters.value > 0:
            o = np.ctypeslib.as_array((ctypes.c_int64 * (iters.value + 1)).from_address(offs.value)).copy()
            self.set_offsets = o
            self.sets = (np.ctypeslib.as_array((ctypes.c_int32 * int(o[-1])).from_address(sets.value)).copy()
                         if o[-1] > 0 else np.zeros(0, dtype=np.int32))
        pf, pt, cnt = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int64()
        _check(lib.chap_run_pairs(handle, ctypes.byref(pf), ctypes.byref(pt), ctypes.byref(cnt)))
        self.pair_feat = None
        self.pair_target = None
        if cnt.value > 0:
            self.pair_feat = np.ctypeslib.as_array(
                (ctypes.c_uint16 * (cnt.value * 16)).from_address(pf.value)).copy().reshape(cnt.value, 16)
            self.pair_target = np.ctypeslib.as_array((ctypes.c_float * cnt.value).from_address(pt.value)).copy()

    def _load_state(self):
        if self._state is None:
            x = np.empty(self._n)
            resid = np.empty(self._mp + 1)
            w = np.empty(self._mp + 1, dtype=np.float32)
            best_x = np.full(self._n, np.nan)
            _check(load_library().chap_run_state(self._h, _ptr(x), _ptr(resid), _ptr(w), None, _ptr(best_x), None))
            self._state = (x, resid, w, None if math.isinf(self.best_obj) else best_x)
        return self._state

    def best_infeasible(self):
        """(point or None, violated rows, iteration; -1 = start, -2 = none)."""
        v, k = ctypes.c_int64(), ctypes.c_int64()
        lib = load_library()
        _check(lib.chap_run_best_infeasible(self._h, None, ctypes.byref(v), ctypes.byref(k)))
        if k.value == -2:
            return None, v.value, k.value
        x = np.empty(self._n)
        _check(lib.chap_run_best_infeasible(self._h, _ptr(x), None, None))
        return x, v.value, k.value

    @property
    def x(self):
        return self._load_state()[0]

    @property
    def resid(self):
        return self._load_state()[1]

    @property
    def w(self):
        return self._load_state()[2]

    @property
    def best_x(self):
        return self._load_state()[3]

    def proposal_set(self, k: int):
        """Original column indices proposed at iteration k (empty for a full
        evaluation); needs a run with log_sets."""
        return self.sets[self.set_offsets[k]:self.set_offsets[k + 1]]

    def __del__(self, _release=_release):
        h = getattr(self, "_h", None)
        if h:
            _release("chap_run_destroy", h)
            self._h = None


class Problem:
    """chap_problem_create on a MIP in original form (host numpy arrays)."""

    def __init__(self, mip, feas_tol: float = 1e-6, graph_iters: int = 0, short_max: int = 0, chunk_min: int = 0,
                 chunk_len: int = 0, row_stage: int = 0, rescore_cap: int = 0):
        lib = load_library()
        self._keep = dict(
            csr_row_ptr=np.ascontiguousarray(mip.csr_row_ptr, dtype=np.int64),
            csr_col=np.ascontiguousarray(mip.csr_col, dtype=np.int32),
            csr_val=np.ascontiguousarray(mip.csr_val, dtype=np.float64),
            csc_col_ptr=np.ascontiguousarray(mip.csc_col_ptr, dtype=np.int64),
            csc_row=np.ascontiguousarray(mip.csc_row, dtype=np.int32),
            csc_val=np.ascontiguousarray(mip.csc_val, dtype=np.float64),
            sense=np.ascontiguousarray(mip.sense, dtype=np.uint8),
            rhs=np.ascontiguousarray(mip.rhs, dtype=np.float64),
            lb=np.ascontiguousarray(mip.lb, dtype=np.float64),
            ub=np.ascontiguousarray(mip.ub, dtype=np.float64),
            is_int=np.ascontiguousarray(mip.is_int, dtype=np.uint8),
            obj=np.ascontiguousarray(mip.obj, dtype=np.float64),
        )
        o = default_options()
        o.feas_tol = feas_tol
        o.graph_iters = graph_iters
        o.short_max = short_max
        o.chunk_min = chunk_min
        o.chunk_len = chunk_len
        o.row_stage = row_stage
        o.rescore_cap = rescore_cap
        h = ctypes.c_void_p()
        k = self._keep
        _check(lib.chap_problem_create(ctypes.byref(h), int(mip.n), int(mip.m), _ptr(k["csr_row_ptr"]),
                                       _ptr(k["csr_col"]), _ptr(k["csr_val"]), _ptr(k["csc_col_ptr"]),
                                       _ptr(k["csc_row"]), _ptr(k["csc_val"]), _ptr(k["sense"]), _ptr(k["rhs"]),
                                       _ptr(k["lb"]), _ptr(k["ub"]), _ptr(k["is_int"]), _ptr(k["obj"]),
                                       ctypes.byref(o)))
        self._h = h
        self._keep = None
        self.n = int(mip.n)
        self.m = int(mip.m)
        self.mp = int(lib.chap_problem_num_norm_rows(h))

    def __del__(self, _release=_release):
        h = getattr(self, "_h", None)
        if h:
            _release("chap_problem_destroy", h)
            self._h = None

    def norm_row_map(self):
        orig = np.empty(self.mp, dtype=np.int32)
        sign = np.empty(self.mp, dtype=np.int8)
        _check(load_library().chap_problem_norm_row_map(self._h, _ptr(orig), _ptr(sign)))
        return orig, sign

    def best_shift(self, x, w, cutoff_rhs: float = math.inf, out_shift=None, out_score=None, stream=None):
        """chap_best_shift on device tensors x (n, float64) and w (m'+1,
        float32); returns (xhat, score) device tensors."""
        import torch
        assert x.is_cuda and x.dtype == torch.float64 and x.is_contiguous() and x.numel() == self.n
        assert w.is_cuda and w.dtype == torch.float32 and w.is_contiguous() and w.numel() == self.mp + 1
        if out_shift is None:
            out_shift = torch.empty_like(x)
        if out_score is None:
            out_score = torch.empty_like(x)
        _check(load_library().chap_best_shift(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                              float(cutoff_rhs), ctypes.c_void_p(out_shift.data_ptr()),
                                              ctypes.c_void_p(out_score.data_ptr()), _stream_handle(stream)))
        return out_shift, out_score

    def best_shift_noalloc(self, x, w, out_shift, out_score, cutoff_rhs: float = math.inf, stream=None):
        """chap_best_shift_noalloc into caller-provided device tensors (no
        allocation anywhere on the call's path)."""
        import torch
        assert x.is_cuda and x.dtype == torch.float64 and x.is_contiguous() and x.numel() == self.n
        assert w.is_cuda and w.dtype == torch.float32 and w.is_contiguous() and w.numel() == self.mp + 1
        for t in (out_shift, out_score):
            assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == self.n
        _check(load_library().chap_best_shift_noalloc(
            self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(w.data_ptr()), float(cutoff_rhs),
            ctypes.c_void_p(out_shift.data_ptr()), ctypes.c_void_p(out_score.data_ptr()), _stream_handle(stream)))
        return out_shift, out_score

    def jump_values(self, x, w, cutoff_rhs: float = math.inf, out_jump=None, out_score=None, stream=None):
        """chap_jump_values on device tensors x (n, float64) and w (m'+1,
        float32); returns (jump value, jump score) device tensors."""
        import torch
        assert x.is_cuda and x.dtype == torch.float64 and x.is_contiguous() and x.numel() == self.n
        assert w.is_cuda and w.dtype == torch.float32 and w.is_contiguous() and w.numel() == self.mp + 1
        if out_jump is None:
            out_jump = torch.empty_like(x)
        if out_score is None:
            out_score = torch.empty_like(x)
        _check(load_library().chap_jump_values(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                               float(cutoff_rhs), ctypes.c_void_p(out_jump.data_ptr()),
                                               ctypes.c_void_p(out_score.data_ptr()), _stream_handle(stream)))
        return out_jump, out_score

    def last_jump_ms(self) -> float:
        """chap_jump_values_ms: HIP-event duration of the last jump kernels."""
        ms = ctypes.c_double()
        _check(load_library().chap_jump_values_ms(self._h, ctypes.byref(ms)))
        return ms.value

    def last_pass_ms(self) -> float:
        """chap_best_shift_pass_ms: HIP-event duration of the last pass."""
        ms = ctypes.c_double()
        _check(load_library().chap_best_shift_pass_ms(self._h, ctypes.byref(ms)))
        return ms.value

    def tabu_run(self, iters: int, tenure: int, seed: int, x0=None, stream=None) -> Run:
        """chap_tabu_run: synchronous; returns the trace and final state."""
        h = ctypes.c_void_p()
        x0p = None
        if x0 is not None:
            x0 = np.ascontiguousarray(x0, dtype=np.float64)
            assert x0.shape[0] == self.n
            x0p = _ptr(x0)
        _check(load_library().chap_tabu_run(self._h, int(iters), int(tenure), int(seed), x0p, ctypes.byref(h),
                                            _stream_handle(stream)))
        return Run(h, self.n, self.mp)


def autotune(problem, candidates=None, walk_iters: int = 64):
    """chap_autotune: returns (best ChapOptions, ms per iteration of every
    candidate). candidates: list of dicts of option overrides, or None for the
    built-in grid."""
    lib = load_library()
    if candidates:
        arr = (ChapOptions * len(candidates))()
        for i, c in enumerate(candidates):
            o = default_options()
            for k, v in c.items():
                setattr(o, k, v)
            arr[i] = o
        ptr, nc = ctypes.cast(arr, ctypes.c_void_p), len(candidates)
    else:
        ptr, nc = None, 0
    ms = np.zeros(max(nc, 8))
    best = ChapOptions()
    _check(lib.chap_autotune(problem._h, ptr, nc, int(walk_iters), ctypes.byref(best), _ptr(ms)))
    return best, ms[:nc if nc else 8]


def learned_options(**kw) -> LearnedOptions:
    o = LearnedOptions()
    load_library().chap_learned_options_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown learned option {k}")
        setattr(o, k, v)
    return o


def learned_run(problem, model, iters: int, tenure: int, seed: int, x0=None, stream=None, **options) -> Run:
    """chap_learned_run: synchronous; options as chap_learned_options
    (topk, full_every, train_steps, train_pairs, lr, log_sets, log_pairs,
    train_seed)."""
    o = learned_options(**options)
    h = ctypes.c_void_p()
    x0p = None
    if x0 is not None:
        x0 = np.ascontiguousarray(x0, dtype=np.float64)
        assert x0.shape[0] == problem.n
        x0p = _ptr(x0)
    _check(load_library().chap_learned_run(problem._h, model._h, ctypes.byref(o), int(iters), int(tenure), int(seed),
                                           x0p, ctypes.byref(h), _stream_handle(stream)))
    return Run(h, problem.n, problem.mp)


def features(problem, x, w, cutoff_rhs, s_last, xhat_last, last_move, moves, k: int, k_last_full: int,
             stream=None):
    """chap_features on device tensors (original order); returns an (n, 16)
    int16 tensor of bfloat16 bit patterns."""
    import torch
    n = problem.n
    out = torch.empty((n, 16), dtype=torch.int16, device=x.device)
    _check(load_library().chap_features(
        problem._h, _dev_ptr(x, torch.float64, n), _dev_ptr(w, torch.float32, problem.mp + 1), float(cutoff_rhs),
        _dev_ptr(s_last, torch.float64, n), _dev_ptr(xhat_last, torch.float64, n), _dev_ptr(last_move, torch.int32, n),
        _dev_ptr(moves, torch.int32, n), int(k), int(k_last_full), _dev_ptr(out, torch.int16, n * 16),
        _stream_handle(stream)))
    return out


def batch_run(problems, walk_prob, walk_seed, iters: int, tenure: int, stream=None, walk_x0=None):
    """chap_batch_run: walk w runs on problems[walk_prob[w]] from walk_x0[w]
    (host array, or None) or else the start point of seed walk_seed[w];
    returns one Run per walk."""
    lib = load_library()
    nprob = len(problems)
    handles = (ctypes.c_void_p * nprob)(*[p._h.value for p in problems])
    wp = np.ascontiguousarray(walk_prob, dtype=np.int32)
    ws = np.ascontiguousarray(walk_seed, dtype=np.uint64)
    nw = wp.shape[0]
    x0p = None
    keep = []
    if walk_x0 is not None:
        x0p = (ctypes.c_void_p * nw)()
        for w in range(nw):
            if walk_x0[w] is not None:
                a = np.ascontiguousarray(walk_x0[w], dtype=np.float64)
                assert a.shape[0] == problems[wp[w]].n
                keep.append(a)
                x0p[w] = a.ctypes.data
        x0p = ctypes.cast(x0p, ctypes.c_void_p)
    out = (ctypes.c_void_p * nw)()
    _check(lib.chap_batch_run(ctypes.cast(handles, ctypes.c_void_p), nprob, _ptr(wp), _ptr(ws), x0p, nw,
                              int(iters), int(tenure), ctypes.cast(out, ctypes.c_void_p), _stream_handle(stream)))
    return [Run(ctypes.c_void_p(out[w]), problems[wp[w]].n, problems[wp[w]].mp) for w in range(nw)]


def batch_restarts(problems, walk_prob, walk_seed, iters: int, tenure: int, restart_every: int, min_distance: int,
                   stream=None):
    """chap_batch_restarts: batched walks with diversity-driven restarts;
    returns one Run per walk (Run.restarts: the iterations at which it
    restarted)."""
    lib = load_library()
    nprob = len(problems)
    handles = (ctypes.c_void_p * nprob)(*[p._h.value for p in problems])
    wp = np.ascontiguousarray(walk_prob, dtype=np.int32)
    ws = np.ascontiguousarray(walk_seed, dtype=np.uint64)
    nw = wp.shape[0]
    out = (ctypes.c_void_p * nw)()
    _check(lib.chap_batch_restarts(ctypes.cast(handles, ctypes.c_void_p), nprob, _ptr(wp), _ptr(ws), nw, int(iters),
                                   int(tenure), int(restart_every), int(min_distance),
                                   ctypes.cast(out, ctypes.c_void_p), _stream_handle(stream)))
    return [Run(ctypes.c_void_p(out[w]), problems[wp[w]].n, problems[wp[w]].mp) for w in range(nw)]


MODEL_NPARAM = 5313


def _dev_ptr(t, dtype, numel=None):
    import torch
    assert t.is_cuda and t.dtype == dtype and t.is_contiguous(), (t.device, t.dtype)
    if numel is not None:
        assert t.numel() == numel, (t.numel(), numel)
    return ctypes.c_void_p(t.data_ptr())


class Model:
    """The candidate-proposal network (chap_model_*). Feature tensors are
    (n, 16) int16 tensors holding bfloat16 bit patterns (or torch.bfloat16)."""

    def __init__(self, seed: int = 0):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.chap_model_create(ctypes.byref(h), int(seed)))
        self._h = h

    def __del__(self, _release=_release):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _release("chap_model_destroy", h)
            self._h = None

    @staticmethod
    def _feat(feat):
        import torch
        if feat.dtype == torch.bfloat16:
            feat = feat.view(torch.int16)
        assert feat.dim() == 2 and feat.shape[1] == 16
        return _dev_ptr(feat, torch.int16)

    def get_params(self) -> np.ndarray:
        out = np.empty(MODEL_NPARAM, dtype=np.float32)
        _check(load_library().chap_model_get_params(self._h, _ptr(out)))
        return out

    def set_params(self, params) -> None:
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.shape == (MODEL_NPARAM,)
        _check(load_library().chap_model_set_params(self._h, _ptr(p)))

    def forward(self, feat, out=None, stream=None):
        import torch
        n = feat.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=feat.device)
        _check(load_library().chap_model_forward(self._h, self._feat(feat), n, _dev_ptr(out, torch.float32, n),
                                                 _stream_handle(stream)))
        return out

    def grad(self, feat, target, out=None, stream=None):
        import torch
        n = feat.shape[0]
        if out is None:
            out = torch.empty(MODEL_NPARAM, dtype=torch.float32, device=feat.device)
        _check(load_library().chap_model_grad(self._h, self._feat(feat), _dev_ptr(target, torch.float32, n), n,
                                              _dev_ptr(out, torch.float32, MODEL_NPARAM), _stream_handle(stream)))
        return out

    def train(self, feat, target, steps: int, batch: int, lr: float, seed: int = 0, stream=None) -> None:
        import torch
        n = feat.shape[0]
        _check(load_library().chap_model_train(self._h, self._feat(feat), _dev_ptr(target, torch.float32, n), n,
                                               int(steps), int(batch), float(lr), int(seed), _stream_handle(stream)))
