"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Bit-exact everywhere. Scores are sums of +-w, +-w/2 with integer weights,
exact in FP64; breakpoints and residuals of ordinary rows use the same IEEE
operations in the same order (rows summed in the caller's CSR order). The
objective row's activity c^T x, a sum over every variable, is the exact
value rounded once on both sides (an exactly rounded sum in the oracle, a
fixed-point exact sum kept incrementally on the GPU), so walks on continuous
data agree bit for bit too, past the first incumbent.
"""
from __future__ import annotations

import math
import os
import sys

import numpy as np
import pytest

import mipgen
import oracle

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def chap():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2605_05086_amd as c

    c.load_library()
    return c


def gpu_best_shift(c, mip, x, w, cutoff=math.inf, **opts):
    import torch

    P = c.Problem(mip, **opts)
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()
    wd = torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).cuda()
    xh, s = P.best_shift(xd, wd, cutoff)
    torch.cuda.synchronize()
    return xh.cpu().numpy(), s.cpu().numpy()


def assert_same(a, b, what):
    a = np.asarray(a)
    b = np.asarray(b)
    bad = np.flatnonzero(~((a == b) | (np.isnan(a) & np.isnan(b))))
    assert bad.size == 0, f"{what}: {bad.size} mismatches, first at {bad[:5]}: gpu {a[bad[:5]]} oracle {b[bad[:5]]}"


ROUTING = [
    dict(),
    dict(short_max=1),
    dict(short_max=4),
    dict(short_max=1, chunk_min=3, chunk_len=2),
    dict(short_max=2, chunk_min=6, chunk_len=7),
]


@pytest.mark.parametrize("route", range(len(ROUTING)))
@pytest.mark.parametrize("cut", [False, True])
def test_best_shift_random_mixed(chap, route, cut):
    opts = ROUTING[route]
    for seed in range(12):
        mip = mipgen.random_mixed(100 + seed, n=60, m=50, max_row_nnz=8, int_width=40 if seed % 2 else 12,
                                  inf_bounds=0.1 if seed % 3 == 0 else 0.0, long_cols=3, long_deg=30)
        P = oracle.OracleProblem(mip)
        x = mipgen.random_point(mip, seed)
        w = mipgen.random_weights(P.mp + 1, seed + 5)
        cutoff = float(np.floor(mip.obj @ x)) - 3.0 if cut else math.inf
        say(f"best_shift random_mixed seed={seed} route={opts} cut={cut}")
        xh, s = gpu_best_shift(chap, mip, x, w, cutoff, **opts)
        oxh, os_ = P.best_shift(x, w, cutoff)
        assert_same(s, os_, f"score seed={seed}")
        assert_same(xh, oxh, f"shift seed={seed}")


@pytest.mark.parametrize("deg", [70, 300, 1500, 2500])
def test_best_shift_long_general_columns(chap, deg):
    """General (continuous / wide integer) columns beyond one wavefront and
    beyond the largest LDS sort (entries > 4096 with equality pairs)."""
    for seed in range(2):
        mip = mipgen.random_mixed(300 + seed, n=40, m=max(3000, deg + 10), max_row_nnz=3, frac_bin=0.2,
                                  frac_int=0.3, int_width=200, long_cols=4, long_deg=deg)
        P = oracle.OracleProblem(mip)
        x = mipgen.random_point(mip, seed)
        w = mipgen.random_weights(P.mp + 1, seed + 9)
        say(f"best_shift long general deg={deg} seed={seed}")
        xh, s = gpu_best_shift(chap, mip, x, w)
        oxh, os_ = P.best_shift(x, w)
        assert_same(s, os_, "score")
        assert_same(xh, oxh, "shift")


@pytest.mark.parametrize("objective", ["plain", "irrational", "wide"])
def test_best_shift_continuous_data(chap, objective):
    """Continuous data with an active cutoff row: the cutoff residual is
    c^T x - b_c rounded once (objective products that are inexact in FP64,
    magnitudes from 1e-9 to 1e9 that cancel), so shifts and scores are
    bit-exact."""
    for seed in range(6):
        mip = mipgen.random_mixed(500 + seed, n=80, m=60, integer_data=False, frac_bin=0.2, frac_int=0.3)
        rng = np.random.default_rng(seed)
        if objective == "irrational":
            mip.obj[:] = mip.obj * np.pi
        elif objective == "wide":
            mip.obj[:] = mip.obj * 10.0 ** rng.integers(-9, 10, size=mip.n)
        P = oracle.OracleProblem(mip)
        x = mipgen.random_point(mip, seed)
        w = mipgen.random_weights(P.mp + 1, seed)
        say(f"best_shift continuous {objective} seed={seed}")
        xh, s = gpu_best_shift(chap, mip, x, w)
        oxh, os_ = P.best_shift(x, w)
        assert_same(s, os_, "score")
        assert_same(xh, oxh, "shift")
        for off in (0.37, -2.5e-7, 1e-3):
            cutoff = P.objective(x) - off
            xh, s = gpu_best_shift(chap, mip, x, w, cutoff)
            oxh, os_ = P.best_shift(x, w, cutoff)
            assert_same(s, os_, f"score (cutoff offset {off})")
            assert_same(xh, oxh, f"shift (cutoff offset {off})")


def test_best_shift_workload_shapes(chap):
    cases = [("tiny_binary", mipgen.tiny_binary(0)),
             ("general n=100k", mipgen.general(0)),
             ("powerlaw n=200k nnz=2M", mipgen.powerlaw(0, n=200_000, m=100_000, nnz=2_000_000, cap=20_000))]
    for name, mip in cases:
        P = oracle.OracleProblem(mip)
        for seed in (0, 3):
            x = P.start_point(seed)
            w = mipgen.random_weights(P.mp + 1, seed + 1, wmax=5)
            say(f"best_shift {name} seed={seed}")
            xh, s = gpu_best_shift(chap, mip, x, w)
            oxh, os_ = P.best_shift(x, w)
            assert_same(s, os_, f"{name} score")
            assert_same(xh, oxh, f"{name} shift")


@pytest.mark.parametrize("n", [1, 4095, 4096, 4097, 8191, 8192, 8193, 12289, 20000])
def test_best_shift_point_permutation_sizes(chap, n):
    """The caller's point enters internal column order, and the results leave
    it, through two-pass permutations over chunks of 8192 and blocks of 4096
    columns: sizes at, around and past those edges, with ragged last chunks
    and blocks."""
    mip = mipgen.random_mixed(900 + n % 97, n=n, m=max(4, n // 2), max_row_nnz=6, int_width=20, long_cols=0)
    P = oracle.OracleProblem(mip)
    x = mipgen.random_point(mip, 1)
    w = mipgen.random_weights(P.mp + 1, 2)
    say(f"best_shift permutation sizes n={n}")
    xh, s = gpu_best_shift(chap, mip, x, w)
    oxh, os_ = P.best_shift(x, w)
    assert_same(s, os_, f"score n={n}")
    assert_same(xh, oxh, f"shift n={n}")


def compare_runs(g, o, what):
    """Trace, final point, residuals, weights, best objective, cutoff and
    best point, bit for bit."""
    gt, ot = g.trace, o["trace"]
    assert gt.shape == ot.shape
    for f in ("iter", "var", "kind", "viol", "x_old", "x_new", "score", "obj"):
        assert_same(gt[f], ot[f], f"{what} trace.{f}")
    assert_same(g.x, o["x"], f"{what} x")
    assert_same(g.resid, o["r"], f"{what} resid")
    assert_same(g.w, o["w"], f"{what} w")
    assert g.best_obj == o["best_obj"] and g.cutoff_rhs == o["cutoff_rhs"]
    if o["best_x"] is not None:
        assert_same(g.best_x, o["best_x"], f"{what} best_x")
    else:
        assert g.best_x is None


def test_tabu_tiny_binary_full(chap):
    mip = mipgen.tiny_binary(0)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip)
    say("tabu tiny_binary 1000 iters tenure 10 seed 0")
    g = G.tabu_run(1000, 10, 0)
    o = P.tabu_run(1000, 10, 0)
    compare_runs(g, o, "tiny_binary")
    for seed in (1, 99):
        say(f"tabu tiny_binary seed={seed}")
        compare_runs(G.tabu_run(300, 7, seed), P.tabu_run(300, 7, seed), f"tiny_binary seed={seed}")


@pytest.mark.parametrize("graph_iters", [1, 5, 64])
def test_tabu_random_mixed(chap, graph_iters):
    for seed in range(6):
        mip = mipgen.random_mixed(700 + seed, n=50, m=40, max_row_nnz=6, long_cols=2, long_deg=20,
                                  frac_bin=0.4, frac_int=0.6, int_width=30 if seed % 2 else 10,
                                  inf_bounds=0.15 if seed % 3 == 0 else 0.0)
        P = oracle.OracleProblem(mip)
        G = chap.Problem(mip, graph_iters=graph_iters, short_max=1 + seed % 8, chunk_min=8, chunk_len=5)
        for ws, tenure in ((0, 3), (seed + 1, 0)):
            say(f"tabu random_mixed seed={seed} walk_seed={ws} tenure={tenure} K={graph_iters}")
            compare_runs(G.tabu_run(150, tenure, ws), P.tabu_run(150, tenure, ws), f"mixed {seed}/{ws}")


def test_tabu_powerlaw_scaled(chap):
    mip = mipgen.powerlaw(0, n=20_000, m=10_000, nnz=200_000, cap=2000)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip)
    for seed in (0, 5):
        say(f"tabu powerlaw scaled seed={seed}")
        compare_runs(G.tabu_run(200, 10, seed), P.tabu_run(200, 10, seed), f"powerlaw seed={seed}")


def test_tabu_continuous_variables(chap):
    """Instances with continuous variables, real right-hand sides and
    fractional objectives. The walk recomputes every touched row from scratch
    in the caller's CSR order and keeps c^T x as an exact sum, so its trace,
    residuals, cutoff and incumbents equal the oracle's bit for bit, also after
    the first feasible point activates the cutoff row."""
    cases = [("general n=4000", mipgen.general(1, n=4000, m=2000), 300),
             ("general n=100k", mipgen.general(0), 60),
             ("mixed", mipgen.random_mixed(41, n=60, m=50, frac_bin=0.3, frac_int=0.3), 300),
             ("mixed 2", mipgen.random_mixed(42, n=80, m=40, frac_bin=0.2, frac_int=0.3, integer_data=False), 300),
             ("mixed 3", mipgen.random_mixed(43, n=40, m=12, frac_bin=0.2, frac_int=0.3, integer_data=False), 400),
             ("mixed 4", mipgen.random_mixed(44, n=30, m=10, frac_bin=0.3, frac_int=0.2, integer_data=False), 400)]
    incumbents = 0
    for name, mip, iters in cases:
        if name.startswith("mixed"):
            mip.obj[:] = mip.obj * np.pi / 3.0   # products inexact in FP64
        P = oracle.OracleProblem(mip)
        G = chap.Problem(mip)
        say(f"tabu continuous {name} {iters} iters")
        g = G.tabu_run(iters, 10, 0)
        o = P.tabu_run(iters, 10, 0)
        feas = np.flatnonzero(o["trace"]["viol"] == 0)
        print(f"{name}: first feasible point after step {int(feas[0]) + 1 if feas.size else None} of {iters}",
              flush=True)
        incumbents += int(o["best_x"] is not None)
        compare_runs(g, o, name)
    assert incumbents >= 2


def test_tabu_edge_cases(chap):
    # no rows at all: every shift scores 0 until the cutoff row exists
    mip = mipgen.random_mixed(11, n=5, m=0, frac_bin=0.5, frac_int=0.5)
    P = oracle.OracleProblem(mip)
    say("tabu edge: m=0")
    compare_runs(chap.Problem(mip).tabu_run(5, 2, 3), P.tabu_run(5, 2, 3), "m=0")
    # zero iterations
    mip = mipgen.random_mixed(12, n=20, m=15, frac_bin=0.5, frac_int=0.5)
    P = oracle.OracleProblem(mip)
    say("tabu edge: iters=0")
    g = chap.Problem(mip).tabu_run(0, 3, 1)
    o = P.tabu_run(0, 3, 1)
    assert g.trace.shape[0] == 0
    assert_same(g.x, o["x"], "x")
    assert_same(g.resid, o["r"], "resid")
    # user start point (all-integer instance)
    mip = mipgen.random_mixed(14, n=25, m=20, frac_bin=0.5, frac_int=0.5)
    P = oracle.OracleProblem(mip)
    x0 = mipgen.random_point(mip, 4)
    say("tabu edge: x0 given")
    compare_runs(chap.Problem(mip).tabu_run(40, 2, 0, x0=x0), P.tabu_run(40, 2, 0, x0=x0), "x0")
    # fixed variables and infinite bounds
    mip = mipgen.random_mixed(13, n=30, m=20, inf_bounds=0.3, frac_bin=0.3, frac_int=0.7)
    mip.ub[:5] = mip.lb[:5] = np.where(np.isfinite(mip.lb[:5]), mip.lb[:5], 0.0)
    P = oracle.OracleProblem(mip)
    say("tabu edge: fixed and unbounded variables")
    compare_runs(chap.Problem(mip).tabu_run(80, 4, 0), P.tabu_run(80, 4, 0), "fixed/inf")


def test_tabu_deterministic(chap):
    mip = mipgen.powerlaw(2, n=5000, m=2500, nnz=50_000, cap=2000)
    G = chap.Problem(mip, chunk_min=64, chunk_len=64)
    say("tabu determinism x3")
    runs = [G.tabu_run(100, 10, 0) for _ in range(3)]
    for r in runs[1:]:
        assert r.trace.tobytes() == runs[0].trace.tobytes()
        assert r.x.tobytes() == runs[0].x.tobytes()


@pytest.mark.slow
def test_full_size_powerlaw(chap):
    """The 20M-nonzero instance at full size: every column's best shift at two
    points, and the first iterations of the walk."""
    mip = mipgen.powerlaw(0)
    P = oracle.OracleProblem(mip)
    for seed in (0, 1):
        x = P.start_point(seed)
        w = mipgen.random_weights(P.mp + 1, seed, wmax=4)
        say(f"best_shift powerlaw full seed={seed}")
        xh, s = gpu_best_shift(chap, mip, x, w)
        oxh, os_ = P.best_shift(x, w)
        assert_same(s, os_, "score")
        assert_same(xh, oxh, "shift")
    G = chap.Problem(mip)
    say("tabu powerlaw full 3 iters")
    compare_runs(G.tabu_run(3, 10, 0), P.tabu_run(3, 10, 0), "powerlaw full")


@pytest.mark.slow
def test_full_size_snapshot_parity(chap):
    """The 20M-nonzero walk at iterations 1000, 5000 and 9999: the GPU walk's
    state (point, weights, tabu list, incumbent, cutoff) is downloaded there;
    every column's best shift at that state equals the oracle's, and the next
    two GPU iterations equal the oracle walk continued from that state, bit
    for bit."""
    import torch

    from helpers import tabu_until_from_trace

    mip = mipgen.powerlaw(0)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip)
    for k0 in (1000, 5000, 9999):
        say(f"snapshot parity at iteration {k0}: GPU walk")
        g = G.tabu_run(k0, 10, 0)
        tb = tabu_until_from_trace(g.trace, mip.n, 10)
        xd = torch.from_numpy(g.x).cuda()
        wd = torch.from_numpy(g.w).cuda()
        xh, s = G.best_shift(xd, wd, g.cutoff_rhs)
        torch.cuda.synchronize()
        say(f"snapshot parity at iteration {k0}: oracle best shift")
        oxh, os_ = P.best_shift(g.x, g.w, g.cutoff_rhs)
        assert_same(s.cpu().numpy(), os_, f"score at {k0}")
        assert_same(xh.cpu().numpy(), oxh, f"shift at {k0}")
        say(f"snapshot parity at iteration {k0}: next two iterations")
        g2 = G.tabu_run(k0 + 2, 10, 0)
        assert g2.trace[:k0].tobytes() == g.trace.tobytes()
        o = P.tabu_resume(2, 10, g.x, g.w, tb, k0, g.best_obj, g.best_x, g.cutoff_rhs)
        for f in ("iter", "var", "kind", "viol", "x_old", "x_new", "score", "obj"):
            assert_same(g2.trace[f][k0:], o["trace"][f], f"trace.{f} after {k0}")
        assert_same(g2.x, o["x"], f"x after {k0}")
        assert_same(g2.resid, o["r"], f"resid after {k0}")
        assert_same(g2.w, o["w"], f"w after {k0}")


def test_best_shift_repeatable(chap):
    """Identical passes on one problem give identical results equal to the
    oracle (catches timing-dependent corruption in the pass kernels)."""
    import torch

    mip = mipgen.powerlaw(0, n=200_000, m=100_000, nnz=2_000_000, cap=20_000)
    P = oracle.OracleProblem(mip)
    w = mipgen.random_weights(P.mp + 1, 1, wmax=5)
    G = chap.Problem(mip)
    wd = torch.from_numpy(w).cuda()
    for seed in (0, 3):
        x = P.start_point(seed)
        oxh, os_ = P.best_shift(x, w)
        xd = torch.from_numpy(x).cuda()
        for rep in range(4):
            say(f"best_shift repeat seed={seed} rep={rep}")
            xh, s = G.best_shift(xd, wd)
            torch.cuda.synchronize()
            assert_same(s.cpu().numpy(), os_, f"score rep={rep}")
            assert_same(xh.cpu().numpy(), oxh, f"shift rep={rep}")


def test_batch_equals_plain(chap):
    """Batched walks over instances of uneven size: every walk's trace and
    final state equal the plain walk's, bit for bit; two walks are also
    checked against the oracle."""
    mips = [mipgen.general(900 + k, n=n, m=n // 2) for k, n in enumerate((3000, 800, 6000))]
    mips.append(mipgen.powerlaw(5, n=8000, m=4000, nnz=80_000, cap=3000))
    probs = [chap.Problem(m) for m in mips]
    walk_prob = [w % len(probs) for w in range(10)]
    walk_seed = [w + 1 for w in range(10)]
    say("batch of 10 walks on 4 instances, 120 iterations")
    runs = chap.batch_run(probs, walk_prob, walk_seed, 120, 10)
    for w, r in enumerate(runs):
        say(f"plain walk {w}")
        g = probs[walk_prob[w]].tabu_run(120, 10, walk_seed[w])
        assert r.trace.tobytes() == g.trace.tobytes(), f"walk {w} trace"
        assert r.x.tobytes() == g.x.tobytes() and r.resid.tobytes() == g.resid.tobytes()
        assert r.w.tobytes() == g.w.tobytes() and r.best_obj == g.best_obj
    for w in (3, 7):
        say(f"oracle walk {w}")
        o = oracle.OracleProblem(mips[walk_prob[w]]).tabu_run(120, 10, walk_seed[w])
        compare_runs(runs[w], o, f"batch walk {w}")


def test_autotune_picks_a_candidate(chap):
    mip = mipgen.random_mixed(77, n=400, m=300, max_row_nnz=8, long_cols=4, long_deg=120)
    G = chap.Problem(mip)
    say("autotune grid")
    best, ms = chap.autotune(G, walk_iters=16)
    assert ms.shape == (8,) and np.all(ms > 0)
    assert best.short_max in (4, 8) and best.chunk_len in (2048, 4096) and best.graph_iters in (32, 64)
    cands = [dict(short_max=2, chunk_min=16, chunk_len=16, graph_iters=8), dict(short_max=8, graph_iters=64)]
    best2, ms2 = chap.autotune(G, cands, walk_iters=16)
    assert ms2.shape == (2,) and (best2.short_max, best2.graph_iters) in ((2, 8), (8, 64))
    # the tuned problem walks exactly as the default one
    T = chap.Problem(mip, short_max=best2.short_max, chunk_min=best2.chunk_min, chunk_len=best2.chunk_len,
                     graph_iters=best2.graph_iters)
    np.testing.assert_array_equal(T.tabu_run(100, 10, 3).trace, G.tabu_run(100, 10, 3).trace)


@pytest.mark.parametrize("wkind", ["integral", "fractional", "large", "cutoff fractional", "cutoff large"])
def test_best_shift_weight_kinds(chap, wkind):
    """All-integer instances let a single pass gather a compact copy of the
    rows when the caller's weights are integers below 65535; fractional or
    large weights must take the full-row path, and so must an active cutoff
    row whose weight alone is fractional or large. Both agree with the
    oracle."""
    mip = mipgen.random_mixed(91, n=300, m=200, max_row_nnz=8, int_width=30, long_cols=3, long_deg=60)
    P = oracle.OracleProblem(mip)
    x = mipgen.random_point(mip, 4)
    w = mipgen.random_weights(P.mp + 1, 5)
    cutoff = math.inf
    if wkind == "fractional":
        w = w + np.float32(0.5)
    elif wkind == "large":
        w[::7] = 70000.0
    elif wkind.startswith("cutoff"):
        w[P.mp] = 2.5 if wkind == "cutoff fractional" else 70000.0
        cutoff = float(np.floor(mip.obj @ x)) - 3.0
    say(f"best_shift weights {wkind}")
    xh, s = gpu_best_shift(chap, mip, x, w, cutoff)
    oxh, os_ = P.best_shift(x, w, cutoff)
    assert_same(xh, oxh, f"shift ({wkind} weights)")
    assert_same(s, os_, f"score ({wkind} weights)")


STAGE_CASES = [
    ("mixed", lambda: mipgen.random_mixed(71, n=400, m=300, max_row_nnz=9, frac_bin=0.2, frac_int=0.8,
                                          int_width=90, long_cols=4, long_deg=120), {}),
    ("few rows", lambda: mipgen.random_mixed(72, n=50, m=5, max_row_nnz=12, frac_bin=0.3, frac_int=0.7), {}),
    ("powerlaw", lambda: mipgen.powerlaw(73, n=30_000, m=15_000, nnz=300_000, cap=5000), {}),
    # many long columns spanning several 8192-row blocks
    ("long", lambda: mipgen.powerlaw(75, n=40_000, m=30_000, nnz=400_000, cap=20_000), dict(chunk_min=24)),
]


@pytest.mark.parametrize("case", range(len(STAGE_CASES)))
@pytest.mark.parametrize("row_stage", [1, -1])
@pytest.mark.parametrize("cut", [False, True])
def test_best_shift_row_stage(chap, case, row_stage, cut):
    """Short and packed narrow columns scored from row-range records (the
    default on all-integer instances) and from direct gathers (row_stage=-1):
    both equal the oracle bit for bit, with and without the cutoff row, with
    empty row ranges (5 rows) and offsets beyond the +-64 clamp."""
    name, make, opts = STAGE_CASES[case]
    mip = make()
    P = oracle.OracleProblem(mip)
    for seed in (0, 2):
        x = mipgen.random_point(mip, seed)
        w = mipgen.random_weights(P.mp + 1, seed + 1, wmax=9)
        cutoff = float(np.dot(mip.obj, x)) + 3.0 if cut else math.inf
        say(f"best_shift staged {name} row_stage={row_stage} cut={cut} seed={seed}")
        xh, s = gpu_best_shift(chap, mip, x, w, cutoff, row_stage=row_stage, **opts)
        oxh, os_ = P.best_shift(x, w, cutoff)
        assert_same(s, os_, f"{name} score")
        assert_same(xh, oxh, f"{name} shift")


def test_tabu_row_stage_long_columns(chap):
    """A walk whose long columns (more than 24 entries) take the row-block
    partials: equal to the oracle and to the unstaged walk."""
    mip = mipgen.powerlaw(76, n=20_000, m=20_000, nnz=200_000, cap=10_000)
    P = oracle.OracleProblem(mip)
    say("tabu staged long columns 60 iters")
    g = chap.Problem(mip, chunk_min=24).tabu_run(60, 5, 2)
    compare_runs(g, P.tabu_run(60, 5, 2), "staged long")
    h = chap.Problem(mip, chunk_min=24, row_stage=-1).tabu_run(60, 5, 2)
    assert g.trace.tobytes() == h.trace.tobytes()


def test_batch_row_stage_long_columns(chap):
    """Batched staged walks where some instances have long columns (their
    partial bins are combined by the move selection's extra workgroups) and
    one has none: every walk equals its plain walk bit for bit, and one
    equals the oracle."""
    mips = [mipgen.powerlaw(77, n=12_000, m=10_000, nnz=120_000, cap=6_000),
            mipgen.powerlaw(78, n=6_000, m=8_000, nnz=40_000, cap=10),
            mipgen.powerlaw(79, n=9_000, m=5_000, nnz=90_000, cap=4_000)]
    probs = [chap.Problem(m, chunk_min=24) for m in mips]
    walk_prob = [0, 1, 2, 0, 2, 1]
    walk_seed = [3, 4, 5, 6, 7, 8]
    say("batch of 6 staged walks on 3 instances, 50 iterations")
    runs = chap.batch_run(probs, walk_prob, walk_seed, 50, 5)
    for w, r in enumerate(runs):
        say(f"plain staged walk {w}")
        g = probs[walk_prob[w]].tabu_run(50, 5, walk_seed[w])
        assert r.trace.tobytes() == g.trace.tobytes(), f"walk {w} trace"
        assert r.x.tobytes() == g.x.tobytes() and r.w.tobytes() == g.w.tobytes()
    say("oracle walk 4")
    o = oracle.OracleProblem(mips[2]).tabu_run(50, 5, walk_seed[4])
    compare_runs(runs[4], o, "batch staged walk 4")


def test_tabu_row_stage_full_rows(chap):
    """A walk of 65540 iterations keeps full rows (weights may pass 65534), so
    the staged records carry row indices instead of weights; the walk equals
    the oracle and the unstaged walk."""
    mip = mipgen.random_mixed(74, n=40, m=30, max_row_nnz=6, frac_bin=0.3, frac_int=0.7)
    P = oracle.OracleProblem(mip)
    iters = 65540
    say(f"tabu staged full rows {iters} iters")
    g = chap.Problem(mip).tabu_run(iters, 3, 1)
    compare_runs(g, P.tabu_run(iters, 3, 1), "staged full rows")
    say(f"tabu unstaged full rows {iters} iters")
    h = chap.Problem(mip, row_stage=-1).tabu_run(iters, 3, 1)
    assert g.trace.tobytes() == h.trace.tobytes()
