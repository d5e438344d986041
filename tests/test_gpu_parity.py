"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Integer data: bit-exact (scores are sums of +-w, +-w/2 with integer weights,
exact in FP64; breakpoints and residuals use the same IEEE operations in the
same order). Continuous data: residuals of ordinary rows are still computed in
the same order and match bit for bit; the cutoff row's activity is a
parallel sum on the GPU, so with an active cutoff the shifts agree to 1e-12
relative and the scores exactly.
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


def test_best_shift_continuous_data(chap):
    for seed in range(6):
        mip = mipgen.random_mixed(500 + seed, n=80, m=60, integer_data=False, frac_bin=0.2, frac_int=0.3)
        P = oracle.OracleProblem(mip)
        x = mipgen.random_point(mip, seed)
        w = mipgen.random_weights(P.mp + 1, seed)
        say(f"best_shift continuous seed={seed}")
        xh, s = gpu_best_shift(chap, mip, x, w)
        oxh, os_ = P.best_shift(x, w)
        assert_same(s, os_, "score")
        assert_same(xh, oxh, "shift")
        cutoff = float(mip.obj @ x) - 0.37
        xh, s = gpu_best_shift(chap, mip, x, w, cutoff)
        oxh, os_ = P.best_shift(x, w, cutoff)
        assert_same(s, os_, "score (cutoff)")
        np.testing.assert_allclose(xh, oxh, rtol=1e-12, atol=1e-12)


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


def compare_runs(g, o, what, exact=True):
    gt, ot = g.trace, o["trace"]
    assert gt.shape == ot.shape
    for f in ("iter", "var", "kind", "viol"):
        assert_same(gt[f], ot[f], f"{what} trace.{f}")
    for f in ("x_old", "x_new", "score", "obj"):
        if exact:
            assert_same(gt[f], ot[f], f"{what} trace.{f}")
        else:
            np.testing.assert_allclose(gt[f], ot[f], rtol=1e-12, atol=1e-9)
    if exact:
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
        mip = mipgen.random_mixed(700 + seed, n=50, m=40, max_row_nnz=6, long_cols=2, long_deg=20)
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


def test_tabu_general_scaled_continuous(chap):
    """Continuous data: the walk keeps residuals incrementally while the oracle
    recomputes them; trajectories agree step for step on these sizes and the
    values to 1e-12 relative."""
    mip = mipgen.general(1, n=4000, m=2000)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip)
    say("tabu general scaled (continuous data) 150 iters")
    g = G.tabu_run(150, 10, 0)
    o = P.tabu_run(150, 10, 0)
    compare_runs(g, o, "general", exact=False)
    # the incremental residual agrees with a from-scratch residual at the final point
    r, _ = P.residual(g.x, g.cutoff_rhs)
    scale = np.abs(r) + 1.0
    assert np.all(np.abs(g.resid - r) <= 1e-9 * scale)


def test_tabu_edge_cases(chap):
    # no rows at all: every shift scores 0; walk only reweights
    mip = mipgen.random_mixed(11, n=5, m=0)
    P = oracle.OracleProblem(mip)
    say("tabu edge: m=0")
    compare_runs(chap.Problem(mip).tabu_run(5, 2, 3), P.tabu_run(5, 2, 3), "m=0")
    # zero iterations
    mip = mipgen.random_mixed(12, n=20, m=15)
    P = oracle.OracleProblem(mip)
    say("tabu edge: iters=0")
    g = chap.Problem(mip).tabu_run(0, 3, 1)
    o = P.tabu_run(0, 3, 1)
    assert g.trace.shape[0] == 0
    assert_same(g.x, o["x"], "x")
    assert_same(g.resid, o["r"], "resid")
    # user start point
    x0 = mipgen.random_point(mip, 4)
    say("tabu edge: x0 given")
    compare_runs(chap.Problem(mip).tabu_run(40, 2, 0, x0=x0), P.tabu_run(40, 2, 0, x0=x0), "x0")
    # fixed variables and infinite bounds
    mip = mipgen.random_mixed(13, n=30, m=20, inf_bounds=0.3)
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
