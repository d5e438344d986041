"""Jump values (weighted-violation minimisers) through the C ABI against the
oracle (section 3.1 "Best Shift Moves"; the oracle's definition is pinned
in test_jump_oracle.py).

Every column of at most 4096 entries sums V in the oracle's order, so the
jump value and score are bit-exact on any data. Longer columns add the
partial sums of 4096-entry chunks: bit-exact on integer data, and on other
data the score within 1e-12 relative and the value one the oracle scores
within that tolerance of its best.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import mipgen
import oracle
from test_gpu_parity import assert_same, chap, say  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def gpu_jump(G, x, w, cutoff=math.inf):
    import torch
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()
    wd = torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).cuda()
    jv, js = G.jump_values(xd, wd, cutoff)
    torch.cuda.synchronize()
    return jv.cpu().numpy(), js.cpu().numpy()


def check_exact(lib, mip, x, w, cutoff, what, G=None):
    P = oracle.OracleProblem(mip)
    G = G or lib.Problem(mip)
    ojv, ojs = P.jump_values(x, w, cutoff)
    gjv, gjs = gpu_jump(G, x, w, cutoff)
    assert_same(gjv, ojv, f"{what} jump value")
    assert_same(gjs, ojs, f"{what} jump score")


@pytest.mark.parametrize("kind", ["narrow", "wide", "continuous", "infinite", "long"])
def test_jump_random_mixed(chap, kind):
    kw = dict(narrow=dict(int_width=12), wide=dict(int_width=300, frac_int=0.6),
              continuous=dict(integer_data=False, frac_int=0.2),
              infinite=dict(inf_bounds=0.2, integer_data=False),
              long=dict(long_cols=5, long_deg=150, int_width=90))[kind]
    for seed in range(4):
        mip = mipgen.random_mixed(300 + seed, n=300, m=200, max_row_nnz=8, **kw)
        P = oracle.OracleProblem(mip)
        x = mipgen.random_point(mip, seed)
        w = mipgen.random_weights(P.mp + 1, seed, wmax=7)
        for cut in (math.inf, P.objective(x) - 2.5):
            say(f"jump {kind} seed={seed} cutoff={cut}")
            check_exact(chap, mip, x, w, cut, f"{kind} {seed}")


def test_jump_workload_shapes(chap):
    cases = [("tiny_binary", mipgen.tiny_binary(0)), ("general 20k", mipgen.general(5, n=20_000, m=10_000)),
             ("powerlaw 200k", mipgen.powerlaw(6, n=200_000, m=100_000, nnz=2_000_000, cap=20_000))]
    for name, mip in cases:
        P = oracle.OracleProblem(mip)
        G = chap.Problem(mip)
        for seed in (0, 1):
            x = mipgen.random_point(mip, seed)
            w = mipgen.random_weights(P.mp + 1, seed, wmax=9)
            say(f"jump {name} seed={seed}")
            check_exact(chap, mip, x, w, math.inf, f"{name} {seed}", G)
        say(f"jump {name} with cutoff")
        x = mipgen.random_point(mip, 2)
        check_exact(chap, mip, x, mipgen.random_weights(P.mp + 1, 2), P.objective(x) + 1.0, f"{name} cutoff", G)


def test_jump_full_size_powerlaw(chap):
    """The 20M-nonzero instance (columns up to 100k entries: chunked, integer
    data) at a random point: every column equals the oracle."""
    mip = mipgen.powerlaw(0)
    oracle.set_threads(16)
    try:
        P = oracle.OracleProblem(mip)
        x = mipgen.random_point(mip, 3)
        w = mipgen.random_weights(P.mp + 1, 3, wmax=6)
        say("jump full-size powerlaw")
        check_exact(chap, mip, x, w, math.inf, "powerlaw 20M")
    finally:
        oracle.set_threads(1)


def test_jump_long_columns_fractional(chap):
    """General columns beyond one 4096-entry chunk on fractional data: the
    score within 1e-12 relative of the oracle's, and the value is one the
    oracle scores within that tolerance of its best."""
    mip = mipgen.random_mixed(321, n=200, m=9000, max_row_nnz=3, frac_bin=0.2, frac_int=0.2, integer_data=False,
                              long_cols=3, long_deg=8500)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip)
    x = mipgen.random_point(mip, 4)
    w = mipgen.random_weights(P.mp + 1, 4)
    say("jump long fractional columns")
    ojv, ojs = P.jump_values(x, w)
    gjv, gjs = gpu_jump(G, x, w)
    tol = 1e-12 * np.maximum(1.0, np.abs(ojs))
    assert np.all(np.abs(gjs - ojs) <= tol), np.max(np.abs(gjs - ojs))
    for j in np.flatnonzero(gjv != ojv):
        vg = P.weighted_violation(x, w, j, gjv[j])
        vo = P.weighted_violation(x, w, j, ojv[j])
        assert vg <= vo + 1e-12 * max(1.0, abs(vo)), (j, gjv[j], ojv[j], vg, vo)
    short = np.diff(mip.csc_col_ptr) <= 4096
    assert np.array_equal(gjv[short], ojv[short]) and np.array_equal(gjs[short], ojs[short])


def test_jump_edge_cases(chap):
    """Empty columns, fixed variables, a cutoff-only column, n with no rows
    touching most columns; repeated calls reuse the problem's buffers."""
    mip = mipgen.random_mixed(331, n=60, m=5, max_row_nnz=3, inf_bounds=0.3)
    mip.lb[:5] = mip.ub[:5] = np.floor(mip.lb[:5]) if np.all(np.isfinite(mip.lb[:5])) else 0.0
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip)
    x = np.clip(mipgen.random_point(mip, 1), mip.lb, mip.ub)
    w = mipgen.random_weights(P.mp + 1, 1)
    for k in range(3):
        say(f"jump edge cases call {k}")
        check_exact(chap, mip, x, w, P.objective(x) - 1.0 if k else math.inf, f"edge {k}", G)
    assert G.last_jump_ms() > 0.0


def test_jump_narrow_long_columns_exact_and_not(chap):
    """Narrow integer columns longer than one lane's entries on integer data:
    with integer weights and an integral cutoff residual they are scored from
    slope and offset bins, with fractional weights or a fractional cutoff
    residual by the wavefront tasks; both equal the oracle bit for bit."""
    mip = mipgen.random_mixed(341, n=400, m=3000, max_row_nnz=6, frac_bin=0.3, frac_int=0.7, int_width=30,
                              long_cols=6, long_deg=2500)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip)
    x = mipgen.random_point(mip, 5)
    w_int = mipgen.random_weights(P.mp + 1, 5, wmax=9)
    w_frac = (w_int * 0.5 + 0.25).astype(np.float32)
    f = P.objective(x)
    for name, w, cut in (("integer weights", w_int, math.inf), ("integral cutoff", w_int, f - 2.0),
                         ("fractional cutoff", w_int, f - 2.5), ("fractional weights", w_frac, math.inf)):
        say(f"jump narrow long columns: {name}")
        check_exact(chap, mip, x, w, cut, name, G)


def test_jump_without_rows(chap):
    """Variables in no row: the cutoff row alone (c != 0) or nothing to
    violate (every value ties at V = 0: the value next to xbar, the smaller
    first)."""
    from helpers import make_mip
    mip = make_mip(4, [({3: 1.0}, "L", 2.0)], [0, -5, 0, 0], [10, 5, 7.5, 4], [1, 1, 0, 1], obj=[3, -2, 1.5, 0])
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip)
    x = np.array([4.0, 0.0, 2.5, 4.0])
    w = np.ones(P.mp + 1, dtype=np.float32)
    for cut in (math.inf, P.objective(x) - 3.0, P.objective(x) + 7.0):
        say(f"jump without rows cutoff={cut}")
        check_exact(chap, mip, x, w, cut, f"no rows {cut}", G)
