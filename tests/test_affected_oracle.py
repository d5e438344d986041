"""Pin of the affected-set claim behind affected rescoring (oracle only).

The best shift of column q is a function of x_q, its bounds, the residuals
and weights of the rows of q and, when the cutoff row is active, of that
row's residual and weight (section 3.1, Algorithm 1 and the scoring
functions). So after a move of column j with the weights and the cutoff
row unchanged (cutoff inactive, or c_j = 0), every column that shares no row
with j keeps its best shift and score. Checked on the oracle by recomputing
every column from scratch before and after random moves; the columns that
do share a row must change in some of the cases (the check has power).
"""
from __future__ import annotations

import numpy as np
import pytest

import mipgen
import oracle


def affected(mip, j):
    rows = mip.csc_row[mip.csc_col_ptr[j]:mip.csc_col_ptr[j + 1]]
    cols = {int(j)}
    for i in rows:
        cols.update(int(c) for c in mip.csr_col[mip.csr_row_ptr[i]:mip.csr_row_ptr[i + 1]])
    return cols


def new_value(mip, x, j, rng):
    lo, hi = mip.lb[j], mip.ub[j]
    lo = lo if np.isfinite(lo) else x[j] - 10.0
    hi = hi if np.isfinite(hi) else x[j] + 10.0
    for _ in range(20):
        v = np.floor(lo + rng.random() * (hi - lo + 1)) if mip.is_int[j] else lo + rng.random() * (hi - lo)
        v = min(v, hi)
        if v != x[j]:
            return float(v)
    return None


@pytest.mark.parametrize("case", ["mixed", "continuous", "long", "cutoff"])
def test_unaffected_columns_keep_their_best_shift(case):
    rng = np.random.default_rng({"mixed": 1, "continuous": 2, "long": 3, "cutoff": 4}[case])
    changed_inside = 0
    for t in range(12):
        seed = 100 * t + len(case)
        if case == "continuous":
            mip = mipgen.random_mixed(seed, n=60, m=40, integer_data=False)
        elif case == "long":
            mip = mipgen.random_mixed(seed, n=80, m=60, max_row_nnz=5, long_cols=2, long_deg=30)
        else:
            mip = mipgen.random_mixed(seed, n=50, m=40, max_row_nnz=5)
        P = oracle.OracleProblem(mip)
        x = mipgen.random_point(mip, seed)
        w = mipgen.random_weights(P.mp + 1, seed)
        cutoff = float("inf")
        if case == "cutoff":
            cutoff = P.objective(x) - 3.0
        xh0, s0 = P.best_shift(x, w, cutoff)
        for _ in range(4):
            j = int(rng.integers(mip.n))
            if case == "cutoff" and mip.obj[j] != 0.0:
                continue
            v = new_value(mip, x, j, rng)
            if v is None:
                continue
            x2 = x.copy()
            x2[j] = v
            xh1, s1 = P.best_shift(x2, w, cutoff)
            A = affected(mip, j)
            out = np.array([q not in A for q in range(mip.n)])
            assert np.array_equal(xh0[out], xh1[out]) and np.array_equal(s0[out], s1[out]), (case, t, j)
            inside = np.array(sorted(A))
            changed_inside += int(np.count_nonzero((xh0[inside] != xh1[inside]) | (s0[inside] != s1[inside])))
    assert changed_inside > 0


def test_cutoff_change_reaches_objective_columns():
    """With the cutoff row active, a move of a column with c_j != 0 changes the
    cutoff residual, and columns outside j's rows with c != 0 can change:
    such steps are left to the full pass."""
    hits = 0
    for t in range(10):
        mip = mipgen.random_mixed(500 + t, n=50, m=40, max_row_nnz=5)
        P = oracle.OracleProblem(mip)
        x = mipgen.random_point(mip, t)
        w = mipgen.random_weights(P.mp + 1, t)
        cutoff = P.objective(x) - 2.0
        xh0, s0 = P.best_shift(x, w, cutoff)
        js = np.flatnonzero(mip.obj != 0.0)
        j = int(js[0])
        rng = np.random.default_rng(t)
        v = new_value(mip, x, j, rng)
        if v is None:
            continue
        x2 = x.copy()
        x2[j] = v
        xh1, s1 = P.best_shift(x2, w, cutoff)
        A = affected(mip, j)
        outside = [q for q in range(mip.n) if q not in A]
        hits += sum(1 for q in outside if (xh0[q], s0[q]) != (xh1[q], s1[q]))
    assert hits > 0
