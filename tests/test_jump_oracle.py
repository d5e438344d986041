"""Pins of the oracle's jump values (weighted violation, after Feasibility
Jump; section 3.1 "Best Shift Moves").

V_j(t) = sum over j's normalised rows of w_i max(0, r_i + a_ij (t - xbar_j)),
the cutoff row included when active. The jump value minimises V_j over the
domain without xbar_j (ties: closest to xbar_j, then smaller); the score is
V_j(xbar_j) - V_j(t*). Pinned by hand-derived closed forms, by exhaustive
search over every integer of the domain in exact rational arithmetic (which
checks the oracle's reduction to kinks, bounds and xbar +- 1 on wide domains),
and on continuous columns by the convexity invariants: t* is no worse than
any point of a dense grid when the score is >= 0, and the slope of V changes
sign at t*.
"""
from __future__ import annotations

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import mipgen
import oracle
from exact import ExactProblem
from helpers import make_mip

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _cases():
    out = []
    for ln in open(os.path.join(GOLDEN, "jump_closed_forms.jsonl")):
        d = json.loads(ln)
        if "name" in d:
            out.append(d)
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda d: d["name"][:40])
def test_jump_closed_forms(case):
    rows = [({int(c): a for c, a in coef.items()}, s, b) for coef, s, b in case["rows"]]
    mip = make_mip(case["n"], rows, [float(v) for v in case["lb"]], [float(v) for v in case["ub"]], case["int"],
                   obj=case.get("obj"))
    P = oracle.OracleProblem(mip)
    w = np.array(case["w"], dtype=np.float32)
    assert w.shape[0] == P.mp + 1
    jv, js = P.jump_values(np.array(case["x"], dtype=np.float64), w, float(case.get("cutoff", math.inf)))
    assert jv[0] == case["jv"] and js[0] == case["js"], (jv[0], js[0])


def exact_V(E, j, xbar, r, rc, w, cutoff_active, t):
    d = Fraction(t) - Fraction(xbar)
    v = Fraction(0)
    for i, a in E.column(j, cutoff_active):
        ri = rc if i == E.mp else r[i]
        y = ri + a * d
        if y > 0:
            v += Fraction(float(w[i])) * y
    return v


def _instances(count, seed0, **kw):
    for k in range(count):
        rng = np.random.default_rng(seed0 + k)
        n = int(rng.integers(2, 10))
        m = int(rng.integers(1, 8))
        yield seed0 + k, mipgen.random_mixed(seed0 + k, n=n, m=m, max_row_nnz=min(n, 4), **kw)


@pytest.mark.parametrize("width", [12, 150])
def test_jump_integer_columns_equal_exhaustive_search(width):
    """Every integer of the domain tried in exact arithmetic: the oracle's
    value and score are the exhaustive ones (integer data, so the oracle's
    FP64 sums are exact)."""
    checked = 0
    for seed, mip in _instances(60, 7000 + width, frac_bin=0.2, frac_int=0.8, int_width=width):
        P = oracle.OracleProblem(mip)
        E = ExactProblem(mip)
        x = mipgen.random_point(mip, seed)
        w = mipgen.random_weights(P.mp + 1, seed, wmax=5)
        cutoff = P.objective(x) - 3.0 if seed % 2 else math.inf
        jv, js = P.jump_values(x, w, cutoff)
        r, rc = E.residual(x, None if math.isinf(cutoff) else cutoff)
        act = not math.isinf(cutoff)
        for j in range(mip.n):
            if not E.is_int[j]:
                continue
            l, u = int(E.lb[j]), int(E.ub[j])
            xb = int(x[j])
            best = None
            for t in range(l, u + 1):
                if t == xb:
                    continue
                key = (exact_V(E, j, xb, r, rc, w, act, t), abs(t - xb), t)
                if best is None or key < best:
                    best = key
            if best is None:
                assert jv[j] == xb and js[j] == 0.0
                continue
            v0 = exact_V(E, j, xb, r, rc, w, act, xb)
            assert jv[j] == best[2], (seed, j, jv[j], best)
            assert Fraction(js[j]) == v0 - best[0], (seed, j)
            checked += 1
    assert checked > 200


def test_jump_continuous_columns_convexity():
    """Continuous columns (kinks at rational points): when the score is >= 0
    no point of a dense grid of the domain has a smaller weighted violation
    than t*, and V's slope is <= 0 just left of an interior t* and >= 0 just
    right of it (exact arithmetic at the FP64 t*, tolerance for its
    rounding)."""
    checked = 0
    for seed, mip in _instances(80, 9100, frac_bin=0.2, frac_int=0.3, cont_ub=20.0):
        P = oracle.OracleProblem(mip)
        E = ExactProblem(mip)
        x = mipgen.random_point(mip, seed)
        w = mipgen.random_weights(P.mp + 1, seed, wmax=5)
        jv, js = P.jump_values(x, w)
        r, rc = E.residual(x)
        for j in range(mip.n):
            if E.is_int[j] or not E.cols[j]:
                continue
            l, u = E.lb[j], E.ub[j]
            xb = x[j]
            vt = exact_V(E, j, xb, r, rc, w, False, jv[j])
            v0 = exact_V(E, j, xb, r, rc, w, False, xb)
            assert abs(float(v0 - vt) - js[j]) <= 1e-9 * max(1.0, abs(js[j]))
            if js[j] >= 0:
                for g in np.linspace(l, u, 401):
                    assert vt <= exact_V(E, j, xb, r, rc, w, False, float(g)) + Fraction(1, 10**6)
            h = Fraction(1, 10**4)
            t = Fraction(jv[j])
            if js[j] > 0 and l + 1e-3 < jv[j] < u - 1e-3:
                left = (exact_V(E, j, xb, r, rc, w, False, t) - exact_V(E, j, xb, r, rc, w, False, t - h)) / h
                right = (exact_V(E, j, xb, r, rc, w, False, t + h) - exact_V(E, j, xb, r, rc, w, False, t)) / h
                assert left <= Fraction(1, 10**6) and right >= -Fraction(1, 10**6), (seed, j, left, right)
            checked += 1
    assert checked > 100
