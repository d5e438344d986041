"""Pins of the CPU oracle against facts that do not come from the oracle.

* published SplitMix64 outputs (start-point generator);
* hand-derived closed forms of single-variable best shifts;
* exhaustive search over every integer of the domain (brute force) with exact
  rational arithmetic, on tiny instances;
* a dense-grid search in exact arithmetic for continuous variables;
* the binary flip equals Algorithm 1 restricted to [0, 1];
* invariance under row order;
* a full tabu walk in exact arithmetic (independent implementation);
* walk invariants: residual identity, violation counts, tabu, aspiration,
  incumbent feasibility.
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
from helpers import make_mip, splitmix64_py, tabu_until_from_trace

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vector():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) if not ln.startswith("#")]
    for idx, hexval in rows:
        want = int(hexval, 16)
        assert oracle.splitmix64(0, int(idx)) == want
        assert splitmix64_py(0, int(idx)) == want
    for seed in (1, 7, 2**63 + 5):
        for i in range(50):
            assert oracle.splitmix64(seed, i) == splitmix64_py(seed, i)


def _closed_form_cases():
    out = []
    for ln in open(os.path.join(GOLDEN, "closed_forms.jsonl")):
        d = json.loads(ln)
        if "name" in d:
            out.append(d)
    return out


@pytest.mark.parametrize("case", _closed_form_cases(), ids=lambda d: d["name"][:40])
def test_closed_forms(case):
    rows = [({0: a}, s, b) for a, s, b in case["rows"]]
    lb = float(case["lb"]) if not isinstance(case["lb"], str) else float(case["lb"])
    mip = make_mip(1, rows, [lb], [float(case["ub"])], [case["int"]])
    P = oracle.OracleProblem(mip)
    w = np.array(case["w"] + [1.0], dtype=np.float32)
    assert w.shape[0] == P.mp + 1
    xh, s = P.best_shift(np.array([float(case["xbar"])]), w)
    assert s[0] == case["s"]
    if "xhat_exact" in case:
        assert abs(xh[0] - float(case["xhat_exact"])) <= 1e-15
    else:
        assert xh[0] == case["xhat"]


def _tiny_instances(count, seed0=0, **kw):
    for k in range(count):
        rng = np.random.default_rng(10_000 + seed0 + k)
        n = int(rng.integers(2, 12))
        m = int(rng.integers(1, 9))
        yield mipgen.random_mixed(seed0 + k, n=n, m=m, max_row_nnz=min(n, 5), int_width=12,
                                  frac_bin=0.3, frac_int=0.7, **kw)


def test_normalisation_map_and_hidden_point():
    for mip in _tiny_instances(30):
        P = oracle.OracleProblem(mip)
        orig, sign = P.norm_rows()
        want = []
        for i, s in enumerate(mip.sense):
            if s == ord("L"):
                want.append((i, 1))
            elif s == ord("G"):
                want.append((i, -1))
            else:
                want += [(i, 1), (i, -1)]
        assert list(zip(orig.tolist(), sign.tolist())) == want
        # the hidden point satisfies every normalised row (integer data: exactly)
        r, v = P.residual(mip.hidden_x)
        assert v == 0 and np.all(r[:-1] <= 0)
        E = ExactProblem(mip)
        rx, _ = E.residual(mip.hidden_x)
        assert [Fraction(float(a)) for a in r[:-1]] == rx


def _exact_inputs(mip, seed):
    x = mipgen.random_point(mip, seed)
    P = oracle.OracleProblem(mip)
    w = mipgen.random_weights(P.mp + 1, seed + 1)
    return P, x, w


@pytest.mark.parametrize("with_cutoff", [False, True])
def test_best_shift_equals_exhaustive_search(with_cutoff):
    checked = 0
    improving = 0
    for mip in _tiny_instances(120, seed0=500 if with_cutoff else 0):
        P, x, w = _exact_inputs(mip, 77)
        cut = None
        if with_cutoff:
            cut = float(np.floor(mip.obj @ x)) - 2.0
        xh, s = P.best_shift(x, w, cutoff_rhs=math.inf if cut is None else cut)
        E = ExactProblem(mip)
        r, rc = E.residual(x, cut)
        r = list(r) + [rc if rc is not None else Fraction(0)]
        active = cut is not None
        for j in range(mip.n):
            ex_x, ex_s = E.best_shift(j, x, r, w, active)
            assert Fraction(float(s[j])) == ex_s, (mip.name, j)
            assert Fraction(float(xh[j])) == ex_x, (mip.name, j)
            if E.is_int[j] and math.isfinite(E.lb[j]) and math.isfinite(E.ub[j]):
                vals = E.brute_force_max(j, x, r, w, active)
                best = max((v for v, _ in vals), default=None)
                if best is not None and best > 0:
                    improving += 1
                    assert ex_s == best
                    # the returned shift is a maximiser over the whole domain
                    assert E.score(j, x[j], xh[j], r, w, active) == best
                else:
                    assert s[j] == 0 and xh[j] == x[j]
            checked += 1
    assert checked > 500 and improving > 100


def test_binary_flip_equals_algorithm1_on_unit_interval():
    for mip in _tiny_instances(80, seed0=900):
        P, x, w = _exact_inputs(mip, 5)
        Q = oracle.OracleProblem(mip, binary_as_general=True)
        xa, sa = P.best_shift(x, w)
        xb, sb = Q.best_shift(x, w)
        assert np.array_equal(xa, xb) and np.array_equal(sa, sb)


def test_row_order_invariance():
    for mip in _tiny_instances(40, seed0=1300):
        P, x, w = _exact_inputs(mip, 9)
        xh, s = P.best_shift(x, w)
        # reverse the original rows and carry the weights along
        perm = np.arange(mip.m)[::-1]
        rows = []
        for i in perm:
            lo, hi = mip.csr_row_ptr[i], mip.csr_row_ptr[i + 1]
            rows.append(({int(c): float(v) for c, v in zip(mip.csr_col[lo:hi], mip.csr_val[lo:hi])},
                         chr(mip.sense[i]), float(mip.rhs[i])))
        mip2 = make_mip(mip.n, rows, mip.lb, mip.ub, mip.is_int, mip.obj)
        P2 = oracle.OracleProblem(mip2)
        orig, sign = P.norm_rows()
        orig2, sign2 = P2.norm_rows()
        key = {(int(o), int(sg)): k for k, (o, sg) in enumerate(zip(orig, sign))}
        w2 = np.empty_like(w)
        for k, (o, sg) in enumerate(zip(orig2, sign2)):
            w2[k] = w[key[(int(perm[o]), int(sg))]]
        w2[-1] = w[-1]
        xh2, s2 = P2.best_shift(x, w2)
        assert np.array_equal(xh, xh2) and np.array_equal(s, s2)


def test_continuous_best_shift_against_dense_grid():
    """Dyadic data and eps = 0 keep every breakpoint exactly representable; the
    supremum of the step function over [l, u] minus the incumbent is then the
    maximum over a grid of step 1/8 (breakpoints are multiples of 1/4)."""
    rng = np.random.default_rng(3)
    checked = 0
    for trial in range(60):
        n = int(rng.integers(1, 5))
        m = int(rng.integers(1, 6))
        rows = []
        for _ in range(m):
            cols = rng.choice(n, size=int(rng.integers(1, n + 1)), replace=False)
            coef = {int(c): float(rng.choice([-4, -2, -1, 1, 2, 4])) for c in cols}
            rows.append((coef, "LGE"[int(rng.integers(0, 3))], float(rng.integers(-6, 7)) / 2))
        lb = rng.integers(-4, 1, size=n).astype(float)
        ub = lb + rng.integers(1, 6, size=n)
        mip = make_mip(n, rows, lb, ub, np.zeros(n, dtype=np.uint8))
        P = oracle.OracleProblem(mip, eps=0.0)
        x = (lb + rng.integers(0, 9, size=n) / 8 * (ub - lb)).astype(float)
        x = np.round(x * 4) / 4
        w = rng.integers(1, 5, size=P.mp + 1).astype(np.float32)
        xh, s = P.best_shift(x, w)
        E = ExactProblem(mip, eps=0.0)
        r, _ = E.residual(x)
        r = list(r) + [Fraction(0)]
        for j in range(n):
            grid = [Fraction(int(lb[j] * 8) + k, 8) for k in range(int((ub[j] - lb[j]) * 8) + 1)]
            vals = [(E.score(j, x[j], p, r, w, False), p) for p in grid if p != Fraction(float(x[j]))]
            best = max((v for v, _ in vals), default=Fraction(0))
            if best > 0:
                assert Fraction(float(s[j])) == best
                assert E.score(j, x[j], xh[j], r, w, False) == best
                ex_x, _ = E.best_shift(j, x, r, w, False)
                assert Fraction(float(xh[j])) == ex_x
            else:
                assert s[j] == 0 and xh[j] == x[j]
            checked += 1
    assert checked > 100


@pytest.mark.parametrize("seed", [0, 7])
def test_tabu_walk_matches_exact_walk(seed):
    walks = 0
    for k, mip in enumerate(_tiny_instances(12, seed0=2000 + 31 * seed)):
        P = oracle.OracleProblem(mip)
        out = P.tabu_run(60, 3, seed)
        E = ExactProblem(mip)
        x0 = E.start_point(seed, splitmix64_py)
        assert [Fraction(float(v)) for v in P.start_point(seed)] == x0
        trace, xe, we, fbest, bc, re = E.tabu_run(60, 3, x0)
        t = out["trace"]
        for rec, ex in zip(t, trace):
            got = (int(rec["iter"]), int(rec["var"]), int(rec["kind"]))
            assert got == ex[:3], (mip.name, got, ex[:3])
            if ex[1] >= 0:
                assert Fraction(float(rec["x_old"])) == ex[3]
                assert Fraction(float(rec["x_new"])) == ex[4]
                assert Fraction(float(rec["score"])) == ex[5]
            assert int(rec["viol"]) == ex[6]
            assert Fraction(float(rec["obj"])) == ex[7]
        assert [Fraction(float(v)) for v in out["x"]] == xe
        assert [Fraction(float(v)) for v in out["w"]] == we
        if bc is None:
            assert out["cutoff_rhs"] == math.inf and out["best_x"] is None
        else:
            assert Fraction(out["cutoff_rhs"]) == bc and Fraction(out["best_obj"]) == fbest
            assert [Fraction(float(v)) for v in out["r"]] == re
        walks += 1
    assert walks == 12


def test_walk_invariants_tiny_binary():
    mip = mipgen.tiny_binary(0)
    P = oracle.OracleProblem(mip)
    out = P.tabu_run(1000, 10, 0)
    t = out["trace"]
    x = P.start_point(0)
    last_move = {}
    best = math.inf
    cutoff = math.inf
    r, v = P.residual(x)
    if v == 0:
        best = float(mip.obj @ x)
        cutoff = best - 1.0
    for rec in t:
        k, j = int(rec["iter"]), int(rec["var"])
        if j >= 0:
            assert rec["score"] > 0
            assert x[j] == rec["x_old"]
            if j in last_move and k - last_move[j] <= 10:
                assert rec["kind"] == 1  # only aspiration may move a tabu variable
            x[j] = rec["x_new"]
            last_move[j] = k
        r, v = P.residual(x, cutoff)
        assert v == rec["viol"]
        assert float(mip.obj @ x) == rec["obj"]
        if rec["kind"] == 1:
            assert rec["viol"] == 0
        if v == 0:
            f = float(mip.obj @ x)
            assert f < best
            best = f
            cutoff = best - 1.0
    assert np.array_equal(x, out["x"])
    assert out["best_obj"] == best
    r, v = P.residual(out["best_x"])
    assert v == 0 and float(mip.obj @ out["best_x"]) == best


def test_generator_shapes():
    a = mipgen.tiny_binary(0)
    assert a.counts() == {"n": 200, "m": 100, "nnz": 1000, "nnz_obj": a.nnz_obj, "rows_L": 100,
                          "rows_G": 0, "rows_E": 0}
    assert np.all(np.diff(a.csr_row_ptr) == 10)
    assert np.all(a.rhs == np.floor(0.5 * np.add.reduceat(a.csr_val, a.csr_row_ptr[:-1])))
    b = mipgen.general(1, n=20_000, m=10_000)
    c = b.counts()
    assert (c["rows_L"], c["rows_G"], c["rows_E"]) == (4000, 4000, 2000)
    assert abs(c["nnz"] / c["m"] - 8.0) < 0.5
    assert np.count_nonzero(b.is_int == 0) == 2000
    assert np.count_nonzero((b.is_int == 1) & (b.ub == 1)) == 12000
    P = oracle.OracleProblem(b)
    r, v = P.residual(b.hidden_x)
    assert v == 0
    d = mipgen.zipf_degrees(2_000_000, 20_000_000)
    assert d.sum() == 20_000_000 or abs(int(d.sum()) - 20_000_000) < 5
    assert d.max() == 100_000 and int((d == 100_000).sum()) == 25
    p = mipgen.powerlaw(0, n=20_000, m=10_000, nnz=200_000, cap=2000)
    assert p.nnz == 200_000 or abs(p.nnz - 200_000) < 5
    P = oracle.OracleProblem(p)
    r, v = P.residual(p.hidden_x)
    assert v == 0
    # CSR and CSC describe the same matrix
    for mip in (a, b, p):
        rows = np.repeat(np.arange(mip.m), np.diff(mip.csr_row_ptr))
        k1 = rows.astype(np.int64) * mip.n + mip.csr_col
        cols = np.repeat(np.arange(mip.n), np.diff(mip.csc_col_ptr))
        k2 = mip.csc_row.astype(np.int64) * mip.n + cols
        o1, o2 = np.argsort(k1), np.argsort(k2)
        assert np.array_equal(k1[o1], k2[o2]) and np.array_equal(mip.csr_val[o1], mip.csc_val[o2])


@pytest.mark.parametrize("k0", [1, 17, 45])
def test_resumed_walk_continues_the_walk(k0):
    """A walk continued from its state at iteration k0 (point, weights, tabu
    list, incumbent, cutoff) is the same walk: trace and final state equal the
    uninterrupted walk's."""
    for mip in list(_tiny_instances(8, seed0=700)) + [mipgen.random_mixed(9, n=60, m=40, integer_data=False)]:
        P = oracle.OracleProblem(mip)
        full = P.tabu_run(60, 3, 2)
        head = P.tabu_run(k0, 3, 2)
        tb = tabu_until_from_trace(head["trace"], mip.n, 3)
        rest = P.tabu_resume(60 - k0, 3, head["x"], head["w"], tb, k0, head["best_obj"], head["best_x"],
                             head["cutoff_rhs"])
        assert rest["trace"].tobytes() == full["trace"][k0:].tobytes(), mip.name
        for f in ("x", "r", "w"):
            assert np.array_equal(rest[f], full[f]), (mip.name, f)
        assert rest["best_obj"] == full["best_obj"] and rest["cutoff_rhs"] == full["cutoff_rhs"]


def test_threads_do_not_change_results():
    """The oracle's per-column and per-row loops split across threads give
    the same best shifts and walks as one thread."""
    mip = mipgen.powerlaw(4, n=20_000, m=10_000, nnz=150_000, cap=3000)
    cont = mipgen.random_mixed(11, n=300, m=200, integer_data=False)
    try:
        for m in (mip, cont):
            P = oracle.OracleProblem(m)
            x = mipgen.random_point(m, 1)
            w = mipgen.random_weights(P.mp + 1, 1)
            oracle.set_threads(1)
            a = P.best_shift(x, w)
            ta = P.tabu_run(40, 5, 3)
            assert oracle.set_threads(4) == 4
            b = P.best_shift(x, w)
            tb = P.tabu_run(40, 5, 3)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
            assert ta["trace"].tobytes() == tb["trace"].tobytes() and np.array_equal(ta["r"], tb["r"])
    finally:
        oracle.set_threads(1)


def test_best_infeasible_point_by_replaying_the_trace():
    """The oracle's best infeasible point against a recount: the points of the
    walk are rebuilt from the start point and the trace's moves, each one's
    violated rows (cutoff row not counted) are counted from scratch, and the
    first point with the fewest (more than zero) must be the one reported."""
    cases = list(_tiny_instances(10, seed0=900)) + [mipgen.random_mixed(14, n=60, m=40, integer_data=False),
                                                   mipgen.tiny_binary(0)]
    for mip in cases:
        P = oracle.OracleProblem(mip)
        for seed in (0, 3):
            iters = 80
            out = P.tabu_run(iters, 3, seed)
            x = P.start_point(seed)
            best_v, best_k, best_x = None, -2, None
            pts = [(-1, x.copy())]
            for rec in out["trace"]:
                if rec["var"] >= 0:
                    x[rec["var"]] = rec["x_new"]
                    pts.append((int(rec["iter"]), x.copy()))
            for k, xk in pts:
                _, v = P.residual(xk)
                if v > 0 and (best_v is None or v < best_v):
                    best_v, best_k, best_x = v, k, xk
            assert out["inf_iter"] == best_k, (mip.name, seed)
            if best_k == -2:
                assert out["inf_viol"] == 0 and out["inf_x"] is None
            else:
                assert out["inf_viol"] == best_v and np.array_equal(out["inf_x"], best_x)
