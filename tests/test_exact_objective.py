"""Pins of the oracle's objective arithmetic.

The objective f = c^T x and the cutoff residual c^T x - b_c are sums over
every variable, so their FP64 values depend on the order of summation unless
they are rounded once. The oracle takes the exact value rounded once to
nearest (ties to even). Pinned here against exact rational arithmetic
(fractions.Fraction, whose float() rounds to nearest) on random, cancelling,
mixed-magnitude, subnormal and half-way cases, and against a tabu walk in
exact arithmetic with fractional objectives, where the cutoff offset
delta = 1e-4 max(1, |f_best|) applies (section 3.2; the offset is a reading).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

import mipgen
import oracle
from exact import ExactProblem
from helpers import splitmix64_py


def rounded(terms) -> float:
    return float(sum((Fraction(t) for t in terms), Fraction(0)))


def check(terms):
    got = oracle.exact_sum(terms)
    want = rounded(terms)
    assert got == want and math.copysign(1.0, got) == math.copysign(1.0, want if want != 0 else 1.0), \
        (terms[:6], got, want)
    return got


def test_exact_sum_random_magnitudes():
    rng = np.random.default_rng(5)
    for k in range(400):
        n = int(rng.integers(1, 40))
        mant = rng.uniform(-1, 1, size=n)
        expo = rng.integers(-60 if k % 2 else -1070, 60 if k % 2 else 1000, size=n)
        check([float(np.ldexp(a, int(e))) for a, e in zip(mant, expo)])


def test_exact_sum_cancellation_and_ties():
    u = 2.0 ** -53
    cases = [
        [1.0, u],                       # half-way, even neighbour below: 1.0
        [1.0 + 2 * u, u],               # half-way, odd: rounds up
        [1.0, u, 2.0 ** -80],           # just above half-way: up
        [1.0, u, -(2.0 ** -80)],        # just below: down
        [1e-16, 1.0, 1e16],
        [1e308, -1e308, 1.0],
        [1e16, 1.0, -1e16, 1e-30],
        [5e-324, 5e-324, 5e-324],
        [3 * 5e-324, -5e-324],
        [2.0 ** -1022, -(2.0 ** -1074)],
        [0.1] * 10 + [-1.0],
        [1.0, -1.0],                    # exact zero is +0
        [-0.0],
        [],
    ]
    for c in cases:
        check(c)
    assert math.copysign(1.0, oracle.exact_sum([1.0, -1.0])) == 1.0
    assert math.copysign(1.0, oracle.exact_sum([-0.0, -0.0])) == 1.0


def test_exact_sum_permutation_invariant_and_fsum():
    rng = np.random.default_rng(11)
    for _ in range(100):
        v = (rng.standard_normal(50) * 10.0 ** rng.integers(-8, 9, size=50)).tolist()
        a = oracle.exact_sum(v)
        assert a == oracle.exact_sum(v[::-1]) == oracle.exact_sum(sorted(v)) == math.fsum(v)


def test_objective_is_the_rounded_exact_dot():
    for seed in range(20):
        mip = mipgen.random_mixed(300 + seed, n=60, m=20, integer_data=False, cont_ub=1000.0)
        mip.obj[:] = mip.obj * np.pi  # inexact products
        P = oracle.OracleProblem(mip)
        x = mipgen.random_point(mip, seed)
        want = float(sum((Fraction(float(c)) * Fraction(float(v)) for c, v in zip(mip.obj, x)), Fraction(0)))
        assert P.objective(x) == want
        bc = float(np.floor(want)) - 0.37
        r, _ = P.residual(x, bc)
        exact_rc = sum((Fraction(float(c)) * Fraction(float(v)) for c, v in zip(mip.obj, x)), Fraction(0)) - \
            Fraction(bc)
        assert r[-1] == float(exact_rc)


def _fractional_instances(count, seed0, small):
    """Tiny all-integer instances with a dyadic fractional objective: every
    FP64 operation of a walk is exact except delta and the cutoff offset.
    small: objective values within (-1, 1), where delta = 1e-4 (not
    1e-4 |f_best|)."""
    for k in range(count):
        rng = np.random.default_rng(20_000 + seed0 + k)
        n = int(rng.integers(3, 12))
        m = int(rng.integers(1, 7))
        mip = mipgen.random_mixed(seed0 + k, n=n, m=m, max_row_nnz=min(n, 5), int_width=12,
                                  frac_bin=0.3, frac_int=0.7)
        if small:
            mip.obj[:] = 0.0
            mip.obj[: min(n, 2)] = rng.choice([-0.125, 0.125, 0.0625, -0.0625], size=min(n, 2))
            mip.lb[:2] = 0.0
            mip.ub[:2] = 3.0
        else:
            mip.obj[:] = rng.integers(-12, 13, size=n) / 4.0
            if not np.any(mip.obj % 1 != 0):
                mip.obj[0] = 0.75
        yield mip


@pytest.mark.parametrize("seed,small", [(0, False), (3, False), (1, True), (5, True)])
def test_walk_with_fractional_objective_matches_exact_walk(seed, small):
    feasible = 0
    walks = 0
    count = 30 if small else 16
    for mip in _fractional_instances(count, seed0=4000 + 97 * seed, small=small):
        P = oracle.OracleProblem(mip)
        out = P.tabu_run(60, 3, seed)
        E = ExactProblem(mip)
        assert not E.obj_integral
        x0 = E.start_point(seed, splitmix64_py)
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
            assert float(rec["obj"]) == float(ex[7])
        assert [Fraction(float(v)) for v in out["x"]] == xe
        assert [Fraction(float(v)) for v in out["w"]] == we
        if bc is None:
            assert out["cutoff_rhs"] == math.inf and out["best_x"] is None
        else:
            feasible += 1
            assert Fraction(out["cutoff_rhs"]) == bc and out["best_obj"] == float(fbest)
            assert list(out["r"]) == [float(v) for v in re]
            # the offset is not 1: a non-integral objective
            assert float(fbest) - out["cutoff_rhs"] == pytest.approx(1e-4 * max(1.0, abs(float(fbest))), rel=1e-9)
        walks += 1
    assert walks == count and feasible >= 12, feasible
