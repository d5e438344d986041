"""Diversity-driven restarts of batched walks through the C ABI against the
oracle's composition (section 3.1 "Parallel Tabu Search Instances"; the
rule is pinned in test_restarts_oracle.py): every walk's trace, final
state, best point, cutoff and restart iterations equal the oracle's.
"""
from __future__ import annotations

import numpy as np
import pytest

import mipgen
import oracle
from test_gpu_parity import assert_same, chap, say  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def compare(g, o, what):
    assert g.restarts == o["restarts"], (what, g.restarts, o["restarts"])
    for f in ("iter", "var", "kind", "viol", "x_old", "x_new", "score", "obj"):
        assert_same(g.trace[f], o["trace"][f], f"{what} trace.{f}")
    assert_same(g.x, o["x"], f"{what} x")
    assert_same(g.w, o["w"], f"{what} w")
    assert_same(g.resid, o["r"], f"{what} resid")
    assert g.best_obj == o["best_obj"] and g.cutoff_rhs == o["cutoff_rhs"], what
    if o["best_x"] is not None:
        assert_same(g.best_x, o["best_x"], f"{what} best_x")


@pytest.mark.parametrize("min_distance", [0, 6, 10**9])
def test_restarts_equal_oracle(chap, min_distance):
    mips = [mipgen.tiny_binary(0), mipgen.random_mixed(401, n=150, m=100, max_row_nnz=6, frac_bin=0.5, frac_int=0.5),
            mipgen.random_mixed(402, n=120, m=60, max_row_nnz=6, integer_data=False)]
    probs = [chap.Problem(m) for m in mips]
    oprobs = [(oracle.OracleProblem(m), m) for m in mips]
    walk_prob = [0, 0, 1, 0, 1, 2, 2, 1]
    walk_seed = [1, 1, 2, 3, 2, 5, 6, 9]
    say(f"batch restarts min_distance={min_distance}")
    runs = chap.batch_restarts(probs, walk_prob, walk_seed, 170, 6, 40, min_distance)
    outs = oracle.batch_restarts(oprobs, walk_prob, walk_seed, 170, 6, 40, min_distance)
    for w, (g, o) in enumerate(zip(runs, outs)):
        compare(g, o, f"walk {w}")
    if min_distance == 0:
        plain = chap.batch_run(probs, walk_prob, walk_seed, 170, 6)
        for g, p in zip(runs, plain):
            assert g.trace.tobytes() == p.trace.tobytes()
    if min_distance > 0:
        assert runs[1].restarts  # same seed as walk 0 on the same problem


def test_restarted_walk_has_no_best_infeasible(chap):
    mip = mipgen.random_mixed(403, n=80, m=50, max_row_nnz=5)
    G = chap.Problem(mip)
    runs = chap.batch_restarts([G], [0, 0], [3, 3], 60, 5, 20, 10**9)
    assert runs[1].restarts == [20, 40]
    with pytest.raises(chap.ChapError, match="CHAP_EINVAL"):
        runs[1].best_infeasible()
    x, v, k = runs[0].best_infeasible()
    assert runs[0].restarts == []


def test_restart_argument_checks(chap):
    G = chap.Problem(mipgen.random_mixed(404, n=20, m=10))
    for every, dmin in ((0, 1), (-5, 1), (10, -1)):
        with pytest.raises(chap.ChapError, match="CHAP_EINVAL"):
            chap.batch_restarts([G], [0], [1], 30, 5, every, dmin)


def test_restart_segments_longer_than_the_walk(chap):
    """restart_every >= iters: one segment, no restart, the plain batch."""
    mips = [mipgen.random_mixed(405, n=60, m=40, max_row_nnz=5), mipgen.tiny_binary(0)]
    probs = [chap.Problem(m) for m in mips]
    wp, ws = [0, 1, 0], [2, 2, 2]
    runs = chap.batch_restarts(probs, wp, ws, 90, 5, 90, 10**9)
    plain = chap.batch_run(probs, wp, ws, 90, 5)
    for g, p in zip(runs, plain):
        assert g.restarts == []
        assert g.trace.tobytes() == p.trace.tobytes()
        assert g.x.tobytes() == p.x.tobytes()
