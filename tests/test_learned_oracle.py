"""Pins of the learned-proposal references (oracle/features.py and the
learned form of the oracle walk) against hand-derived values and against the
plain walk, which is itself pinned to an exact-arithmetic walk."""
from __future__ import annotations

import math

import numpy as np
import pytest

import mipgen
import oracle
from oracle import features as F
from helpers import make_mip


def hand_mip():
    # x0 binary, x1 integer in [0, 10], x2 continuous in [0, inf)
    rows = [({0: 1, 1: 2, 2: -1}, "L", 5), ({1: 3, 2: 1}, "E", 7)]
    return make_mip(3, rows, [0, 0, 0], [1, 10, math.inf], [1, 1, 0], obj=[1, -2, 4])


def test_features_hand_derived():
    mip = hand_mip()
    P = oracle.OracleProblem(mip)
    # normalised rows: 0 = row 0, 1 = row 1, 2 = -(row 1); at x = (1, 3, 0)
    # residuals are 2, 2, -2: rows 0 and 1 violated, V = 2, m' = 3
    x = np.array([1.0, 3.0, 0.0])
    w = np.array([1.0, 2.0, 3.0, 1.0], dtype=np.float32)
    s_last = np.array([10.0, 3.0, -1.5])
    xhat_last = np.array([0.0, 5.0, 0.0])
    last_move = np.array([9, 4, -1024])
    moves = np.array([1, 3, 0])
    got, ok = F.inputs(mip, P, x, w, math.inf, s_last, xhat_last, last_move, moves, 10, 8)
    assert ok.all()
    two3 = 0.66796875          # bfloat16(2/3)
    want = np.array([
        # x0: one row (a = 1, r = 2, w = 1)
        [1.0, 1.0, 0.25, 4.0, 1, 0, 0, 1.0, 1.0, 1.0, 131 / 65536, -1.0, 1 / 1024, 1 / 32, two3, 1.0],
        # x1: rows a = 2, 3, -3 with w = 1, 2, 3; violated: the first two
        [0.5, 203 / 128, -0.5, 0.5, 0, 1, 0, 154 / 512, 221 / 64, two3, 164 / 131072, 1.0, 6 / 1024, 1 / 32, two3,
         2.0],
        # x2: rows a = -1, 1, -1; infinite upper bound
        [0.5, 203 / 128, 1.0, -0.25, 0, 0, 1, 0.5, 20.0, two3, 175 / 131072, 0.0, 1.0, 1 / 32, two3, 0.0],
    ])
    np.testing.assert_array_equal(got, want)


def test_features_refresh_point_and_eligibility():
    mip = mipgen.random_mixed(3, n=40, m=30, max_row_nnz=6, integer_data=True)
    P = oracle.OracleProblem(mip)
    rng = np.random.default_rng(0)
    lb, ub, _ = P.bounds()
    x0 = P.start_point(0)
    x1 = x0.copy()
    x1[5] = lb[5] if x1[5] != lb[5] else ub[5] if math.isfinite(ub[5]) else lb[5] + 1
    w = rng.integers(1, 4, P.mp + 1).astype(np.float32)
    z = np.zeros(mip.n)
    lm = np.full(mip.n, -1024)
    mv = np.zeros(mip.n, dtype=np.int64)
    now, _ = F.inputs(mip, P, x1, w, math.inf, z, x0, lm, mv, 3, 0)
    ref, _ = F.inputs(mip, P, x1, w, math.inf, z, x0, lm, mv, 3, 0, refresh=(x0, w, math.inf))
    # only the row aggregates (0, 3, 9, 10) come from the refresh point
    np.testing.assert_array_equal(np.delete(now, [0, 3, 9, 10], axis=1), np.delete(ref, [0, 3, 9, 10], axis=1))
    r0, _ = F.inputs(mip, P, x0, w, math.inf, z, x0, lm, mv, 3, 0)
    np.testing.assert_array_equal(ref[:, [0, 3, 9, 10]], r0[:, [0, 3, 9, 10]])
    # a general column with 4094 normalised entries is proposable, one more
    # is not; binary and narrow integer columns are proposable at any length
    for cnt, ub, expect in ((4094, 100, True), (4095, 100, False), (5000, 63, True), (5000, 1, True)):
        rows = [({0: 1}, "L", 1)] * cnt
        m2 = make_mip(1, rows, [0], [ub], [1])
        O2 = oracle.OracleProblem(m2)
        lb2, ub2, _ = O2.bounds()
        assert F.proposable(m2, F.column_rows(m2, *O2.norm_rows()), lb2, ub2)[0] == expect


def _walk_pair(mip, iters, full_every, sets_fn):
    P = oracle.OracleProblem(mip)
    offs = [0]
    sets = []
    for k in range(iters):
        s = sets_fn(k)
        sets.extend(s)
        offs.append(len(sets))
    plain = P.tabu_run(iters, 10, 1)
    learned = P.learned_replay(iters, 10, 1, full_every, np.array(sets, dtype=np.int32), np.array(offs))
    return plain, learned


def test_learned_all_columns_equals_plain_until_first_reweight():
    mip = mipgen.random_mixed(5, n=60, m=40, max_row_nnz=6, integer_data=True)
    n = mip.n
    plain, learned = _walk_pair(mip, 150, 8, lambda k: list(range(n)))
    tp, tl = plain["trace"], learned["trace"]
    first = int(np.argmax(tp["kind"] == 2)) if (tp["kind"] == 2).any() else len(tp)
    assert first > 10
    for k in range(first):
        full = k % 8 == 0
        assert tl["kind"][k] == tp["kind"][k] + (0 if full else 8)
        for f in ("var", "x_old", "x_new", "score", "viol", "obj"):
            assert tl[f][k] == tp[f][k], (k, f)
    if first < len(tp):
        # the plain walk reweights; a proposal iteration stalls there instead
        # (no move, no reweight) unless it is a full evaluation
        if first % 8 != 0:
            assert tl["kind"][first] == 3 and tl["var"][first] == -1
            assert tl["kind"][first + 1] == 2   # the next iteration is full and reweights


def test_learned_empty_sets_stall_then_full():
    mip = mipgen.random_mixed(6, n=30, m=20, max_row_nnz=5, integer_data=True)
    _, learned = _walk_pair(mip, 40, 4, lambda k: [])
    kinds = learned["trace"]["kind"]
    # full, stall, full, stall, ... : each stall ends its block
    for k in range(40):
        assert (kinds[k] in (0, 1, 2)) == (k % 2 == 0), (k, kinds[:8])
        if k % 2 == 1:
            assert kinds[k] == 3 and learned["trace"]["var"][k] == -1


def test_learned_full_every_one_is_plain():
    mip = mipgen.random_mixed(7, n=50, m=30, max_row_nnz=6, integer_data=True)
    plain, learned = _walk_pair(mip, 80, 1, lambda k: [0])
    np.testing.assert_array_equal(plain["trace"], learned["trace"])
    np.testing.assert_array_equal(plain["x"], learned["x"])
    np.testing.assert_array_equal(plain["w"], learned["w"])
