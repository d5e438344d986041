"""Pins of the oracle's diversity-driven restarts (section 3.1 "Parallel
Tabu Search Instances"; the restart rule, seeds and what a restart keeps are
readings). Walks run in segments composed from resumed walks; these checks
tie the composition to plain walks and the restart rule to its definition.
"""
from __future__ import annotations

import numpy as np

import mipgen
import oracle


def _prob(mip):
    return (oracle.OracleProblem(mip), mip)


def test_hamming_counts_discrete_variables_only():
    mip = mipgen.random_mixed(1, n=30, m=10, frac_bin=0.3, frac_int=0.3)
    x = mipgen.random_point(mip, 1)
    y = x.copy()
    cont = np.flatnonzero(mip.is_int == 0)
    ints = np.flatnonzero(mip.is_int == 1)
    y[cont] += 0.25
    assert oracle.hamming_discrete(x, y, mip.is_int) == 0
    y[ints[:3]] = np.where(y[ints[:3]] == mip.lb[ints[:3]], mip.ub[ints[:3]], mip.lb[ints[:3]])
    assert oracle.hamming_discrete(x, y, mip.is_int) == int(np.count_nonzero(x[ints[:3]] != y[ints[:3]]))


def test_no_restarts_is_the_plain_walks():
    mips = [mipgen.random_mixed(2, n=60, m=40, max_row_nnz=5), mipgen.tiny_binary(0)]
    probs = [_prob(m) for m in mips]
    wp, ws = [0, 1, 0, 1], [1, 2, 3, 0]
    out = oracle.batch_restarts(probs, wp, ws, 130, 7, every=40, min_distance=0)
    for w in range(4):
        o = probs[wp[w]][0].tabu_run(130, 7, ws[w])
        assert out[w]["restarts"] == []
        assert out[w]["trace"].tobytes() == o["trace"].tobytes(), w
        assert np.array_equal(out[w]["x"], o["x"]) and np.array_equal(out[w]["w"], o["w"])
        assert out[w]["best_obj"] == o["best_obj"] and out[w]["cutoff_rhs"] == o["cutoff_rhs"]


def test_identical_walks_restart_the_later_one():
    mip = mipgen.random_mixed(3, n=80, m=50, max_row_nnz=5, frac_bin=0.5, frac_int=0.5)
    probs = [_prob(mip)]
    out = oracle.batch_restarts(probs, [0, 0], [4, 4], 120, 5, every=50, min_distance=1)
    plain = probs[0][0].tabu_run(120, 5, 4)
    assert out[0]["restarts"] == []
    assert out[0]["trace"].tobytes() == plain["trace"].tobytes()
    assert out[1]["restarts"][0] == 50
    assert out[1]["trace"][:50].tobytes() == plain["trace"][:50].tobytes()
    # the restart point is the start point of the walk's next restart seed:
    # the first move after the boundary leaves that point's value
    x1 = probs[0][0].start_point(oracle.restart_seed(4, 1))
    tr = out[1]["trace"][50:]
    first = tr[tr["var"] >= 0][0]
    assert first["x_old"] == x1[first["var"]]


def test_walks_on_different_problems_are_not_compared():
    mip = mipgen.random_mixed(5, n=40, m=30, max_row_nnz=4)
    probs = [_prob(mip), _prob(mip)]
    out = oracle.batch_restarts(probs, [0, 1], [9, 9], 90, 5, every=30, min_distance=10**9)
    assert out[0]["restarts"] == [] and out[1]["restarts"] == []


def test_close_walks_restart_at_every_boundary():
    mip = mipgen.random_mixed(6, n=50, m=30, max_row_nnz=4, frac_bin=0.6, frac_int=0.4)
    probs = [_prob(mip)]
    out = oracle.batch_restarts(probs, [0, 0, 0], [1, 2, 3], 100, 5, every=25, min_distance=10**9)
    assert out[0]["restarts"] == []
    assert out[1]["restarts"] == [25, 50, 75] and out[2]["restarts"] == [25, 50, 75]
    assert all(len(o["trace"]) == 100 for o in out)
