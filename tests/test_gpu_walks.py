"""GPU walks on cached buffers and mixed batches, through the C ABI.

chap_tabu_run keeps one walk's device buffers and captured iteration graphs
with its problem between calls and reads the final state back only when it
is asked for. These tests run many walks of different lengths, seeds and
start points on one problem, with earlier runs kept alive or released, and
compare each with the oracle bit for bit. A batch mixing staged walks
(all-integer, row-block records) and unstaged walks (row_stage=-1, or
continuous variables) with long narrow columns must equal the plain walks.
"""
from __future__ import annotations

import numpy as np
import pytest

import mipgen
import oracle
from test_gpu_parity import chap, compare_runs, say  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def test_repeated_runs_on_one_problem(chap):
    mip = mipgen.random_mixed(81, n=300, m=200, max_row_nnz=8, frac_bin=0.3, frac_int=0.7, int_width=30,
                              long_cols=4, long_deg=80)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip, graph_iters=16, chunk_min=24, chunk_len=16)
    kept = []
    for k, (iters, seed) in enumerate([(0, 0), (1, 3), (5, 0), (37, 2), (16, 1), (100, 4), (3, 5), (70, 2)]):
        say(f"cached slot run {k}: iters={iters} seed={seed}")
        g = G.tabu_run(iters, 7, seed)
        o = P.tabu_run(iters, 7, seed)
        if k % 2:
            kept.append((g, o, iters, seed))   # state read later, after other runs used the problem
        else:
            compare_runs(g, o, f"run {k}")
    x0 = mipgen.random_point(mip, 9)
    say("cached slot run with x0")
    compare_runs(G.tabu_run(45, 5, 0, x0=x0), P.tabu_run(45, 5, 0, x0=x0), "x0")
    for g, o, iters, seed in kept:
        say(f"deferred state of run iters={iters} seed={seed}")
        compare_runs(g, o, f"kept run iters={iters} seed={seed}")


def test_run_outlives_problem(chap):
    mip = mipgen.powerlaw(82, n=6000, m=3000, nnz=60_000, cap=2000)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip)
    say("run outliving its problem")
    g = G.tabu_run(50, 10, 1)
    del G
    import gc
    gc.collect()
    compare_runs(g, P.tabu_run(50, 10, 1), "after problem release")


def test_compact_rows_toggle_on_one_slot(chap):
    """A walk of 65540 iterations cannot keep compact rows; short walks before
    and after it on the same problem do. All equal the oracle."""
    mip = mipgen.random_mixed(74, n=40, m=30, max_row_nnz=6, frac_bin=0.3, frac_int=0.7)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip)
    say("short walk (compact rows)")
    compare_runs(G.tabu_run(200, 3, 1), P.tabu_run(200, 3, 1), "before")
    say("65540-iteration walk on the same slot (full rows)")
    compare_runs(G.tabu_run(65540, 3, 1), P.tabu_run(65540, 3, 1), "long")
    say("short walk again (compact rows)")
    compare_runs(G.tabu_run(300, 3, 2), P.tabu_run(300, 3, 2), "after")


def test_mixed_batch_staged_and_unstaged(chap):
    """Staged walks (long columns scored by k_stage_score, combined in the move
    selection when alone) batched with unstaged walks whose long narrow
    columns go through k_narrow_chunk: every walk equals its plain walk, and
    walks of each kind equal the oracle."""
    base = mipgen.powerlaw(83, n=9000, m=6000, nnz=90_000, cap=4000)
    cont = mipgen.general(84, n=6000, m=3000)
    probs = [chap.Problem(base, chunk_min=24), chap.Problem(base, chunk_min=24, row_stage=-1),
             chap.Problem(cont, chunk_min=24)]
    walk_prob = [0, 1, 2, 0, 1, 2]
    walk_seed = [3, 3, 4, 5, 6, 7]
    say("mixed batch: staged + unstaged + continuous, 60 iterations")
    runs = chap.batch_run(probs, walk_prob, walk_seed, 60, 5)
    for w, r in enumerate(runs):
        say(f"plain walk {w} (problem {walk_prob[w]})")
        g = probs[walk_prob[w]].tabu_run(60, 5, walk_seed[w])
        assert r.trace.tobytes() == g.trace.tobytes(), f"walk {w} trace"
        assert r.x.tobytes() == g.x.tobytes() and r.w.tobytes() == g.w.tobytes()
        assert r.resid.tobytes() == g.resid.tobytes()
    assert runs[0].trace.tobytes() == runs[1].trace.tobytes()
    for w in (0, 4):
        say(f"oracle walk {w}")
        o = oracle.OracleProblem(base).tabu_run(60, 5, walk_seed[w])
        compare_runs(runs[w], o, f"mixed batch walk {w}")
    # the same mixture with only staged walks and unstaged walks of integer data
    say("mixed batch: staged + unstaged only")
    runs2 = chap.batch_run(probs[:2], [0, 1, 1, 0], [9, 9, 10, 10], 40, 5)
    assert runs2[0].trace.tobytes() == runs2[1].trace.tobytes()
    assert runs2[2].trace.tobytes() == runs2[3].trace.tobytes()
    compare_runs(runs2[2], oracle.OracleProblem(base).tabu_run(40, 5, 10), "staged+unstaged walk 2")


def test_byte_copy_of_x(chap):
    """Instances whose variables are all integers with bounds in [-128, 127]
    let residuals from scratch gather a byte copy of x. Points at the bounds
    (the ends of the byte range, and a narrow domain whose columns take the
    staged path) give passes and walks equal to the oracle."""
    import torch

    for lo, hi in ((-128.0, 127.0), (-20.0, 43.0)):
        mip = mipgen.powerlaw(85, n=20_000, m=10_000, nnz=200_000, cap=3000)
        mip.lb[:] = lo
        mip.ub[:] = hi
        P = oracle.OracleProblem(mip)
        G = chap.Problem(mip)
        w = mipgen.random_weights(P.mp + 1, 2, wmax=6)
        wd = torch.from_numpy(w).cuda()
        base = np.clip(mipgen.random_point(mip, 3), lo, hi)
        j = np.arange(mip.n)
        cases = [("random", base), ("lower bounds", np.full(mip.n, lo)), ("upper bounds", np.full(mip.n, hi)),
                 ("mixed ends", np.where(j % 3 == 0, lo, np.where(j % 3 == 1, hi, base)))]
        for name, x in cases:
            say(f"best_shift byte copy [{lo}, {hi}]: {name}")
            xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
            xh, s = G.best_shift(xd, wd)
            torch.cuda.synchronize()
            oxh, os_ = P.best_shift(x, w)
            assert np.array_equal(s.cpu().numpy(), os_), name
            assert np.array_equal(xh.cpu().numpy(), oxh), name
        say(f"walk byte copy [{lo}, {hi}] from the upper bounds")
        x0 = np.full(mip.n, hi)
        compare_runs(G.tabu_run(30, 5, 0, x0=x0), P.tabu_run(30, 5, 0, x0=x0), f"x0 at {hi}")


def test_start_point_validation(chap):
    """A start point must lie within the bounds and be integral on integer
    variables (CHAP_EINVAL otherwise)."""
    mip = mipgen.random_mixed(86, n=30, m=20)
    G = chap.Problem(mip)
    ok = np.clip(np.zeros(mip.n), mip.lb, mip.ub)
    G.tabu_run(3, 2, 0, x0=ok)
    ints = np.flatnonzero(mip.is_int == 1)
    bad_frac = ok.copy()
    bad_frac[ints[0]] += 0.5
    bad_high = ok.copy()
    bad_high[0] = mip.ub[0] + 1.0
    for bad in (bad_frac, bad_high):
        with pytest.raises(chap.ChapError, match="CHAP_EINVAL"):
            G.tabu_run(3, 2, 0, x0=bad)


def test_best_infeasible_point(chap):
    """The best infeasible point a walk visited (fewest violated rows, the
    cutoff row not counted, first reached) equals the oracle's: its point,
    row count and iteration, for walks that reach feasibility and walks that
    do not."""
    cases = [("tiny_binary", mipgen.tiny_binary(0), 400),
             ("mixed integer", mipgen.random_mixed(87, n=300, m=200, max_row_nnz=8, frac_bin=0.3, frac_int=0.7,
                                                   long_cols=3, long_deg=60), 300),
             ("continuous", mipgen.random_mixed(88, n=80, m=40, integer_data=False), 300),
             ("powerlaw", mipgen.powerlaw(89, n=20_000, m=10_000, nnz=200_000, cap=3000), 200)]
    for name, mip, iters in cases:
        P = oracle.OracleProblem(mip)
        G = chap.Problem(mip)
        for seed in (0, 2):
            say(f"best infeasible {name} seed={seed}")
            g = G.tabu_run(iters, 10, seed)
            o = P.tabu_run(iters, 10, seed)
            x, v, k = g.best_infeasible()
            assert (v, k) == (o["inf_viol"], o["inf_iter"]), (name, seed, v, k, o["inf_viol"], o["inf_iter"])
            if k == -2:
                assert x is None and o["inf_x"] is None
            else:
                assert np.array_equal(x, o["inf_x"]), (name, seed)


def test_batch_with_start_points(chap):
    """Batched walks from given start points (some walks seeded): each equals
    the plain walk from the same start, and one equals the oracle."""
    mips = [mipgen.random_mixed(90, n=400, m=250, max_row_nnz=8, frac_bin=0.3, frac_int=0.7),
            mipgen.general(91, n=3000, m=1500)]
    probs = [chap.Problem(m) for m in mips]
    walk_prob = [0, 1, 0, 1, 0]
    walk_seed = [1, 2, 3, 4, 5]
    walk_x0 = [mipgen.random_point(mips[0], 7), None, None, mipgen.random_point(mips[1], 8),
               mipgen.random_point(mips[0], 9)]
    say("batch with start points")
    runs = chap.batch_run(probs, walk_prob, walk_seed, 60, 5, walk_x0=walk_x0)
    for w, r in enumerate(runs):
        g = probs[walk_prob[w]].tabu_run(60, 5, walk_seed[w], x0=walk_x0[w])
        assert r.trace.tobytes() == g.trace.tobytes(), f"walk {w}"
        assert r.x.tobytes() == g.x.tobytes() and r.w.tobytes() == g.w.tobytes()
        assert r.best_infeasible()[1:] == g.best_infeasible()[1:]
    o = oracle.OracleProblem(mips[0]).tabu_run(60, 5, 0, x0=walk_x0[0])
    compare_runs(runs[0], o, "batch walk from x0")


def _two_class_instance(seed: int) -> mipgen.MIP:
    """150,000 binary columns in one row each and 150,000 integer columns in
    [0, 10] in three rows each; the first 15,000 rows hold only binaries, the
    other 45,000 only integers. Internal column order puts the two classes
    in separate ranges, so with x held in 131,072-column blocks the row groups
    of binary rows have no entries in the last block and those of integer
    rows none in the first."""
    rng = np.random.default_rng(seed)
    nb, ni, mb, mi = 150_000, 150_000, 15_000, 45_000
    rows_b = np.repeat(np.arange(mb), 10)
    cols_b = rng.permutation(nb)
    rows_i = np.repeat(np.arange(mb, mb + mi), 10)
    cols_i = nb + rng.permutation(np.repeat(np.arange(ni), 3))
    # rows of one integer row must not repeat a column: redraw until none do
    while True:
        key = rows_i.astype(np.int64) * (nb + ni) + cols_i
        o = np.argsort(key, kind="stable")
        dup = np.zeros(key.shape[0], dtype=bool)
        dup[o[1:]] = key[o[1:]] == key[o[:-1]]
        if not dup.any():
            break
        cols_i[dup] = nb + rng.integers(0, ni, size=int(dup.sum()))
    rows = np.concatenate([rows_b, rows_i])
    cols = np.concatenate([cols_b, cols_i])
    vals = rng.integers(1, 6, size=rows.shape[0]) * (rng.integers(0, 2, size=rows.shape[0]) * 2 - 1)
    n, m = nb + ni, mb + mi
    lb = np.zeros(n)
    ub = np.concatenate([np.ones(nb), np.full(ni, 10.0)])
    is_int = np.ones(n, dtype=np.uint8)
    hidden = np.concatenate([rng.integers(0, 2, size=nb), rng.integers(0, 11, size=ni)]).astype(np.float64)
    sense = rng.choice(np.array([mipgen.SENSE_L, mipgen.SENSE_G, mipgen.SENSE_E]), size=m, p=[0.45, 0.45, 0.1])
    obj = rng.integers(-3, 4, size=n).astype(np.float64)
    return mipgen._finish(n, m, rows, cols, vals.astype(np.float64), sense, lambda act: act, lb, ub, is_int, obj,
                          hidden, "two classes")


def test_residuals_with_empty_x_blocks(chap):
    """Residuals from scratch of an all-integer instance whose row groups
    leave whole blocks of x without entries (skipped at the start and at the
    end of a group's sweep): single passes and a walk equal the oracle."""
    import torch

    mip = _two_class_instance(91)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip)
    for seed in (1, 2):
        x = mipgen.random_point(mip, seed)
        w = mipgen.random_weights(P.mp + 1, seed + 3, wmax=5)
        say(f"best_shift two-class instance seed={seed}")
        xh, s = G.best_shift(torch.from_numpy(x).cuda(), torch.from_numpy(w).cuda())
        torch.cuda.synchronize()
        oxh, os_ = P.best_shift(x, w)
        assert np.array_equal(s.cpu().numpy(), os_)
        assert np.array_equal(xh.cpu().numpy(), oxh)
    say("walk two-class instance")
    compare_runs(G.tabu_run(25, 5, 3), P.tabu_run(25, 5, 3), "two classes")


@pytest.mark.parametrize("n", [131071, 131072, 131073, 262145])
def test_residuals_at_x_block_edges(chap, n):
    """All-integer instances whose column count falls at and around the
    residual kernel's 131,072-column blocks of x (a last block of one column,
    an exact fit, a ragged tail) with 8,193 rows (a last row group of one
    row): single passes and a short walk equal the oracle."""
    import torch

    mip = mipgen.random_mixed(700 + n % 11, n=n, m=8193, max_row_nnz=8, frac_bin=0.5, frac_int=0.5,
                              int_width=40)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip)
    x = mipgen.random_point(mip, 5)
    w = mipgen.random_weights(P.mp + 1, 6, wmax=5)
    say(f"best_shift at x-block edges n={n}")
    xh, s = G.best_shift(torch.from_numpy(x).cuda(), torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    oxh, os_ = P.best_shift(x, w)
    assert np.array_equal(s.cpu().numpy(), os_)
    assert np.array_equal(xh.cpu().numpy(), oxh)
    say(f"walk at x-block edges n={n}")
    compare_runs(G.tabu_run(6, 5, 2), P.tabu_run(6, 5, 2), f"n={n}")
