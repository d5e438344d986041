"""Affected rescoring (rescore_cap > 0) through the C ABI.

After a move that changes no weight, no incumbent and no cutoff residual,
a walk scores again only the columns sharing a row with the moved column
(section 3.1 "Memory Considerations", first paragraph; the claim is pinned
on the oracle in test_affected_oracle.py). The trajectory must be the one of
full rescoring: every walk here equals the oracle bit for bit and the same
walk on a problem without the option, and reports how many iterations took
the subset pass.
"""
from __future__ import annotations

import numpy as np
import pytest

import mipgen
import oracle
from test_gpu_parity import chap, compare_runs, say  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def same_walk(a, b, what):
    assert a.trace.tobytes() == b.trace.tobytes(), f"{what}: trace"
    assert a.x.tobytes() == b.x.tobytes() and a.w.tobytes() == b.w.tobytes(), what
    assert a.resid.tobytes() == b.resid.tobytes(), what
    assert a.best_obj == b.best_obj and a.cutoff_rhs == b.cutoff_rhs, what


def test_rescore_tiny_binary(chap):
    """From x = 0 the point is feasible at once, the cutoff row is active and
    nearly every column has c != 0, so nearly every iteration is a full pass;
    from x = 1 the walk first moves through infeasible points, where moves
    rescore only the affected columns. Both reach feasible points, update the
    incumbent and reweight."""
    mip = mipgen.tiny_binary(0)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip, rescore_cap=256)
    F = chap.Problem(mip)
    for name, x0 in (("x=0", None), ("x=1", np.ones(mip.n))):
        say(f"rescore tiny_binary 1000 iterations from {name}")
        g = G.tabu_run(1000, 10, 0, x0=x0)
        compare_runs(g, P.tabu_run(1000, 10, 0, x0=x0), f"tiny_binary {name}")
        same_walk(g, F.tabu_run(1000, 10, 0, x0=x0), f"tiny_binary full {name}")
        assert (g.trace["kind"] == 2).any() and np.isfinite(g.best_obj)
        if x0 is not None:
            assert 0 < g.rescored < 1000, g.rescored


@pytest.mark.parametrize("cap", [1, 4, 64, 4096])
def test_rescore_mixed_caps(chap, cap):
    """Mixed instances with long narrow and general columns, infinite bounds,
    all senses; cap 1 and 4 force most iterations to the full pass."""
    mip = mipgen.random_mixed(131, n=400, m=300, max_row_nnz=8, frac_bin=0.3, frac_int=0.4, int_width=40,
                              inf_bounds=0.05, long_cols=4, long_deg=120)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip, rescore_cap=cap, chunk_min=24, chunk_len=16)
    say(f"rescore mixed cap={cap}")
    for seed in (0, 3):
        g = G.tabu_run(300, 7, seed)
        compare_runs(g, P.tabu_run(300, 7, seed), f"mixed cap={cap} seed={seed}")
        if cap >= 64:
            assert g.rescored > 0
        if cap == 1:
            assert g.rescored == 0


def test_rescore_continuous_data(chap):
    """Fractional coefficients and objective: incumbents and the cutoff row
    (delta = 1e-4 max(1, |f_best|)); rows are summed again on every move."""
    for seed in (141, 142, 143):
        mip = mipgen.random_mixed(seed, n=120, m=60, max_row_nnz=6, integer_data=False)
        P = oracle.OracleProblem(mip)
        G = chap.Problem(mip, rescore_cap=512)
        say(f"rescore continuous seed={seed}")
        g = G.tabu_run(400, 5, 1)
        compare_runs(g, P.tabu_run(400, 5, 1), f"continuous {seed}")
        assert g.rescored > 0


def test_rescore_general_columns_beyond_the_subset_sort(chap):
    """General columns with more than 4094 entries have no subset form: a
    move touching one of them leaves the iteration to the full pass."""
    mip = mipgen.random_mixed(151, n=300, m=5000, max_row_nnz=4, frac_bin=0.2, frac_int=0.1, long_cols=3,
                              long_deg=4600)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip, rescore_cap=4096)
    say("rescore with long general columns")
    g = G.tabu_run(150, 5, 2)
    compare_runs(g, P.tabu_run(150, 5, 2), "long general")


def test_rescore_general_workload(chap):
    """The general workload's shape at 20k variables: 2000 iterations equal
    the walk of full rescoring, the first 300 equal the oracle, and nearly
    every iteration takes the subset pass."""
    mip = mipgen.general(161, n=20_000, m=10_000)
    G = chap.Problem(mip, rescore_cap=1024)
    F = chap.Problem(mip)
    say("rescore general 2000 iterations")
    g = G.tabu_run(2000, 10, 0)
    same_walk(g, F.tabu_run(2000, 10, 0), "general full")
    assert g.rescored >= 1900, g.rescored
    say("rescore general vs oracle 300 iterations")
    compare_runs(G.tabu_run(300, 10, 4), oracle.OracleProblem(mip).tabu_run(300, 10, 4), "general oracle")


def test_rescore_repeated_runs_and_start_points(chap):
    """Stamps of earlier runs on the cached walk buffers do not leak into
    later runs (iteration tags restart at each run)."""
    mip = mipgen.random_mixed(171, n=200, m=150, max_row_nnz=6, frac_bin=0.4, frac_int=0.4)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip, rescore_cap=128, graph_iters=16)
    for k, (iters, seed) in enumerate([(50, 0), (200, 1), (7, 2), (120, 0)]):
        say(f"rescore repeated run {k}")
        compare_runs(G.tabu_run(iters, 5, seed), P.tabu_run(iters, 5, seed), f"run {k}")
    x0 = mipgen.random_point(mip, 5)
    compare_runs(G.tabu_run(90, 5, 0, x0=x0), P.tabu_run(90, 5, 0, x0=x0), "x0")


def test_rescore_problem_in_batches_and_single_passes(chap):
    """A problem created with rescore_cap scores every column in batched
    walks and single passes (the option only changes chap_tabu_run walks),
    with the same results as a problem without it and as the oracle."""
    import math

    import torch

    mip = mipgen.random_mixed(181, n=300, m=200, max_row_nnz=6, frac_bin=0.4, frac_int=0.4, long_cols=3, long_deg=60)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip, rescore_cap=256)
    F = chap.Problem(mip, row_stage=-1)
    say("rescore problem in a batch")
    runs = chap.batch_run([G, F], [0, 1, 0], [3, 3, 4], 80, 5)
    assert runs[0].trace.tobytes() == runs[1].trace.tobytes()
    compare_runs(runs[2], P.tabu_run(80, 5, 4), "batch walk on the rescore problem")
    say("rescore problem single pass")
    x = mipgen.random_point(mip, 2)
    w = mipgen.random_weights(P.mp + 1, 2)
    xd = torch.from_numpy(x).cuda()
    wd = torch.from_numpy(w).cuda()
    for cut in (math.inf, P.objective(x) - 1.0):
        xh, s = G.best_shift(xd, wd, cut)
        torch.cuda.synchronize()
        oxh, os_ = P.best_shift(x, w, cut)
        assert np.array_equal(xh.cpu().numpy(), oxh) and np.array_equal(s.cpu().numpy(), os_)
