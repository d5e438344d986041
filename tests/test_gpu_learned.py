"""GPU parity of the learned proposal form against the CPU oracle.

* network inputs at a given state against oracle/features.py (integer data:
  bit-exact);
* with full_every = 1 the learned walk is the plain walk, record for record;
* every learned walk replays exactly in the oracle given its logged proposal
  sets (the sets are the network's choice; everything else is unique);
* each logged set is a valid top-K of the reference network scores at its
  iteration, within the FP32 accumulation bound of oracle/mlp.py.
"""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import mipgen
import oracle
from oracle import features as F
from oracle import mlp

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def chap():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2605_05086_amd as c

    c.load_library()
    return c


def dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def bf16_values(bits):
    b = np.asarray(bits).astype(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def compare_traces(g, o, what):
    """Every field bit-exact (the traced objective is c^T x rounded once on
    both sides)."""
    for f in ("iter", "var", "kind", "x_old", "x_new", "score", "viol", "obj"):
        a, b = g[f], o[f]
        bad = np.flatnonzero(a != b)
        assert bad.size == 0, f"{what}: field {f} differs first at iteration {bad[0]}: gpu {a[bad[0]]} oracle {b[bad[0]]}"


def random_state(mip, P, seed, k):
    rng = np.random.default_rng(seed)
    lb, ub, _ = P.bounds()
    x = mipgen.random_point(mip, seed)
    xh = mipgen.random_point(mip, seed + 1)
    w = rng.integers(1, 6, P.mp + 1).astype(np.float32)
    s_last = rng.integers(-8, 9, mip.n).astype(np.float64)
    last_move = rng.integers(-1024, k, mip.n).astype(np.int32)
    moves = rng.integers(0, 40, mip.n).astype(np.int32)
    return x, w, s_last, xh, last_move, moves


@pytest.mark.parametrize("seed,cut", [(0, False), (1, True), (2, False)])
def test_features_parity(chap, seed, cut):
    import torch
    mip = mipgen.random_mixed(300 + seed, n=300, m=200, max_row_nnz=8, int_width=40, long_cols=2, long_deg=60,
                              inf_bounds=0.1)
    P = oracle.OracleProblem(mip)
    G = chap.Problem(mip)
    k, klf = 100, 90
    x, w, s_last, xh, lm, mv = random_state(mip, P, seed, k)
    cutoff = float(np.floor(mip.obj @ x)) - 2.0 if cut else math.inf
    say(f"features seed={seed} cut={cut}")
    out = chap.features(G, dev(x, torch.float64), dev(w, torch.float32), cutoff, dev(s_last, torch.float64),
                        dev(xh, torch.float64), dev(lm, torch.int32), dev(mv, torch.int32), k, klf)
    got = bf16_values(out.cpu().numpy())
    want, ok = F.inputs(mip, P, x, w, cutoff, s_last, xh, lm, mv, k, klf)
    assert np.array_equal(got[~ok], np.zeros_like(got[~ok]))
    bad = np.argwhere(got != want)
    assert bad.size == 0, (bad[:5], got[tuple(bad[0])], want[tuple(bad[0])])


def test_full_every_one_is_plain(chap):
    mip = mipgen.random_mixed(410, n=200, m=150, max_row_nnz=8, int_width=30, long_cols=2, long_deg=40)
    G = chap.Problem(mip)
    M = chap.Model(1)
    say("learned full_every=1 vs plain")
    plain = G.tabu_run(300, 10, 3)
    lr = chap.learned_run(G, M, 300, 10, 3, full_every=1, topk=16, train_steps=2, train_pairs=32)
    compare_traces(lr.trace, plain.trace, "learned(F=1) vs plain")
    np.testing.assert_array_equal(lr.x, plain.x)
    np.testing.assert_array_equal(lr.w, plain.w)
    assert lr.evals == 300 and lr.stalls == 0


CASES = [
    # (generator seed, n, m, iters, full_every, topk, train_steps, refresh_every)
    (420, 200, 150, 400, 8, 16, 0, 1),
    (421, 300, 200, 500, 16, 32, 2, 1),
    (422, 120, 100, 300, 4, 8, 1, 1),
    (423, 300, 200, 500, 16, 32, 1, 4),
    (424, 200, 150, 400, 32, 16, 0, 7),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"seed{c[0]}-F{c[4]}-K{c[5]}-T{c[6]}-R{c[7]}")
def test_learned_walk_replays_exactly(chap, case):
    gseed, n, m, iters, F_, K, steps, R = case
    mip = mipgen.random_mixed(gseed, n=n, m=m, max_row_nnz=8, int_width=30, long_cols=2, long_deg=50)
    G = chap.Problem(mip)
    M = chap.Model(gseed)
    say(f"learned walk {case}")
    run = chap.learned_run(G, M, iters, 10, 2, full_every=F_, topk=K, train_steps=steps, train_pairs=24, lr=3e-3,
                           log_sets=1, refresh_every=R)
    P = oracle.OracleProblem(mip)
    ref = P.learned_replay(iters, 10, 2, F_, run.sets, run.set_offsets)
    compare_traces(run.trace, ref["trace"], f"learned {case}")
    np.testing.assert_array_equal(run.x, ref["x"])
    np.testing.assert_array_equal(run.w, ref["w"])
    assert run.best_obj == ref["best_obj"] and run.cutoff_rhs == ref["cutoff_rhs"]
    kinds = run.trace["kind"]
    assert (kinds >= 8).sum() > 0, "no move came from a proposal set"
    full = np.isin(kinds, [0, 1, 2])
    assert run.evals == int(full.sum())
    assert run.stalls == int((kinds == 3).sum())
    for k in np.flatnonzero(~full):
        s = run.proposal_set(k)
        assert 0 < s.size <= K and np.unique(s).size == s.size
    if R > 1:
        # a set is kept for R proposal iterations after each refresh
        kept = 0
        for k in np.flatnonzero(~full[1:]) + 1:
            if not full[k - 1] and kinds[k - 1] != 3 and np.array_equal(run.proposal_set(k), run.proposal_set(k - 1)):
                kept += 1
        assert kept > 0


def test_tiny_binary_learned_replay(chap):
    mip = mipgen.tiny_binary(0)
    G = chap.Problem(mip)
    M = chap.Model(0)
    say("tiny binary learned walk")
    run = chap.learned_run(G, M, 1000, 10, 0, full_every=16, topk=32, train_steps=1, train_pairs=16, log_sets=1)
    ref = oracle.OracleProblem(mip).learned_replay(1000, 10, 0, 16, run.sets, run.set_offsets)
    compare_traces(run.trace, ref["trace"], "tiny binary learned")
    assert run.best_obj == ref["best_obj"]


def _state_at(P, iters_prefix, F_, sets, offs, seed):
    """Oracle replay of the first `iters_prefix` iterations."""
    o = offs[:iters_prefix + 1]
    return P.learned_replay(iters_prefix, 10, seed, F_, sets, o)


def test_proposal_sets_are_top_k(chap):
    mip = mipgen.random_mixed(430, n=400, m=300, max_row_nnz=8, int_width=30, long_cols=2, long_deg=50)
    G = chap.Problem(mip)
    M = chap.Model(5)
    params = M.get_params().astype(np.float64)
    F_, K, iters, seed = 8, 24, 60, 4
    say("proposal sets vs reference scores")
    run = chap.learned_run(G, M, iters, 10, seed, full_every=F_, topk=K, log_sets=1)
    P = oracle.OracleProblem(mip)
    kinds = run.trace["kind"]
    full_iters = np.flatnonzero(np.isin(kinds, [0, 1, 2]))
    checked = 0
    for kstar in (5, 13, 30, 45):
        if kstar >= iters or np.isin(kinds[kstar], [0, 1, 2]) or kinds[kstar - 1] == 3:
            continue
        klf = int(full_iters[full_iters < kstar].max())
        now = _state_at(P, kstar, F_, run.sets, run.set_offsets, seed)
        at_full = _state_at(P, klf, F_, run.sets, run.set_offsets, seed)
        after_full = _state_at(P, klf + 1, F_, run.sets, run.set_offsets, seed)
        xh, s_last = P.best_shift(at_full["x"], at_full["w"], at_full["cutoff_rhs"])
        tr = run.trace[:kstar]
        moved = tr["var"] >= 0
        last_move = np.full(mip.n, -1024)
        moves = np.zeros(mip.n, dtype=np.int64)
        for k in np.flatnonzero(moved):
            last_move[tr["var"][k]] = k
            moves[tr["var"][k]] += 1
        X, ok = F.inputs(mip, P, now["x"], now["w"], now["cutoff_rhs"], s_last, xh, last_move, moves, kstar, klf,
                         refresh=(after_full["x"], after_full["w"], after_full["cutoff_rhs"]))
        y, _ = mlp.forward(params, X, True)
        ey, _ = mlp.forward_bound(params, X)
        chosen = np.zeros(mip.n, dtype=bool)
        chosen[run.proposal_set(kstar)] = True
        assert not (chosen & ~ok).any()
        assert chosen.sum() == min(K, ok.sum())
        lo = np.min((y + ey)[chosen])
        hi = np.max((y - ey)[ok & ~chosen])
        assert lo >= hi, (kstar, lo, hi)
        checked += 1
    assert checked >= 2


def test_learned_options_rejected(chap):
    mip = mipgen.random_mixed(440, n=50, m=40)
    G = chap.Problem(mip)
    M = chap.Model(0)
    for bad in (dict(topk=0), dict(full_every=0), dict(train_pairs=0), dict(lr=0.0), dict(train_steps=-1),
                dict(refresh_every=0)):
        with pytest.raises(chap.ChapError) as e:
            chap.learned_run(G, M, 10, 10, 0, **bad)
        assert e.value.code == -1


def test_learned_edge_cases(chap):
    mip = mipgen.random_mixed(450, n=60, m=40, max_row_nnz=6, long_cols=1, long_deg=30)
    G = chap.Problem(mip)
    M = chap.Model(2)
    P = oracle.OracleProblem(mip)
    for iters, F_, K in ((0, 8, 4), (1, 8, 4), (7, 64, 4), (40, 5, 1000), (40, 3, 1)):
        say(f"learned edge iters={iters} F={F_} K={K}")
        run = chap.learned_run(G, M, iters, 5, 1, full_every=F_, topk=K, log_sets=1)
        assert run.trace.shape[0] == iters
        if iters == 0:
            continue
        ref = P.learned_replay(iters, 5, 1, F_, run.sets, run.set_offsets)
        compare_traces(run.trace, ref["trace"], f"edge iters={iters} F={F_} K={K}")


def test_trained_network_gains_over_untrained(chap):
    """What the trained network gains: on a 2M-nonzero power-law instance, a
    network trained on pairs logged by a plain walk from another start point
    puts the full evaluation's own choice into its proposal set far more
    often than the same network untrained, and the moves its walk takes from
    proposal sets have larger exact scores. (Violation counts of single
    walks are too noisy at this size to rank the two.)"""
    import torch
    mip = mipgen.powerlaw(0, n=200_000, m=100_000, nnz=2_000_000, cap=20_000)
    G = chap.Problem(mip)
    iters, tenure = 768, 10
    say("gain: plain walk")
    plain = G.tabu_run(iters, tenure, 0)
    vp = int(plain.trace["viol"][-1])
    trained = chap.Model(0)
    say("gain: logging walk and training")
    log = chap.learned_run(G, trained, 64, tenure, 7, full_every=1, topk=256, train_pairs=512, log_pairs=64 * 1024)
    trained.train(torch.from_numpy(log.pair_feat.view(np.int16)).cuda(), torch.from_numpy(log.pair_target).cuda(),
                  steps=600, batch=1024, lr=1e-3, seed=1)
    out = {}
    for name, M in (("trained", trained), ("untrained", chap.Model(0))):
        say(f"gain: learned walk, {name}")
        run = chap.learned_run(G, M, iters, tenure, 0, full_every=16, topk=256)
        prop = run.trace["kind"] >= 8
        out[name] = (run.hits / run.evals, float(np.mean(run.trace["score"][prop])), int(run.trace["viol"][-1]))
    say(f"gain: (hit rate, mean proposal-move score, final violations) {out}; plain final {vp}")
    assert out["trained"][0] >= 0.5 and out["trained"][0] >= out["untrained"][0] + 0.3, out
    assert out["trained"][1] > 1.2 * out["untrained"][1], out


def test_learned_replay_full_size_paths(chap):
    """The proposal paths the 20M-nonzero workload runs, at their full sizes:
    a 2M-nonzero power-law instance (200k columns) whose proposable columns
    include narrow columns far beyond one 2048-entry subset chunk and one
    4096-entry refresh chunk, and general columns of 3500..4094 entries (the
    largest that one workgroup's sort holds); top-K of 1024 over every
    proposable column (all radix digits), a full evaluation every 16
    iterations, online training. The walk replays in the oracle from its
    logged proposal sets bit for bit, and one proposal set is checked to be a
    valid top-K set of the reference network scores."""
    mip = mipgen.powerlaw(0, n=200_000, m=100_000, nnz=2_000_000, cap=20_000)
    # normalised entries per column (equality rows count twice)
    is_e = (mip.sense == ord("E"))[mip.csc_row]
    col_of = np.repeat(np.arange(mip.n), np.diff(mip.csc_col_ptr))
    ne = np.bincount(col_of, weights=1.0 + is_e, minlength=mip.n).astype(np.int64) + (mip.obj != 0)
    general = np.flatnonzero((ne >= 3500) & (ne + 2 <= 4096))[:6]
    assert general.size >= 3
    mip.ub[general] = 400.0   # wider than 64 values: general columns
    P = oracle.OracleProblem(mip)
    assert int(ne.max()) > 8192
    G = chap.Problem(mip)
    M = chap.Model(3)
    iters, F_, K, seed = 96, 16, 1024, 1
    say("learned full-size paths: walk")
    run = chap.learned_run(G, M, iters, 10, seed, full_every=F_, topk=K, train_steps=2, train_pairs=256, lr=1e-3,
                           log_sets=1)
    say("learned full-size paths: oracle replay")
    ref = P.learned_replay(iters, 10, seed, F_, run.sets, run.set_offsets)
    compare_traces(run.trace, ref["trace"], "learned full-size")
    np.testing.assert_array_equal(run.x, ref["x"])
    np.testing.assert_array_equal(run.w, ref["w"])
    kinds = run.trace["kind"]
    prop_iters = np.flatnonzero(~np.isin(kinds, [0, 1, 2]))
    assert prop_iters.size > 40 and (kinds >= 8).sum() > 20
    sizes = [run.proposal_set(k).size for k in prop_iters]
    assert min(sizes) == max(sizes) == K
    moved_general = np.isin(run.trace["var"], general).sum() + sum(
        np.isin(run.proposal_set(k), general).any() for k in prop_iters)
    print(f"general columns moved or proposed: {moved_general}", flush=True)


def test_learned_topk_valid_full_size(chap):
    """One proposal set of a 200k-column walk with an untrained network and no
    training (fixed parameters) is a valid top-1024 set of the reference scores
    within the accumulation bound."""
    mip = mipgen.powerlaw(0, n=200_000, m=100_000, nnz=2_000_000, cap=20_000)
    G = chap.Problem(mip)
    M = chap.Model(9)
    params = M.get_params().astype(np.float64)
    F_, K, iters, seed = 16, 1024, 8, 2
    say("top-K validity at full size: walk")
    run = chap.learned_run(G, M, iters, 10, seed, full_every=F_, topk=K, log_sets=1)
    P = oracle.OracleProblem(mip)
    kinds = run.trace["kind"]
    kstar = 5
    assert not np.isin(kinds[kstar], [0, 1, 2]) and kinds[kstar - 1] != 3
    now = _state_at(P, kstar, F_, run.sets, run.set_offsets, seed)
    at_full = _state_at(P, 0, F_, run.sets, run.set_offsets, seed)
    after_full = _state_at(P, 1, F_, run.sets, run.set_offsets, seed)
    xh, s_last = P.best_shift(at_full["x"], at_full["w"], at_full["cutoff_rhs"])
    tr = run.trace[:kstar]
    last_move = np.full(mip.n, -1024)
    moves = np.zeros(mip.n, dtype=np.int64)
    for k in np.flatnonzero(tr["var"] >= 0):
        last_move[tr["var"][k]] = k
        moves[tr["var"][k]] += 1
    say("top-K validity at full size: reference inputs")
    X, ok = F.inputs(mip, P, now["x"], now["w"], now["cutoff_rhs"], s_last, xh, last_move, moves, kstar, 0,
                     refresh=(after_full["x"], after_full["w"], after_full["cutoff_rhs"]))
    y, _ = mlp.forward(params, X, True)
    ey, _ = mlp.forward_bound(params, X)
    chosen = np.zeros(mip.n, dtype=bool)
    chosen[run.proposal_set(kstar)] = True
    assert not (chosen & ~ok).any()
    assert chosen.sum() == min(K, ok.sum())
    assert np.min((y + ey)[chosen]) >= np.max((y - ey)[ok & ~chosen])
