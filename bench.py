"""Benchmark of the GPU tabu-search hot path on one MI355X.

One step = one tabu iteration (a best-shift pass over every variable, move
selection under tabu/aspiration, sparse residual update or reweight) on the
large power-law instance: 2M integer variables in [0, 50], 1M rows (80 % '<=',
20 % '='), 20M nonzeros with rank-Zipf(1.1) column degrees capped at 100k,
coefficients U{-9..9}\\{0}, generated with seed 0.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per best-shift pass on the 20M-nonzero instance, from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) over the pass kernels, scaled
# by the counters of a 1 GiB device copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0);
# see profiles/best_shift_pass_hbm_counters_powerlaw_20M.md. Valid for the
# pass kernels as they are; None until they are measured again after a change.
PASS_TRAFFIC_BYTES = 499_200_000
METRIC = "tabu moves/s, best-shift nnz/s, % HBM peak; plain vs batched/learned"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(mip, cutoff_active: bool) -> int:
    """Bytes one best-shift pass must move with int32 indices and FP64 values:
    12 per stored nonzero (index + coefficient, objective entries counted when
    the cutoff row is active), 12 per row (residual + weight), 4 per equality
    row (second weight), 48 per column (offset, incumbent, bounds, result
    shift and score, tabu entry)."""
    nnz = mip.nnz + (mip.nnz_obj if cutoff_active else 0)
    m_e = int(np.count_nonzero(mip.sense == ord("E")))
    return 12 * nnz + 12 * mip.m + 4 * m_e + 48 * mip.n


def cpu_info():
    """Host cores the oracle may use (the machine's CPU share: OMP_NUM_THREADS when
    set, else every core up to 16), the core count and the CPU model."""
    nproc = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(16, nproc)
    return threads, nproc, model


def cpu_baseline(mip, iters_single: int, iters_all: int):
    """The oracle walk on the host: iters_single iterations on one core, then
    iters_all iterations with its per-column and per-row loops on every core
    the box gives this job (same results)."""
    import oracle

    threads, nproc, model = cpu_info()
    P = oracle.OracleProblem(mip)
    oracle.set_threads(1)
    t0 = time.perf_counter()
    out1 = P.tabu_run(iters_single, 10, 0)
    dt1 = time.perf_counter() - t0
    used = oracle.set_threads(threads)
    t0 = time.perf_counter()
    out = P.tabu_run(iters_all, 10, 0)
    dt = time.perf_counter() - t0
    oracle.set_threads(1)
    assert out["trace"][:iters_single].tobytes() == out1["trace"].tobytes()
    return {"value": iters_all / dt, "unit": "moves/s", "cores": used, "kind": "oracle",
            "sample": f"{iters_all} tabu iterations (tenure 10, seed 0) of the same 20M-nonzero instance with "
                      f"{used} threads ({dt:.1f} s), and {iters_single} on one core ({dt1:.1f} s); the oracle "
                      f"recomputes every residual and every best shift each iteration",
            "single_core_value": iters_single / dt1, "nproc": nproc, "cpu_model": model,
            "last_viol": int(out["trace"]["viol"][-1])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--pass-reps", type=int, default=20)
    ap.add_argument("--cpu-iters", type=int, default=3, help="oracle iterations on one core")
    ap.add_argument("--cpu-iters-all", type=int, default=24, help="oracle iterations on all cores")
    ap.add_argument("--compare-iters", type=int, default=2000,
                    help="length of the plain walk the learned forms are compared against")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--small", action="store_true", help="reduced instance for quick checks")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (reference for HBM counters)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the learned-proposal and batched-walk comparisons against the plain walk")
    ap.add_argument("--batch-iters", type=int, default=1000)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-walk comparison")
    ap.add_argument("--configs-only", action="store_true",
                    help="run only configurations 1 and 2 (plain and affected rescoring) and print them")
    ap.add_argument("--batched-only", action="store_true",
                    help="of the comparisons run only the batch itself (no learned forms, no one-by-one "
                         "walks); for kernel traces of the batched iteration")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (this path does not "
              f"shard across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch

    import mipgen
    import paper_2605_05086_amd as chap

    assert torch.cuda.is_available()
    chap.load_library()
    if args.configs_only:
        # configurations 1 and 2 alone (kernel traces of their paths); not the bench line
        print(json.dumps({"configs": small_configs(chap, 10)}), flush=True)
        return
    t0 = time.perf_counter()
    if args.small:
        mip = mipgen.powerlaw(0, n=200_000, m=100_000, nnz=2_000_000, cap=20_000)
        wname = "powerlaw n=200k m=100k nnz=2M (Zipf 1.1, cap 20k), integer [0,50]"
    else:
        mip = mipgen.powerlaw(0)
        wname = "powerlaw n=2M m=1M nnz=20M (Zipf 1.1 column degrees, cap 100k), integer [0,50]"
    log(f"generated {mip.name} in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    G = chap.Problem(mip)
    log(f"problem created and uploaded in {time.perf_counter() - t0:.1f} s")

    tenure, seed = 10, 0
    # warm-up: W iterations, then one untimed call of the timed length, which
    # instantiates the iteration graphs that call uses (a problem keeps its
    # walk buffers and graphs between calls)
    w_run = G.tabu_run(args.warmup, tenure, seed)
    del w_run
    w_run = G.tabu_run(args.steps, tenure, seed)
    del w_run
    log(f"warmup {args.warmup} iterations (+ one untimed call of {args.steps}) done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run = G.tabu_run(args.steps, tenure, seed)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tr = run.trace
    moves = int(np.count_nonzero(tr["var"] >= 0))
    log(f"timed {args.steps} iterations: {wall:.3f} s wall, graphs {run.elapsed_ms:.1f} ms, {moves} moves, "
        f"violated rows {int(tr['viol'][0])} -> {int(tr['viol'][-1])}")

    # best-shift pass at the final point of the timed walk, HIP events on its stream
    xd = torch.from_numpy(run.x).cuda()
    wd = torch.from_numpy(run.w).cuda()
    cutoff = run.cutoff_rhs
    out_x = torch.empty_like(xd)
    out_s = torch.empty_like(xd)
    times, calls = [], []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(args.pass_reps + 3):
        ev0.record()
        G.best_shift(xd, wd, cutoff, out_x, out_s)
        ev1.record()
        times.append(G.last_pass_ms())
        ev1.synchronize()
        calls.append(ev0.elapsed_time(ev1))
    pass_ms = float(np.mean(times[3:]))
    call_ms = float(np.mean(calls[3:]))
    cut_active = math.isfinite(cutoff)
    B = algorithmic_bytes(mip, cut_active)
    nnz_pass = mip.nnz + (mip.nnz_obj if cut_active else 0)
    achieved = B / (pass_ms * 1e-3) / 1e9
    log(f"best-shift pass {pass_ms * 1e3:.1f} us (whole call {call_ms * 1e3:.1f} us), {B / 1e6:.1f} MB algorithmic, "
        f"{achieved:.0f} GB/s")

    # jump values at the same point: the second pass on the same primitives
    jump = jump_values_leg(G, mip, xd, wd, cutoff, args.pass_reps)

    if args.calibrate_copy_mb > 0:
        src = torch.ones(args.calibrate_copy_mb * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calibrate_copy_mb} MiB done")
        del src, dst

    value = args.steps / wall
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wname, "iters": args.steps, "tenure": tenure, "seed": seed,
                   "parallelism": "single GPU"},
        "applied_moves_per_s": moves / wall,
        "graph_ms_per_step": run.elapsed_ms / args.steps,
        "best_shift_pass_us": pass_ms * 1e3,
        "best_shift_call_us": call_ms * 1e3,
        "best_shift_nnz_per_s": nnz_pass / (pass_ms * 1e-3),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": PASS_TRAFFIC_BYTES if not args.small else None,
                     "kernel": "best-shift pass (k_stage_rows + k_stage_score + k_narrow_combine on the 20M "
                               "instance)",
                     "bytes_per_launch": B},
    }
    result["jump_values"] = jump
    if args.batched_only:
        result["batched"] = compare_batched(chap, args.batch_iters, tenure, args.small, plain=False)
    elif not args.no_compare:
        result["learned"] = compare_learned(chap, G, args.compare_iters, tenure, seed)
        del G
        if not args.no_batched:
            result["batched"] = compare_batched(chap, args.batch_iters, tenure, args.small)
        result["configs"] = small_configs(chap, tenure)
    if not args.no_cpu:
        log(f"cpu baseline: {args.cpu_iters} oracle iterations on one core, {args.cpu_iters_all} on all")
        result["cpu_baseline"] = cpu_baseline(mip, args.cpu_iters, args.cpu_iters_all)
    print(json.dumps(result), flush=True)


def jump_values_leg(G, mip, xd, wd, cutoff, reps):
    """chap_jump_values on the walk's final point: kernel time (HIP events),
    nonzeros per second, and the pass's algorithmic bytes (the data of the
    best-shift pass: every nonzero's index, value and row state, every
    column's bounds, point and results) against the HBM peak."""
    import torch

    times = []
    for _ in range(reps + 3):
        G.jump_values(xd, wd, cutoff)
        times.append(G.last_jump_ms())
    torch.cuda.synchronize()
    ms = float(np.mean(times[3:]))
    act = math.isfinite(cutoff)
    B = algorithmic_bytes(mip, act)
    nnz = mip.nnz + (mip.nnz_obj if act else 0)
    achieved = B / (ms * 1e-3) / 1e9
    out = {"pass_us": ms * 1e3, "nnz_per_s": nnz / (ms * 1e-3),
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "bytes_per_launch": B}}
    log(f"jump values {ms * 1e3:.1f} us, {achieved:.0f} GB/s algorithmic ({100 * achieved / HBM_PEAK_GBS:.1f} % "
        f"of 8 TB/s)")
    return out


def heuristic_params():
    """Parameters of a hand-set network that outputs input 3, the last exact
    score of the column per unit of its row weight (clamped to [-4, 4]), as
    relu(relu(x3)) - relu(relu(-x3)) (exact in bfloat16). Its top-K set is the
    K columns that scored best at the last full evaluation: the heuristic
    top-k baseline."""
    p = np.zeros(5313, dtype=np.float32)
    w1, b1, w2, b2, w3 = 0, 1024, 1088, 1088 + 4096, 1088 + 4096 + 64
    p[w1 + 0 * 16 + 3] = 1.0
    p[w1 + 1 * 16 + 3] = -1.0
    p[w2 + 0 * 64 + 0] = 1.0
    p[w2 + 1 * 64 + 1] = 1.0
    p[w3 + 0] = 1.0
    p[w3 + 1] = -1.0
    assert b1 == 1024 and b2 == 5184 and w3 + 64 == 5312
    return p


def compare_learned(chap, G, iters, tenure, seed):
    """The learned proposal against the plain walk on the same instance and
    start point: violation reduction per second at equal final score. The
    plain walk runs `iters` iterations; each proposal form runs until it
    reaches the plain walk's final violation count (at most 2 iters), and
    the time to get there is measured by a second run of exactly that many
    iterations. Forms: a network trained offline on pairs logged by a plain
    walk from another start point (seed + 7), the same network untrained,
    the heuristic top-k (hand-set network ranking by the last exact score),
    an untrained network trained online during the walk, and the trained and
    heuristic forms with a proposal set kept for 8 proposal iterations."""
    import torch

    chap.learned_run(G, chap.Model(0), 64, tenure, seed, full_every=64, topk=1024)   # warm-up
    G.tabu_run(iters, tenure, seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = G.tabu_run(iters, tenure, seed)
    torch.cuda.synchronize()
    pwall = time.perf_counter() - t0
    v0 = int(plain.trace["viol"][0])
    vp = int(plain.trace["viol"][-1])
    t0 = time.perf_counter()
    trained = chap.Model(0)
    logrun = chap.learned_run(G, trained, 100, tenure, seed + 7, full_every=1, topk=1024, train_pairs=1024,
                              log_pairs=100 * 2048)
    feat = torch.from_numpy(logrun.pair_feat.view(np.int16)).cuda()
    tgt = torch.from_numpy(logrun.pair_target).cuda()
    trained.train(feat, tgt, steps=1000, batch=1024, lr=1e-3, seed=1)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    heur = chap.Model(0)
    heur.set_params(heuristic_params())
    forms = [("trained", trained, {}), ("untrained", chap.Model(0), {}), ("heuristic_topk", heur, {}),
             ("online", chap.Model(0), dict(train_steps=4, train_pairs=512, lr=1e-3)),
             ("trained_refresh8", trained, dict(refresh_every=8)),
             ("heuristic_topk_refresh8", heur, dict(refresh_every=8))]
    out = {"instance": "the same 20M-nonzero instance and start point", "plain_iters": iters,
           "plain_seconds": pwall, "plain_ms_per_iter": pwall * 1e3 / iters, "plain_final_viol": vp,
           "options": dict(full_every=64, topk=1024),
           "training": f"offline: 1000 Adam steps (batch 1024, lr 1e-3) on {logrun.pair_target.shape[0]} pairs from "
                       f"100 full evaluations of a plain walk from seed {seed + 7}; {train_s:.1f} s, not timed; "
                       f"online: 4 Adam steps on 512 pairs at every full evaluation, timed"}
    for name, M, extra in forms:
        opts = dict(full_every=64, topk=1024, **extra)
        probe = chap.learned_run(G, M if name != "online" else chap.Model(0), 2 * iters, tenure, seed, **opts)
        viol = probe.trace["viol"]
        reach = np.flatnonzero(viol <= vp)
        rec = {"final_viol_at_2x": int(viol[-1]), "judge_hits": probe.hits, "judge_evals": probe.evals,
               "stalls": probe.stalls}
        if reach.size:
            it = int(reach[0]) + 1
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            again = chap.learned_run(G, M if name != "online" else chap.Model(0), it, tenure, seed, **opts)
            torch.cuda.synchronize()
            treach = time.perf_counter() - t0
            assert int(again.trace["viol"][-1]) <= vp
            rec.update({"iters_to_plain_final": it, "seconds_to_plain_final": treach,
                        "ms_per_iter": treach * 1e3 / it,
                        "violation_reduction_per_s": (v0 - vp) / treach,
                        "speedup_at_equal_final_score": pwall / treach})
        else:
            rec.update({"iters_to_plain_final": None, "speedup_at_equal_final_score": None})
        out[name] = rec
        log(f"learned {name}: reaches plain final at {rec['iters_to_plain_final']}, "
            f"speedup {rec['speedup_at_equal_final_score']}")
    out["plain_violation_reduction_per_s"] = (v0 - vp) / pwall
    return out


def small_configs(chap, tenure):
    """Configurations 1 and 2: iterations per second of the walk and the
    best-shift pass time (HIP events), with nonzeros per second; and the same
    walks with affected rescoring."""
    import torch

    import mipgen

    out = {}
    for name, mip, iters in (("tiny_binary n=200 m=100 (1000 iterations)", mipgen.tiny_binary(0), 1000),
                             ("general n=100k m=50k (10000 iterations)", mipgen.general(0), 10000)):
        G = chap.Problem(mip)
        G.tabu_run(iters, tenure, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run = G.tabu_run(iters, tenure, 0)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        xd = torch.from_numpy(run.x).cuda()
        wd = torch.from_numpy(run.w).cuda()
        ox, os_ = torch.empty_like(xd), torch.empty_like(xd)
        times = []
        for _ in range(23):
            G.best_shift(xd, wd, run.cutoff_rhs, ox, os_)
            times.append(G.last_pass_ms())
        pass_ms = float(np.mean(times[3:]))
        nnz = mip.nnz + (mip.nnz_obj if math.isfinite(run.cutoff_rhs) else 0)
        out[name] = {"iters_per_s": iters / wall, "ms_per_iter": wall * 1e3 / iters,
                     "graph_ms_per_iter": run.elapsed_ms / iters, "best_shift_pass_us": pass_ms * 1e3,
                     "best_shift_nnz_per_s": nnz / (pass_ms * 1e-3),
                     "final_viol": int(run.trace["viol"][-1]), "best_obj": run.best_obj}
        log(f"{name}: {iters / wall:.0f} it/s, pass {pass_ms * 1e3:.1f} us")
        # affected rescoring: the same walk, scoring after each plain move only
        # the columns that share a row with the moved column
        R = chap.Problem(mip, rescore_cap=1024)
        R.tabu_run(iters, tenure, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rr = R.tabu_run(iters, tenure, 0)
        torch.cuda.synchronize()
        rwall = time.perf_counter() - t0
        out[name]["affected_rescoring"] = {
            "rescore_cap": 1024, "iters_per_s": iters / rwall, "ms_per_iter": rwall * 1e3 / iters,
            "graph_ms_per_iter": rr.elapsed_ms / iters, "rescored_iters": int(rr.rescored),
            "identical_trajectory": bool(np.array_equal(rr.trace, run.trace)),
            "speedup": (iters / rwall) / (iters / wall)}
        log(f"{name} affected rescoring: {iters / rwall:.0f} it/s ({rr.rescored} of {iters} iterations rescored "
            f"the affected columns only), identical={out[name]['affected_rescoring']['identical_trajectory']}")
        del G, R
    return out


def compare_batched(chap, iters, tenure, small, plain=True):
    """256 walks over the pool of general instances (walk w on instance
    w mod P, start seed w + 1) as one batch, against the same walks run one by
    one (plain=False: the batch alone). Both give identical trajectories (same
    final score); the ratio of GPU times is the speedup at equal final score."""
    import torch

    import mipgen

    t0 = time.perf_counter()
    pool = mipgen.batch_pool(total_nnz=2_000_000 if small else 20_000_000)
    probs = [chap.Problem(m) for m in pool]
    # per-instance plan chosen by chap_autotune (short-column threshold; the
    # pool's columns are short and general, so the long-column knobs do not
    # apply), timed on a 32-iteration walk of each instance
    t1 = time.perf_counter()
    chosen = {}
    for i, m in enumerate(pool):
        best, _ = chap.autotune(probs[i], candidates=[{"short_max": 4}, {"short_max": 8}], walk_iters=32)
        chosen[int(best.short_max)] = chosen.get(int(best.short_max), 0) + 1
        if best.short_max != 8:
            probs[i] = chap.Problem(m, short_max=int(best.short_max))
    tune = {"candidates": [{"short_max": 4}, {"short_max": 8}], "chosen_short_max": chosen,
            "seconds": time.perf_counter() - t1}
    log(f"autotune over the pool: {chosen} in {tune['seconds']:.1f} s")
    nw = 256
    wp = np.arange(nw) % len(pool)
    ws = np.arange(nw) + 1
    log(f"batch pool: {len(pool)} instances, {sum(m.nnz for m in pool)} nonzeros, set up in "
        f"{time.perf_counter() - t0:.1f} s")
    chap.batch_run(probs, wp, ws, 4, tenure)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = chap.batch_run(probs, wp, ws, iters, tenure)
    bwall = time.perf_counter() - t0
    bms = runs[0].elapsed_ms
    # algorithmic bytes of one batched iteration: every walk's pass (cutoff
    # rows counted where a walk's cutoff is active at its end)
    bpi = sum(algorithmic_bytes(pool[wp[w]], math.isfinite(runs[w].cutoff_rhs)) for w in range(nw))
    roof = {"bytes_per_batched_iter": int(bpi), "achieved_GBps": bpi * iters / (bms * 1e-3) / 1e9,
            "peak_GBps": 8000.0}
    roof["frac"] = roof["achieved_GBps"] / roof["peak_GBps"]
    log(f"batched roofline: {bpi / 1e6:.1f} MB per batched iteration, {roof['achieved_GBps']:.0f} GB/s "
        f"({100 * roof['frac']:.1f} % of 8 TB/s, graph time including walk set-up)")
    # diversity-driven restarts: the same batch in segments of 50 iterations,
    # restarting walks that come within 64 discrete variables of another walk
    # on the same instance
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rruns = chap.batch_restarts(probs, wp, ws, iters, tenure, 50, 64)
    rwall = time.perf_counter() - t0
    restarts = {"restart_every": 50, "min_distance": 64, "restarts": int(sum(len(r.restarts) for r in rruns)),
                "gpu_ms": rruns[0].elapsed_ms, "wall_s": rwall, "batched_wall_s": bwall,
                "wall_overhead_vs_batched": rwall / bwall}
    log(f"batched with restarts: {rruns[0].elapsed_ms:.1f} ms GPU, {rwall:.3f} s wall vs {bwall:.3f} s, "
        f"{restarts['restarts']} restarts")
    if not plain:
        log(f"batched: {bms:.1f} ms (GPU graphs), {bms / iters:.3f} ms per batched iteration")
        return {"walks": nw, "instances": len(pool), "pool_nnz": int(sum(m.nnz for m in pool)), "iters": iters,
                "batched_gpu_ms": bms, "batched_wall_s": bwall, "roofline": roof, "restarts": restarts, "autotune": tune,
                "walk_iters_per_s": {"batched": nw * iters / (bms * 1e-3)}}
    pms = 0.0
    pwall = 0.0
    same = True
    for w in range(nw):
        t0 = time.perf_counter()
        r = probs[wp[w]].tabu_run(iters, tenure, int(ws[w]))
        pwall += time.perf_counter() - t0
        pms += r.elapsed_ms
        same = same and np.array_equal(r.trace, runs[w].trace)
    out = {"walks": nw, "instances": len(pool), "pool_nnz": int(sum(m.nnz for m in pool)), "iters": iters,
           "batched_gpu_ms": bms, "plain_gpu_ms_sum": pms, "batched_wall_s": bwall, "plain_wall_s": pwall,
           "identical_trajectories": bool(same), "speedup_at_equal_final_score": pms / bms, "roofline": roof,
           "restarts": restarts, "autotune": tune,
           "walk_iters_per_s": {"batched": nw * iters / (bms * 1e-3), "plain": nw * iters / (pms * 1e-3)}}
    log(f"batched: {bms:.1f} ms vs plain {pms:.1f} ms (GPU graphs), identical={same}")
    return out


if __name__ == "__main__":
    main()
