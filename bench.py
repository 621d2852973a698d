"""Benchmark: one step = one whole pass of the hot path over the dense workload.

Workload: 1 scene x 1024 goals, 50 obstacles, 6 lanes, T = 100 samples over
10 s, 100 iterations of Algorithm 1 per goal (cold start), then meta-cost
scoring and argmin. Operator setup (the FP64 KKT inverses) is done once before
the timed region: it depends only on (T, m), not on the batch.

Prints ONE JSON line. `value` is goal-trajectories x iterations per second on
this GPU with inputs resident in HBM. `roofline` is for the dominant kernel
(the fused AM kernel), from its average duration measured with HIP events on
the stream it is launched on; `cpu_baseline` is the FP64 oracle on the host's
cores (all of them, one process per core, and one core alone) over a bounded
sample of the same workload, with the CPU model and core count.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_COEF = 11
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector peak (AMD datasheet; needs packed FP32 instructions)
PEAK_FP32_UNPACKED_TFLOPS = 78.65  # the same without packed FP32, which this library is built without

# HBM bytes per launch of the dominant kernel of each workload, from rocprofv3
# FETCH_SIZE / WRITE_SIZE, scaled by the same counters over a plain 256 MiB copy
# (fetch x2.00, write x1.00); see profiles/. Valid only for the kernel sources
# they were taken on: when the hash of those sources differs, traffic is null.
MEASURED_TRAFFIC = {
    "dense": {"sources": ("paper_2109_10392_amd/csrc/traj_solve.hip", "paper_2109_10392_amd/csrc/traj_internal.h",
                          "paper_2109_10392_amd/csrc/traj_device.h"),
              "sha256": "4193d025e3eed1e9ea8ab120a2ce1e179ab1460202e762810672a87d4e0b88d8",
              "bytes_per_launch": int((242.5 * 2.0 + 284.0) * 1024),
              "profile": "profiles/k_am_wave2_dense1024.md"},
    "uneven": {"sources": ("paper_2109_10392_amd/csrc/traj_group.hip", "paper_2109_10392_amd/csrc/traj_internal.h",
                           "paper_2109_10392_amd/csrc/traj_device.h", "paper_2109_10392_amd/csrc/traj_mma.h"),
               "sha256": "7d1f120b983d3441d256ca93687cd90bde63e82e8b929b6aa8b81407ef833698",
               "bytes_per_launch": int((87925.4 * 2.0 + 277450.9) * 1024),
               "profile": "profiles/k_am_group_uneven512.md"},
}


def sources_hash(files):
    import hashlib
    h = hashlib.sha256()
    for rel in files:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, kernel, waves, precision):
    """Bytes per launch if the profiled kernel (FP32 form) and sources are what runs, else None."""
    m = MEASURED_TRAFFIC.get(workload)
    expected = {"dense": ("wave", 2), "uneven": ("group", None)}[workload]
    if m is None or precision != "fp32" or kernel != expected[0] or (expected[1] is not None and waves != expected[1]):
        return None
    return m["bytes_per_launch"] if sources_hash(m["sources"]) == m["sha256"] else None


def algorithmic_flops_per_goal_iter(n, m, N=N_COEF):
    """Algorithmic FP32 work of one AM iteration of one goal (FMA = 2).

    contractions 28 N n (basis evaluation 12 N n, x/y transposed contraction
    12 N n, heading 4 N n) + 11x11 applies 16 N^2 + element-wise 30 n +
    obstacle test 8 m n.
    """
    return 28 * N * n + 16 * N * N + 30 * n + 8 * m * n


def _oracle_chunk(args):
    """One worker of the CPU baseline: the FP64 oracle on goals [lo, hi) of the
    dense scene of `seed`, one BLAS thread, with every goal's final lateral
    position moved by `shift` metres; returns the seconds of the solve and the
    coefficients [3][11][hi - lo]."""
    seed, lo, hi, iters = args[:4]
    shift = args[4] if len(args) > 4 else 0.0
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import traj_oracle as O
    from paper_2109_10392_amd import scenes as S
    sc = S.workload_dense(seed).scenes[0]
    goals = sc.goals[lo:hi].astype(np.float64)
    goals[:, 1] += shift
    with threadpool_limits(1):
        prob = O.Problem(sc.n_time, sc.t_f, sc.obs.shape[0], S.DEFAULT_PARAMS)
        t0 = time.perf_counter()
        st = O.solve(prob, sc.ego, sc.obs, goals, iters)
        return time.perf_counter() - t0, np.stack([st.c_x, st.c_y, st.c_psi])


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(seed, iters, one_core_goals, max_workers=16):
    """The FP64 oracle (explicit F, NumPy/SciPy) on the host: one core on
    `one_core_goals` goals of the dense scene, then every goal of the scene split
    over one process per usable core (at most max_workers), one BLAS thread each.
    Runs before the GPU is initialised (the worker processes are started fresh)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    workers = max(1, min(cores, max_workers))
    n_goals = 1024
    dt1 = _oracle_chunk((seed, 0, one_core_goals, iters))[0]
    chunks = [(seed, n_goals * w // workers, n_goals * (w + 1) // workers, iters) for w in range(workers)]
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        list(ex.map(_oracle_chunk, [(seed, 0, 1, 1)] * workers))  # start every worker and import first
        t0 = time.perf_counter()
        parts = list(ex.map(_oracle_chunk, chunks))
        dtn = time.perf_counter() - t0
        # the same goals moved by 1e-6 m (below FP32's resolution of the inputs): where
        # that moves the FP64 result by more than 2e-6 the goal sits at a bifurcation
        shifted = list(ex.map(_oracle_chunk, [ch + (1e-6,) for ch in chunks]))
    import numpy as np

    from oracle import traj_oracle as O
    from paper_2109_10392_amd import scenes as S
    c = np.concatenate([p[1] for p in parts], axis=2)
    c_shift = np.concatenate([p[1] for p in shifted], axis=2)
    bifurcating = _rel_coef_err(c_shift, c) > 2e-6
    sc = S.workload_dense(seed).scenes[0]
    prob = O.Problem(sc.n_time, sc.t_f, sc.obs.shape[0], S.DEFAULT_PARAMS)
    best = O.best_goal(O.meta_cost(prob, c[0], c[1], c[2], v_ref=float(sc.ego[2])))
    model = cpu_model()
    return {"value": n_goals * iters / dtn, "unit": "goal-trajectories*iters/s", "cores": workers, "kind": "oracle",
            "sample": f"all {n_goals} goals of the dense scene (seed {seed}), {iters} iterations, FP64 NumPy/SciPy "
                      f"oracle, {workers} processes x 1 BLAS thread, {dtn:.1f} s wall on {model} "
                      f"({cores} usable cores, {os.cpu_count()} logical CPUs)",
            "cpu_model": model, "host_cores": cores,
            "single_core": {"value": one_core_goals * iters / dt1, "cores": 1,
                            "sample": f"{one_core_goals} of the 1024 goals, {iters} iterations, 1 BLAS thread, "
                                      f"{dt1:.1f} s"},
            "_oracle_c": c, "_oracle_best": best, "_bifurcating": bifurcating}


def _rel_coef_err(c, c_ref):
    """Per goal, the largest relative coefficient difference over the three axes:
    max |c - c_ref| / max(max |c_ref|, 1) per axis ([3][11][B] arrays)."""
    import numpy as np
    num = np.abs(np.asarray(c, np.float64) - c_ref).max(axis=1)
    den = np.maximum(np.abs(c_ref).max(axis=1), 1.0)
    return (num / den).max(axis=0)


def parity_vs_oracle(c_gpu, c_ref, bifurcating, best_gpu, best_ref):
    """The timed solve's result against the oracle's on the same scene and
    iteration count: the distribution over the goals of _rel_coef_err, over all
    goals and over those whose FP64 result is determined (not moved past 2e-6 by a
    1e-6 m goal shift; at a bifurcation FP32 and FP64 may take different
    branches, each correct), and both best goals."""
    import numpy as np
    err = _rel_coef_err(c_gpu, c_ref)
    det = err[~bifurcating]
    q = lambda e, p: float(f"{np.percentile(e, p):.3g}") if e.size else None
    return {"goals": int(err.size), "rel_coef_err_median": q(err, 50), "p90": q(err, 90), "max": q(err, 100),
            "within_1e-4": int(np.count_nonzero(err <= 1e-4)), "within_1e-3": int(np.count_nonzero(err <= 1e-3)),
            "determined_goals": int(det.size), "determined_max": q(det, 100),
            "determined_within_1e-4": int(np.count_nonzero(det <= 1e-4)),
            "determined_within_1e-3": int(np.count_nonzero(det <= 1e-3)),
            "best_goal_gpu": int(best_gpu), "best_goal_oracle": int(best_ref)}


def uneven_extras(T, S, solver, batch, db, st, v_ref, cost, best, args, kernel, group, persistent, one_launch_ms,
                  waves=1):
    """The uneven batch as one hipGraph replay and as one launch per scene.

    graph: the whole step (work list, persistent solve, scoring) captured once and
    replayed; separate: the same kernels and tile, each scene solved and scored by
    its own calls (its own one-scene batch and state), back to back on one stream.
    """
    import torch

    def step():
        solver.solve(db, st, args.iters, precision=args.precision)
        solver.score(db, st, v_ref, cost, best)

    step()
    torch.cuda.synchronize()
    ref_c = st.c.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    g.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.steps):
        g.replay()
    b.record()
    torch.cuda.synchronize()
    graph_ms = a.elapsed_time(b) / args.steps
    graph_equal = bool(torch.equal(st.c, ref_c))

    # the single tile: every shape at the tile's group size (the per-bucket sizes off)
    groups = solver.get_shape_groups()
    single_ms, single_equal = None, None
    if kernel == "group" and any(groups):
        solver.set_shape_groups(None)
        step()
        torch.cuda.synchronize()
        a.record()
        for _ in range(args.steps):
            step()
        b.record()
        torch.cuda.synchronize()
        single_ms = a.elapsed_time(b) / args.steps
        single_equal = bool(torch.equal(st.c, ref_c))
        solver.set_shape_groups(groups)

    # one launch per scene: per-scene batches and states (goal-fastest layouts do
    # not allow views of one scene inside the batch state)
    parts = []
    for sc in batch.scenes:
        one = S.Batch([sc])
        dbs = T.DeviceBatch.from_batch(one, shapes=batch.shapes())
        sts = T.DeviceState.empty(one.n_goals)
        vr = torch.tensor([float(sc.ego[2])], device="cuda")
        parts.append((dbs, sts, vr, torch.zeros(one.n_goals, device="cuda"),
                      torch.zeros(1, device="cuda", dtype=torch.int32)))

    def separate():
        for dbs, sts, vr, cs, bs in parts:
            solver.solve(dbs, sts, args.iters, precision=args.precision)
            solver.score(dbs, sts, vr, cs, bs)

    separate()
    torch.cuda.synchronize()
    reps = max(1, min(args.steps, 3))
    a.record()
    for _ in range(reps):
        separate()
    b.record()
    torch.cuda.synchronize()
    sep_ms = a.elapsed_time(b) / reps
    off = batch.goal_off()
    sep_equal = all(torch.equal(p[1].c, ref_c[:, :, off[i]:off[i + 1]]) for i, p in enumerate(parts))
    return {"one_launch_ms": one_launch_ms, "graph_replay_ms": graph_ms, "separate_launches_ms": sep_ms,
            "speedup_vs_separate": sep_ms / graph_ms, "graph_equals_eager": graph_equal,
            "separate_equals_batched": bool(sep_equal), "tile": [kernel, group, persistent, waves],
            "single_tile_step_ms": single_ms,
            "gain_over_single_tile": None if single_ms is None else single_ms / one_launch_ms,
            "single_tile_equals": single_equal}


def residual_curve(seeds=range(100), chunk=5, total=300, tol=1e-3):
    """Residuals over the iterations (the quantity of Fig. 3a) at the paper's scene
    scale, batched: the 11-goal scenes of `seeds` (10 obstacles, 4 lanes, T = 100)
    in one batch, a cold FP32 solve resumed chunk by chunk (bitwise the continuous
    solve) and scored after every chunk. Per chunk: the median over the scenes of
    max(r_obs, r_acc, r_nh) of each scene's meta-cost-best goal (eq. 25), and the
    share of scenes where it is at or below `tol`. Runs after the timed region."""
    import numpy as np
    import torch
    from paper_2109_10392_amd import scenes as S
    from paper_2109_10392_amd import traj as T
    batch = S.Batch([S.workload_small(s).scenes[0] for s in seeds])
    solver = T.Solver(S.DEFAULT_PARAMS, batch.shapes())
    solver.set_tile("wave", 16, True, 2)
    db = T.DeviceBatch.from_batch(batch)
    st = T.DeviceState.empty(batch.n_goals)
    v_ref = torch.tensor([float(s.ego[2]) for s in batch.scenes], device="cuda")
    cost = torch.zeros(batch.n_goals, device="cuda")
    best = torch.zeros(batch.n_scenes, device="cuda", dtype=torch.int32)
    first = torch.as_tensor(np.asarray(batch.goal_off()[:-1], np.int64), device="cuda")
    med, share = [], []
    for k in range(total // chunk):
        solver.solve(db, st, chunk, from_state=k > 0)
        solver.score(db, st, v_ref, cost, best)
        r = st.resid[:3].amax(0)
        rb = torch.where(best >= 0, r[first + best.clamp(min=0).long()], torch.full_like(r[:1], float("inf")))
        med.append(rb.median())
        share.append((rb <= tol).float().mean())
    torch.cuda.synchronize()
    solver.close()
    return {"scenes": f"the 11-goal scenes of seeds {seeds[0]}-{seeds[-1]} in one batch ({batch.n_scenes} scenes, "
                      f"{batch.n_goals} goals), cold start, FP32",
            "iterations": list(range(chunk, total + 1, chunk)),
            "best_goal_max_residual_median": [float(f"{x:.3g}") for x in torch.stack(med).tolist()],
            "share_at_or_below_1e-3": [round(x, 3) for x in torch.stack(share).tolist()]}


def run_warmstart(args):
    """Learned warm start: train on solved template scenes, then time cold FP32 and
    warm + split-BF16 solves of held-out scenes to residual 1e-3 (ms per scene)."""
    import torch

    from paper_2109_10392_amd import warmstart as W
    torch.cuda.set_device(0)
    prob = W.Problem()
    train_seeds = range(1000, 1000 + args.train_scenes)
    net, mean, std, info = W.fit(prob, train_seeds, epochs=args.epochs, lr=2e-3, log=None)
    res = W.evaluate(prob, net, mean, std, list(range(args.test_scenes)), restart_at=args.restart_at or None)
    return {
        "metric": "ms/scene to residual 1e-3 (warm+mixed vs cold FP32)",
        "value": res["warm"]["ms_per_scene"],
        "unit": "ms/scene",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": res["warm"]["ms_per_scene"] * args.test_scenes,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3",
        "data": "synthetic",
        "config": {"workload": f"learned warm start: template scenes (4 lanes x 64 goal slots, 10 obstacles, T=100 "
                               f"over 10 s), network trained on {args.train_scenes} solved scenes, "
                               f"{args.test_scenes} held-out scenes; stop when the best goal's max(r_obs, r_acc, "
                               f"r_nh) <= 1e-3 (checked every 5 iterations, at most 300)",
                   "train_scenes": args.train_scenes, "test_scenes": args.test_scenes, "epochs": args.epochs},
        "cold_fp32": res["cold"], "warm_fp32": res["warm_fp32"], "warm_mixed": res["warm"],
        "iters_ratio": res["iters_ratio"], "ms_ratio": res["ms_ratio"], "training": info,
        "converged_only_cold": res.get("converged_only_cold"), "converged_only_warm": res.get("converged_only_warm"),
        "common": res.get("common"), "restart_at": args.restart_at,
    }


def warm_leg(train_scenes, test_scenes, epochs, restart_at):
    """The metric's second half at reduced size: a network trained on the solved
    template scenes `1000 .. 1000 + train_scenes`, then cold FP32 and warm + mixed
    precision (split-BF16 solver, cold fallback) on `test_scenes` held-out scenes to
    the stopping rule (best goal at max(r_obs, r_acc, r_nh) <= 1e-3, at most 300
    iterations): ms per scene, converged share, and both timed again on only the
    scenes both forms bring to 1e-3."""
    from paper_2109_10392_amd import warmstart as W
    prob = W.Problem()
    net, mean, std, info = W.fit(prob, range(1000, 1000 + train_scenes), epochs=epochs, lr=2e-3, log=None)
    res = W.evaluate(prob, net, mean, std, list(range(test_scenes)), restart_at=restart_at,
                     modes=("cold", "warm"))
    out = {"metric": "ms/scene to residual 1e-3 (warm+mixed vs cold FP32)", "unit": "ms/scene",
           "higher_is_better": False,
           "sample": f"template scenes (4 lanes x 64 goal slots, 10 obstacles, T=100 over 10 s); network trained "
                     f"on the converged scenes among {train_scenes} solved ones ({epochs} epochs), "
                     f"{test_scenes} held-out scenes; warm: split-BF16 solver, cold start as fallback per goal"
                     + (f", unconverged scenes restarted cold after {restart_at} iterations" if restart_at else ""),
           "cold_fp32": res["cold"], "warm_mixed": res["warm"], "ms_ratio": res["ms_ratio"],
           "iters_ratio": res["iters_ratio"], "converged_cold": res["cold"]["converged"],
           "converged_warm": res["warm"]["converged"], "converged_only_cold": res.get("converged_only_cold"),
           "converged_only_warm": res.get("converged_only_warm"), "common": res.get("common"),
           "training": info}
    prob.solver.close()
    return out


def run_mpc(args):
    """Closed loop: E episodes (4 lanes, 10 IDM vehicles each) replanned every cycle
    (goal template, solve to residual 1e-3 with at most --iters iterations, scoring,
    IDM traffic step); timed over --steps cycles after --warmup cycles."""
    import torch

    from paper_2109_10392_amd import mpc
    torch.cuda.set_device(0)
    cl = mpc.ClosedLoop(range(args.episodes), iters=args.iters, warm=args.warm, clear_min=args.clear_min,
                        scenario=args.scenario, precision=args.precision)
    for _ in range(args.warmup):
        cl.cycle()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.steps):
        cl.cycle()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.steps
    m = cl.metrics(args.warmup + args.steps)
    return {
        "metric": "closed-loop episode-cycles/s", "value": args.episodes / (ms / 1e3), "unit": "episode-cycles/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else "bf16x3",
        "data": "synthetic",
        "config": {"workload": f"closed loop: {args.episodes} episodes, 4 lanes, 10 IDM vehicles each, 256 goals "
                               f"per plan, replanning every sample interval (0.101 s), at most {args.iters} "
                               f"iterations per plan (stop at residual 1e-3), start: {args.warm}, "
                               f"collision post-check at {args.clear_min}, scenario: {args.scenario}, "
                               f"precision: {args.precision}",
                   "episodes": args.episodes, "warm": args.warm, "clear_min": args.clear_min,
                   "precision": args.precision,
                   "scenario": args.scenario},
        "closed_loop": m,
    }


def run_plan(args):
    """One plan at the paper's scale (latency-bound): the 11-goal scene (10
    obstacles, 4 lanes, T = 100) of each seed 0 .. --steps-1, solved alone:
    (a) --iters iterations and scoring, (b) the chunked solve to the stopping
    rule (best goal at max(r_obs, r_acc, r_nh) <= 1e-3, chunks of 5, at most 300
    iterations). Each plan is timed on its own with HIP events after --warmup
    untimed plans of seed 0; the wave kernel with two waves per goal."""
    import numpy as np
    import torch

    from paper_2109_10392_amd import scenes as S
    from paper_2109_10392_amd import traj as T
    torch.cuda.set_device(0)
    seeds = list(range(args.steps))
    batches = [S.workload_small(s) for s in seeds]
    solver = T.Solver(S.DEFAULT_PARAMS, batches[0].shapes())
    solver.set_tile("wave", 16, True, 2)
    dbs = [T.DeviceBatch.from_batch(b) for b in batches]
    st = T.DeviceState.empty(batches[0].n_goals)        # plain solves (no skip mask)
    st_rule = T.DeviceState.empty(batches[0].n_goals)   # chunked solves (their own scene_done)
    cost = torch.zeros(batches[0].n_goals, device="cuda")
    best = torch.zeros(1, device="cuda", dtype=torch.int32)
    its = torch.zeros(1, device="cuda", dtype=torch.int32)
    v_refs = [torch.tensor([float(b.scenes[0].ego[2])], device="cuda") for b in batches]

    def plan(k):
        solver.solve(dbs[k], st, args.iters)
        solver.score(dbs[k], st, v_refs[k], cost, best)

    def to_rule(k):
        solver.converge(dbs[k], st_rule, v_refs[k], cost, best, its, max_iters=300, chunk=5, tol=1e-3)

    def timed(fn, k):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn(k)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    for _ in range(args.warmup):
        plan(0)
        to_rule(0)
    torch.cuda.synchronize()
    ms_plan = [timed(plan, k) for k in range(len(seeds))]
    ms_rule, it_rule, conv = [], [], []
    for k in range(len(seeds)):
        ms_rule.append(timed(to_rule, k))
        it_rule.append(int(its[0].item()))
        conv.append(bool(st_rule.scene_done[0].item()))
    solver.close()
    med = float(np.median(ms_plan))
    conv_ms = [m for m, c in zip(ms_rule, conv) if c]
    return {
        "metric": "ms per plan (11 goals, 100 iterations + scoring)", "value": med, "unit": "ms",
        "n_gpus": 1, "steps": len(seeds), "warmup": args.warmup, "ms_per_step": med, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"one plan at a time: the 11-goal scene (10 obstacles, 4 lanes, T=100 over 10 s) of "
                               f"seeds 0-{len(seeds) - 1}, {args.iters} iterations + scoring; then the chunked "
                               f"solve to residual 1e-3 (chunks of 5, at most 300 iterations)",
                   "seeds": len(seeds), "iters": args.iters, "kernel": "wave", "waves": 2},
        "plan_ms_p10_median_p90": [float(np.percentile(ms_plan, 10)), med, float(np.percentile(ms_plan, 90))],
        "to_rule": {"converged": sum(conv), "of": len(seeds),
                    "ms_median_converged": float(np.median(conv_ms)) if conv_ms else None,
                    "iterations_median_converged": (float(np.median([i for i, c in zip(it_rule, conv) if c]))
                                                    if conv_ms else None),
                    "ms_median_all": float(np.median(ms_rule))},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the runs after the timed region (profiling): dense: the residual curve; "
                         "uneven: the graph-replay and separate-launch comparisons")
    ap.add_argument("--cpu-goals", type=int, default=320,
                    help="goals of the one-core CPU oracle sample (about 8 s; the all-core leg solves all 1024)")
    ap.add_argument("--kernel", choices=["auto", "wave", "mfma", "group"], default="auto",
                    help="auto: the tile chosen by the autotuner for this workload (tuning.json), else wave")
    ap.add_argument("--precision", choices=["fp32", "bf16x3"], default="fp32")
    ap.add_argument("--group", type=int, default=None, help="goals per matrix-core workgroup")
    ap.add_argument("--waves", type=int, default=None, choices=[1, 2], help="wave kernel: wavefronts per goal")
    ap.add_argument("--workload", choices=["dense", "uneven", "warmstart", "mpc", "plan"], default="dense",
                    help="plan: one 11-goal scene at a time (latency; --steps seeds)")
    ap.add_argument("--episodes", type=int, default=1024, help="mpc: episodes run together")
    ap.add_argument("--warm", choices=["cold", "previous", "shifted"], default="shifted",
                    help="mpc: start of every plan after the first (the previous cycle's solutions advanced by "
                         "one period, the same unshifted, or the cold start)")
    ap.add_argument("--scenario", choices=["cruise", "right_lane"], default="cruise",
                    help="mpc: cruise (template goals, eq. 25) or high speed near the right lane (eq. 26)")
    ap.add_argument("--clear-min", type=float, default=1.0,
                    help="mpc: collision post-check of the ranking (scaled obstacle distance; 0 = off)")
    ap.add_argument("--no-warm", action="store_true", help="dense: skip the reduced warm-start leg")
    ap.add_argument("--obstacle-range", type=float, default=80.0,
                    help="dense: obstacles placed over [0, L] m (80: the benchmark; 266.7: the 11-goal scenes' "
                         "density, the sensitivity variant)")
    ap.add_argument("--warm-train", type=int, default=20000, help="dense: training scenes of the warm-start leg")
    ap.add_argument("--warm-test", type=int, default=2048, help="dense: held-out scenes of the warm-start leg")
    ap.add_argument("--warm-epochs", type=int, default=30, help="dense: training epochs of the warm-start leg")
    ap.add_argument("--restart-at", type=int, default=10,
                    help="warm start: restart the scenes still unconverged after this many iterations from the cold "
                         "start (within the same 300-iteration budget; 0 = never)")
    ap.add_argument("--train-scenes", type=int, default=100000, help="warmstart: solved scenes to train on")
    ap.add_argument("--test-scenes", type=int, default=10000, help="warmstart: held-out scenes timed")
    ap.add_argument("--epochs", type=int, default=30, help="warmstart: training epochs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "goals are independent, so a multi-GPU run would shard scenes with no exchange inside the loop.",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "warmstart":
        print(json.dumps(run_warmstart(args)), flush=True)
        return
    if args.workload == "mpc":
        print(json.dumps(run_mpc(args)), flush=True)
        return
    if args.workload == "plan":
        print(json.dumps(run_plan(args)), flush=True)
        return

    # the CPU oracle first, before anything initialises the GPU (its workers are new processes)
    cpu = cpu_baseline(args.seed, args.iters, args.cpu_goals) if not args.no_cpu and args.workload == "dense" else None

    import numpy as np
    import torch

    from paper_2109_10392_amd import scenes as S
    from paper_2109_10392_amd import traj as T

    torch.cuda.set_device(0)
    x_range = (0.0, args.obstacle_range)
    batch = S.workload_dense(args.seed, x_range) if args.workload == "dense" else S.workload_uneven(args.seed)
    sc = batch.scenes[0]
    n, m, B = sc.n_time, sc.obs.shape[0], batch.n_goals
    solver = T.Solver(S.DEFAULT_PARAMS, batch.shapes())
    kernel = args.kernel
    persistent, waves = True, 1
    if kernel == "auto":
        from paper_2109_10392_amd import autotune
        tile = autotune.lookup(args.workload, args.precision)
        kernel, group, persistent, waves = (tile if tile is not None else ("wave", 16, True, 1))
    else:
        group = 16
    if args.group is not None:
        group = args.group
    if args.waves is not None:
        waves = args.waves
    if args.precision == "bf16x3" and kernel == "wave":
        kernel = "mfma"
    solver.set_tile(kernel, group, persistent, waves)
    buckets = None
    if args.kernel == "auto" and kernel == "group" and args.group is None:
        # the group kernel's per-(T, m) bucket group sizes, where the autotuner stored any
        from paper_2109_10392_amd import autotune
        buckets = autotune.lookup_buckets(args.workload, args.precision)
        if buckets:
            solver.set_shape_groups(autotune.shape_groups(batch.shapes(), buckets))
    db = T.DeviceBatch.from_batch(batch)
    st = T.DeviceState.empty(B)
    v_ref = torch.tensor([float(s.ego[2]) for s in batch.scenes], device="cuda")
    cost = torch.zeros(B, device="cuda")
    best = torch.zeros(batch.n_scenes, device="cuda", dtype=torch.int32)

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        solver.solve(db, st, args.iters, precision=args.precision)
        if ev is not None:
            ev[1].record()
        solver.score(db, st, v_ref, cost, best)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record()
    for k in range(args.steps):
        step(evs[k])
    t_end.record()
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    solve_ms = [a.elapsed_time(b) for a, b in evs]
    ms_per_step = total_ms / args.steps
    value = B * args.iters * args.steps / (total_ms / 1e3)
    solve_avg_s = sum(solve_ms) / len(solve_ms) / 1e3
    flops = sum(algorithmic_flops_per_goal_iter(s.n_time, s.obs.shape[0]) * s.goals.shape[0]
                for s in batch.scenes) * args.iters
    achieved = flops / solve_avg_s / 1e12
    # the same count without the 8 m n obstacle tests, which exact culling skips for
    # most pairs: a lower bound of the arithmetic the kernel really executes
    flops_no_obs = sum(algorithmic_flops_per_goal_iter(s.n_time, 0) * s.goals.shape[0]
                       for s in batch.scenes) * args.iters
    out = {
        "metric": "goal-trajectories*iters/s",
        "value": value,
        "unit": "goal-trajectories*iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # FP32 arithmetic with the 11x11 x/y applies in FP64; the split-BF16 form's
        # evaluations and contractions in BF16 (hi + lo) on the matrix cores
        "dtype": "f32+f64" if args.precision == "fp32" else "bf16x3+f32+f64",
        "data": "synthetic",
        "config": ({"workload": "dense highway scene: 1 scene x 1024 goals, 50 obstacles, 6 lanes, "
                                "T=100 over 10 s, Bernstein-10 basis, 100 AM iterations (cold start) + scoring"
                                + ("" if args.obstacle_range == 80.0 else
                                   f"; obstacles placed over {args.obstacle_range:.0f} m"),
                    "goals": B, "obstacles": m, "n_time": n, "obstacle_range_m": args.obstacle_range}
                   if args.workload == "dense" else
                   {"workload": "uneven batch: 512 scenes, goals log-uniform 16-1024, obstacles U{4..64}, "
                                "T in {50,100,150}, 100 AM iterations (cold start) + scoring",
                    "goals": B, "scenes": batch.n_scenes})
        | {"iters": args.iters, "seed": args.seed, "kernel": kernel, "group": group, "persistent": persistent,
           "waves": waves} | ({"bucket_groups": buckets} if buckets else {}),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": (measured_traffic(args.workload, kernel, waves, args.precision)
                                 if args.obstacle_range == 80.0 else None),
                     "kernel": {"wave": "k_am (wave kernel)", "mfma": "k_am_mfma", "group": "k_am_group"}[kernel],
                     "kernel_ms": solve_avg_s * 1e3,
                     "kernel_ms_p10_median_p90": [float(np.percentile(solve_ms, 10)), float(np.median(solve_ms)),
                                                  float(np.percentile(solve_ms, 90))],
                     "algorithmic_flop_per_launch": flops,
                     "frac_without_obstacle_tests": flops_no_obs / solve_avg_s / 1e12 / PEAK_FP32_TFLOPS,
                     "frac_of_unpacked_fp32_peak": achieved / PEAK_FP32_UNPACKED_TFLOPS,
                     "target_frac": 0.5},
        "best_goal": int(best[0].item()),
    }
    if cpu is not None:
        ref_c, ref_best, bif = cpu.pop("_oracle_c"), cpu.pop("_oracle_best"), cpu.pop("_bifurcating")
        if args.workload == "dense" and args.obstacle_range == 80.0:
            cpu["parity"] = parity_vs_oracle(st.c.cpu().numpy(), ref_c, bif, best[0].item(), ref_best)
    if args.workload == "dense" and not args.no_extras:
        out["residual_curve"] = residual_curve()
    if args.workload == "uneven" and not args.no_extras:
        out["uneven"] = uneven_extras(T, S, solver, batch, db, st, v_ref, cost, best, args, kernel, group, persistent,
                                      total_ms / args.steps, waves)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    if args.workload == "dense" and not args.no_warm:
        out["warmstart"] = warm_leg(args.warm_train, args.warm_test, args.warm_epochs, args.restart_at or None)
    solver.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
