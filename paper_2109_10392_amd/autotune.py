"""Tile autotuner: time the solver's kernel tiles on a workload, keep the fastest.

A tile is (kernel, group, persistent, waves): the wave kernel with one or two
wavefronts per goal; the
matrix-core kernel with `group` goals per workgroup (1..16 MFMA columns used)
and one wave per 16-sample time tile; or the group kernel, one wave per goal
group sweeping its own time tiles over a cost-sorted work list, consumed by a
persistent grid or one wave per listed group. The result is stored per
(workload, precision) in tuning.json next to this file and read back by
`lookup`, which the benchmark uses for TRAJ_KERNEL_AUTO.

Per (T, m) bucket (`--buckets`, group kernel): the shapes of a batch fall into
buckets of equal horizon T and obstacle counts m in [16 i, 16 i + 15]; starting
from the tile's group size everywhere, each bucket in turn (most goals first)
tries the other group sizes on the whole batch and keeps one only if the solve
gets faster by more than the noise margin. The table is stored with the tile
and applied through traj_set_shape_groups (`lookup_buckets`).
"""
from __future__ import annotations

import json
import os

TUNING_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")

CANDIDATES = [("wave", 16, True, 1), ("wave", 16, True, 2), ("mfma", 16, True, 1), ("mfma", 4, True, 1),
              ("group", 16, True, 1), ("group", 16, False, 1), ("group", 8, True, 1), ("group", 4, True, 1)]


def lookup(workload: str, precision: str = "fp32"):
    if not os.path.exists(TUNING_PATH):
        return None
    with open(TUNING_PATH) as f:
        table = json.load(f)
    entry = table.get(f"{workload}/{precision}")
    if entry is None:
        return None
    return entry["kernel"], int(entry["group"]), bool(entry.get("persistent", True)), int(entry.get("waves", 1))


def bucket_of(shape):
    """(T, m) bucket of a (n_time, t_f, n_obs) shape: 'T<n>/m<lo>-<hi>'."""
    n, _, m = shape
    lo = 16 * (int(m) // 16)
    return f"T{int(n)}/m{lo}-{lo + 15}"


def lookup_buckets(workload: str, precision: str = "fp32"):
    """{bucket: group size} stored for the workload, or None."""
    if not os.path.exists(TUNING_PATH):
        return None
    with open(TUNING_PATH) as f:
        entry = json.load(f).get(f"{workload}/{precision}")
    return None if entry is None else entry.get("buckets")


def shape_groups(shapes, buckets):
    """Per-shape group sizes (0 = the tile's) from a bucket table."""
    return [int(buckets.get(bucket_of(sh), 0)) for sh in shapes] if buckets else [0] * len(shapes)


def time_solve(solver, db, st, iters, precision, reps):
    """Median ms of `reps` solves after one warm-up."""
    import numpy as np
    import torch
    solver.solve(db, st, iters, precision=precision)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        solver.solve(db, st, iters, precision=precision)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def tune_buckets(solver, db, st, iters, shapes, goals_per_shape, precision="fp32", options=(8, 12), reps=5,
                 margin=0.02, log=print):
    """Coordinate descent over per-bucket group sizes of the group kernel on the
    whole batch. A size is kept when the solve gets faster than the best so far by
    more than `margin`; at the end the kept table and the single tile are timed
    again, alternately, and the table survives only if it still wins by `margin`.
    Returns (buckets {bucket: group}, ms with them, ms of the single tile,
    sweep {bucket: {group: ms}})."""
    keys = {}
    for i, sh in enumerate(shapes):
        keys.setdefault(bucket_of(sh), []).append(i)
    order = sorted(keys, key=lambda k: -sum(goals_per_shape[i] for i in keys[k]))
    tile_group = solver.get_tile()[1]
    chosen = {k: tile_group for k in order}

    def groups_of(ch):
        return [ch[bucket_of(sh)] for sh in shapes]

    solver.set_shape_groups(None)
    single = time_solve(solver, db, st, iters, precision, reps)
    best = single
    sweep = {}
    log(f"  single tile (group {tile_group}): {single:.3f} ms")
    for k in order:
        sweep[k] = {}
        for g in options:
            if g == chosen[k]:
                continue
            trial = dict(chosen)
            trial[k] = g
            solver.set_shape_groups(groups_of(trial))
            ms = time_solve(solver, db, st, iters, precision, reps)
            sweep[k][g] = ms
            log(f"  {k:14s} ({sum(goals_per_shape[i] for i in keys[k]):6d} goals) group {g:2d}: {ms:.3f} ms")
            if ms < best * (1.0 - margin):
                best, chosen = ms, trial
    # confirm against the single tile, alternating the two settings
    t_b, t_1 = [], []
    for _ in range(3):
        solver.set_shape_groups(groups_of(chosen))
        t_b.append(time_solve(solver, db, st, iters, precision, reps))
        solver.set_shape_groups(None)
        t_1.append(time_solve(solver, db, st, iters, precision, reps))
    import numpy as np
    with_buckets, single = float(np.median(t_b)), float(np.median(t_1))
    if not with_buckets < single * (1.0 - margin):
        log(f"  kept table {with_buckets:.3f} ms against the single tile {single:.3f} ms: not kept")
        chosen = {k: tile_group for k in order}
        with_buckets = single
    solver.set_shape_groups(groups_of(chosen))
    return chosen, with_buckets, single, sweep


def tune(solver, db, st, iters, precision="fp32", candidates=None, reps=3):
    """Return [(ms, kernel, group, persistent, waves)] sorted fastest first for this batch."""
    import torch
    res = []
    for kernel, group, persistent, waves in (candidates or CANDIDATES):
        if precision == "bf16x3" and kernel == "wave":
            continue
        solver.set_tile(kernel, group, persistent, waves)
        solver.solve(db, st, iters, precision=precision)  # warm-up
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            solver.solve(db, st, iters, precision=precision)
        b.record()
        torch.cuda.synchronize()
        res.append((a.elapsed_time(b) / reps, kernel, group, persistent, waves))
        print(f"  {kernel:5s} group {group:2d} persistent {int(persistent)} waves {waves}: {res[-1][0]:8.3f} ms",
              flush=True)
    res.sort()
    return res


def store(workload: str, precision: str, sweep, path=TUNING_PATH):
    table = {}
    if os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
    ms, kernel, group, persistent, waves = sweep[0]
    table[f"{workload}/{precision}"] = {"kernel": kernel, "group": group, "persistent": persistent, "waves": waves,
                                         "ms": ms,
                                         "sweep": [{"ms": t, "kernel": k, "group": g, "persistent": p, "waves": w}
                                                   for t, k, g, p, w in sweep]}
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def store_buckets(workload: str, precision: str, buckets, ms_buckets, ms_single, sweep=None, path=TUNING_PATH):
    """Add the per-bucket group sizes to the workload's stored tile (which must exist).
    Only buckets that differ from the tile's group size are kept; the sweep's
    timings are stored beside them."""
    with open(path) as f:
        table = json.load(f)
    entry = table[f"{workload}/{precision}"]
    entry["buckets"] = {k: g for k, g in sorted(buckets.items()) if g != entry["group"]}
    entry["buckets_ms"] = ms_buckets
    entry["single_tile_ms"] = ms_single
    if sweep is not None:
        entry["bucket_sweep"] = {k: {str(g): round(ms, 3) for g, ms in v.items()} for k, v in sorted(sweep.items())}
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def main():
    import argparse
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch

    from paper_2109_10392_amd import scenes as S
    from paper_2109_10392_amd import traj as T

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["dense", "uneven"], default="dense")
    ap.add_argument("--precision", choices=["fp32", "bf16x3"], default="fp32")
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--write", action="store_true", help="store the winner in tuning.json")
    ap.add_argument("--out", default=TUNING_PATH, help="table to store into (default: tuning.json of the package)")
    ap.add_argument("--kernels", default="wave,mfma,group", help="comma-separated kernels to sweep")
    ap.add_argument("--buckets", action="store_true",
                    help="tune the group kernel's group size per (T, m) bucket on top of the stored tile")
    args = ap.parse_args()
    kernels = set(args.kernels.split(","))
    batch = S.workload_dense(0) if args.workload == "dense" else S.workload_uneven(0)
    solver = T.Solver(S.DEFAULT_PARAMS, batch.shapes())
    db = T.DeviceBatch.from_batch(batch)
    st = T.DeviceState.empty(batch.n_goals)
    if args.buckets:
        tile = lookup(args.workload, args.precision)
        if tile is None or tile[0] != "group":
            raise SystemExit("per-bucket tuning needs a stored group-kernel tile for this workload")
        solver.set_tile(*tile)
        sid = batch.shape_id()
        goals = [0] * len(batch.shapes())
        for sc, i in zip(batch.scenes, sid):
            goals[int(i)] += sc.goals.shape[0]
        buckets, ms_b, ms_1, sweep = tune_buckets(solver, db, st, args.iters, batch.shapes(), goals, args.precision)
        print(f"{args.workload}/{args.precision}: single tile {ms_1:.3f} ms, per-bucket groups {ms_b:.3f} ms "
              f"(gain x{ms_1 / ms_b:.3f}); buckets changed: "
              f"{ {k: g for k, g in buckets.items() if g != tile[1]} }", flush=True)
        if args.write:
            store_buckets(args.workload, args.precision, buckets, ms_b, ms_1, sweep, args.out)
            print(f"stored the bucket table in {args.out}", flush=True)
        solver.close()
        return
    sweep = tune(solver, db, st, args.iters, args.precision, [c for c in CANDIDATES if c[0] in kernels])
    for ms, k, g, p, w in sweep:
        print(f"{args.workload}/{args.precision} {k:5s} group {g:2d} persistent {int(p)} waves {w}: {ms:8.3f} ms",
              flush=True)
    if args.write:
        store(args.workload, args.precision, sweep, args.out)
        print(f"stored {sweep[0][1:]} in {args.out}", flush=True)
    solver.close()


if __name__ == "__main__":
    main()
