"""Tile autotuner: time the solver's kernel tiles on a workload, keep the fastest.

A tile is (kernel, group, persistent, waves): the wave kernel with one or two
wavefronts per goal; the
matrix-core kernel with `group` goals per workgroup (1..16 MFMA columns used)
and one wave per 16-sample time tile; or the group kernel, one wave per goal
group sweeping its own time tiles over a cost-sorted work list, consumed by a
persistent grid or one wave per listed group. The result is stored per
(workload, precision) in tuning.json next to this file and read back by
`lookup`, which the benchmark uses for TRAJ_KERNEL_AUTO.
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
    args = ap.parse_args()
    kernels = set(args.kernels.split(","))
    batch = S.workload_dense(0) if args.workload == "dense" else S.workload_uneven(0)
    solver = T.Solver(S.DEFAULT_PARAMS, batch.shapes())
    db = T.DeviceBatch.from_batch(batch)
    st = T.DeviceState.empty(batch.n_goals)
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
