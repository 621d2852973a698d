"""Tile autotuner: time the solver's kernel tiles on a workload, keep the fastest.

A tile is (kernel, group): the one-wave-per-goal kernel, or the matrix-core
kernel with `group` goals per workgroup (1..16 MFMA columns used). The result
is stored per (workload, precision) in tuning.json next to this file and read
back by `lookup`, which the benchmark and the binding use for
TRAJ_KERNEL_AUTO.
"""
from __future__ import annotations

import json
import os

TUNING_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")

CANDIDATES = [("wave", 16), ("mfma", 16), ("mfma", 8), ("mfma", 4), ("mfma", 2)]


def lookup(workload: str, precision: str = "fp32"):
    if not os.path.exists(TUNING_PATH):
        return None
    with open(TUNING_PATH) as f:
        table = json.load(f)
    entry = table.get(f"{workload}/{precision}")
    return None if entry is None else (entry["kernel"], int(entry["group"]))


def tune(solver, db, st, iters, precision="fp32", candidates=None, reps=3):
    """Return [(ms, kernel, group)] sorted fastest first for this batch."""
    import torch
    res = []
    for kernel, group in (candidates or CANDIDATES):
        if precision == "bf16x3" and kernel == "wave":
            continue
        solver.set_tile(kernel, group)
        solver.solve(db, st, iters, precision=precision)  # warm-up
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            solver.solve(db, st, iters, precision=precision)
        b.record()
        torch.cuda.synchronize()
        res.append((a.elapsed_time(b) / reps, kernel, group))
    res.sort()
    return res


def store(workload: str, precision: str, kernel: str, group: int, ms: float, sweep):
    table = {}
    if os.path.exists(TUNING_PATH):
        with open(TUNING_PATH) as f:
            table = json.load(f)
    table[f"{workload}/{precision}"] = {"kernel": kernel, "group": group, "ms": ms,
                                         "sweep": [{"ms": t, "kernel": k, "group": g} for t, k, g in sweep]}
    with open(TUNING_PATH, "w") as f:
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
    args = ap.parse_args()
    batch = S.workload_dense(0) if args.workload == "dense" else S.workload_uneven(0)
    solver = T.Solver(S.DEFAULT_PARAMS, batch.shapes())
    db = T.DeviceBatch.from_batch(batch)
    st = T.DeviceState.empty(batch.n_goals)
    sweep = tune(solver, db, st, args.iters, args.precision)
    for ms, k, g in sweep:
        print(f"{args.workload}/{args.precision} {k:5s} group {g:2d}: {ms:8.3f} ms", flush=True)
    if args.write:
        ms, k, g = sweep[0]
        store(args.workload, args.precision, k, g, ms, sweep)
        print(f"stored {k} group {g} in {TUNING_PATH}", flush=True)
    solver.close()


if __name__ == "__main__":
    main()
