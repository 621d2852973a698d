"""A plain device-to-device copy of known size, for calibrating HBM traffic counters.

rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) over this program reports what
the counters read for exactly `--mib` MiB read and written; the ratio scales
the same counters taken over the solver kernels.
"""
import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=256)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    n = args.mib * (1 << 20) // 4
    src = torch.ones(n, device="cuda", dtype=torch.float32)
    dst = torch.empty_like(src)
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {args.mib} MiB x {args.reps}", flush=True)


if __name__ == "__main__":
    main()
