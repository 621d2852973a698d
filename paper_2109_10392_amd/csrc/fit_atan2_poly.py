"""Fit the first-octant polynomial of the device atan2 (atan2_heading).

atan(a) = a p(a^2) on a in [0, 1], p of degree 9 in s = a^2 with p(0) = 1 held
exactly (so atan(a) -> a for small a). The nine free coefficients minimise the
largest relative error |a p(a^2) - atan(a)| / atan(a) over the interval, found
by Lawson's iteratively reweighted least squares on Chebyshev nodes in s.
The FP32-rounded coefficients are then checked by evaluating the Horner form
with FP32 fused multiply-adds (emulated in FP64 and rounded once) against
atan in FP64 on a dense grid of FP32 arguments, and the result printed in
units in the last place of the FP32 result.

Usage: python fit_atan2_poly.py [--nodes N] [--iters K]
Prints the coefficients, highest degree first, in the order the device code's
Horner form uses them.
"""
from __future__ import annotations

import argparse

import numpy as np

DEGREE = 9


def target(s):
    """atan(sqrt(s)) / sqrt(s), the function p approximates (limit 1 at s = 0)."""
    a = np.sqrt(s)
    with np.errstate(invalid="ignore", divide="ignore"):
        r = np.arctan(a) / a
    return np.where(s == 0.0, 1.0, r)


def lawson(nodes=2000, iters=50):
    """Minimax-relative fit of p(s) - 1 = s q(s) by Lawson's weight updates."""
    k = np.arange(nodes)
    s = 0.5 - 0.5 * np.cos(np.pi * (k + 0.5) / nodes)  # Chebyshev nodes on [0, 1]
    f = target(s)
    # p(s) = 1 + sum_{i=1..DEGREE} c_i s^i; relative error (p - f) / f
    V = np.stack([s ** i for i in range(1, DEGREE + 1)], axis=1) / f[:, None]
    rhs = (f - 1.0) / f
    w = np.full(nodes, 1.0 / nodes)
    for _ in range(iters):
        sw = np.sqrt(w)
        c, *_ = np.linalg.lstsq(V * sw[:, None], rhs * sw, rcond=None)
        err = np.abs(V @ c - rhs)
        w = w * err
        w /= w.sum()
    return np.concatenate([[1.0], c])  # lowest degree first


def fmaf(a, b, c):
    """FP32 fused multiply-add: the product of two FP32 numbers is exact in FP64."""
    return np.float32(a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64))


def horner_fp32(coef_lo_first, a):
    """a p(a^2) with FP32 operations in the device code's order."""
    c = [np.float32(v) for v in coef_lo_first]
    a = a.astype(np.float32)
    s = (a * a).astype(np.float32)
    p = np.full_like(s, c[-1])
    for v in reversed(c[:-1]):
        p = fmaf(p, s, np.full_like(s, v))
    return (a * p).astype(np.float32)


def ulp_error(coef_lo_first, samples=1 << 20):
    a = np.linspace(0.0, 1.0, samples, dtype=np.float64).astype(np.float32)
    a = a[a > 0]
    got = horner_fp32(coef_lo_first, a).astype(np.float64)
    ref = np.arctan(a.astype(np.float64))
    ulp = np.spacing(np.float32(ref)).astype(np.float64)
    return float(np.max(np.abs(got - ref) / ulp))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nodes", type=int, default=2000)
    ap.add_argument("--iters", type=int, default=50)
    args = ap.parse_args()
    coef = lawson(args.nodes, args.iters)
    c32 = [float(np.float32(v)) for v in coef]
    print("coefficients, highest degree first (FP32):")
    for v in reversed(c32):
        print(f"  {v:.8e}")
    print(f"max error of the FP32 Horner form on [0, 1]: {ulp_error(c32):.2f} ulp")


if __name__ == "__main__":
    main()
