"""FP64 reference of the learned warm start (test infrastructure only).

The method (arXiv 2109.10392) is initialisation-agnostic (Remark 4): any
(c, lambda) may start Algorithm 1. The warm start here is a multilayer
perceptron from 64 scene features to the iterate of the 256 template goals
(6 x 11 values per goal: c_x, c_y, c_psi, lambda_x, lambda_y, lambda_psi),
trained by regression on solutions of the optimizer itself. This module is the
plain definition of what the GPU kernels compute, to check them against:

* bf16(x): round to nearest even of an FP32 value to BF16 (8-bit mantissa).
* features(ego, obs): ego speed and the 10 nearest obstacles (FP32 arithmetic,
  the ordering decided on FP32 squared distances, ties by index).
* forward: each layer input is rounded to BF16, weights are BF16 values,
  products are summed exactly here (FP32 on the GPU), bias and ReLU after.
* loss: mean squared error against standardised targets; dy rounded to BF16.
* backward: gradients of that network with the same BF16 rounding points
  (straight through the roundings), the ReLU derivative read off the stored
  activation (a > 0).
* adam: Kingma and Ba (2015), with bias correction, on the FP32 master weights.

Pinned in tests/test_mlp_oracle.py by central finite differences of the loss
(with the rounding switched off), a BF16 conversion of another library, a
closed form of the first Adam step and hand-built feature cases.
"""
from __future__ import annotations

import numpy as np

N_FEAT = 64
N_NEAR = 10
POS_SCALE = np.float32(0.01)       # 1 / 100 m
VEL_SCALE = np.float32(1.0 / 30.0)  # 1 / (30 m/s)


def bf16(x):
    """Round FP32 values to BF16 (nearest, ties to even); returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    nan = np.isnan(a)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def features(ego, obs):
    """64 features of one scene: [v0 / 30, then per nearest obstacle (dx, dy) / 100 m
    and (dvx, dvy) / 30 m/s, relative to the ego at t = 0], zero padded."""
    ego = np.asarray(ego, np.float32)
    obs = np.asarray(obs, np.float32).reshape(-1, 4)
    f = np.zeros(N_FEAT, np.float32)
    f[0] = ego[2] * VEL_SCALE
    if obs.shape[0] == 0:
        return f
    dx = (obs[:, 0] - ego[0]).astype(np.float32)
    dy = (obs[:, 1] - ego[1]).astype(np.float32)
    d2 = (dx * dx).astype(np.float32) + (dy * dy).astype(np.float32)  # FP32, no fused multiply-add
    order = sorted(range(obs.shape[0]), key=lambda j: (float(d2[j]), j))[:N_NEAR]
    for r, j in enumerate(order):
        f[1 + 4 * r] = dx[j] * POS_SCALE
        f[2 + 4 * r] = dy[j] * POS_SCALE
        f[3 + 4 * r] = np.float32(obs[j, 2] - ego[2]) * VEL_SCALE
        f[4 + 4 * r] = np.float32(obs[j, 3] - ego[3]) * VEL_SCALE
    return f


def layer_sizes(n_in=64, n_hidden=256, n_layers=3, n_out=16896):
    return [n_in] + [n_hidden] * n_layers + [n_out]


def unpack(params, sizes):
    """Packed parameters [W1 (in x out row-major), b1, W2, b2, ...] -> [(W, b)]."""
    out, off = [], 0
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        W = params[off:off + fi * fo].reshape(fi, fo)
        off += fi * fo
        b = params[off:off + fo]
        off += fo
        out.append((W, b))
    assert off == params.size
    return out


def forward(layers, x, rounding=True):
    """Returns (y, acts): acts[l] is the (rounded) input of layer l+1; y the output.
    With rounding=False every rounding point is the identity (exact network)."""
    rnd = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    a = rnd(x)
    acts = [a]
    for i, (W, b) in enumerate(layers):
        Wq = rnd(W)
        z = a @ Wq + np.asarray(b, np.float64)
        if i < len(layers) - 1:
            a = rnd(np.maximum(z, 0.0))
            acts.append(a)
        else:
            y = z
    return y, acts


def loss(y, target, mean, std, rounding=True):
    """Mean squared error against (target - mean) / std; returns (L, dy)."""
    rnd = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    t = (np.asarray(target, np.float64) - mean) / std
    d = y - t
    n = d.size
    return float(np.sum(d * d) / n), rnd(2.0 * d / n)


def backward(layers, acts, dy, rounding=True):
    """Gradients [(dW, db)] given the stored layer inputs and dy (already rounded)."""
    rnd = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    grads = [None] * len(layers)
    g = np.asarray(dy, np.float64)
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        a = acts[i]
        grads[i] = (a.T @ g, g.sum(axis=0))
        if i > 0:
            dh = g @ rnd(W).T
            g = rnd(dh * (acts[i] > 0))
    return grads


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (in place on copies); returns (p, m, v)."""
    p = np.asarray(p, np.float64).copy()
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    p -= lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def colstats(rows):
    """Per-column mean and standard deviation (population); columns whose spread
    is below 1e-5 max(1, |mean|) get std 1 (constant outputs, e.g. x(0) = 0)."""
    r = np.asarray(rows, np.float64)
    mean = r.mean(axis=0)
    std = np.sqrt(((r - mean) ** 2).mean(axis=0))
    std = np.where(std < 1e-5 * np.maximum(1.0, np.abs(mean)), 1.0, std)
    return mean, std
