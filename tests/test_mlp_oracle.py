"""Pins of the warm-start reference (oracle/mlp_oracle.py), CPU only.

Each pin comes from outside the code it checks: central finite differences of
the loss for the backward pass, another library's BF16 conversion for the
rounding, the closed form of Adam's first step, and hand-built scenes for the
features.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as M


def tiny_net(rng, sizes):
    n = sum(fi * fo + fo for fi, fo in zip(sizes[:-1], sizes[1:]))
    return rng.normal(0, 0.5, n)


def total_loss(params, sizes, x, t, mean, std):
    layers = M.unpack(params, sizes)
    y, _ = M.forward(layers, x, rounding=False)
    return M.loss(y, t, mean, std, rounding=False)[0]


def test_backward_matches_central_finite_differences():
    rng = np.random.default_rng(0)
    sizes = [5, 7, 6, 4]
    p = tiny_net(rng, sizes)
    x = rng.normal(0, 1, (3, 5))
    t = rng.normal(0, 2, (3, 4))
    mean, std = rng.normal(0, 1, 4), rng.uniform(0.5, 2, 4)
    layers = M.unpack(p, sizes)
    y, acts = M.forward(layers, x, rounding=False)
    _, dy = M.loss(y, t, mean, std, rounding=False)
    grads = M.backward(layers, acts, dy, rounding=False)
    analytic = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (total_loss(p + e, sizes, x, t, mean, std) - total_loss(p - e, sizes, x, t, mean, std)) / (2 * h)
    assert np.max(np.abs(fd - analytic)) <= 1e-7 * max(1.0, np.max(np.abs(fd)))


def test_backward_a_dropped_term_would_fail():
    """The finite-difference pin is sensitive: zeroing one layer's bias gradient fails it."""
    rng = np.random.default_rng(1)
    sizes = [4, 5, 3]
    p = tiny_net(rng, sizes)
    x, t = rng.normal(0, 1, (2, 4)), rng.normal(0, 1, (2, 3))
    layers = M.unpack(p, sizes)
    y, acts = M.forward(layers, x, rounding=False)
    _, dy = M.loss(y, t, np.zeros(3), np.ones(3), rounding=False)
    grads = M.backward(layers, acts, dy, rounding=False)
    broken = np.concatenate([np.concatenate([dW.ravel(), 0 * db]) for dW, db in grads])
    h = 1e-6
    fd = np.array([(total_loss(p + h * np.eye(p.size)[i], sizes, x, t, np.zeros(3), np.ones(3))
                    - total_loss(p - h * np.eye(p.size)[i], sizes, x, t, np.zeros(3), np.ones(3))) / (2 * h)
                   for i in range(p.size)])
    assert np.max(np.abs(fd - broken)) > 1e-4


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e6, 100), [0.0, -0.0, 1.0, 65504.0, 1e-30]])
    # exact ties: 1 + 2^-8 (rounds down to even), 1 + 3 * 2^-8 (rounds up to even)
    x = np.concatenate([x, [1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8)]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(x), ref)
    assert M.bf16(np.float32(1 + 2 ** -8)) == 1.0 and M.bf16(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p0 = np.array([1.0, 2.0, 3.0, 4.0])
    lr, eps = 1e-3, 1e-8
    p, m, v = M.adam(p0, g, np.zeros(4), np.zeros(4), 1, lr, eps=eps)
    assert np.allclose(p, p0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_of_a_hand_built_scene():
    ego = np.array([0, 0, 15, 0, 0, 0, 0, 0], np.float32)
    # 12 obstacles at distinct distances (index 11 nearest), two at equal distance (3 and 4)
    obs = np.array([[80, 3.5, 5, 0], [70, 0, 6, 0], [60, -3.5, 7, 0], [50, 3.5, 8, 0], [50, -3.5, 9, 0],
                    [40, 0, 10, 0], [35, 3.5, 11, 0], [30, -3.5, 12, 0], [25, 0, 13, 0], [20, 3.5, 14, 0],
                    [90, 0, 5, 0], [10, 0, 6, 1]], np.float32)
    f = M.features(ego, obs)
    assert f[0] == np.float32(15) * np.float32(1 / 30)
    order = [11, 9, 8, 7, 6, 5, 3, 4, 2, 1]  # ties (3, 4) by index; 0 and 10 are the farthest
    for r, j in enumerate(order):
        assert f[1 + 4 * r] == np.float32(obs[j, 0] * np.float32(0.01))
        assert f[2 + 4 * r] == np.float32(obs[j, 1] * np.float32(0.01))
        assert f[3 + 4 * r] == np.float32(np.float32(obs[j, 2] - 15) * np.float32(1 / 30))
        assert f[4 + 4 * r] == np.float32(obs[j, 3] * np.float32(1 / 30))
    assert np.all(f[41:] == 0)
    few = M.features(ego, obs[:3])
    assert np.all(few[13:] == 0) and few[1] == np.float32(60 * np.float32(0.01))


def test_colstats_constant_and_known_columns():
    rows = np.array([[0.0, 1.0, 5.0], [0.0, 3.0, 5.0], [0.0, 5.0, 5.0]])
    mean, std = M.colstats(rows)
    assert np.allclose(mean, [0, 3, 5]) and np.allclose(std, [1.0, np.sqrt(8 / 3), 1.0])


@pytest.mark.parametrize("sizes", [[64, 256, 256, 256, 16896]])
def test_parameter_count_of_the_warm_start_network(sizes):
    n = sum(fi * fo + fo for fi, fo in zip(sizes[:-1], sizes[1:]))
    assert n == 4_490_496
    assert M.layer_sizes() == sizes
