"""Warm-start kernels against the FP64 reference (oracle/mlp_oracle.py).

The products sum BF16 x BF16 terms in FP32 on the GPU and exactly in the
reference, so a product agrees to FP32 rounding of its sum. A layer's BF16
output can then differ by one BF16 unit where the sum lies at a rounding
boundary; layers are therefore checked one at a time, each fed the GPU's own
input, and the gradients of the lower layers (which see such one-unit
differences of the GPU's intermediate gradient) to a norm tolerance.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_2109_10392_amd import scenes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_10392_amd import traj, warmstart
    traj.lib()
    return warmstart


def bf16_bits(x):
    """BF16 bit patterns (int16 tensor on the GPU) of FP32 values, rounded as the oracle does."""
    import torch
    v = np.ascontiguousarray(M.bf16(x).astype(np.float32))
    return torch.from_numpy((v.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)).cuda()


def from_bits(t):
    return (t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30)


@pytest.mark.parametrize("ta,tb,M_,N_,K_", [(0, 0, 40, 72, 104), (0, 1, 136, 24, 200), (1, 0, 64, 200, 88),
                                             (1, 1, 8, 8, 8), (0, 0, 130 * 8, 16, 16896)])
def test_gemm_all_layouts_against_exact_sums(W, ta, tb, M_, N_, K_):
    rng = np.random.default_rng(M_ + N_ + K_)
    A = rng.normal(0, 1, (K_, M_) if ta else (M_, K_)).astype(np.float32)
    B = rng.normal(0, 1, (N_, K_) if tb else (K_, N_)).astype(np.float32)
    bias = rng.normal(0, 1, N_).astype(np.float32)
    import torch
    C = W.gemm_bf16(ta, tb, M_, N_, K_, bf16_bits(A), bf16_bits(B), torch.from_numpy(bias).cuda(), relu=False)
    Aq, Bq = M.bf16(A), M.bf16(B)
    ref = (Aq.T if ta else Aq) @ (Bq.T if tb else Bq) + bias
    # FP32 sums of K terms of size ~1: absolute error ~ sqrt(K) 2^-24 |terms|
    assert np.max(np.abs(C.cpu().numpy() - ref)) <= 1e-6 * np.sqrt(K_) * 8
    Cr = W.gemm_bf16(ta, tb, M_, N_, K_, bf16_bits(A), bf16_bits(B), None, relu=True).cpu().numpy()
    assert np.all(Cr >= 0) and np.max(np.abs(Cr - np.maximum(ref - bias, 0))) <= 1e-6 * np.sqrt(K_) * 8


def test_features_bit_exact(W):
    from paper_2109_10392_amd import traj as T
    scenes = [S.make_template_scene(s) for s in range(20)]
    ego = np.array([0, 0, 15, 0, 0, 0, 0, 0], np.float32)
    hand = S.make_template_scene(99)
    hand.ego = ego
    hand.obs = np.array([[80, 3.5, 5, 0], [70, 0, 6, 0], [60, -3.5, 7, 0], [50, 3.5, 8, 0], [50, -3.5, 9, 0],
                         [40, 0, 10, 0], [35, 3.5, 11, 0], [30, -3.5, 12, 0], [25, 0, 13, 0], [20, 3.5, 14, 0],
                         [90, 0, 5, 0], [10, 0, 6, 1]], np.float32)
    few = S.make_scene(7, n_goals=3, n_obs=3)
    none = S.make_scene(8, n_goals=2, n_obs=0)
    batch = S.Batch(scenes + [hand, few, none])
    db = T.DeviceBatch.from_batch(batch)
    got = W.features(db).cpu().numpy()
    for i, sc in enumerate(batch.scenes):
        assert np.array_equal(got[i], M.features(sc.ego, sc.obs)), i


def small_net(W, seed=3):
    net = W.Network(seed=seed)
    rng = np.random.default_rng(seed)
    p = net.initial(seed)
    p[:] += rng.normal(0, 0.01, p.size).astype(np.float32)  # non-zero biases too
    net.load(p)
    return net, p


def test_forward_layer_by_layer(W):
    import torch
    net, p = small_net(W)
    layers = M.unpack(p.astype(np.float64), M.layer_sizes())
    B = 24
    rng = np.random.default_rng(5)
    x = rng.normal(0, 1, (B, 64)).astype(np.float32)
    acts = torch.zeros(net.acts_size(B), dtype=torch.int16, device="cuda")
    y = torch.zeros(B, 16896, device="cuda")
    net.forward(torch.from_numpy(x).cuda(), acts, y)
    a = from_bits(acts)
    sizes = M.layer_sizes()
    offs = [0, B * 64] + [B * 64 + l * B * 256 for l in range(1, 3)]
    got = [a[offs[0]:offs[1]].reshape(B, 64)] + [a[offs[l]:offs[l] + B * 256].reshape(B, 256) for l in range(1, 4)]
    assert np.array_equal(got[0], M.bf16(x))
    for l in range(3):
        W_, b_ = layers[l]
        z = got[l] @ M.bf16(W_.astype(np.float32)) + b_.astype(np.float32)
        ref = M.bf16(np.maximum(z, 0).astype(np.float32))
        # identical except where the FP32 sum sits at a BF16 rounding boundary (one unit apart)
        diff = np.abs(got[l + 1] - ref)
        assert np.all(diff <= 2 ** -7 * np.abs(ref) + 1e-30), l
        assert np.mean(diff > 0) < 0.01, l
    W4, b4 = layers[3]
    yref = got[3] @ M.bf16(W4.astype(np.float32)) + b4.astype(np.float32)
    assert rel(y.cpu().numpy(), yref) < 1e-5


def test_loss_and_gradient_of_the_output(W):
    import torch
    B, N = 24, 16896
    rng = np.random.default_rng(6)
    y = rng.normal(0, 1, (B, N)).astype(np.float32)
    t = rng.normal(3, 2, (B, N)).astype(np.float32)
    mean = rng.normal(3, 0.1, N).astype(np.float32)
    std = rng.uniform(1, 3, N).astype(np.float32)
    from paper_2109_10392_amd import traj as T
    dy = torch.zeros(B, N, dtype=torch.int16, device="cuda")
    row_loss = torch.zeros(B, device="cuda")
    loss = torch.zeros(1, device="cuda")
    import ctypes
    # device copies held by name for the duration of the call
    yd, td, md, sd = (torch.from_numpy(a).cuda() for a in (y, t, mean, std))
    T._check(T.lib().traj_mlp_loss(ctypes.byref(T.MlpDims(*W.DIMS)), W._p(yd), W._p(td), W._p(md), W._p(sd), B,
                                   W._p(dy), W._p(row_loss), W._p(loss), T._stream(None)))
    torch.cuda.synchronize()
    L_ref, dy_ref = M.loss(y.astype(np.float64), t, mean.astype(np.float64), std.astype(np.float64))
    assert abs(float(loss.item()) - L_ref) <= 1e-5 * L_ref
    got = from_bits(dy).reshape(B, N)
    diff = np.abs(got - dy_ref)
    assert np.all(diff <= 2 ** -7 * np.abs(dy_ref) + 1e-30) and np.mean(diff > 0) < 0.01


def test_backward_gradients(W):
    import torch
    net, p = small_net(W, seed=4)
    layers = M.unpack(p.astype(np.float64), M.layer_sizes())
    B = 40
    rng = np.random.default_rng(7)
    x = rng.normal(0, 1, (B, 64)).astype(np.float32)
    acts = torch.zeros(net.acts_size(B), dtype=torch.int16, device="cuda")
    y = torch.zeros(B, 16896, device="cuda")
    net.forward(torch.from_numpy(x).cuda(), acts, y)
    dyf = (rng.normal(0, 1e-4, (B, 16896))).astype(np.float32)
    dy = bf16_bits(dyf)
    work = torch.zeros(2 * B * 256, dtype=torch.int16, device="cuda")
    net.backward(acts, dy, B, work)
    g = net.grad.cpu().numpy().astype(np.float64)
    a = from_bits(acts)
    offs = [0, B * 64] + [B * 64 + l * B * 256 for l in range(1, 3)]
    acts_l = [a[offs[0]:offs[1]].reshape(B, 64)] + [a[offs[l]:offs[l] + B * 256].reshape(B, 256) for l in range(1, 4)]
    ref = M.backward(layers, acts_l, M.bf16(dyf))
    gl = M.unpack(g, M.layer_sizes())
    # top layer: same inputs on both sides, FP32 sums
    assert rel(gl[3][0], ref[3][0]) < 1e-5 and rel(gl[3][1], ref[3][1]) < 1e-5
    # lower layers: intermediate BF16 gradients may differ by one unit in a few entries
    for l in range(3):
        for k in range(2):
            err = np.linalg.norm(gl[l][k] - ref[l][k]) / max(np.linalg.norm(ref[l][k]), 1e-30)
            assert err < 1e-2, (l, k, err)


def test_adam_steps_match_the_reference(W):
    import torch
    net, p = small_net(W, seed=8)
    rng = np.random.default_rng(9)
    m = np.zeros(net.n)
    v = np.zeros(net.n)
    pr = p.astype(np.float64)
    for step in range(1, 4):
        g = rng.normal(0, 1e-2, net.n).astype(np.float32)
        net.grad.copy_(torch.from_numpy(g))
        net.adam(1e-3)
        pr, m, v = M.adam(pr, g.astype(np.float64), m, v, step, 1e-3)
    got = net.params.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - pr)) <= 1e-6 * max(1.0, np.max(np.abs(pr)))
    assert np.array_equal(from_bits(net.params_bf16), M.bf16(net.params.cpu().numpy()))


def test_colstats_and_state_row_moves(W):
    import torch
    from paper_2109_10392_amd import traj as T
    rng = np.random.default_rng(10)
    rows = rng.normal(5, 2, (300, 136)).astype(np.float32)
    rows[:, 3] = 0.0
    mean, std = W.colstats(torch.from_numpy(rows).cuda())
    mr, sr = M.colstats(rows)
    assert rel(mean.cpu().numpy(), mr) < 1e-6 and rel(std.cpu().numpy(), sr) < 1e-6
    # gather / scatter between the solver state and the rows (3 template scenes, 256 goals each)
    batch = W.template_batch([1, 2, 3])
    db = T.DeviceBatch.from_batch(batch, shapes=[(100, 10.0, 10)])
    st = T.DeviceState.empty(batch.n_goals)
    st.c.copy_(torch.randn_like(st.c))
    st.lam.copy_(torch.randn_like(st.lam))
    r = W.state_rows(db, st).cpu().numpy()
    c, lam = st.c.cpu().numpy(), st.lam.cpu().numpy()
    for s in range(3):
        for i in (0, 17, 255):
            g = 256 * s + i
            blk = r[s, 66 * i:66 * i + 66].reshape(6, 11)
            assert np.array_equal(blk[:3], c[:, :, g]) and np.array_equal(blk[3:], lam[:, :, g])
    st2 = T.DeviceState.empty(batch.n_goals)
    W.rows_state(db, st2, torch.from_numpy(r).cuda(), torch.zeros(r.shape[1], device="cuda"),
                 torch.ones(r.shape[1], device="cuda"))
    assert torch.equal(st2.c, st.c) and torch.equal(st2.lam, st.lam)
