"""Learned warm start: binding of the network kernels (include/traj_mlp.h) and the
driver that trains the network on the optimizer's own solutions and measures
what it gains.

Algorithm 1 may start from any iterate (Remark 4 of arXiv 2109.10392). The
network maps 64 features of a scene (ego speed, the 10 nearest obstacles) to
the iterate (c, lambda) of the scene's 256 template goals (4 lanes x 64
longitudinal slots). Every step runs in the library's kernels: features,
forward, loss, backward and Adam on the GPU, the solver for the training
targets and for the evaluation. PyTorch holds the buffers and shuffles the
minibatch indices.

Evaluation (the stopping rule of traj_converge: the best goal of a scene at
max(r_obs, r_acc, r_nh) <= 1e-3, checked every 5 iterations, at most 300):
  cold: FP32 solver from the cold start;
  warm: features -> network -> (c, lambda), then the split-BF16 solver with the
        cold start as fallback twice: per goal, after one iteration, whichever
        start has the lower residual; per scene, a scene not converged after
        RESTART_AT iterations starts again from the cold start for the rest of
        the budget. The network, the features and the extra fallback iteration
        are all inside the warm timing.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import scenes as S
from . import traj as T

DIMS = (64, 256, 3, 16896)
# Second fallback: the scenes a warm start has not brought to the tolerance after
# this many iterations start again from the cold start for the rest of the budget
# (a warm start that converges does so in about 55 iterations; one that has not by
# 30 is more often stalled than slow).
RESTART_AT = 10
GOALS = 256  # template goals per scene (4 lanes x 64 slots)
ROW = 6 * T.N_COEF * GOALS


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Network:
    """Parameters (FP32 master, BF16 copy) and, for training, gradient and Adam moments."""

    def __init__(self, dims=DIMS, seed=0, train=True, device="cuda"):
        import torch
        self.dims = T.MlpDims(*dims)
        n = ctypes.c_int64()
        T._check(T.lib().traj_mlp_param_count(ctypes.byref(self.dims), ctypes.byref(n)))
        self.n = n.value
        z = lambda dt: torch.zeros(self.n, dtype=dt, device=device)
        self.params, self.params_bf16 = z(torch.float32), z(torch.int16)
        self.grad = z(torch.float32) if train else None
        self.m = z(torch.float32) if train else None
        self.v = z(torch.float32) if train else None
        self.step = 0
        self.load(self.initial(seed))

    def sizes(self):
        d = self.dims
        return [d.n_in] + [d.n_hidden] * d.n_layers + [d.n_out]

    def initial(self, seed):
        """He-normal hidden weights, a smaller output layer, zero biases (host array)."""
        rng = np.random.default_rng(seed)
        sizes = self.sizes()
        parts = []
        for i, (fi, fo) in enumerate(zip(sizes[:-1], sizes[1:])):
            std = np.sqrt(2.0 / fi) if i < len(sizes) - 2 else 0.1 / np.sqrt(fi)
            parts += [rng.normal(0, std, fi * fo), np.zeros(fo)]
        return np.concatenate(parts).astype(np.float32)

    def load(self, flat):
        import torch
        self.params.copy_(torch.as_tensor(np.asarray(flat, np.float32)))
        T._check(T.lib().traj_mlp_sync_bf16(ctypes.byref(self.c()), T._stream(None)))

    def c(self):
        return T.MlpC(self.dims, _p(self.params), _p(self.params_bf16), _p(self.grad), _p(self.m), _p(self.v))

    def acts_size(self, batch):
        d = self.dims
        return batch * (d.n_in + d.n_layers * d.n_hidden)

    def forward(self, x, acts, y):
        T._check(T.lib().traj_mlp_forward(ctypes.byref(self.c()), _p(x), int(x.shape[0]), _p(acts), _p(y),
                                          T._stream(None)))

    def loss(self, y, target, mean, std, dy, row_loss, loss):
        T._check(T.lib().traj_mlp_loss(ctypes.byref(self.dims), _p(y), _p(target), _p(mean), _p(std), int(y.shape[0]),
                                       _p(dy), _p(row_loss), _p(loss), T._stream(None)))

    def backward(self, acts, dy, batch, work):
        T._check(T.lib().traj_mlp_backward(ctypes.byref(self.c()), _p(acts), _p(dy), int(batch), _p(work),
                                           T._stream(None)))

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        T._check(T.lib().traj_mlp_adam(ctypes.byref(self.c()), self.step, float(lr), float(b1), float(b2), float(eps),
                                       T._stream(None)))


def features(db):
    import torch
    f = torch.empty(max(db.n_scenes, 1), 64, device="cuda")
    T._check(T.lib().traj_features(ctypes.byref(db.c_struct()), _p(f), T._stream(None)))
    return f[:db.n_scenes]


def state_rows(db, st, gps=GOALS):
    import torch
    rows = torch.empty(db.n_scenes, 6 * T.N_COEF * gps, device="cuda")
    T._check(T.lib().traj_state_rows(ctypes.byref(db.c_struct()), ctypes.byref(st.c_struct()), int(gps), _p(rows),
                                     T._stream(None)))
    return rows


def rows_state(db, st, y, mean, std, gps=GOALS):
    T._check(T.lib().traj_rows_state(ctypes.byref(db.c_struct()), ctypes.byref(st.c_struct()), int(gps), _p(y),
                                     _p(mean), _p(std), T._stream(None)))


def colstats(rows):
    import torch
    mean = torch.empty(rows.shape[1], device="cuda")
    std = torch.empty(rows.shape[1], device="cuda")
    T._check(T.lib().traj_colstats(_p(rows), int(rows.shape[0]), int(rows.shape[1]), _p(mean), _p(std),
                                   T._stream(None)))
    return mean, std


def gemm_bf16(ta, tb, M, N, K, A, B, bias=None, relu=False):
    import torch
    C = torch.empty(M, N, device="cuda")
    T._check(T.lib().traj_gemm_bf16(int(ta), int(tb), M, N, K, _p(A), _p(B), _p(bias), int(relu), _p(C),
                                    T._stream(None)))
    return C


# ---------------------------------------------------------------- data and driver
def template_batch(seeds, n_obs=10):
    return S.Batch([S.make_template_scene(int(s), n_obs=n_obs) for s in seeds])


class Problem:
    """Solver handle and per-batch buffers for template scenes."""

    def __init__(self, kernel=("group", 16, True)):
        self.shape = (100, 10.0, 10)
        self.solver = T.Solver(S.DEFAULT_PARAMS, [self.shape])
        self.solver.set_tile(*kernel)

    def device(self, batch):
        import torch
        db = T.DeviceBatch.from_batch(batch, shapes=[self.shape])
        st = T.DeviceState.empty(batch.n_goals)
        v_ref = torch.tensor([float(s.ego[2]) for s in batch.scenes], device="cuda")
        cost = torch.zeros(batch.n_goals, device="cuda")
        best = torch.zeros(batch.n_scenes, device="cuda", dtype=torch.int32)
        its = torch.zeros(batch.n_scenes, device="cuda", dtype=torch.int32)
        return db, st, v_ref, cost, best, its

    def solve_cold(self, bufs, max_iters=300, tol=1e-3, precision="fp32"):
        db, st, v_ref, cost, best, its = bufs
        self.solver.converge(db, st, v_ref, cost, best, its, max_iters=max_iters, chunk=5, tol=tol,
                             precision=precision)

    def solve_warm(self, bufs, net, mean, std, max_iters=300, tol=1e-3, precision="bf16x3", scratch=None,
                   restart_at=RESTART_AT):
        """Network start with the cold start as fallback; with restart_at, the scenes
        still unconverged after restart_at iterations start again from the cold
        start for the rest of the max_iters budget."""
        import torch
        db, st, v_ref, cost, best, its = bufs
        x = features(db)
        if scratch is None:
            scratch = (torch.empty(net.acts_size(db.n_scenes), dtype=torch.int16, device="cuda"),
                       torch.empty(db.n_scenes, net.dims.n_out, device="cuda"))
        acts, y = scratch
        net.forward(x, acts, y)
        rows_state(db, st, y, mean, std)
        first = max_iters if restart_at is None else min(restart_at, max_iters)
        self.solver.converge(db, st, v_ref, cost, best, its, max_iters=first, chunk=5, tol=tol,
                             from_state=True, fallback=True, precision=precision)
        if first < max_iters:
            self.solver.converge(db, st, v_ref, cost, best, its, max_iters=max_iters - first, chunk=5, tol=tol,
                                 precision=precision, keep_done=True)


def make_dataset(prob, seeds, chunk=4096, max_iters=300, tol=1e-3, log=print, converged_only=False):
    """Features [N][64] and solved iterates [N][16896] of the template scenes `seeds`
    (with converged_only, only the scenes that met the tolerance)."""
    import torch
    feats, rows = [], []
    for i in range(0, len(seeds), chunk):
        t0 = time.time()
        batch = template_batch(seeds[i:i + chunk])
        bufs = prob.device(batch)
        prob.solve_cold(bufs, max_iters, tol)
        f, r = features(bufs[0]), state_rows(bufs[0], bufs[1])
        if converged_only:
            keep = bufs[1].scene_done[:batch.n_scenes] != 0
            f, r = f[keep], r[keep]
        feats.append(f)
        rows.append(r)
        torch.cuda.synchronize()
        if log:
            log(f"  data {i + len(batch.scenes)}/{len(seeds)} scenes ({time.time() - t0:.1f} s)")
    return torch.cat(feats), torch.cat(rows)


def train(net, feats, targets, mean, std, epochs=10, batch=256, lr=1e-3, seed=0, log=print, cosine=True):
    """Adam on the mean squared error of standardised targets, learning rate on a
    cosine schedule from lr to 0 (or constant); returns the loss per epoch."""
    import torch
    N = feats.shape[0]
    nb = N // batch
    acts = torch.empty(net.acts_size(batch), dtype=torch.int16, device="cuda")
    y = torch.empty(batch, net.dims.n_out, device="cuda")
    dy = torch.empty(batch, net.dims.n_out, dtype=torch.int16, device="cuda")
    row_loss = torch.empty(batch, device="cuda")
    loss = torch.empty(1, device="cuda")
    work = torch.empty(2 * batch * net.dims.n_hidden, dtype=torch.int16, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    curve = []
    for ep in range(epochs):
        perm = torch.randperm(N, device="cuda", generator=g)
        tot = torch.zeros(1, device="cuda")
        for b in range(nb):
            idx = perm[b * batch:(b + 1) * batch]
            x, t = feats.index_select(0, idx), targets.index_select(0, idx)
            net.forward(x, acts, y)
            net.loss(y, t, mean, std, dy, row_loss, loss)
            net.backward(acts, dy, batch, work)
            k = ep * nb + b
            net.adam(lr * 0.5 * (1.0 + np.cos(np.pi * k / (epochs * nb))) if cosine else lr)
            tot += loss
        curve.append(float(tot.item()) / max(nb, 1))
        if log:
            log(f"  epoch {ep + 1}/{epochs}: train loss {curve[-1]:.4f}")
    return curve


def fit(prob, seeds, epochs=30, batch=256, lr=2e-3, seed=0, log=print):
    """Train a network on the solved template scenes `seeds` (the scenes the cold
    solver brings to the tolerance); returns (net, mean, std, info)."""
    import torch
    t0 = time.time()
    feats, rows = make_dataset(prob, list(seeds), log=None, converged_only=True)
    torch.cuda.synchronize()
    t1 = time.time()
    mean, std = colstats(rows)
    net = Network(seed=seed)
    curve = train(net, feats, rows, mean, std, epochs=epochs, batch=batch, lr=lr, seed=seed, log=log)
    torch.cuda.synchronize()
    info = {"train_scenes": len(seeds), "train_samples": int(feats.shape[0]), "epochs": epochs, "lr": lr,
            "final_loss": curve[-1], "data_s": t1 - t0, "train_s": time.time() - t1}
    return net, mean, std, info


def evaluate(prob, net, mean, std, seeds, max_iters=300, tol=1e-3, warm_precision="bf16x3", restart_at=RESTART_AT,
             modes=("cold", "warm_fp32", "warm"), common=True):
    """Cold FP32, warm FP32 and warm + mixed precision on the template scenes
    `seeds`: iterations and ms per scene to the tolerance (capped at max_iters),
    the share of scenes that meet it, and (common) the same timings repeated on
    only the scenes that both the cold FP32 and the warm + mixed forms bring to
    the tolerance."""
    import torch

    def timed(mode, batch):
        prec = warm_precision if mode == "warm" else "fp32"
        bufs = prob.device(batch)
        run = (lambda: prob.solve_cold(bufs, max_iters, tol)) if mode == "cold" else \
            (lambda: prob.solve_warm(bufs, net, mean, std, max_iters, tol, prec, restart_at=restart_at))
        run()  # warm-up (also sizes the solver's scratch)
        torch.cuda.synchronize()
        bufs = prob.device(batch)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        run()
        b.record()
        torch.cuda.synchronize()
        its = bufs[5].cpu().numpy()
        done = bufs[1].scene_done.cpu().numpy()[:batch.n_scenes] != 0
        return {"ms_per_scene": a.elapsed_time(b) / batch.n_scenes, "iters_mean": float(its.mean()),
                "iters_median": float(np.median(its)), "converged": float(done.mean()),
                "iters_mean_converged": float(its[done].mean()) if done.any() else None,
                "precision": prec, "scenes": batch.n_scenes}, done, its

    batch = template_batch(seeds)
    out, done = {}, {}
    for mode in modes:
        out[mode], done[mode], _ = timed(mode, batch)
    if restart_at is not None:
        out["restart_at"] = restart_at
    if "warm" in out and "cold" in out:
        out["iters_ratio"] = out["warm"]["iters_mean"] / out["cold"]["iters_mean"]
        out["ms_ratio"] = out["warm"]["ms_per_scene"] / out["cold"]["ms_per_scene"]
    if "warm_fp32" in out and "cold" in out:
        out["iters_ratio_fp32"] = out["warm_fp32"]["iters_mean"] / out["cold"]["iters_mean"]
    if common and "warm" in done and "cold" in done:
        both = done["cold"] & done["warm"]
        sub = [seeds[i] for i in np.flatnonzero(both)]
        if sub:
            sb = template_batch(sub)
            c, _, ci = timed("cold", sb)
            w, _, wi = timed("warm", sb)
            out["common"] = {"scenes": len(sub), "cold_ms_per_scene": c["ms_per_scene"],
                             "warm_ms_per_scene": w["ms_per_scene"], "cold_iters_mean": c["iters_mean"],
                             "warm_iters_mean": w["iters_mean"], "ms_ratio": w["ms_per_scene"] / c["ms_per_scene"],
                             "iters_ratio": w["iters_mean"] / c["iters_mean"]}
        out["converged_only_cold"] = int(np.count_nonzero(done["cold"] & ~done["warm"]))
        out["converged_only_warm"] = int(np.count_nonzero(done["warm"] & ~done["cold"]))
    return out
