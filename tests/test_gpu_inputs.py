"""Inputs a solve cannot use, on every kernel and precision form.

A scene whose ego state (the boundary values of eq. 8b) or any obstacle state
is not finite has every goal marked; a goal whose target is not finite is
marked alone. A marked goal's coefficients, multipliers and residuals are NaN
and its iteration count 0, so scoring never picks it. Every other goal is
solved exactly as in a batch without the bad inputs: bitwise, since goals are
independent instances (Remark 1) and no kernel's result depends on which goals
share a group.
"""
import dataclasses

import numpy as np
import pytest

from paper_2109_10392_amd import scenes as S
from tests.test_gpu_parity import PARAMS

pytestmark = pytest.mark.gpu

ITERS = 30
CASES = [("wave", 1, "fp32"), ("wave", 2, "fp32"), ("mfma", 1, "fp32"), ("mfma", 1, "bf16x3"),
         ("group", 1, "fp32"), ("group", 1, "bf16x3")]


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_10392_amd import traj
    traj.lib()
    return traj


def _with(sc, **kw):
    return dataclasses.replace(sc, **{k: np.array(v, dtype=np.float32) for k, v in kw.items()})


def _solve(T, batch, kernel, waves, precision):
    import torch
    solver = T.Solver(PARAMS, batch.shapes())
    solver.set_tile(kernel, 16, True, waves)
    db = T.DeviceBatch.from_batch(batch)
    st = T.DeviceState.empty(batch.n_goals)
    solver.solve(db, st, ITERS, kernel=kernel, precision=precision)
    v_ref = torch.tensor([float(s.ego[2]) if np.isfinite(s.ego[2]) else 15.0 for s in batch.scenes], device="cuda")
    cost = torch.zeros(batch.n_goals, device="cuda")
    best = torch.zeros(batch.n_scenes, device="cuda", dtype=torch.int32)
    solver.score(db, st, v_ref, cost, best)
    torch.cuda.synchronize()
    out = dict(c=st.c.cpu().numpy(), lam=st.lam.cpu().numpy(), resid=st.resid.cpu().numpy(),
               iters=st.iters.cpu().numpy(), cost=cost.cpu().numpy(), best=best.cpu().numpy())
    solver.close()
    return out


@pytest.mark.parametrize("kernel,waves,precision", CASES)
def test_non_finite_inputs_mark_only_their_goals(T, kernel, waves, precision):
    good = S.make_scene(31, 20, 8)
    other = S.make_scene(32, 20, 8)
    obs = good.obs.copy()
    obs[5, 1] = np.nan
    ego = good.ego.copy()
    ego[2] = np.inf
    goals = other.goals.copy()
    goals[3, 0] = np.nan
    bad_goal = 3
    batch = S.Batch([good, _with(good, obs=obs), _with(other, goals=goals), _with(good, ego=ego)])
    out = _solve(T, batch, kernel, waves, precision)
    off = batch.goal_off()

    # reference: the same scenes without the bad inputs (the marked goal dropped)
    keep = [g for g in range(other.goals.shape[0]) if g != bad_goal]
    ref = _solve(T, S.Batch([good, _with(other, goals=other.goals[keep])]), kernel, waves, precision)
    ref_off = [0, good.goals.shape[0], good.goals.shape[0] + len(keep)]

    def cols(d, sl):
        return {k: d[k][..., sl] for k in ("c", "lam", "resid", "iters", "cost")}

    # scene 0: untouched by its neighbours
    for k, v in cols(out, slice(off[0], off[1])).items():
        assert np.array_equal(v, cols(ref, slice(ref_off[0], ref_off[1]))[k], equal_nan=True), k
    # scenes 1 (obstacle) and 3 (ego): every goal marked, no best goal
    for s in (1, 3):
        sl = slice(off[s], off[s + 1])
        assert np.all(np.isnan(out["c"][..., sl])) and np.all(np.isnan(out["lam"][..., sl]))
        assert np.all(np.isnan(out["resid"][:, sl])) and np.all(out["iters"][sl] == 0)
        assert np.all(np.isnan(out["cost"][sl])) and out["best"][s] == -1
    # scene 2: only the goal with the non-finite target is marked
    g2 = off[2] + bad_goal
    assert np.all(np.isnan(out["c"][..., g2])) and np.all(np.isnan(out["resid"][:, g2]))
    assert out["iters"][g2] == 0 and np.isnan(out["cost"][g2])
    rest = [off[2] + g for g in keep]
    ref_rest = slice(ref_off[1], ref_off[2])
    for k in ("c", "lam", "resid", "iters", "cost"):
        assert np.array_equal(out[k][..., rest], ref[k][..., ref_rest], equal_nan=True), k
    assert out["best"][2] != bad_goal
    b_ref = ref["best"][1]
    assert out["best"][2] == (keep[b_ref] if b_ref >= 0 else -1)
    assert out["best"][0] == ref["best"][0]


@pytest.mark.parametrize("kernel,waves,precision", CASES)
def test_obstacle_range_before_the_array_marks_its_scene(T, kernel, waves, precision):
    """A scene whose obstacle range starts before the obstacle array (its count
    still that of its shape) is marked like one of unknown shape: NaN residuals,
    a NaN cost with the collision post-check, no best goal; its obstacles are never
    read. The next scene is solved exactly as on its own."""
    import torch
    s0, s1 = S.make_scene(41, 12, 12), S.make_scene(42, 12, 12)
    batch = S.Batch([s0, s1])
    all_obs = batch.obs()
    solver = T.Solver(PARAMS, batch.shapes())
    solver.set_tile(kernel, 16, True, waves)
    db = T.DeviceBatch.from_batch(batch)
    # ranges [-6, 6) and [6, 18): both of the shape's 12 obstacles, the first out of the array
    db.obs_off.copy_(torch.tensor([-6, 6, 18], dtype=torch.int32, device="cuda"))
    st = T.DeviceState.empty(batch.n_goals)
    solver.solve(db, st, ITERS, kernel=kernel, precision=precision)
    v_ref = torch.tensor([float(s.ego[2]) for s in batch.scenes], device="cuda")
    cost = torch.zeros(batch.n_goals, device="cuda")
    best = torch.zeros(batch.n_scenes, device="cuda", dtype=torch.int32)
    solver.score(db, st, v_ref, cost, best, clear_min=1.0)
    torch.cuda.synchronize()
    resid, c, cost, best = st.resid.cpu().numpy(), st.c.cpu().numpy(), cost.cpu().numpy(), best.cpu().numpy()
    solver.close()
    n0 = s0.goals.shape[0]
    assert np.all(np.isnan(resid[:, :n0])) and np.all(np.isnan(cost[:n0])) and best[0] == -1

    ref_scene = dataclasses.replace(s1, obs=all_obs[6:18].copy())
    solver = T.Solver(PARAMS, S.Batch([ref_scene]).shapes())
    solver.set_tile(kernel, 16, True, waves)
    rdb = T.DeviceBatch.from_batch(S.Batch([ref_scene]))
    rst = T.DeviceState.empty(ref_scene.goals.shape[0])
    solver.solve(rdb, rst, ITERS, kernel=kernel, precision=precision)
    rcost = torch.zeros(ref_scene.goals.shape[0], device="cuda")
    rbest = torch.zeros(1, device="cuda", dtype=torch.int32)
    solver.score(rdb, rst, v_ref[1:], rcost, rbest, clear_min=1.0)
    torch.cuda.synchronize()
    assert np.array_equal(c[..., n0:], rst.c.cpu().numpy(), equal_nan=True)
    assert np.array_equal(resid[:, n0:], rst.resid.cpu().numpy(), equal_nan=True)
    assert np.array_equal(cost[n0:], rcost.cpu().numpy(), equal_nan=True)
    assert best[1] == int(rbest.item())
    solver.close()
