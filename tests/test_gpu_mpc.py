"""Closed loop on the GPU: one cycle against the oracle (goal template, IDM
traffic, the ego one sample into its chosen trajectory, re-centring, collision
count), then a short batched run."""
import numpy as np
import pytest

from oracle import traj_oracle as O
from tests.test_gpu_parity import PARAMS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_10392_amd import mpc
    return mpc


def test_one_cycle_matches_the_oracle(M):
    import torch
    cl = M.ClosedLoop(range(40, 72), iters=30)
    # perturb the start so the ego is not at rest in its lane and traffic is mixed
    rng = np.random.default_rng(3)
    ego = cl.db.ego.cpu().numpy()
    ego[:, 3] = rng.normal(0, 0.3, ego.shape[0])
    ego[:, 1] = rng.normal(0, 0.5, ego.shape[0])
    cl.db.ego.copy_(torch.from_numpy(ego))
    ego0, obs0 = cl.db.ego.cpu().numpy().astype(np.float64), cl.db.obs.cpu().numpy().astype(np.float64)
    cl.goals()
    goals = cl.db.goal.cpu().numpy()
    cl.plan()
    torch.cuda.synchronize()
    c = cl.st.c.cpu().numpy().astype(np.float64)
    best = cl.best.cpu().numpy()
    cl.step()
    torch.cuda.synchronize()
    ego1, obs1 = cl.db.ego.cpu().numpy(), cl.db.obs.cpu().numpy()
    tr, col = cl.travelled.cpu().numpy(), cl.collisions.cpu().numpy()
    prob = O.Problem(100, 10.0, 10, PARAMS)
    off, ooff = cl.batch.goal_off(), cl.batch.obs_off()
    v_des = cl.v_des.cpu().numpy().astype(np.float64)
    p = dict(O.IDM_DEFAULTS)
    dt = prob.t[1]
    for s in range(cl.batch.n_scenes):
        g_ref = O.mpc_goals(ego0[s])
        assert np.allclose(goals[off[s]:off[s + 1]], g_ref, rtol=1e-6, atol=1e-4), s
        o_ref = O.idm_step(obs0[ooff[s]:ooff[s + 1]], ego0[s], v_des[ooff[s]:ooff[s + 1]], dt, p)
        assert best[s] >= 0
        g = off[s] + best[s]
        e_ref = O.ego_advance(prob, c[0, :, g], c[1, :, g], c[2, :, g])
        shift = e_ref[0]
        assert abs(tr[s] - shift) <= 1e-4 * max(1.0, abs(shift)), s
        e_ref[0] = 0.0
        assert np.allclose(ego1[s], e_ref, rtol=1e-4, atol=1e-4), (s, ego1[s], e_ref)
        o_ref[:, 0] -= shift
        assert np.allclose(obs1[ooff[s]:ooff[s + 1]], o_ref, rtol=1e-5, atol=1e-4), s
        dx = o_ref[:, 0] / PARAMS["a"]
        dy = (o_ref[:, 1] - e_ref[1]) / PARAMS["b"]
        assert col[s] == int(np.sum(dx * dx + dy * dy < 1.0)), s


def test_batched_closed_loop_run(M):
    import torch
    cl = M.ClosedLoop(range(64), iters=100)
    for _ in range(40):
        cl.cycle()
    torch.cuda.synchronize()
    m = cl.metrics(40)
    print(m)
    assert np.all(np.isfinite(cl.db.ego.cpu().numpy())) and np.all(np.isfinite(cl.db.obs.cpu().numpy()))
    assert m["mean_speed"] > 5.0
    assert 0 < m["mean_iterations_per_cycle"] <= 100


def test_shift_matches_the_oracle(M):
    """traj_mpc_shift (every goal's coefficients advanced by one period, the frame
    moved back by the ego's advance; multipliers untouched) against the oracle's
    collocation form."""
    import torch
    cl = M.ClosedLoop(range(3), iters=5)
    rng = np.random.default_rng(11)
    G = cl.batch.n_goals
    c = rng.normal(size=(3, 11, G)) * np.array([80.0, 4.0, 0.1])[:, None, None]
    cl.st.c.copy_(torch.tensor(c, dtype=torch.float32).reshape(cl.st.c.shape))
    cl.st.lam.copy_(torch.tensor(rng.normal(size=(3, 11, G)), dtype=torch.float32).reshape(cl.st.lam.shape))
    lam0 = cl.st.lam.clone()
    dx = np.array([1.3, 0.0, 2.1])
    cl.shift.copy_(torch.tensor(dx, dtype=torch.float32))
    c = cl.st.c.cpu().numpy().astype(np.float64).reshape(3, 11, G)
    cl.shift_state()
    torch.cuda.synchronize()
    c1 = cl.st.c.cpu().numpy().astype(np.float64).reshape(3, 11, G)
    assert torch.equal(cl.st.lam, lam0)
    off = cl.batch.goal_off()
    u0 = 1.0 / (cl.shape[0] - 1)
    Smat = np.abs(O.shift_matrix(11, u0))
    for s in range(3):
        sl = slice(off[s], off[s + 1])
        rc = O.shift_solution(c[:, :, sl], u0, dx[s])
        # FP32 products of FP32-rounded entries: a few ulp of the absolute sums
        bc = 4e-7 * (np.einsum("ik,akg->aig", Smat, np.abs(c[:, :, sl])) + np.array([dx[s], 0, 0])[:, None, None])
        assert np.all(np.abs(c1[:, :, sl] - rc) <= bc + 1e-30), s


@pytest.mark.parametrize("warm", ["previous", "shifted"])
def test_closed_loop_warm_starts_run(M, warm):
    import torch
    cl = M.ClosedLoop(range(64), iters=100, warm=warm, clear_min=1.0)
    for _ in range(20):
        cl.cycle()
    torch.cuda.synchronize()
    m = cl.metrics(20)
    print(warm, m)
    assert np.all(np.isfinite(cl.db.ego.cpu().numpy()))
    assert m["mean_speed"] > 5.0
    assert 0 < m["mean_iterations_per_cycle"] <= 100


def test_closed_loop_with_the_split_bf16_solver(M):
    """The same 64 cold-started episodes in FP32 and with the split-BF16 solver
    over 10 cycles: the plans take the same iterations to the stopping rule and
    the loop's statistics agree (the solver forms differ by rounding only)."""
    import torch
    ms = {}
    for precision in ("fp32", "bf16x3"):
        cl = M.ClosedLoop(range(64), iters=100, warm="cold", clear_min=1.0, precision=precision)
        for _ in range(10):
            cl.cycle()
        torch.cuda.synchronize()
        assert np.all(np.isfinite(cl.db.ego.cpu().numpy()))
        ms[precision] = cl.metrics(10)
        print(precision, ms[precision])
    a, b = ms["fp32"], ms["bf16x3"]
    assert abs(a["mean_iterations_per_cycle"] - b["mean_iterations_per_cycle"]) <= 0.02 * a["mean_iterations_per_cycle"]
    assert abs(a["mean_speed"] - b["mean_speed"]) <= 0.01 * a["mean_speed"]
    assert a["episodes_with_collision"] == b["episodes_with_collision"]


def test_right_lane_goals_match_the_oracle(M):
    import torch
    cl = M.ClosedLoop(range(5), iters=5, scenario="right_lane", v_max=25.0)
    rng = np.random.default_rng(4)
    ego = cl.db.ego.cpu().numpy()
    ego[:, 0] = rng.normal(0, 2.0, ego.shape[0])
    cl.db.ego.copy_(torch.from_numpy(ego))
    cl.goals()
    goals = cl.db.goal.cpu().numpy()
    off = cl.batch.goal_off()
    for s in range(cl.batch.n_scenes):
        ref = O.right_lane_goals(ego[s].astype(np.float64), 25.0)
        assert np.allclose(goals[off[s]:off[s + 1]], ref, rtol=1e-6, atol=1e-4), s


def test_right_lane_closed_loop_run(M):
    import torch
    cl = M.ClosedLoop(range(64), iters=100, warm="shifted", clear_min=1.0, scenario="right_lane", v_max=25.0)
    for _ in range(20):
        cl.cycle()
    torch.cuda.synchronize()
    m = cl.metrics(20)
    print(m)
    assert np.all(np.isfinite(cl.db.ego.cpu().numpy()))
    assert m["mean_speed"] > 5.0 and np.isfinite(m["right_lane_distance_mean"])


def test_brake_fallback_matches_the_oracle(M):
    """Episodes whose goals are all filtered (best < 0) brake along the road and
    stop moving sideways; the others advance along their plans."""
    import torch
    cl = M.ClosedLoop(range(12), iters=10)
    rng = np.random.default_rng(6)
    ego = cl.db.ego.cpu().numpy()
    ego[:, 3] = rng.normal(0, 0.5, ego.shape[0])
    ego[:, 1] = rng.normal(0, 0.8, ego.shape[0])
    ego[5, 2] = 0.1  # stops within the period
    cl.db.ego.copy_(torch.from_numpy(ego))
    cl.goals()
    cl.plan()
    best = cl.best.cpu().numpy()
    forced = [0, 3, 5, 11]
    best[forced] = -1
    cl.best.copy_(torch.from_numpy(best))
    ego0 = cl.db.ego.cpu().numpy().astype(np.float64)
    fb0 = cl.fallbacks.cpu().numpy().copy()
    cl.step()
    torch.cuda.synchronize()
    ego1, tr = cl.db.ego.cpu().numpy(), cl.travelled.cpu().numpy()
    dt = cl.period
    for s in forced:
        ref = O.ego_brake(ego0[s], 4.0, dt)
        assert abs(tr[s] - ref[0]) <= 1e-5 * max(1.0, ref[0]), s
        ref[0] = 0.0
        assert np.allclose(ego1[s], ref, rtol=1e-5, atol=1e-5), (s, ego1[s], ref)
    fb = cl.fallbacks.cpu().numpy()
    assert np.array_equal(fb - fb0, np.isin(np.arange(12), forced).astype(fb.dtype))
