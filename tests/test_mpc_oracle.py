"""Pins of the closed-loop oracle: IDM closed forms (free road, equilibrium gap,
standstill), goal placement, and the ego's state one sample into a known
trajectory."""
import numpy as np

from oracle import traj_oracle as O
from paper_2109_10392_amd import scenes as S

P = O.IDM_DEFAULTS


def test_idm_free_road_equilibrium_and_standstill():
    v, v0 = 10.0, 15.0
    assert abs(O.idm_accel(v, v0, None, 0.0, P) - P["a"] * (1 - (v / v0) ** 4)) < 1e-15
    # a follower at the equilibrium gap of its speed, same speed as its leader, does not accelerate
    s_e = (P["s0"] + v * P["T"]) / np.sqrt(1 - (v / v0) ** 4)
    assert abs(O.idm_accel(v, v0, s_e, 0.0, P)) < 1e-12
    # standing still at the minimum gap behind a stopped leader
    assert abs(O.idm_accel(0.0, v0, P["s0"], 0.0, P)) < 1e-15
    # closing in brakes harder than keeping pace
    assert O.idm_accel(v, v0, 15.0, 3.0, P) < O.idm_accel(v, v0, 15.0, 0.0, P) < 0  # gap below s* = 17 m


def test_idm_step_follows_the_lane_leader_only():
    ego = np.array([0.0, 0.0, 12.0, 0.0, 0, 0, 0, 0])
    obs = np.array([[-30.0, 0.0, 14.0, 0.0],   # behind the ego in its lane: ego leads
                    [40.0, 3.5, 8.0, 0.0],     # free road (nothing ahead in its lane)
                    [25.0, 3.5, 9.0, 0.0]])    # led by obstacle 1
    v_des = np.array([15.0, 10.0, 12.0])
    dt = 0.1
    out = O.idm_step(obs, ego, v_des, dt, P)
    a0 = O.idm_accel(14.0, 15.0, 30.0 - P["length"], 2.0, P)
    a1 = O.idm_accel(8.0, 10.0, None, 0.0, P)
    a2 = O.idm_accel(9.0, 12.0, 15.0 - P["length"], 1.0, P)
    for j, a in enumerate((a0, a1, a2)):
        v_new = max(obs[j, 2] + a * dt, 0.0)
        assert abs(out[j, 2] - v_new) < 1e-12
        assert abs(out[j, 0] - (obs[j, 0] + 0.5 * (obs[j, 2] + v_new) * dt)) < 1e-12
    assert np.array_equal(out[:, 1], obs[:, 1])


def test_goals_and_ego_advance():
    g = O.mpc_goals(np.array([3.0, 0.0, 20.0, 0.0, 0, 0, 0, 0]))
    assert g.shape == (256, 2) and np.allclose(g[0], [3.0 + 160.0, -3.5]) and np.allclose(g[255], [3.0 + 240.0, 7.0])
    prob = O.Problem(100, 10.0, 0, S.DEFAULT_PARAMS)
    k = np.arange(11)
    v, a = 12.0, 0.5
    c_x = v * 10.0 * k / 10 + 0.5 * a * 100.0 * k * (k - 1) / 90
    t1 = prob.t[1]
    e = O.ego_advance(prob, c_x, np.zeros(11), np.zeros(11))
    assert np.allclose(e, [v * t1 + 0.5 * a * t1 ** 2, 0, v + a * t1, 0, a, 0, 0, 0], atol=1e-12)
