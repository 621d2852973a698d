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


def test_shift_closed_forms():
    """The warm start of the next cycle (the solution advanced by one period) on
    polynomials whose shifted Bernstein coefficients are known in closed form."""
    k = np.arange(11)
    u0 = 1.0 / 99.0
    # no shift: identity
    c = np.random.default_rng(0).normal(size=(3, 11, 5))
    assert np.allclose(O.shift_solution(c, 0.0, 0.0), c, atol=1e-12)
    # a line x = x0 + L tau has coefficients x0 + L k/10 (linear precision);
    # advanced by u0 and moved back by dx: x0 + L u0 - dx + L k/10
    x0, L, dx = 2.0, 150.0, 1.7
    c = np.zeros((3, 11, 1))
    c[0, :, 0] = x0 + L * k / 10
    c1 = O.shift_solution(c, u0, dx)
    assert np.allclose(c1[0, :, 0], x0 + L * u0 - dx + L * k / 10, atol=1e-11)
    assert np.allclose(c1[1:], 0.0, atol=1e-12)
    # y = tau^2 has coefficients k(k-1)/90; (u + u0)^2 = u^2 + 2 u0 u + u0^2
    c = np.zeros((3, 11, 1))
    c[1, :, 0] = k * (k - 1) / 90.0
    c1 = O.shift_solution(c, u0, 0.0)
    assert np.allclose(c1[1, :, 0], k * (k - 1) / 90.0 + 2 * u0 * k / 10 + u0 ** 2, atol=1e-12)


def test_shift_keeps_the_trajectory():
    rng = np.random.default_rng(5)
    c = rng.normal(size=(3, 11, 4)) * 10
    u0, dx = 0.05, 0.8
    c1 = O.shift_solution(c, u0, dx)

    # evaluated by de Casteljau's algorithm (also valid outside [0, 1]): the new
    # polynomial at u is the old one at u0 + u, less dx for x
    def casteljau(coef, u):
        b = list(coef)
        while len(b) > 1:
            b = [(1 - u) * b[i] + u * b[i + 1] for i in range(len(b) - 1)]
        return b[0]
    for u in (0.0, 0.3, 0.99, 1.0):
        for g in range(4):
            for a in range(3):
                want = casteljau(c[a, :, g], u0 + u) - (dx if a == 0 else 0.0)
                assert abs(casteljau(c1[a, :, g], u) - want) < 1e-9
    # advancing by u0 and then by -u0 returns the start
    assert np.allclose(O.shift_solution(c1, -u0, -dx), c, atol=1e-9)


def test_traffic_scenes_keep_headways():
    """The closed-loop starts: in every lane, each follower has at least the
    standstill gap, a 1.5 s headway and room to shed its closing speed at 3 m/s^2."""
    for seed in range(200):
        sc = S.make_traffic_scene(seed)
        veh = [(0.0, 0.0, float(sc.ego[2]))] + [(float(o[0]), float(o[1]), float(o[2])) for o in sc.obs]
        assert len(veh) == 11
        for i in range(len(veh)):
            for j in range(len(veh)):
                (xr, yr, vr), (xf, yf, vf) = veh[i], veh[j]
                if i == j or abs(yr - yf) >= S.LANE_WIDTH / 2 or xr > xf:
                    continue
                need = 2.0 + 1.5 * vr + max(0.0, vr - vf) ** 2 / 6.0
                assert xf - xr - 4.5 >= need - 1e-4, (seed, i, j)
        assert sc.goals.shape == (256, 2)


def test_right_lane_sampler_counts_and_distances():
    """Sec. III-F: about 60% of the goals on the right lane at different
    distances, the rest over the other lanes at v_max t_f."""
    ego = np.array([1.0, 0.0, 15.0, 0.0, 0, 0, 0, 0])
    g = O.right_lane_goals(ego, 25.0)
    assert g.shape == (256, 2)
    right = g[:, 1] == -3.5
    assert right.sum() == 154 and abs(right.mean() - 0.6) < 0.01
    assert np.allclose(np.sort(g[right, 0]), 1.0 + 250.0 * np.linspace(0.2, 1.0, 154))
    for y in (0.0, 3.5, 7.0):
        sel = g[:, 1] == y
        assert sel.sum() in (34, 35)
        assert np.all((g[sel, 0] >= 1.0 + 0.9 * 250.0 - 1e-9) & (g[sel, 0] <= 1.0 + 250.0 + 1e-9))
    assert len({tuple(r) for r in g}) == 256


def test_brake_fallback():
    dt, a = 0.1, 4.0
    e = O.ego_brake([0.0, 1.2, 15.0, 0.8, 0.3, -0.2, 0.05, 0.01], a, dt)
    assert np.allclose(e, [0.5 * (15.0 + 14.6) * dt, 1.2, 14.6, 0, -4.0, 0, 0, 0])
    # at standstill it stays put; a speed below a_max dt stops within the period
    assert np.allclose(O.ego_brake([0.0, -3.5, 0.0, 0.0, 0, 0, 0, 0], a, dt), [0, -3.5, 0, 0, 0, 0, 0, 0])
    e = O.ego_brake([0.0, 0.0, 0.2, 0.0, 0, 0, 0, 0], a, dt)
    assert np.allclose(e, [0.5 * 0.2 * dt, 0, 0, 0, -4.0, 0, 0, 0])
