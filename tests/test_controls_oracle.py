"""Pins of the control extraction and collision post-check of the oracle
(closed forms): a heading linear in time steers by arctan(omega h / v); a
longitudinal profile with constant acceleration has v' equal to it; an
obstacle moving with the trajectory at a fixed gap has clearance gap / a."""
import numpy as np

from oracle import traj_oracle as O
from paper_2109_10392_amd import scenes as S

PARAMS = S.DEFAULT_PARAMS


def test_linear_heading_and_constant_acceleration():
    prob = O.Problem(100, 10.0, 0, PARAMS)
    k = np.arange(11)
    v0, a, w, h = 12.0, 0.8, 0.05, 2.5
    # Bernstein coefficients (degree 10 on tau = t/t_f) of t and t^2: t_f k/10, t_f^2 k(k-1)/90
    c_x = v0 * 10.0 * k / 10 + 0.5 * a * 100.0 * k * (k - 1) / 90
    c_y = np.zeros(11)
    c_psi = w * 10.0 * k / 10
    acc, steer, clear = O.controls(prob, np.zeros((0, 4)), c_x, c_y, c_psi, h, 0.1)
    v = v0 + a * prob.t
    assert np.allclose(acc, a, rtol=0, atol=1e-12)
    assert np.allclose(steer, np.arctan(w * h / v), rtol=0, atol=1e-12)
    assert clear == np.inf


def test_clearance_of_an_obstacle_at_a_fixed_gap():
    prob = O.Problem(100, 10.0, 1, PARAMS)
    k = np.arange(11)
    v, gap = 15.0, 9.0
    c_x = v * 10.0 * k / 10
    zeros = np.zeros(11)
    obs = np.array([[gap, 0.0, v, 0.0]])
    _, _, clear = O.controls(prob, obs, c_x, zeros, zeros, 2.5, 0.1)
    assert abs(clear - gap / PARAMS["a"]) < 1e-12
    obs_side = np.array([[0.0, 2.0, v, 0.0]])
    _, _, clear = O.controls(prob, obs_side, c_x, zeros, zeros, 2.5, 0.1)
    assert abs(clear - 2.0 / PARAMS["b"]) < 1e-12 and clear < 1.0  # inside the ellipse: a collision
