"""Pins of the road-frame oracle (Sec. III, assumption 1) against closed forms:
a straight road is a rotation and a translation; on a circular road of radius R
a point at radius r and polar angle phi has s = R phi, d = +-(R - r), and
uniform circular motion at speed v has s' = v R / r with d' = s'' = d'' = 0 and
no heading rate relative to the road."""
import math

import numpy as np

from oracle.frenet_oracle import RoadOracle


def test_straight_road_is_a_rigid_motion():
    th0, x0, y0 = 0.3, 5.0, -2.0
    R = RoadOracle([(100.0, 0.0)], x0, y0, th0)
    T = np.array([math.cos(th0), math.sin(th0)])
    N = np.array([-math.sin(th0), math.cos(th0)])
    for s, d in [(0.0, 0.0), (37.5, 3.5), (99.0, -7.0), (-20.0, 1.0), (140.0, 2.0)]:
        p = np.array([x0, y0]) + s * T + d * N
        assert np.allclose(R.to_global(s, d), [p[0], p[1], th0], atol=1e-10)
        ss, dd = R.project(*p)
        assert abs(ss - s) < 1e-7 and abs(dd - d) < 1e-9
    v, a = np.array([12.0, -1.0]), np.array([0.5, 0.2])
    p = np.array([x0, y0]) + 40 * T + 1.5 * N
    out = R.from_global([p[0], p[1], v[0], v[1], a[0], a[1], 0.4, 0.02])
    assert np.allclose(out[2:4], [v @ T, v @ N], atol=1e-6)
    assert np.allclose(out[4:6], [a @ T, a @ N], atol=1e-4)
    assert np.allclose(out[6:8], [0.4 - th0, 0.02], atol=1e-6)


def test_circular_road_closed_forms():
    for k in (1 / 100.0, -1 / 80.0):
        Rr = 1 / abs(k)
        road = RoadOracle([(120.0, k)], 0.0, 0.0, 0.0)
        cy = 1 / k  # centre of curvature (0, 1/k)
        for phi, r in [(0.2, Rr - 3.5), (0.9, Rr + 2.0), (1.1, Rr)]:
            # point at angle phi along the arc from the start, radius r from the centre
            ang = -math.pi / 2 + phi if k > 0 else math.pi / 2 - phi
            p = np.array([r * math.cos(ang), cy + r * math.sin(ang)])
            s, d = road.project(*p)
            assert abs(s - Rr * phi) < 1e-7
            assert abs(d - (Rr - r if k > 0 else r - Rr)) < 1e-9
            g = road.to_global(s, d)
            assert np.allclose(g[:2], p, atol=1e-9) and abs(g[2] - k * Rr * phi) < 1e-12
            # uniform circular motion at radius r along the road at speed v
            v = 15.0
            tdir = np.array([-math.sin(ang), math.cos(ang)]) * (1 if k > 0 else -1)
            acc = -(p - np.array([0.0, cy])) / r * v * v / r
            psi = k * Rr * phi
            out = road.from_global([p[0], p[1], *(v * tdir), *acc, psi, math.copysign(v / r, k)])
            assert abs(out[2] - v * Rr / r) < 1e-6, out
            assert abs(out[3]) < 1e-6 and abs(out[4]) < 2e-4 and abs(out[5]) < 2e-4, out
            assert abs(out[6]) < 1e-9 and abs(out[7]) < 1e-6, out


def test_round_trip_on_a_mixed_road():
    road = RoadOracle([(50, 0.0), (100, 1 / 80), (30, 0.0), (80, -1 / 60), (40, 0.0)], 10.0, 20.0, -0.2)
    rng = np.random.default_rng(0)
    for _ in range(25):
        s, d = rng.uniform(-20, road.length + 20), rng.uniform(-8, 8)
        g = road.to_global(s, d)
        ss, dd = road.project(g[0], g[1])
        assert abs(ss - s) < 1e-6 and abs(dd - d) < 1e-8, (s, d, ss, dd)


def test_lane_keeping_trajectory_maps_to_the_lane():
    k = 1 / 150.0
    road = RoadOracle([(300.0, k)], 0.0, 0.0, 0.0)
    d0, v = -3.5, 20.0
    times = np.linspace(0.5, 10, 11)  # away from the road's start, where the curvature jumps
    out = road.trajectory_to_global(lambda t: v * t, lambda t: d0, times)
    for i, t in enumerate(times):
        # on the circle of radius R - d0 around (0, 1/k), heading = the road's
        assert abs(math.hypot(out[i, 0], out[i, 1] - 1 / k) - (1 / k - d0)) < 1e-7
        assert abs(out[i, 2] - k * v * t) < 1e-7
