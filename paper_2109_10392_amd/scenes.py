"""Seeded synthetic highway scenes: the inputs both the HIP path and the oracle consume.

This module holds no arithmetic of the optimizer itself. It only draws the
quantities the paper's problem statement takes as given (Sec. III intro and
Sec. III-F): the ego state, obstacle ellipses with a constant-velocity
prediction (position and velocity at t = 0), and goal positions at the end
of the horizon. Everything is drawn from numpy's PCG64 in a fixed order so
that a (seed, recipe) pair always yields the same scene.

Recipe (the paper's data sets -- IDM traffic and NGSIM -- are not available;
these draws stand in for them with the shapes the workloads name):

* road: ``n_lanes`` straight lanes 3.5 m wide, lane k centred at
  ``(k - (n_lanes - 1) // 2) * 3.5`` so the ego starts on y = 0;
* ego: at the origin, heading 0, speed v0 ~ U(10, 20) m/s, no acceleration;
* obstacles: lane ~ U{0..n_lanes-1}, x ~ U(0, 80) m, vx ~ U(5, 15) m/s,
  vy = 0 (cars move parallel to the centre-line); an obstacle whose ellipse
  (a = 5.6, b = 3.1) contains the ego start is drawn again;
* goals: goal i targets lane ``i mod n_lanes`` at x_f = v0 * t_f * U(0.8, 1.2).

Closed-loop traffic (``make_traffic_scene``) must also be drivable by the
traffic model, so vehicles keep headways: obstacles are drawn as above but with
x ~ U(-40, 120) m (followers behind the ego too), and a draw is rejected unless,
against every vehicle already placed in its lane (the ego included), the
bumper-to-bumper gap (centre distance less 4.5 m) is at least
2 + 1.5 v_rear + max(0, v_rear - v_front)^2 / 6 m (a standstill gap, a 1.5 s
headway and the distance to shed the closing speed at 3 m/s^2).

Arrays are float32 (what the device path consumes); the oracle promotes them
to float64 itself.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

LANE_WIDTH = 3.5
ELLIPSE_A = 5.6  # inflated semi-axes used in the paper's experiments (Sec. IV)
ELLIPSE_B = 3.1

# Ego state layout shared by both sides: x0, y0, vx0, vy0, ax0, ay0, psi0, psidot0.
EGO_FIELDS = 8


def lane_centres(n_lanes: int) -> np.ndarray:
    k = np.arange(n_lanes, dtype=np.float64)
    return (k - (n_lanes - 1) // 2) * LANE_WIDTH


@dataclass
class Scene:
    """One scene: ego, obstacles and goals (float32 arrays)."""

    ego: np.ndarray      # [8]
    obs: np.ndarray      # [m, 4]  x, y, vx, vy at t = 0
    goals: np.ndarray    # [B, 2]  x_f, y_f
    n_time: int
    t_f: float
    n_lanes: int
    seed: int


@dataclass
class Batch:
    """Several scenes concatenated (goal index fastest, scene-major)."""

    scenes: list = field(default_factory=list)

    @property
    def n_scenes(self) -> int:
        return len(self.scenes)

    @property
    def n_goals(self) -> int:
        return int(sum(s.goals.shape[0] for s in self.scenes))

    def goal_off(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum([s.goals.shape[0] for s in self.scenes])]).astype(np.int32)

    def obs_off(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum([s.obs.shape[0] for s in self.scenes])]).astype(np.int32)

    def ego(self) -> np.ndarray:
        return np.stack([s.ego for s in self.scenes]).astype(np.float32)

    def obs(self) -> np.ndarray:
        parts = [s.obs for s in self.scenes]
        if not parts or sum(p.shape[0] for p in parts) == 0:
            return np.zeros((0, 4), np.float32)
        return np.concatenate(parts).astype(np.float32)

    def goals(self) -> np.ndarray:
        return np.concatenate([s.goals for s in self.scenes]).astype(np.float32)

    def shapes(self) -> list:
        """Distinct (n_time, t_f, n_obs) triples in first-seen order."""
        out = []
        for s in self.scenes:
            key = (s.n_time, float(s.t_f), int(s.obs.shape[0]))
            if key not in out:
                out.append(key)
        return out

    def shape_id(self) -> np.ndarray:
        shapes = self.shapes()
        return np.array([shapes.index((s.n_time, float(s.t_f), int(s.obs.shape[0])))
                         for s in self.scenes], np.int32)


def make_scene(seed: int, n_goals: int, n_obs: int, n_lanes: int = 4,
               n_time: int = 100, t_f: float = 10.0, x_range=(0.0, 80.0),
               v0_range=(10.0, 20.0), vobs_range=(5.0, 15.0)) -> Scene:
    """Draw one scene. Draw order: v0, then per obstacle (lane, x, vx), then goal scales."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = lane_centres(n_lanes)
    v0 = rng.uniform(*v0_range)
    obs = np.zeros((n_obs, 4), np.float64)
    for j in range(n_obs):
        while True:
            lane = int(rng.integers(0, n_lanes))
            x = rng.uniform(*x_range)
            vx = rng.uniform(*vobs_range)
            y = centres[lane]
            # keep the ego start outside every obstacle ellipse
            if (x / ELLIPSE_A) ** 2 + (y / ELLIPSE_B) ** 2 >= 1.0:
                break
        obs[j] = (x, y, vx, 0.0)
    scale = rng.uniform(0.8, 1.2, size=n_goals)
    goals = np.zeros((n_goals, 2), np.float64)
    for i in range(n_goals):
        goals[i, 0] = v0 * t_f * scale[i]
        goals[i, 1] = centres[i % n_lanes]
    ego = np.array([0.0, 0.0, v0, 0.0, 0.0, 0.0, 0.0, 0.0])
    return Scene(ego=ego.astype(np.float32), obs=obs.astype(np.float32),
                 goals=goals.astype(np.float32), n_time=n_time, t_f=t_f,
                 n_lanes=n_lanes, seed=seed)


def template_goals(v0: float, t_f: float, n_lanes: int = 4, per_lane: int = 64) -> np.ndarray:
    """Fixed goal slots for the learned warm start: lanes x linspace(0.8, 1.2) * v0 * t_f, lane-major."""
    centres = lane_centres(n_lanes)
    fr = np.linspace(0.8, 1.2, per_lane)
    goals = np.zeros((n_lanes * per_lane, 2), np.float64)
    for lane in range(n_lanes):
        goals[lane * per_lane:(lane + 1) * per_lane, 0] = v0 * t_f * fr
        goals[lane * per_lane:(lane + 1) * per_lane, 1] = centres[lane]
    return goals.astype(np.float32)


def make_template_scene(seed: int, n_obs: int = 10, n_lanes: int = 4, n_time: int = 100,
                        t_f: float = 10.0, per_lane: int = 64) -> Scene:
    """A scene whose goals are the deterministic warm-start template (same draws as make_scene)."""
    s = make_scene(seed, n_goals=1, n_obs=n_obs, n_lanes=n_lanes, n_time=n_time, t_f=t_f)
    s.goals = template_goals(float(s.ego[2]), t_f, n_lanes, per_lane)
    return s


def make_traffic_scene(seed: int, n_obs: int = 10, n_lanes: int = 4, n_time: int = 100, t_f: float = 10.0,
                       per_lane: int = 64, x_range=(-40.0, 120.0), v0_range=(10.0, 20.0),
                       vobs_range=(5.0, 15.0)) -> Scene:
    """A closed-loop start: headway-respecting traffic around the ego (module recipe),
    goals = the template. Draw order: v0, then per obstacle attempt (lane, x, vx)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = lane_centres(n_lanes)
    v0 = rng.uniform(*v0_range)
    placed = [(0.0, 0.0, v0)]  # (x, y, v), the ego first
    obs = np.zeros((n_obs, 4), np.float64)
    for j in range(n_obs):
        for _attempt in range(10000):
            lane = int(rng.integers(0, n_lanes))
            x = rng.uniform(*x_range)
            vx = rng.uniform(*vobs_range)
            y = centres[lane]
            if (x / ELLIPSE_A) ** 2 + (y / ELLIPSE_B) ** 2 < 1.0:
                continue
            ok = True
            for (px, py, pv) in placed:
                if abs(py - y) >= LANE_WIDTH / 2:
                    continue
                (rx, rv), (fx, fv) = ((x, vx), (px, pv)) if x < px else ((px, pv), (x, vx))
                need = 2.0 + 1.5 * rv + max(0.0, rv - fv) ** 2 / 6.0
                if fx - rx - 4.5 < need:
                    ok = False
                    break
            if ok:
                break
        else:
            raise RuntimeError(f"traffic scene {seed}: no room for obstacle {j}")
        placed.append((x, y, vx))
        obs[j] = (x, y, vx, 0.0)
    ego = np.array([0.0, 0.0, v0, 0.0, 0.0, 0.0, 0.0, 0.0])
    return Scene(ego=ego.astype(np.float32), obs=obs.astype(np.float32),
                 goals=template_goals(v0, t_f, n_lanes, per_lane).astype(np.float32), n_time=n_time, t_f=t_f,
                 n_lanes=n_lanes, seed=seed)


# ---------------------------------------------------------------- workloads
def workload_small(seed: int) -> Batch:
    """1 scene x 11 goals, 10 obstacles, 4 lanes, T = 100 over 10 s."""
    return Batch([make_scene(seed, n_goals=11, n_obs=10, n_lanes=4, n_time=100, t_f=10.0)])


# Obstacle placement range of the dense scene's density-sensitivity variant: the
# 11-goal scenes' density (10 obstacles over 4 lanes x 80 m) with 50 obstacles on
# 6 lanes, 80 * (50 / 10) * (4 / 6) m.
SPARSE_DENSE_RANGE = (0.0, 80.0 * (50 / 10) * (4 / 6))


def workload_dense(seed: int, x_range=(0.0, 80.0)) -> Batch:
    """1 scene x 1024 goals, 50 obstacles, 6 lanes, T = 100 over 10 s; obstacles
    placed over x_range (the default is the 11-goal scenes' 0-80 m, so five times
    their density per lane x 4/6; SPARSE_DENSE_RANGE keeps their density)."""
    return Batch([make_scene(seed, n_goals=1024, n_obs=50, n_lanes=6, n_time=100, t_f=10.0, x_range=x_range)])


def workload_uneven(seed: int = 0, n_scenes: int = 512, lo: int = 16, hi: int = 1024) -> Batch:
    """Many scenes: goals log-uniform in [lo, hi], obstacles U{4..64}, T in {50, 100, 150}, t_f = T/10."""
    rng = np.random.Generator(np.random.PCG64(seed))
    scenes = []
    for s in range(n_scenes):
        g = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        m = int(rng.integers(4, 65))
        T = int(rng.choice([50, 100, 150]))
        sub_seed = int(rng.integers(0, 2 ** 31 - 1))
        scenes.append(make_scene(sub_seed, n_goals=g, n_obs=m, n_lanes=6, n_time=T, t_f=T / 10.0))
    return Batch(scenes)


# Solver constants the paper leaves open (rho, bounds); a and b are the paper's.
DEFAULT_PARAMS = dict(n_coef=11, rho=1.0, a=ELLIPSE_A, b=ELLIPSE_B, v_min=0.1, v_max=30.0,
                      a_max=4.0, psi_max=13.0 * math.pi / 180.0)
