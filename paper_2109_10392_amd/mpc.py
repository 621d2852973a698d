"""Closed-loop (receding-horizon) driver: binding of include/traj_mpc.h and a
batched episode runner.

Every cycle, for all episodes at once on the GPU: place the goal template from
the ego's current state (traj_mpc_goals), solve to the stopping rule with at
most `iters` iterations (traj_converge; from the cold start, the previous
cycle's solutions, those advanced by one period (traj_mpc_shift) or the learned
warm start), rank (traj_score, optionally with the collision post-check), then
move the ego one sample into its chosen trajectory and the traffic one period
by IDM (traj_mpc_step). The host only launches.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import scenes as S
from . import traj as T


class MpcParams(ctypes.Structure):
    _fields_ = [("idm_a", ctypes.c_float), ("idm_b", ctypes.c_float), ("idm_s0", ctypes.c_float),
                ("idm_T", ctypes.c_float), ("idm_delta", ctypes.c_float), ("car_length", ctypes.c_float),
                ("lane_width", ctypes.c_float), ("n_lanes", ctypes.c_int32), ("per_lane", ctypes.c_int32),
                ("goal_v_floor", ctypes.c_float), ("sampler", ctypes.c_int32), ("v_max", ctypes.c_float)]


class EpisodesC(ctypes.Structure):
    _fields_ = [("ego", ctypes.c_void_p), ("obs", ctypes.c_void_p), ("goal", ctypes.c_void_p),
                ("v_des", ctypes.c_void_p), ("obs_next", ctypes.c_void_p), ("travelled", ctypes.c_void_p),
                ("collisions", ctypes.c_void_p), ("fallbacks", ctypes.c_void_p), ("shift", ctypes.c_void_p)]


# IDM parameters (Treiber, Hennecke and Helbing 2000: typical highway values)
IDM = dict(idm_a=1.0, idm_b=1.5, idm_s0=2.0, idm_T=1.5, idm_delta=4.0, car_length=4.5, lane_width=3.5)


def params(n_lanes=4, per_lane=64, goal_v_floor=5.0, sampler=0, v_max=25.0, **over):
    p = dict(IDM, **over)
    return MpcParams(p["idm_a"], p["idm_b"], p["idm_s0"], p["idm_T"], p["idm_delta"], p["car_length"],
                     p["lane_width"], n_lanes, per_lane, goal_v_floor, sampler, v_max)


def _bind():
    L = T.lib()
    if getattr(L, "_mpc_bound", False):
        return L
    vp, i32 = ctypes.c_void_p, ctypes.c_int
    L.traj_mpc_goals.argtypes = [vp, ctypes.POINTER(T.BatchC), ctypes.POINTER(EpisodesC), ctypes.POINTER(MpcParams),
                                 vp]
    L.traj_mpc_step.argtypes = [vp, ctypes.POINTER(T.BatchC), ctypes.POINTER(T.StateC), vp,
                                ctypes.POINTER(EpisodesC), ctypes.POINTER(MpcParams), i32, vp]
    L.traj_mpc_shift.argtypes = [vp, ctypes.POINTER(T.BatchC), ctypes.POINTER(T.StateC), ctypes.POINTER(EpisodesC),
                                 vp]
    L.traj_mpc_goals.restype = ctypes.c_int
    L.traj_mpc_step.restype = ctypes.c_int
    L.traj_mpc_shift.restype = ctypes.c_int
    L._mpc_bound = True
    return L


class ClosedLoop:
    """Episodes on 4-lane roads with 10 vehicles each (headway-respecting traffic
    around the ego, goals = the template), driven by the planner every cycle."""

    def __init__(self, seeds, tile=("group", 16, True, 1), precision="fp32", iters=100, tol=1e-3, net=None,
                 warm="cold", clear_min=0.0, scenario="cruise", v_max=25.0, w1=1.0, w2=1.0):
        """warm: start of every plan after the first: "cold"; "previous" (the
        previous cycle's iterate of the same goal slot); "shifted" (that iterate
        advanced by one period, traj_mpc_shift); or "learned" (the network `net` =
        (Network, mean, std)). The warm starts keep the cold start as per-goal
        fallback. clear_min: the collision post-check of the ranking (0 = off).
        scenario: "cruise" (template goals, eq. 25 with v_cruise = the initial
        speed) or "right_lane" (the right-lane sampler, eq. 26 with v_max, y_rl =
        the right lane's centre and weights w1, w2)."""
        import torch
        self.L = _bind()
        self.batch = S.Batch([S.make_traffic_scene(int(s)) for s in seeds])
        self.shape = (100, 10.0, 10)
        self.solver = T.Solver(S.DEFAULT_PARAMS, [self.shape])
        self.solver.set_tile(*tile)
        self.db = T.DeviceBatch.from_batch(self.batch, shapes=[self.shape])
        self.st = T.DeviceState.empty(self.batch.n_goals)
        n_s, n_o = self.batch.n_scenes, int(self.batch.obs_off()[-1])
        self.n_obs = n_o
        z = lambda *s, dt=torch.float32: torch.zeros(*s, device="cuda", dtype=dt)
        # IDM desired speed of every vehicle: its initial speed
        self.v_des = self.db.obs[:, 2].clone()
        self.obs_next = z(max(n_o, 1), 4)
        self.travelled, self.collisions, self.fallbacks = z(n_s), z(n_s, dt=torch.int32), z(n_s, dt=torch.int32)
        self.shift = z(n_s)
        if scenario not in ("cruise", "right_lane"):
            raise ValueError(f"unknown scenario {scenario!r}")
        self.scenario, self.kind, self.w1, self.w2 = scenario, int(scenario == "right_lane"), float(w1), float(w2)
        if self.kind == 0:
            self.v_ref = self.db.ego[:, 2].clone()  # cruise speed of the meta-cost: the initial speed
        else:
            self.v_ref = torch.full((n_s,), float(v_max), device="cuda")
        self.y_rl = torch.full((n_s,), float(S.lane_centres(4)[0]), device="cuda")
        self.cost, self.best = z(self.batch.n_goals), z(n_s, dt=torch.int32)
        self.its = z(n_s, dt=torch.int32)
        self.p = params(sampler=self.kind, v_max=v_max)
        # closed-loop statistics, accumulated on the device every cycle
        self.stats = {k: z(n_s) for k in ("v_res", "v_res_max", "lat", "acc", "acc_max", "ang", "ang_max")}
        # closest approach: smallest scaled distance sqrt((dx/a)^2 + (dy/b)^2) of any
        # obstacle centre to the ego after a cycle (below 1: inside the inflated ellipse)
        self.closest = torch.full((n_s,), float("inf"), device="cuda")
        self.obs_scene = torch.repeat_interleave(torch.arange(n_s, device="cuda"),
                                                 torch.tensor(np.diff(self.batch.obs_off()), device="cuda"))
        self.ell = (float(S.DEFAULT_PARAMS["a"]), float(S.DEFAULT_PARAMS["b"]))
        self.psid_prev = self.db.ego[:, 7].clone()
        self.precision, self.iters, self.tol, self.net = precision, iters, tol, net
        if warm not in ("cold", "previous", "shifted", "learned"):
            raise ValueError(f"unknown warm start {warm!r}")
        self.warm = warm if net is None else "learned"
        self.clear_min = float(clear_min)
        self.cycles_done = 0
        self.iters_total = z(n_s, dt=torch.int32)

    def episodes(self):
        return EpisodesC(T._ptr(self.db.ego), T._ptr(self.db.obs), T._ptr(self.db.goal), T._ptr(self.v_des),
                         T._ptr(self.obs_next), T._ptr(self.travelled), T._ptr(self.collisions),
                         T._ptr(self.fallbacks), T._ptr(self.shift))

    def goals(self):
        T._check(self.L.traj_mpc_goals(self.solver.handle, ctypes.byref(self.db.c_struct()),
                                       ctypes.byref(self.episodes()), ctypes.byref(self.p), T._stream(None)))

    def shift_state(self):
        T._check(self.L.traj_mpc_shift(self.solver.handle, ctypes.byref(self.db.c_struct()),
                                       ctypes.byref(self.st.c_struct()), ctypes.byref(self.episodes()),
                                       T._stream(None)))

    def plan(self):
        kw = dict(max_iters=self.iters, chunk=5, tol=self.tol, precision=self.precision, clear_min=self.clear_min,
                  kind=self.kind, w1=self.w1, w2=self.w2, y_rl=self.y_rl)
        if self.warm in ("previous", "shifted") and self.cycles_done > 0:
            # the previous cycle's (c, lambda) of every goal slot (for "shifted" the coefficients advanced by one period,
            # for "shifted"); the x/y step of the first iteration enforces the new
            # boundary values (eq. 8b)
            if self.warm == "shifted":
                self.shift_state()
            self.solver.converge(self.db, self.st, self.v_ref, self.cost, self.best, self.its, from_state=True,
                                 fallback=True, **kw)
        elif self.warm != "learned":
            self.solver.converge(self.db, self.st, self.v_ref, self.cost, self.best, self.its, **kw)
        else:
            from . import warmstart as W
            net, mean, std = self.net
            x = W.features(self.db)
            import torch
            acts = torch.empty(net.acts_size(self.db.n_scenes), dtype=torch.int16, device="cuda")
            y = torch.empty(self.db.n_scenes, net.dims.n_out, device="cuda")
            net.forward(x, acts, y)
            W.rows_state(self.db, self.st, y, mean, std)
            self.solver.converge(self.db, self.st, self.v_ref, self.cost, self.best, self.its, from_state=True,
                                 fallback=True, **kw)
        self.iters_total += self.its

    def step(self):
        T._check(self.L.traj_mpc_step(self.solver.handle, ctypes.byref(self.db.c_struct()),
                                      ctypes.byref(self.st.c_struct()), T._ptr(self.best),
                                      ctypes.byref(self.episodes()), ctypes.byref(self.p), self.n_obs,
                                      T._stream(None)))

    def accumulate(self):
        """Executed-motion statistics after a step (speed residual to v_ref, lateral
        distance to the right lane, |linear acceleration| (x' x'' + y' y'') / v,
        |angular acceleration| as the change of psi' over the period)."""
        import torch
        e, st = self.db.ego, self.stats
        v = torch.hypot(e[:, 2], e[:, 3])
        r = (v - self.v_ref) ** 2
        st["v_res"] += r
        torch.maximum(st["v_res_max"], r, out=st["v_res_max"])
        st["lat"] += (e[:, 1] - self.y_rl).abs()
        acc = ((e[:, 2] * e[:, 4] + e[:, 3] * e[:, 5]) / v.clamp_min(1e-6)).abs()
        st["acc"] += acc
        torch.maximum(st["acc_max"], acc, out=st["acc_max"])
        ang = ((e[:, 7] - self.psid_prev) / self.period).abs()
        st["ang"] += ang
        torch.maximum(st["ang_max"], ang, out=st["ang_max"])
        self.psid_prev.copy_(e[:, 7])
        if self.n_obs > 0:
            o = self.db.obs[: self.n_obs]
            q = torch.hypot(o[:, 0] / self.ell[0], (o[:, 1] - e[self.obs_scene, 1]) / self.ell[1])
            self.closest.scatter_reduce_(0, self.obs_scene, q, reduce="amin")

    @property
    def period(self):
        return self.shape[1] / (self.shape[0] - 1)

    def cycle(self):
        self.goals()
        self.plan()
        self.step()
        self.accumulate()
        self.cycles_done += 1

    def metrics(self, cycles):
        n = self.batch.n_scenes
        tr = self.travelled.cpu().numpy()
        dt = self.period
        st = {k: v.cpu().numpy() for k, v in self.stats.items()}
        c = max(self.cycles_done, 1)
        return {"episodes": n, "cycles": cycles, "scenario": self.scenario,
                "mean_speed": float(tr.mean() / (cycles * dt)),
                "speed_residual_mean": float(st["v_res"].mean() / c), "speed_residual_max": float(st["v_res_max"].max()),
                "right_lane_distance_mean": float(st["lat"].mean() / c),
                "linear_acc_mean": float(st["acc"].mean() / c), "linear_acc_max": float(st["acc_max"].max()),
                "angular_acc_mean": float(st["ang"].mean() / c), "angular_acc_max": float(st["ang_max"].max()),
                "closest_approach": float(self.closest.min().item()),
                "collision_events": int(self.collisions.sum().item()),
                "episodes_with_collision": int((self.collisions > 0).sum().item()),
                "fallback_cycles": int(self.fallbacks.sum().item()),
                "mean_iterations_per_cycle": float(self.iters_total.float().mean().item()) / max(cycles, 1)}
