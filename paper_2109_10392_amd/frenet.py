"""Road-attached frame: binding of include/traj_frenet.h.

The planner works along a road's centre-line (x = arc length s, y = signed
lateral offset d, Sec. III assumption 1). A Road holds the centre-line (segments
of constant curvature from a start pose); its methods map device tensors
between the global and the road frame on the current stream. Arithmetic runs in
the library's kernels; this module only marshals pointers.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import traj as T


class RoadC(ctypes.Structure):
    _fields_ = [("n_seg", ctypes.c_int32), ("seg", ctypes.c_void_p), ("x0", ctypes.c_float),
                ("y0", ctypes.c_float), ("theta0", ctypes.c_float)]


def _bind():
    L = T.lib()
    if getattr(L, "_frenet_bound", False):
        return L
    vp, i32 = ctypes.c_void_p, ctypes.c_int
    L.traj_road_from_global.argtypes = [ctypes.POINTER(RoadC), i32, i32, vp, vp, vp]
    L.traj_road_to_global.argtypes = [ctypes.POINTER(RoadC), i32, vp, vp, vp]
    L.traj_trajectory_to_global.argtypes = [vp, ctypes.POINTER(T.BatchC), ctypes.POINTER(T.StateC), vp,
                                            ctypes.POINTER(RoadC), i32, vp, vp]
    for f in (L.traj_road_from_global, L.traj_road_to_global, L.traj_trajectory_to_global):
        f.restype = ctypes.c_int
    L._frenet_bound = True
    return L


class Road:
    """Centre-line: segments [(length, curvature), ...] from (x0, y0) heading theta0."""

    def __init__(self, segments, x0=0.0, y0=0.0, theta0=0.0):
        self.seg = np.ascontiguousarray(np.asarray(segments, np.float32).reshape(-1, 2))
        self.x0, self.y0, self.theta0 = float(x0), float(y0), float(theta0)
        self.L = _bind()

    def c_struct(self):
        return RoadC(int(self.seg.shape[0]), self.seg.ctypes.data, self.x0, self.y0, self.theta0)

    def from_global(self, states, out=None, stream=None):
        """[n][4] (x, y, vx, vy) or [n][8] ego states -> the road frame (same width)."""
        kind = {4: 0, 8: 1}[int(states.shape[-1])]
        out = states if out is None else out
        r = self.c_struct()
        T._check(self.L.traj_road_from_global(ctypes.byref(r), kind, int(states.shape[0]), T._ptr(states),
                                              T._ptr(out), T._stream(stream)))
        return out

    def to_global(self, sd, stream=None):
        """[n][2] (s, d) -> [n][3] (X, Y, centre-line heading)."""
        import torch
        out = torch.empty(sd.shape[0], 3, device=sd.device, dtype=torch.float32)
        r = self.c_struct()
        T._check(self.L.traj_road_to_global(ctypes.byref(r), int(sd.shape[0]), T._ptr(sd), T._ptr(out),
                                            T._stream(stream)))
        return out

    def trajectory(self, solver, batch, state, best, stride=None, stream=None):
        """Each scene's chosen trajectory in the global frame: [S][stride][3] (X, Y, heading),
        NaN where nothing was written."""
        import torch
        stride = stride or max(n for n, _, _ in solver.shapes)
        out = torch.full((max(batch.n_scenes, 1), stride, 3), float("nan"), device=state.c.device)
        r = self.c_struct()
        T._check(self.L.traj_trajectory_to_global(solver.handle, ctypes.byref(batch.c_struct()),
                                                  ctypes.byref(state.c_struct()), T._ptr(best), ctypes.byref(r),
                                                  int(stride), T._ptr(out), T._stream(stream)))
        return out
