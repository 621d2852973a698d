"""Python binding of libtraj (ctypes): argument marshalling only.

Every step of the solver runs in the HIP library; this module moves pointers,
sizes and the current HIP stream across the C-ABI declared in include/traj.h.
PyTorch supplies device memory and the stream. There is no fallback: if
libtraj.so is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtraj.so")

TRAJ_OK = 0
TRAJ_INIT_COLD = 0x0
TRAJ_INIT_FROM_STATE = 0x1
TRAJ_WARM_FALLBACK = 0x2
TRAJ_KEEP_DONE = 0x4
TRAJ_PREC_FP32 = 0x0
TRAJ_PREC_BF16X3 = 0x10
TRAJ_KERNEL_AUTO = 0x0
TRAJ_KERNEL_WAVE = 0x100
TRAJ_KERNEL_MFMA = 0x200
TRAJ_KERNEL_GROUP = 0x400
N_COEF = 11
_KERNELS = {"auto": TRAJ_KERNEL_AUTO, "wave": TRAJ_KERNEL_WAVE, "mfma": TRAJ_KERNEL_MFMA,
            "group": TRAJ_KERNEL_GROUP}
_PRECISIONS = {"fp32": TRAJ_PREC_FP32, "bf16x3": TRAJ_PREC_BF16X3}


class Params(ctypes.Structure):
    _fields_ = [("n_coef", ctypes.c_int32), ("rho", ctypes.c_float), ("a", ctypes.c_float),
                ("b", ctypes.c_float), ("v_min", ctypes.c_float), ("v_max", ctypes.c_float),
                ("a_max", ctypes.c_float), ("psi_max", ctypes.c_float)]


class Shape(ctypes.Structure):
    _fields_ = [("n_time", ctypes.c_int32), ("t_f", ctypes.c_float), ("n_obs", ctypes.c_int32)]


class BatchC(ctypes.Structure):
    _fields_ = [("n_scenes", ctypes.c_int32), ("n_goals", ctypes.c_int32),
                ("goal_off", ctypes.c_void_p), ("obs_off", ctypes.c_void_p), ("shape_id", ctypes.c_void_p),
                ("ego", ctypes.c_void_p), ("obs", ctypes.c_void_p), ("goal", ctypes.c_void_p)]


class StateC(ctypes.Structure):
    _fields_ = [("c", ctypes.c_void_p), ("lam", ctypes.c_void_p), ("resid", ctypes.c_void_p),
                ("iters", ctypes.c_void_p), ("work", ctypes.c_void_p), ("work_ints", ctypes.c_int64),
                ("scene_done", ctypes.c_void_p)]


class TileC(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("group", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("waves", ctypes.c_int32)]


class MetaC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("v_ref", ctypes.c_void_p), ("w1", ctypes.c_float),
                ("w2", ctypes.c_float), ("y_rl", ctypes.c_void_p), ("clear_min", ctypes.c_float)]


class MlpDims(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32), ("n_layers", ctypes.c_int32),
                ("n_out", ctypes.c_int32)]


class MlpC(ctypes.Structure):
    _fields_ = [("dims", MlpDims), ("params", ctypes.c_void_p), ("params_bf16", ctypes.c_void_p),
                ("grad", ctypes.c_void_p), ("adam_m", ctypes.c_void_p), ("adam_v", ctypes.c_void_p)]


MLP_EXPORTS = ("traj_mlp_param_count", "traj_mlp_sync_bf16", "traj_features", "traj_mlp_forward", "traj_mlp_loss",
               "traj_mlp_backward", "traj_mlp_adam", "traj_colstats", "traj_state_rows", "traj_rows_state",
               "traj_gemm_bf16")

EXPORTS = ("traj_setup", "traj_solve_batch", "traj_solve_batch_noalloc", "traj_score", "traj_destroy", "traj_last_error",
           "traj_debug_operators", "traj_debug_table_size", "traj_debug_reduce", "traj_set_tile", "traj_get_tile",
           "traj_work_ints", "traj_converge", "traj_debug_atan2", "traj_controls", "traj_set_shape_groups",
           "traj_get_shape_groups")

_lib = None


def lib():
    """Load libtraj.so once; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2109_10392_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, f32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_float
    L.traj_setup.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Shape), i32, vp, ctypes.POINTER(vp)]
    L.traj_solve_batch.argtypes = [vp, ctypes.POINTER(BatchC), ctypes.POINTER(StateC), i32, f32, ctypes.c_uint32, vp]
    L.traj_solve_batch_noalloc.argtypes = [vp, ctypes.POINTER(BatchC), ctypes.POINTER(StateC), i32, f32,
                                           ctypes.c_uint32, vp]
    L.traj_score.argtypes = [vp, ctypes.POINTER(BatchC), ctypes.POINTER(StateC), ctypes.POINTER(MetaC), vp, vp, vp]
    L.traj_destroy.argtypes = [vp]
    L.traj_last_error.restype = ctypes.c_char_p
    L.traj_debug_operators.argtypes = [vp, i32, vp, vp, vp]
    L.traj_debug_table_size.argtypes = [vp, i32]
    L.traj_debug_reduce.argtypes = [vp, vp, i32, vp]
    L.traj_debug_atan2.argtypes = [vp, vp, vp, i32, vp]
    L.traj_controls.argtypes = [vp, ctypes.POINTER(BatchC), ctypes.POINTER(StateC), vp, f32, i32, vp, vp, vp, vp]
    L.traj_set_tile.argtypes = [vp, ctypes.POINTER(TileC)]
    L.traj_get_tile.argtypes = [vp, ctypes.POINTER(TileC)]
    L.traj_work_ints.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_int64)]
    L.traj_set_shape_groups.argtypes = [vp, vp]
    L.traj_get_shape_groups.argtypes = [vp, vp]
    L.traj_converge.argtypes = [vp, ctypes.POINTER(BatchC), ctypes.POINTER(StateC), ctypes.POINTER(MetaC), i32, i32,
                                f32, ctypes.c_uint32, vp, vp, vp, vp]
    P = ctypes.POINTER
    L.traj_mlp_param_count.argtypes = [P(MlpDims), P(ctypes.c_int64)]
    L.traj_mlp_sync_bf16.argtypes = [P(MlpC), vp]
    L.traj_features.argtypes = [P(BatchC), vp, vp]
    L.traj_mlp_forward.argtypes = [P(MlpC), vp, i32, vp, vp, vp]
    L.traj_mlp_loss.argtypes = [P(MlpDims), vp, vp, vp, vp, i32, vp, vp, vp, vp]
    L.traj_mlp_backward.argtypes = [P(MlpC), vp, vp, i32, vp, vp]
    L.traj_mlp_adam.argtypes = [P(MlpC), i32, f32, f32, f32, f32, vp]
    L.traj_colstats.argtypes = [vp, i32, i32, vp, vp, vp]
    L.traj_state_rows.argtypes = [P(BatchC), P(StateC), i32, vp, vp]
    L.traj_rows_state.argtypes = [P(BatchC), P(StateC), i32, vp, vp, vp, vp]
    L.traj_gemm_bf16.argtypes = [i32, i32, i32, i32, i32, vp, vp, vp, i32, vp, vp]
    for name in EXPORTS + MLP_EXPORTS:
        getattr(L, name).restype = ctypes.c_char_p if name == "traj_last_error" else ctypes.c_int
    _lib = L
    return L


class TrajError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libtraj error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != TRAJ_OK:
        raise TrajError(rc, lib().traj_last_error().decode())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def make_params(p: dict) -> Params:
    return Params(int(p["n_coef"]), float(p["rho"]), float(p["a"]), float(p["b"]), float(p["v_min"]),
                  float(p["v_max"]), float(p["a_max"]), float(p["psi_max"]))


@dataclass
class DeviceBatch:
    """Device copy of a scenes.Batch (or any arrays of the same layout)."""
    n_scenes: int
    n_goals: int
    goal_off: object
    obs_off: object
    shape_id: object
    ego: object
    obs: object
    goal: object
    shapes: list

    @staticmethod
    def from_batch(batch, device="cuda", shapes=None):
        import torch
        shapes = list(shapes) if shapes is not None else batch.shapes()
        sid = np.array([shapes.index((s.n_time, float(s.t_f), int(s.obs.shape[0]))) for s in batch.scenes], np.int32)

        def t(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)

        obs = batch.obs()
        if obs.shape[0] == 0:
            obs = np.zeros((1, 4), np.float32)
        return DeviceBatch(batch.n_scenes, batch.n_goals, t(batch.goal_off(), torch.int32),
                           t(batch.obs_off(), torch.int32), t(sid, torch.int32), t(batch.ego(), torch.float32),
                           t(obs, torch.float32), t(batch.goals(), torch.float32), shapes)

    def c_struct(self) -> BatchC:
        return BatchC(self.n_scenes, self.n_goals, _ptr(self.goal_off), _ptr(self.obs_off), _ptr(self.shape_id),
                      _ptr(self.ego), _ptr(self.obs), _ptr(self.goal))


@dataclass
class DeviceState:
    c: object      # [3, 11, G] float32
    lam: object    # [3, 11, G] float32
    resid: object  # [4, G] float32
    iters: object  # [G] int32
    work: object = None  # int32 scratch of the group kernel (Solver.solve sizes it)
    scene_done: object = None  # [S] int32: scenes to leave untouched (set by converge)

    @staticmethod
    def empty(n_goals, device="cuda"):
        import torch
        z = lambda *s: torch.zeros(*s, device=device, dtype=torch.float32)
        return DeviceState(z(3, N_COEF, n_goals), z(3, N_COEF, n_goals), z(4, n_goals),
                           torch.zeros(n_goals, device=device, dtype=torch.int32))

    def c_struct(self) -> StateC:
        w = self.work
        return StateC(_ptr(self.c), _ptr(self.lam), _ptr(self.resid), _ptr(self.iters), _ptr(w),
                      0 if w is None else int(w.numel()), _ptr(self.scene_done))


class Solver:
    """Owns a libtraj handle set up for a list of (n_time, t_f, n_obs) shapes."""

    def __init__(self, params: dict, shapes, stream=None):
        L = lib()
        self.params = dict(params)
        self.shapes = [(int(n), float(tf), int(m)) for (n, tf, m) in shapes]
        arr = (Shape * len(self.shapes))(*[Shape(n, tf, m) for (n, tf, m) in self.shapes])
        h = ctypes.c_void_p()
        _check(L.traj_setup(ctypes.byref(make_params(params)), arr, len(self.shapes), _stream(stream),
                            ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle is not None and self.handle.value:
            lib().traj_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _flags(self, from_state, fallback, precision, kernel):
        return ((TRAJ_INIT_FROM_STATE if from_state else TRAJ_INIT_COLD) | (TRAJ_WARM_FALLBACK if fallback else 0)
                | _PRECISIONS[precision] | _KERNELS[kernel])

    def converge(self, batch: DeviceBatch, state: DeviceState, v_ref, cost, best, scene_iters, max_iters=300,
                 chunk=5, tol=1e-3, from_state=False, fallback=False, precision="fp32", kernel="auto", kind=0,
                 w1=1.0, w2=1.0, y_rl=None, clear_min=0.0, stream=None, keep_done=False):
        """Chunked solve until each scene's best goal meets the residual tolerance
        (device-side bookkeeping; state.scene_done and scene_iters hold the outcome).
        keep_done: continue an earlier call (only the scenes it left unconverged run)."""
        import torch
        if kernel == "group" or (kernel == "auto" and self.get_tile()[0] == "group"):
            self.ensure_work(batch, state)
        if state.scene_done is None or state.scene_done.numel() < batch.n_scenes:
            state.scene_done = torch.zeros(max(batch.n_scenes, 1), dtype=torch.int32, device=state.c.device)
        b = batch.c_struct()
        s = state.c_struct()
        mc = MetaC(int(kind), _ptr(v_ref), float(w1), float(w2), _ptr(y_rl), float(clear_min))
        flags = self._flags(from_state, fallback, precision, kernel) | (TRAJ_KEEP_DONE if keep_done else 0)
        _check(lib().traj_converge(self.handle, ctypes.byref(b), ctypes.byref(s), ctypes.byref(mc), int(max_iters),
                                   int(chunk), float(tol), flags,
                                   _ptr(cost), _ptr(best), _ptr(scene_iters), _stream(stream)))

    def solve(self, batch: DeviceBatch, state: DeviceState, iters: int, tol: float = 0.0,
              from_state: bool = False, precision: str = "fp32", kernel: str = "auto", stream=None,
              fallback: bool = False):
        if kernel == "group" or (kernel == "auto" and self.get_tile()[0] == "group"):
            self.ensure_work(batch, state)
        b = batch.c_struct()
        s = state.c_struct()
        flags = self._flags(from_state, fallback, precision, kernel)
        _check(lib().traj_solve_batch(self.handle, ctypes.byref(b), ctypes.byref(s), int(iters), float(tol),
                                      flags, _stream(stream)))

    def solve_noalloc(self, batch: DeviceBatch, state: DeviceState, iters: int, tol: float = 0.0,
                      from_state: bool = False, precision: str = "fp32", kernel: str = "auto", stream=None,
                      fallback: bool = False):
        """solve() through traj_solve_batch_noalloc: the group kernel's work list lives
        in the library's own device scratch (state.work is not used)."""
        b = batch.c_struct()
        s = state.c_struct()
        flags = self._flags(from_state, fallback, precision, kernel)
        _check(lib().traj_solve_batch_noalloc(self.handle, ctypes.byref(b), ctypes.byref(s), int(iters), float(tol),
                                              flags, _stream(stream)))

    def set_tile(self, kernel: str, group: int = 16, persistent: bool = True, waves: int = 1):
        t = TileC(_KERNELS[kernel], int(group), 1 if persistent else 0, int(waves))
        _check(lib().traj_set_tile(self.handle, ctypes.byref(t)))

    def set_shape_groups(self, groups=None):
        """Goals per group of the group kernel per shape (0 = the tile's); None clears."""
        if groups is None:
            _check(lib().traj_set_shape_groups(self.handle, None))
            return
        n = len(self.shapes)
        if len(groups) != n:
            raise ValueError(f"need {n} group sizes, got {len(groups)}")
        arr = (ctypes.c_int32 * n)(*[int(g) for g in groups])
        _check(lib().traj_set_shape_groups(self.handle, arr))

    def get_shape_groups(self):
        arr = (ctypes.c_int32 * len(self.shapes))()
        _check(lib().traj_get_shape_groups(self.handle, arr))
        return list(arr)

    def get_tile(self):
        """(kernel, group, persistent, waves) of the handle's tile."""
        t = TileC()
        _check(lib().traj_get_tile(self.handle, ctypes.byref(t)))
        inv = {v: k for k, v in _KERNELS.items()}
        return inv[t.kernel], t.group, bool(t.persistent), t.waves

    def work_ints(self, n_scenes: int, n_goals: int) -> int:
        """int32 scratch entries a group-kernel solve of this batch size needs."""
        out = ctypes.c_int64()
        _check(lib().traj_work_ints(self.handle, int(n_scenes), int(n_goals), ctypes.byref(out)))
        return out.value

    def ensure_work(self, batch, state):
        """Give `state` a group-kernel scratch buffer of sufficient size (allocated by
        torch outside any solve; solves themselves never allocate)."""
        import torch
        need = self.work_ints(batch.n_scenes, batch.n_goals)
        if state.work is None or state.work.numel() < need:
            state.work = torch.zeros(need, dtype=torch.int32, device=state.c.device)

    def score(self, batch: DeviceBatch, state: DeviceState, v_ref, cost, best, kind=0, w1=1.0, w2=1.0,
              y_rl=None, clear_min=0.0, stream=None):
        b = batch.c_struct()
        s = state.c_struct()
        mc = MetaC(int(kind), _ptr(v_ref), float(w1), float(w2), _ptr(y_rl), float(clear_min))
        _check(lib().traj_score(self.handle, ctypes.byref(b), ctypes.byref(s), ctypes.byref(mc), _ptr(cost),
                                _ptr(best), _stream(stream)))

    def controls(self, batch: DeviceBatch, state: DeviceState, best, wheelbase=2.5, stride=None, stream=None):
        """(accel [S][stride], steer [S][stride], clearance [S]) of each scene's chosen trajectory."""
        import torch
        stride = stride or max(n for n, _, _ in self.shapes)
        S_ = max(batch.n_scenes, 1)
        acc = torch.zeros(S_, stride, device=state.c.device)
        steer = torch.zeros(S_, stride, device=state.c.device)
        clear = torch.zeros(S_, device=state.c.device)
        _check(lib().traj_controls(self.handle, ctypes.byref(batch.c_struct()), ctypes.byref(state.c_struct()),
                                   _ptr(best), float(wheelbase), int(stride), _ptr(acc), _ptr(steer), _ptr(clear),
                                   _stream(stream)))
        return acc, steer, clear

    def operators(self, shape: int):
        """FP64 KKT inverses [5, 17, 17] and the FP32 table of one shape (host arrays)."""
        L = lib()
        n32 = L.traj_debug_table_size(self.handle, shape)
        if n32 < 0:
            _check(n32)
        f64 = np.zeros(5 * 17 * 17, np.float64)
        f32 = np.zeros(n32, np.float32)
        _check(L.traj_debug_operators(self.handle, shape, f64.ctypes.data_as(ctypes.c_void_p),
                                      f32.ctypes.data_as(ctypes.c_void_p), _stream(None)))
        return f64.reshape(5, 17, 17), f32


def debug_atan2(y_dev, x_dev, out_dev, stream=None):
    _check(lib().traj_debug_atan2(_ptr(y_dev), _ptr(x_dev), _ptr(out_dev), int(y_dev.numel()), _stream(stream)))


def debug_reduce(values_dev, out_dev, r, stream=None):
    _check(lib().traj_debug_reduce(_ptr(values_dev), _ptr(out_dev), int(r), _stream(stream)))
