"""The C-ABI end to end without PyTorch: device memory from the HIP runtime
through ctypes, the null stream, traj_setup / traj_set_tile / traj_solve_batch /
traj_score. The results equal those of the PyTorch-plumbed binding bitwise, so
PyTorch only supplies memory and streams."""
import ctypes

import numpy as np
import pytest

from paper_2109_10392_amd import traj as T
from tests.test_gpu_parity import PARAMS, ragged_batch

pytestmark = pytest.mark.gpu

ITERS = 40
H2D, D2H = 1, 2  # hipMemcpyKind


def _hip():
    for name in ("libamdhip64.so", "/opt/rocm/lib/libamdhip64.so"):
        try:
            hip = ctypes.CDLL(name)
            break
        except OSError:
            hip = None
    if hip is None:
        pytest.skip("no HIP runtime")
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    hip.hipMalloc.argtypes = [ctypes.POINTER(vp), sz]
    hip.hipMemcpy.argtypes = [vp, vp, sz, ctypes.c_int]
    hip.hipFree.argtypes = [vp]
    hip.hipGetDeviceCount.argtypes = [ctypes.POINTER(ctypes.c_int)]
    n = ctypes.c_int(0)
    if hip.hipGetDeviceCount(ctypes.byref(n)) != 0 or n.value < 1:
        pytest.skip("no GPU")
    return hip


class Device:
    """Device buffers from hipMalloc, freed by close()."""

    def __init__(self, hip):
        self.hip, self.ptrs = hip, []

    def alloc(self, nbytes):
        """Device address (an int) of a new buffer of nbytes."""
        p = ctypes.c_void_p()
        assert self.hip.hipMalloc(ctypes.byref(p), max(int(nbytes), 4)) == 0
        self.ptrs.append(p)
        return p.value

    def put(self, arr):
        arr = np.ascontiguousarray(arr)
        p = self.alloc(arr.nbytes)
        assert self.hip.hipMemcpy(p, arr.ctypes.data_as(ctypes.c_void_p), arr.nbytes, H2D) == 0
        return p

    def get(self, p, shape, dtype):
        out = np.empty(shape, dtype)
        assert self.hip.hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), p, out.nbytes, D2H) == 0
        return out

    def close(self):
        for p in self.ptrs:
            self.hip.hipFree(p)
        self.ptrs = []


def _torch_path(batch):
    import torch
    solver = T.Solver(PARAMS, batch.shapes())
    solver.set_tile("wave", 16, True, 2)
    db = T.DeviceBatch.from_batch(batch)
    st = T.DeviceState.empty(batch.n_goals)
    solver.solve(db, st, ITERS, kernel="wave")
    v_ref = torch.tensor([float(s.ego[2]) for s in batch.scenes], device="cuda")
    cost = torch.zeros(batch.n_goals, device="cuda")
    best = torch.zeros(batch.n_scenes, device="cuda", dtype=torch.int32)
    solver.score(db, st, v_ref, cost, best)
    torch.cuda.synchronize()
    out = dict(c=st.c.cpu().numpy(), lam=st.lam.cpu().numpy(), resid=st.resid.cpu().numpy(),
               iters=st.iters.cpu().numpy(), cost=cost.cpu().numpy(), best=best.cpu().numpy())
    solver.close()
    return out


def test_c_abi_end_to_end_without_torch():
    hip = _hip()
    L = T.lib()
    batch = ragged_batch()
    shapes = batch.shapes()
    sid = np.array([shapes.index((s.n_time, float(s.t_f), int(s.obs.shape[0]))) for s in batch.scenes], np.int32)
    G, Sn = batch.n_goals, batch.n_scenes
    dev = Device(hip)
    h = ctypes.c_void_p()
    try:
        arr = (T.Shape * len(shapes))(*[T.Shape(n, tf, m) for (n, tf, m) in shapes])
        assert L.traj_setup(ctypes.byref(T.make_params(PARAMS)), arr, len(shapes), None, ctypes.byref(h)) == 0
        assert L.traj_set_tile(h, ctypes.byref(T.TileC(T.TRAJ_KERNEL_WAVE, 16, 1, 2))) == 0
        obs = batch.obs() if batch.obs().shape[0] else np.zeros((1, 4), np.float32)
        b = T.BatchC(Sn, G, dev.put(batch.goal_off().astype(np.int32)), dev.put(batch.obs_off().astype(np.int32)),
                     dev.put(sid), dev.put(batch.ego().astype(np.float32)), dev.put(obs.astype(np.float32)),
                     dev.put(batch.goals().astype(np.float32)))
        c, lam = dev.alloc(3 * 11 * G * 4), dev.alloc(3 * 11 * G * 4)
        resid, iters = dev.alloc(4 * G * 4), dev.alloc(G * 4)
        s = T.StateC(c, lam, resid, iters, None, 0, None)
        assert L.traj_solve_batch(h, ctypes.byref(b), ctypes.byref(s), ITERS, 0.0, T.TRAJ_KERNEL_WAVE, None) == 0
        v_ref = dev.put(np.array([float(sc.ego[2]) for sc in batch.scenes], np.float32))
        cost, best = dev.alloc(G * 4), dev.alloc(Sn * 4)
        mc = T.MetaC(0, v_ref, 1.0, 1.0, None, 0.0)
        assert L.traj_score(h, ctypes.byref(b), ctypes.byref(s), ctypes.byref(mc), cost, best, None) == 0
        got = dict(c=dev.get(c, (3, 11, G), np.float32), lam=dev.get(lam, (3, 11, G), np.float32),
                   resid=dev.get(resid, (4, G), np.float32), iters=dev.get(iters, (G,), np.int32),
                   cost=dev.get(cost, (G,), np.float32), best=dev.get(best, (Sn,), np.int32))
    finally:
        if h.value:
            L.traj_destroy(h)
        dev.close()
    ref = _torch_path(batch)
    for k in ("c", "lam", "resid", "iters", "cost", "best"):
        assert np.array_equal(got[k], ref[k].reshape(got[k].shape), equal_nan=True), k
    assert np.all(np.isfinite(got["c"]))
