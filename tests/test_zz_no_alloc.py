"""traj_solve_batch_noalloc (the group kernel's work list in the library's own
device scratch) against traj_solve_batch with a caller-owned work buffer, through
the C-ABI: bitwise equal results on two calls in a row, the second on a smaller
batch, with per-shape group sizes too, and the size limit rejected before any
device work."""
import ctypes

import numpy as np
import pytest

from paper_2109_10392_amd import scenes as S

pytestmark = pytest.mark.gpu

PARAMS = S.DEFAULT_PARAMS


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_10392_amd import traj
    traj.lib()
    return traj


def _batches():
    big = S.Batch([S.make_scene(31, 300, 40, n_lanes=6), S.make_scene(32, 17, 5, n_lanes=4),
                   S.make_scene(33, 90, 64, n_lanes=6, n_time=150, t_f=15.0),
                   S.make_scene(34, 45, 0, n_lanes=4, n_time=50, t_f=5.0)])
    small = S.Batch([S.make_scene(35, 23, 12, n_lanes=4), S.make_scene(36, 7, 3, n_lanes=4, n_time=50, t_f=5.0)])
    return big, small


def _run(T, solver, batch, iters, noalloc, precision="fp32"):
    import torch
    db = T.DeviceBatch.from_batch(batch, shapes=solver.shapes)
    st = T.DeviceState.empty(batch.n_goals)
    # both start from NaN-filled outputs, so every value compared was written by the solve
    for t in (st.c, st.lam, st.resid):
        t.fill_(float("nan"))
    st.iters.fill_(-1)
    if noalloc:
        solver.solve_noalloc(db, st, iters, kernel="group", precision=precision)
    else:
        solver.solve(db, st, iters, kernel="group", precision=precision)
    torch.cuda.synchronize()
    return {k: getattr(st, k).cpu().numpy() for k in ("c", "lam", "resid", "iters")}


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_noalloc_equals_the_work_buffer_solve_on_two_calls(T, precision):
    big, small = _batches()
    shapes = sorted(set(big.shapes()) | set(small.shapes()))
    solver = T.Solver(PARAMS, shapes)
    try:
        solver.set_tile("group", 16, True)
        for i, batch in enumerate((big, small)):  # the second call is smaller: stale list entries must not leak
            print(f"call {i}: {batch.n_scenes} scenes, {batch.n_goals} goals, {precision}", flush=True)
            ref = _run(T, solver, batch, 30, noalloc=False, precision=precision)
            out = _run(T, solver, batch, 30, noalloc=True, precision=precision)
            for k in ("c", "lam", "resid", "iters"):
                assert np.array_equal(out[k], ref[k], equal_nan=True), (i, k)
            assert np.all(np.isfinite(out["c"])) and np.all(out["iters"] == 30)
    finally:
        solver.close()


def test_noalloc_small_group_size_and_listed_schedule(T):
    """Group size 3, one wavefront per listed group: more list entries than the
    default tile, the same results as the caller-owned buffer."""
    big, small = _batches()
    solver = T.Solver(PARAMS, sorted(set(big.shapes()) | set(small.shapes())))
    try:
        solver.set_tile("group", 3, False)
        for batch in (big, small):
            ref = _run(T, solver, batch, 20, noalloc=False)
            out = _run(T, solver, batch, 20, noalloc=True)
            for k in ("c", "lam", "resid", "iters"):
                assert np.array_equal(out[k], ref[k], equal_nan=True), k
    finally:
        solver.close()


def test_noalloc_with_per_shape_group_sizes(T):
    """Group sizes set per shape (traj_set_shape_groups): the scratch list is sized
    by the smallest, and the results equal the caller-owned buffer's."""
    big, small = _batches()
    shapes = sorted(set(big.shapes()) | set(small.shapes()))
    solver = T.Solver(PARAMS, shapes)
    try:
        solver.set_tile("group", 16, True)
        solver.set_shape_groups([(2, 5, 0, 11, 7, 3)[i % 6] for i in range(len(shapes))])
        for batch in (big, small):
            ref = _run(T, solver, batch, 20, noalloc=False)
            out = _run(T, solver, batch, 20, noalloc=True)
            for k in ("c", "lam", "resid", "iters"):
                assert np.array_equal(out[k], ref[k], equal_nan=True), k
    finally:
        solver.close()


def test_noalloc_rejects_a_work_list_beyond_the_scratch(T):
    """One scene of 400,000 goals at group size 1 needs more than the 524,288-int32
    scratch: TRAJ_E_INVAL before any device work (all arrays are real, sized for
    the batch, so even a launch would stay in bounds); at group size 16 it fits."""
    import torch
    solver = T.Solver(PARAMS, [(100, 10.0, 0)])
    try:
        solver.set_tile("group", 1, True)
        G = 400_000
        need = solver.work_ints(1, G)
        assert need > 524_288
        dev = "cuda"
        goal_off = torch.tensor([0, G], dtype=torch.int32, device=dev)
        obs_off = torch.zeros(2, dtype=torch.int32, device=dev)
        sid = torch.zeros(1, dtype=torch.int32, device=dev)
        ego = torch.zeros(1, 8, device=dev)
        ego[0, 2] = 15.0
        obs = torch.zeros(1, 4, device=dev)
        goal = torch.zeros(G, 2, device=dev)
        goal[:, 0] = 150.0
        c = torch.zeros(3, 11, G, device=dev)
        lam = torch.zeros(3, 11, G, device=dev)
        b = T.BatchC(1, G, goal_off.data_ptr(), obs_off.data_ptr(), sid.data_ptr(), ego.data_ptr(),
                     obs.data_ptr(), goal.data_ptr())
        s = T.StateC(c.data_ptr(), lam.data_ptr(), None, None, None, 0, None)
        c.fill_(7.0)
        torch.cuda.synchronize()
        rc = T.lib().traj_solve_batch_noalloc(solver.handle, ctypes.byref(b), ctypes.byref(s), 5, 0.0,
                                              T.TRAJ_KERNEL_GROUP, T._stream(None))
        assert rc == -1
        assert b"scratch" in T.lib().traj_last_error()
        torch.cuda.synchronize()
        assert bool(torch.all(c == 7.0))  # nothing ran
        # the same batch at group size 16 fits and runs
        solver.set_tile("group", 16, True)
        assert solver.work_ints(1, G) <= 524_288
        rc = T.lib().traj_solve_batch_noalloc(solver.handle, ctypes.byref(b), ctypes.byref(s), 2, 0.0,
                                              T.TRAJ_KERNEL_GROUP, T._stream(None))
        assert rc == 0, T.lib().traj_last_error()
        torch.cuda.synchronize()
        assert bool(torch.all(torch.isfinite(c)))
    finally:
        solver.close()
