"""Controls of the chosen trajectory and the collision post-check on the GPU,
against the oracle evaluated on the same coefficients (FP32 evaluation vs FP64:
agreement to FP32 rounding of 11-term sums)."""
import numpy as np
import pytest

from oracle import traj_oracle as O
from paper_2109_10392_amd import scenes as S
from tests.test_gpu_parity import PARAMS, ragged_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_10392_amd import traj
    traj.lib()
    return traj


def test_controls_and_clearance_match_the_oracle(T):
    import torch
    batch = ragged_batch()
    solver = T.Solver(PARAMS, batch.shapes())
    db = T.DeviceBatch.from_batch(batch)
    st = T.DeviceState.empty(batch.n_goals)
    solver.solve(db, st, 60)
    v_ref = torch.tensor([float(s.ego[2]) for s in batch.scenes], device="cuda")
    cost = torch.zeros(batch.n_goals, device="cuda")
    best = torch.zeros(batch.n_scenes, device="cuda", dtype=torch.int32)
    solver.score(db, st, v_ref, cost, best)
    acc, steer, clear = solver.controls(db, st, best, wheelbase=2.5, stride=160)
    torch.cuda.synchronize()
    c = st.c.cpu().numpy().astype(np.float64)
    off = batch.goal_off()
    b = best.cpu().numpy()
    acc, steer, clear = acc.cpu().numpy(), steer.cpu().numpy(), clear.cpu().numpy()
    for s, sc in enumerate(batch.scenes):
        if b[s] < 0:
            assert np.isnan(clear[s])
            continue
        prob = O.Problem(sc.n_time, sc.t_f, sc.obs.shape[0], PARAMS)
        g = off[s] + b[s]
        a_ref, s_ref, c_ref = O.controls(prob, sc.obs, c[0, :, g], c[1, :, g], c[2, :, g], 2.5, PARAMS["v_min"])
        n = sc.n_time
        scale_a = max(1.0, np.max(np.abs(a_ref)))
        assert np.max(np.abs(acc[s, :n] - a_ref)) <= 1e-3 * scale_a, s
        assert np.max(np.abs(steer[s, :n] - s_ref)) <= 1e-5, s
        if np.isinf(c_ref):
            assert np.isinf(clear[s])
        else:
            assert abs(clear[s] - c_ref) <= 1e-5 * max(1.0, c_ref), s
        print(f"scene {s}: best {b[s]}, clearance {clear[s]:.4f}, max |steer| {np.max(np.abs(s_ref)):.4f} rad")
    solver.close()


def test_controls_reject_a_short_stride(T):
    import ctypes

    import torch
    batch = S.workload_small(0)
    solver = T.Solver(PARAMS, batch.shapes())
    db = T.DeviceBatch.from_batch(batch)
    st = T.DeviceState.empty(batch.n_goals)
    best = torch.zeros(1, device="cuda", dtype=torch.int32)
    out = torch.zeros(1, 50, device="cuda")
    rc = T.lib().traj_controls(solver.handle, ctypes.byref(db.c_struct()), ctypes.byref(st.c_struct()), T._ptr(best),
                               2.5, 50, T._ptr(out), T._ptr(out), T._ptr(out), T._stream(None))
    assert rc == -1
    solver.close()


def test_collision_post_check_in_the_ranking_matches_the_oracle(T):
    """traj_score with clear_min: goals whose trajectory comes closer than
    clear_min to an obstacle are discarded. After a few iterations many
    trajectories still cross obstacles, so both outcomes occur."""
    import torch
    batch = ragged_batch()
    solver = T.Solver(PARAMS, batch.shapes())
    db = T.DeviceBatch.from_batch(batch)
    st = T.DeviceState.empty(batch.n_goals)
    solver.solve(db, st, 8)
    v_ref = torch.tensor([float(s.ego[2]) for s in batch.scenes], device="cuda")
    cost = torch.zeros(batch.n_goals, device="cuda")
    best = torch.zeros(batch.n_scenes, device="cuda", dtype=torch.int32)
    n_cut = n_kept = 0
    for clear_min in (1.0, 1.2):
        solver.score(db, st, v_ref, cost, best, clear_min=clear_min)
        torch.cuda.synchronize()
        c = st.c.cpu().numpy().astype(np.float64)
        cg, bg = cost.cpu().numpy(), best.cpu().numpy()
        off = batch.goal_off()
        for s, sc in enumerate(batch.scenes):
            prob = O.Problem(sc.n_time, sc.t_f, sc.obs.shape[0], PARAMS)
            sl = slice(off[s], off[s + 1])
            ref = O.meta_cost(prob, c[0][:, sl], c[1][:, sl], c[2][:, sl], 0, v_ref=float(sc.ego[2]),
                              obs=sc.obs, clear_min=clear_min)
            clear = np.array([O.controls(prob, sc.obs, c[0][:, g], c[1][:, g], c[2][:, g], 1.0, 1.0)[2]
                              for g in range(off[s], off[s + 1])])
            # the decision is compared where FP32 cannot flip it
            sure = np.abs(clear - clear_min) > 1e-4 * clear_min
            assert np.array_equal(np.isinf(cg[sl])[sure], np.isinf(ref)[sure]), s
            fin = np.isfinite(ref) & np.isfinite(cg[sl])
            assert np.allclose(cg[sl][fin], ref[fin], rtol=2e-4, atol=1e-3), s
            if sure.all():
                assert bg[s] == O.best_goal(ref), s
            n_cut += int(np.sum(np.isinf(ref) & sure))
            n_kept += int(np.sum(np.isfinite(ref) & sure))
    print(f"post-check: {n_cut} goals discarded, {n_kept} kept")
    assert n_cut > 0 and n_kept > 0
    solver.close()
