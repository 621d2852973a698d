"""Chunked solve to a residual tolerance, the per-scene skip mask and the
cold-start fallback of a warm start.

Stopping rule: a scene stops after the first chunk of 5 iterations at which its
current best goal has max(r_obs, r_acc, r_nh) <= tol. Solves resume bitwise, so
a converged scene's state equals a plain cold solve of the same iteration count,
and one chunk earlier the rule must not have held yet.
Fallback: after one iteration from the given state and one from the cold start,
each goal keeps the one with the lower residual; the result then equals, goal by
goal, the plain warm or the plain cold solve.
"""
import numpy as np
import pytest

from paper_2109_10392_amd import scenes as S
from tests.test_gpu_parity import PARAMS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_10392_amd import traj
    traj.lib()
    return traj


def small_batch():
    return S.Batch([S.make_scene(31 + i, n_goals=g, n_obs=m, n_lanes=4) for i, (g, m) in
                    enumerate([(11, 10), (7, 4), (16, 10), (3, 0), (20, 12)])])


def run(T, batch, iters, kernel="group", init=None, fallback=False, skip=None, precision="fp32"):
    import torch
    solver = T.Solver(PARAMS, batch.shapes())
    solver.set_tile(kernel, 16, True)
    db = T.DeviceBatch.from_batch(batch)
    st = T.DeviceState.empty(batch.n_goals)
    if init is not None:
        st.c.copy_(torch.as_tensor(init[0], device="cuda"))
        st.lam.copy_(torch.as_tensor(init[1], device="cuda"))
    if skip is not None:
        st.scene_done = torch.as_tensor(np.asarray(skip, np.int32), device="cuda")
    solver.solve(db, st, iters, from_state=init is not None, fallback=fallback, precision=precision)
    torch.cuda.synchronize()
    out = (st.c.cpu().numpy(), st.lam.cpu().numpy(), st.resid.cpu().numpy())
    solver.close()
    return out


@pytest.mark.parametrize("kernel", ["group", "wave", "mfma"])
def test_skipped_scenes_are_left_untouched(T, kernel):
    batch = small_batch()
    off = batch.goal_off()
    ref = run(T, batch, 20, kernel)
    sentinel = (np.full((3, 11, batch.n_goals), 7.0, np.float32), np.full((3, 11, batch.n_goals), -2.0, np.float32))
    skip = [0, 1, 0, 1, 0]
    import torch
    solver = T.Solver(PARAMS, batch.shapes())
    solver.set_tile(kernel, 16, True)
    db = T.DeviceBatch.from_batch(batch)
    st = T.DeviceState.empty(batch.n_goals)
    st.c.fill_(7.0)
    st.lam.fill_(-2.0)
    st.scene_done = torch.as_tensor(np.asarray(skip, np.int32), device="cuda")
    solver.solve(db, st, 20)
    torch.cuda.synchronize()
    c, lam = st.c.cpu().numpy(), st.lam.cpu().numpy()
    solver.close()
    for s in range(batch.n_scenes):
        sl = slice(off[s], off[s + 1])
        if skip[s]:
            assert np.all(c[:, :, sl] == sentinel[0][:, :, sl]) and np.all(lam[:, :, sl] == sentinel[1][:, :, sl])
        else:
            assert np.array_equal(c[:, :, sl], ref[0][:, :, sl]), s


@pytest.mark.parametrize("kernel,waves,precision", [("group", 1, "fp32"), ("group", 1, "bf16x3"),
                                                    ("wave", 2, "fp32"), ("mfma", 1, "bf16x3")])
def test_converge_stops_at_the_first_chunk_meeting_the_rule(T, kernel, waves, precision):
    """Every scene stops at the first chunk of 5 iterations where its best goal
    meets the rule (R10), and its state equals a plain solve of that many
    iterations bitwise; on each kernel and precision form."""
    import torch
    batch = S.Batch([S.workload_small(s).scenes[0] for s in range(6)])
    solver = T.Solver(PARAMS, batch.shapes())
    solver.set_tile(kernel, 16, True, waves)
    db = T.DeviceBatch.from_batch(batch)
    st = T.DeviceState.empty(batch.n_goals)
    v_ref = torch.tensor([float(s.ego[2]) for s in batch.scenes], device="cuda")
    cost = torch.zeros(batch.n_goals, device="cuda")
    best = torch.zeros(batch.n_scenes, device="cuda", dtype=torch.int32)
    its = torch.zeros(batch.n_scenes, device="cuda", dtype=torch.int32)
    tol, cap = 1e-3, 300
    solver.converge(db, st, v_ref, cost, best, its, max_iters=cap, chunk=5, tol=tol, precision=precision)
    torch.cuda.synchronize()
    c = st.c.cpu().numpy()
    done = st.scene_done.cpu().numpy()
    iters = its.cpu().numpy()
    print("scene iterations:", iters.tolist(), "converged:", done.tolist())
    assert np.all(iters % 5 == 0) and np.all(iters <= cap) and np.all(iters > 0)
    assert np.all((done == 1) | (iters == cap))
    off = batch.goal_off()

    def plain(s, k):
        one = S.Batch([batch.scenes[s]])
        dbs = T.DeviceBatch.from_batch(one, shapes=batch.shapes())
        sts = T.DeviceState.empty(one.n_goals)
        solver.solve(dbs, sts, k, precision=precision)
        vr = v_ref[s:s + 1]
        cs = torch.zeros(one.n_goals, device="cuda")
        bs = torch.zeros(1, device="cuda", dtype=torch.int32)
        solver.score(dbs, sts, vr, cs, bs)
        torch.cuda.synchronize()
        b = int(bs.item())
        worst = float(sts.resid[:3, b].max().item()) if b >= 0 else float("inf")
        return sts.c.cpu().numpy(), worst

    for s in range(batch.n_scenes):
        cs, worst = plain(s, int(iters[s]))
        assert np.array_equal(cs, c[:, :, off[s]:off[s + 1]]), s
        if done[s]:
            assert worst <= tol
            if iters[s] > 5:
                _, worst_before = plain(s, int(iters[s]) - 5)
                assert worst_before > tol, s
    solver.close()


@pytest.mark.parametrize("bad,precision", [("far", "fp32"), ("nan", "fp32"), ("huge", "fp32"), ("nan", "bf16x3"),
                                           ("huge", "bf16x3")])
def test_warm_fallback_keeps_the_better_start_per_goal(T, bad, precision):
    """Every third goal starts from a corrupted state (values of order 1e3, NaN,
    or 1e30 whose products overflow). Each goal keeps the start whose residual
    max(r_obs, r_acc, r_nh) after one iteration is lower (a NaN residual loses),
    read here from plain one-iteration solves, and then ends exactly where the
    plain solve from that start ends. The corrupted goals always fall back; the
    others, started near the fixed point, keep the warm start except where both
    residuals are at rounding level (a straight goal: either start may win)."""
    batch = small_batch()
    n = batch.n_goals
    good = run(T, batch, 150)                      # near the fixed point: warm wins
    rng = np.random.default_rng(0)
    if bad == "far":
        bad_c = rng.normal(0, 1e3, (3, 11, n)).astype(np.float32)
        bad_l = rng.normal(0, 1e3, (3, 11, n)).astype(np.float32)
    elif bad == "nan":
        bad_c = np.full((3, 11, n), np.nan, np.float32)
        bad_l = rng.normal(0, 1.0, (3, 11, n)).astype(np.float32)
    else:
        bad_c = np.full((3, 11, n), 1e30, np.float32)
        bad_l = np.full((3, 11, n), -1e30, np.float32)
    use_good = (np.arange(n) % 3) != 0
    init_c = np.where(use_good[None, None], good[0], bad_c)
    init_l = np.where(use_good[None, None], good[1], bad_l)
    r_warm = run(T, batch, 1, init=(init_c, init_l), precision=precision)[2][:3].max(0)
    r_cold = run(T, batch, 1, precision=precision)[2][:3].max(0)
    keep_warm = r_warm <= r_cold                   # NaN compares false: the cold start
    assert not keep_warm[~use_good].any()
    assert np.count_nonzero(keep_warm[use_good]) >= 0.8 * np.count_nonzero(use_good)
    flipped = [(g, float(r_warm[g]), float(r_cold[g])) for g in np.flatnonzero(use_good & ~keep_warm)]
    print(f"good goals that keep the cold start (index, warm, cold residual): {flipped}")
    for g, rw, rc in flipped:
        assert rc < 1e-4, (g, rw, rc)              # only where both are at rounding level
    got = run(T, batch, 25, init=(init_c, init_l), fallback=True, precision=precision)
    warm = run(T, batch, 25, init=(init_c, init_l), precision=precision)
    cold = run(T, batch, 25, precision=precision)
    for g in range(n):
        ref = warm if keep_warm[g] else cold
        assert np.array_equal(got[0][:, :, g], ref[0][:, :, g]), g
        assert np.array_equal(got[1][:, :, g], ref[1][:, :, g]), g


def test_warm_fallback_needs_the_group_kernel(T):
    import ctypes
    batch = small_batch()
    solver = T.Solver(PARAMS, batch.shapes())
    solver.set_tile("wave", 16)
    db = T.DeviceBatch.from_batch(batch)
    st = T.DeviceState.empty(batch.n_goals)
    b, s = db.c_struct(), st.c_struct()
    rc = T.lib().traj_solve_batch(solver.handle, ctypes.byref(b), ctypes.byref(s), 5, 0.0,
                                  T.TRAJ_INIT_FROM_STATE | T.TRAJ_WARM_FALLBACK, T._stream(None))
    assert rc == -1
    rc = T.lib().traj_solve_batch(solver.handle, ctypes.byref(b), ctypes.byref(s), 5, 0.0, T.TRAJ_WARM_FALLBACK,
                                  T._stream(None))
    assert rc == -1
    solver.close()
