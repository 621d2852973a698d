"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Gate (per goal and axis, after a fixed iteration count):
    max_k |c_gpu - c_oracle| / max(max_k |c_oracle|, 1) <= 1e-4
and the same best-goal index (or a near-tie of the meta-cost). The oracle runs
on the same seeded scenes; at the dense size only a sample of goals is checked
(goals are independent instances, Remark 1), in the same launch configuration
the benchmark times.
"""
import math

import numpy as np
import pytest

from oracle import traj_oracle as O
from paper_2109_10392_amd import scenes as S

pytestmark = pytest.mark.gpu

PARAMS = S.DEFAULT_PARAMS
TOL = 1e-4
# The split-BF16 form keeps about 16 of FP32's 24 significant bits in its split
# evaluations and contractions (the x/y applies stay FP64, the heading path FP32,
# positions are split relative to their end-to-end line); its gate on the same
# measure, for determined goals, is a decade above FP32's.
TOL_BF16X3 = 1e-3


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_10392_amd import traj
    traj.lib()
    return traj


def gpu_solve(T, batch, iters, init=None, tol=0.0, params=PARAMS, shapes=None, kernel="auto", precision="fp32",
              group=16, persistent=True, waves=1):
    import torch
    solver = T.Solver(params, shapes or batch.shapes())
    solver.set_tile("wave" if kernel == "auto" else kernel, group, persistent, waves)
    db = T.DeviceBatch.from_batch(batch, shapes=shapes)
    st = T.DeviceState.empty(batch.n_goals)
    if init is not None:
        st.c.copy_(torch.from_numpy(init["c"]).cuda())
        st.lam.copy_(torch.from_numpy(init["lam"]).cuda())
    solver.solve(db, st, iters, tol=tol, from_state=init is not None, kernel=kernel, precision=precision)
    torch.cuda.synchronize()
    out = dict(c=st.c.cpu().numpy(), lam=st.lam.cpu().numpy(), resid=st.resid.cpu().numpy(),
               iters=st.iters.cpu().numpy())
    solver.close()
    return out


def oracle_scene(sc, iters, goals=None):
    prob = O.Problem(sc.n_time, sc.t_f, sc.obs.shape[0], PARAMS)
    g = sc.goals if goals is None else sc.goals[goals]
    return prob, O.solve(prob, sc.ego, sc.obs, g, iters)


def undetermined_goals(prob, sc, st, iters, goals=None, shift=1e-6, thresh=1e-5):
    """Goals whose FP64 result is not determined at single precision.

    The oracle is re-run with every goal's final lateral position moved by
    `shift` metres (far below FP32 resolution of the inputs' scale). Where that
    changes the FP64 coefficients by more than `thresh` (relative), the instance
    sits on a bifurcation (e.g. an obstacle centred in the goal's own lane makes
    swerving left and right equally good) and any rounding decides the branch:
    several results are correct there.
    """
    g = (sc.goals if goals is None else sc.goals[goals]).astype(np.float64).copy()
    g[:, 1] += shift
    st2 = O.solve(prob, sc.ego, sc.obs, g, iters)
    c64 = np.stack([st.c_x, st.c_y, st.c_psi])
    return coef_err(c64, st2).max(0) > thresh


def check_gate(out_c, prob, sc, st, iters, goals=None, max_undetermined=0.35, tol=TOL):
    err = coef_err(out_c, st).max(0)
    und = undetermined_goals(prob, sc, st, iters, goals)
    print(f"  gated goals: {np.count_nonzero(~und)}/{und.size}, max rel err {err[~und].max() if (~und).any() else 0:.2e}; "
          f"undetermined (bifurcating) goals {np.flatnonzero(und).tolist()} err {np.array2string(err[und], precision=1)}")
    assert np.all(err[~und] <= tol), err
    assert np.count_nonzero(und) <= max_undetermined * und.size
    # undetermined goals: still a valid iterate (finite, boundary rows of eq. 8b met)
    assert np.all(np.isfinite(out_c))
    c = out_c.astype(np.float64)
    g = sc.goals if goals is None else sc.goals[goals]
    b_x, b_y, b_psi = O.boundary_values(sc.ego, g)
    for A, ax, b in ((prob.A_x, 0, b_x), (prob.A_y, 1, b_y), (prob.A_psi, 2, b_psi)):
        assert np.max(np.abs(A @ c[ax] - b)) <= 1e-3 * max(1.0, np.max(np.abs(b)))
    return err, und


def coef_err(c_gpu, st):
    """[3, B] relative error per axis and goal; c_gpu is [3, 11, B]."""
    errs = []
    for ax, name in enumerate(("c_x", "c_y", "c_psi")):
        ref = getattr(st, name)
        num = np.max(np.abs(c_gpu[ax].astype(np.float64) - ref), axis=0)
        den = np.maximum(np.max(np.abs(ref), axis=0), 1.0)
        errs.append(num / den)
    return np.array(errs)


def test_reduce_lane_layout(T):
    import torch
    rng = np.random.default_rng(0)
    for r in (16, 32):
        vals = rng.integers(-1000, 1000, size=(r, 64)).astype(np.float32)
        out = torch.zeros(64, device="cuda")
        T.debug_reduce(torch.from_numpy(vals).cuda(), out, r)
        torch.cuda.synchronize()
        sums = vals.astype(np.float64).sum(axis=1)
        expect = sums[np.arange(64) // (64 // r)]
        assert np.array_equal(out.cpu().numpy().astype(np.float64), expect)


def test_heading_atan2_accuracy_and_special_cases(T):
    """The solver's atan2 against FP64 arctan2: at most 3 units in the last place
    over all octants and magnitudes, and IEEE results on the special cases."""
    import torch
    rng = np.random.default_rng(11)
    ang = rng.uniform(-np.pi, np.pi, 200000)
    mag = 10.0 ** rng.uniform(-30, 30, ang.size)
    y = np.concatenate([mag * np.sin(ang), rng.normal(0, 1, 50000)]).astype(np.float32)
    x = np.concatenate([mag * np.cos(ang), rng.normal(0, 1, 50000)]).astype(np.float32)
    sp = [(0.0, 0.0), (-0.0, 0.0), (0.0, -0.0), (-0.0, -0.0), (1.0, 0.0), (-1.0, 0.0), (0.0, 1.0), (0.0, -1.0),
          (np.inf, np.inf), (-np.inf, np.inf), (np.inf, -np.inf), (-np.inf, -np.inf), (3.0, np.inf), (3.0, -np.inf),
          (np.inf, 2.0), (-np.inf, 2.0), (1e-40, 1e-40), (1e-40, 0.0), (np.nan, 1.0), (1.0, np.nan), (5.0, 5.0),
          (-5.0, 5.0), (2.0, 1e-39)]
    y = np.concatenate([y, np.array([p[0] for p in sp], np.float32)])
    x = np.concatenate([x, np.array([p[1] for p in sp], np.float32)])
    out = torch.empty(y.size, device="cuda")
    T.debug_atan2(torch.from_numpy(y).cuda(), torch.from_numpy(x).cuda(), out)
    got = out.cpu().numpy()
    ref = np.arctan2(y.astype(np.float64), x.astype(np.float64))
    fin = np.isfinite(ref)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ulp = np.abs(got[fin] - ref[fin]) / np.spacing(np.abs(ref[fin]).astype(np.float32)).astype(np.float64)
    assert ulp.max() <= 3.0, ulp.max()
    k = y.size - len(sp)
    assert np.array_equal(np.signbit(got[k:k + 4]), np.signbit(ref[k:k + 4]))  # signed zeros and pi


@pytest.mark.parametrize("shape", [(100, 10.0, 10), (50, 5.0, 4), (150, 15.0, 64), (100, 10.0, 0)])
def test_setup_inverses_match_oracle(T, shape):
    n, tf, m = shape
    solver = T.Solver(PARAMS, [shape])
    inv64, tab = solver.operators(0)
    solver.close()
    prob = O.Problem(n, tf, m, PARAMS)
    N = 11
    ix = list(range(N)) + list(range(2 * N, 2 * N + 4))
    iy = list(range(N, 2 * N)) + list(range(2 * N + 4, 2 * N + 10))
    Jxy = np.linalg.inv(prob.Q_xy)
    J0 = np.linalg.inv(prob.Q_0)
    refs = [Jxy[np.ix_(ix, ix)], Jxy[np.ix_(iy, iy)], np.linalg.inv(prob.Q_psi), J0[np.ix_(ix, ix)],
            J0[np.ix_(iy, iy)]]
    for sys, ref in enumerate(refs):
        k = ref.shape[0]
        got = inv64[sys, :k, :k]
        assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-9, sys
    # FP32 basis table against the oracle's basis
    P32 = tab[:11 * n].reshape(11, n).T
    assert np.max(np.abs(P32 - prob.P)) < 1e-6


@pytest.mark.parametrize("seed", range(10))
def test_small_workload_parity(T, seed):
    batch = S.workload_small(seed)
    out = gpu_solve(T, batch, 100)
    prob, st = oracle_scene(batch.scenes[0], 100)
    print(f"seed {seed}:")
    err, und = check_gate(out["c"], prob, batch.scenes[0], st, 100)
    # residuals agree to the same scale on the determined goals
    assert np.allclose(out["resid"][:3, ~und], st.resid[:3, ~und], rtol=1e-2, atol=1e-3)
    # same best goal (meta-cost of eq. 25 recomputed in FP64 from the GPU coefficients)
    cg = out["c"].astype(np.float64)
    v0 = float(batch.scenes[0].ego[2])
    cost_g = O.meta_cost(prob, cg[0], cg[1], cg[2], 0, v_ref=v0)
    cost_o = O.meta_cost(prob, st.c_x, st.c_y, st.c_psi, 0, v_ref=v0)
    bg, bo = O.best_goal(cost_g), O.best_goal(cost_o)
    if bg != bo and not (und[bg] or und[bo]):
        assert bg >= 0 and bo >= 0 and abs(cost_o[bg] - cost_o[bo]) <= 1e-6 * max(1.0, abs(cost_o[bo]))


def test_dense_workload_sampled_goals(T):
    batch = S.workload_dense(0)
    out = gpu_solve(T, batch, 100)
    sample = [0, 1, 2, 3, 4, 5, 63, 64, 255, 256, 511, 700, 1000, 1021, 1022, 1023]
    prob, st = oracle_scene(batch.scenes[0], 100, goals=sample)
    print("dense, sampled goals:")
    check_gate(out["c"][:, :, sample], prob, batch.scenes[0], st, 100, goals=sample)
    assert np.all(np.isfinite(out["c"])) and np.all(np.isfinite(out["resid"]))


def ragged_batch():
    scenes = [S.make_scene(11, n_goals=7, n_obs=4, n_lanes=6, n_time=50, t_f=5.0),
              S.make_scene(12, n_goals=5, n_obs=0, n_lanes=4, n_time=100, t_f=10.0),
              S.make_scene(13, n_goals=9, n_obs=64, n_lanes=6, n_time=150, t_f=15.0),
              S.make_scene(14, n_goals=1, n_obs=10, n_lanes=4, n_time=100, t_f=10.0),
              S.make_scene(15, n_goals=6, n_obs=23, n_lanes=6, n_time=73, t_f=7.3)]
    return S.Batch(scenes)


def test_ragged_multi_shape_batch(T):
    batch = ragged_batch()
    out = gpu_solve(T, batch, 40)
    off = batch.goal_off()
    for i, sc in enumerate(batch.scenes):
        prob, st = oracle_scene(sc, 40)
        print(f"scene {i} (n={sc.n_time}, m={sc.obs.shape[0]}, B={sc.goals.shape[0]}):")
        check_gate(out["c"][:, :, off[i]:off[i + 1]], prob, sc, st, 40, max_undetermined=0.5)


def test_zero_iterations_is_the_cold_start(T):
    batch = S.workload_small(3)
    out = gpu_solve(T, batch, 0)
    _, st = oracle_scene(batch.scenes[0], 0)
    assert coef_err(out["c"], st).max() <= 1e-5
    assert np.all(out["lam"] == 0)
    assert np.allclose(out["resid"], st.resid, rtol=1e-3, atol=1e-4)


def test_resume_equals_continuous_run_bitwise(T):
    batch = S.workload_small(5)
    full = gpu_solve(T, batch, 100)
    part = gpu_solve(T, batch, 40)
    rest = gpu_solve(T, batch, 60, init=dict(c=part["c"], lam=part["lam"]))
    for k in ("c", "lam", "resid"):
        assert np.array_equal(full[k], rest[k]), k


def test_duplicate_goals_are_bitwise_identical(T):
    sc = S.workload_small(6).scenes[0]
    sc.goals = sc.goals[[2, 5, 2, 2, 9]]
    out = gpu_solve(T, S.Batch([sc]), 50)
    assert np.array_equal(out["c"][:, :, 0], out["c"][:, :, 2])
    assert np.array_equal(out["c"][:, :, 0], out["c"][:, :, 3])


def test_unknown_shape_marks_scene_nan_without_touching_others(T):
    import torch
    batch = S.Batch([S.make_scene(1, 5, 10), S.make_scene(2, 3, 10)])
    solver = T.Solver(PARAMS, batch.shapes())
    db = T.DeviceBatch.from_batch(batch)
    db.shape_id[1] = 7  # not set up
    st = T.DeviceState.empty(batch.n_goals)
    solver.solve(db, st, 20)
    torch.cuda.synchronize()
    r = st.resid.cpu().numpy()
    assert np.all(np.isnan(r[:, 5:])) and np.all(np.isfinite(r[:, :5]))
    solver.close()


def test_empty_batch_is_a_no_op(T):
    import torch
    solver = T.Solver(PARAMS, [(100, 10.0, 10)])
    db = T.DeviceBatch.from_batch(S.Batch([S.make_scene(1, 1, 10)]))
    db.n_goals = 0
    db.n_scenes = 0
    st = T.DeviceState.empty(1)
    solver.solve(db, st, 10)
    torch.cuda.synchronize()
    solver.close()


def test_tolerance_stop(T):
    batch = S.workload_small(2)
    out = gpu_solve(T, batch, 300, tol=1e-3)
    it = out["iters"]
    assert np.all(it % 5 == 0) and np.all((it > 0) & (it <= 300))
    stopped = it < 300
    assert stopped.any()
    assert np.all(out["resid"][:3, stopped].max(0) <= 1e-3)


def test_score_matches_oracle(T):
    import torch
    batch = S.Batch([S.workload_small(s).scenes[0] for s in range(4)] + [S.make_scene(9, 16, 10)])
    solver = T.Solver(PARAMS, batch.shapes())
    db = T.DeviceBatch.from_batch(batch)
    st = T.DeviceState.empty(batch.n_goals)
    solver.solve(db, st, 60)
    v_ref = torch.tensor([float(s.ego[2]) for s in batch.scenes], device="cuda")
    y_rl = torch.full((batch.n_scenes,), -3.5, device="cuda")
    for kind in (0, 1):
        cost = torch.zeros(batch.n_goals, device="cuda")
        best = torch.zeros(batch.n_scenes, device="cuda", dtype=torch.int32)
        solver.score(db, st, v_ref, cost, best, kind=kind, w1=1.0, w2=0.5, y_rl=y_rl)
        torch.cuda.synchronize()
        c = st.c.cpu().numpy().astype(np.float64)
        cg, bg = cost.cpu().numpy(), best.cpu().numpy()
        off = batch.goal_off()
        for i, sc in enumerate(batch.scenes):
            prob = O.Problem(sc.n_time, sc.t_f, sc.obs.shape[0], PARAMS)
            sl = slice(off[i], off[i + 1])
            ref = O.meta_cost(prob, c[0][:, sl], c[1][:, sl], c[2][:, sl], kind, v_ref=float(sc.ego[2]),
                              w1=1.0, w2=0.5, y_rl=-3.5)
            fin = np.isfinite(ref)
            assert np.array_equal(np.isfinite(cg[sl]), fin)
            assert np.allclose(cg[sl][fin], ref[fin], rtol=1e-4, atol=1e-3)
            bo = O.best_goal(ref)
            if bg[i] != bo:
                assert bo >= 0 and abs(ref[bg[i]] - ref[bo]) <= 1e-4 * max(1.0, abs(ref[bo]))
    solver.close()


@pytest.mark.parametrize("tile", [("wave", 1, 192), ("wave", 2, 192), ("group", 1, 192), ("mfma", 1, 176)])
def test_largest_horizon_and_obstacle_count(T, tile):
    """The largest shape each kernel takes with 64 obstacles against the oracle:
    n_time = 192 (the handle's limit, three 64-lane slots) on the wave and group
    kernels, 176 on the MFMA kernel (its LDS budget)."""
    kernel, waves, n = tile
    sc = S.make_scene(17, n_goals=6, n_obs=64, n_lanes=6, n_time=n, t_f=(n - 1) / 10.0)
    batch = S.Batch([sc])
    out = gpu_solve(T, batch, 60, kernel=kernel, waves=waves)
    prob, st = oracle_scene(sc, 60)
    print(f"n={n}, m=64, {tile}:")
    check_gate(out["c"], prob, sc, st, 60, max_undetermined=0.5)


@pytest.mark.parametrize("tile", [("wave", 1), ("group", 1)])
def test_smallest_horizon_is_valid(T, tile):
    """n_time = 11 (as many samples as coefficients; the x/y system's condition
    number is ~6e7, so FP32 is not held to the 1e-4 gate): finite iterates that
    meet the boundary rows."""
    kernel, waves = tile
    sc = S.make_scene(18, n_goals=5, n_obs=4, n_lanes=4, n_time=11, t_f=1.0)
    batch = S.Batch([sc])
    out = gpu_solve(T, batch, 30, kernel=kernel, waves=waves)
    assert np.all(np.isfinite(out["c"]))
    prob = O.Problem(sc.n_time, sc.t_f, sc.obs.shape[0], PARAMS)
    b_x, b_y, b_psi = O.boundary_values(sc.ego, sc.goals)
    c = out["c"].astype(np.float64)
    for A, ax, b in ((prob.A_x, 0, b_x), (prob.A_y, 1, b_y), (prob.A_psi, 2, b_psi)):
        assert np.max(np.abs(A @ c[ax] - b)) <= 1e-2 * max(1.0, np.max(np.abs(b)))


def test_mfma_kernel_rejects_a_horizon_beyond_its_lds_budget(T):
    sc = S.make_scene(17, n_goals=3, n_obs=64, n_lanes=6, n_time=192, t_f=19.1)
    with pytest.raises(T.TrajError, match="MFMA kernel keeps every obstacle prediction"):
        gpu_solve(T, S.Batch([sc]), 5, kernel="mfma")
