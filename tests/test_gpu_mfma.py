"""Matrix-core kernel: FP32 parity with the oracle, invariances, and the split-BF16 precision report.

The FP32 form runs the same gate as the wave kernel (1e-4 per goal and axis,
bifurcating goals checked for validity). The split-BF16 form (basis evaluations
and contractions on split-BF16 MFMA with FP32 accumulation, x/y applies in FP64,
the heading path in FP32) is held to 1e-3 on the same measure; its coefficient
and residual errors against the FP64 oracle are reported per scene, and the test
checks that they are finite and that the best goal is the oracle's (or a near-tie).
"""
import json

import numpy as np
import pytest

from tests.conftest import report_path

from oracle import traj_oracle as O
from paper_2109_10392_amd import scenes as S
from tests.test_gpu_parity import (TOL, TOL_BF16X3, check_gate, coef_err, gpu_solve, oracle_scene, ragged_batch,
                                   undetermined_goals)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_10392_amd import traj
    traj.lib()
    return traj


@pytest.mark.parametrize("seed", range(5))
def test_mfma_fp32_small_parity(T, seed):
    batch = S.workload_small(seed)
    out = gpu_solve(T, batch, 100, kernel="mfma")
    prob, st = oracle_scene(batch.scenes[0], 100)
    print(f"seed {seed}:")
    check_gate(out["c"], prob, batch.scenes[0], st, 100)


_DENSE_ORACLE = {}


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_mfma_dense_sampled(T, precision):
    """Dense scene (1024 goals, 50 obstacles), sampled goals against the oracle:
    FP32 at 1e-4, the split-BF16 form at 1e-3."""
    batch = S.workload_dense(0)
    out = gpu_solve(T, batch, 100, kernel="mfma", precision=precision)
    sample = [0, 1, 2, 3, 4, 5, 63, 64, 255, 256, 511, 700, 1000, 1021, 1022, 1023]
    if "ref" not in _DENSE_ORACLE:
        _DENSE_ORACLE["ref"] = oracle_scene(batch.scenes[0], 100, goals=sample)
    prob, st = _DENSE_ORACLE["ref"]
    print(f"dense, sampled goals ({precision}):")
    check_gate(out["c"][:, :, sample], prob, batch.scenes[0], st, 100, goals=sample,
               tol=TOL if precision == "fp32" else TOL_BF16X3)
    assert np.all(np.isfinite(out["c"]))


_RAGGED_ORACLE = {}


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_mfma_ragged(T, precision):
    """Scenes of different horizons, obstacle and goal counts in one launch, each
    against the oracle: FP32 at 1e-4, the split-BF16 form at 1e-3."""
    batch = ragged_batch()
    out = gpu_solve(T, batch, 40, kernel="mfma", precision=precision)
    off = batch.goal_off()
    for i, sc in enumerate(batch.scenes):
        if i not in _RAGGED_ORACLE:
            _RAGGED_ORACLE[i] = oracle_scene(sc, 40)
        prob, st = _RAGGED_ORACLE[i]
        print(f"scene {i} (n={sc.n_time}, m={sc.obs.shape[0]}, B={sc.goals.shape[0]}, {precision}):")
        check_gate(out["c"][:, :, off[i]:off[i + 1]], prob, sc, st, 40, max_undetermined=0.5,
                   tol=TOL if precision == "fp32" else TOL_BF16X3)


def test_mfma_group_size_does_not_change_results(T):
    batch = S.Batch([S.make_scene(21, 37, 12, n_lanes=6), S.make_scene(22, 5, 3, n_lanes=4)])
    ref = gpu_solve(T, batch, 30, kernel="mfma", group=16)
    for group in (1, 4, 7):
        out = gpu_solve(T, batch, 30, kernel="mfma", group=group)
        for k in ("c", "lam", "resid"):
            assert np.array_equal(out[k], ref[k]), (group, k)


def test_mfma_resume_equals_continuous_bitwise(T):
    batch = S.workload_small(5)
    full = gpu_solve(T, batch, 100, kernel="mfma")
    part = gpu_solve(T, batch, 40, kernel="mfma")
    rest = gpu_solve(T, batch, 60, init=dict(c=part["c"], lam=part["lam"]), kernel="mfma")
    for k in ("c", "lam", "resid"):
        assert np.array_equal(full[k], rest[k]), k


def test_mfma_zero_iterations_is_the_cold_start(T):
    batch = S.workload_small(3)
    out = gpu_solve(T, batch, 0, kernel="mfma")
    _, st = oracle_scene(batch.scenes[0], 0)
    assert coef_err(out["c"], st).max() <= TOL
    assert np.all(out["lam"] == 0)


def test_mfma_tolerance_stop(T):
    batch = S.workload_small(2)
    out = gpu_solve(T, batch, 300, tol=1e-3, kernel="mfma", group=1)
    it = out["iters"]
    assert np.all(it % 5 == 0) and np.all((it > 0) & (it <= 300))
    stopped = it < 300
    assert stopped.any()
    assert np.all(out["resid"][:3, stopped].max(0) <= 1e-3)


def test_bf16x3_precision_report(T):
    """Precision form on the 11-goal scenes: error vs FP64 reported per scene and
    held to the split form's gate."""
    rows = []
    for seed in range(10):
        batch = S.workload_small(seed)
        sc = batch.scenes[0]
        out = gpu_solve(T, batch, 100, kernel="mfma", precision="bf16x3")
        prob, st = oracle_scene(sc, 100)
        und = undetermined_goals(prob, sc, st, 100)
        err = coef_err(out["c"], st).max(0)
        res_err = np.abs(out["resid"][:3] - st.resid[:3]).max(0)
        assert np.all(np.isfinite(out["c"])) and np.all(np.isfinite(out["resid"]))
        cg = out["c"].astype(np.float64)
        # boundary constraints of eq. 8b at the computed coefficients (relative to max(|b|, 1))
        b_x, b_y, b_psi = O.boundary_values(sc.ego, sc.goals)
        cons = max(float(np.max(np.abs(A @ cg[ax] - b)) / max(1.0, float(np.max(np.abs(b)))))
                   for A, ax, b in ((prob.A_x, 0, b_x), (prob.A_y, 1, b_y), (prob.A_psi, 2, b_psi)))
        v0 = float(sc.ego[2])
        cost_g = O.meta_cost(prob, cg[0], cg[1], cg[2], 0, v_ref=v0)
        cost_o = O.meta_cost(prob, st.c_x, st.c_y, st.c_psi, 0, v_ref=v0)
        bg, bo = O.best_goal(cost_g), O.best_goal(cost_o)
        near = bg == bo or (bg >= 0 and bo >= 0 and abs(cost_o[bg] - cost_o[bo]) <= 1e-3 * max(1.0, abs(cost_o[bo])))
        rows.append(dict(seed=seed, coef_err_max=float(err[~und].max()), coef_err_median=float(np.median(err[~und])),
                         resid_abs_err_max=float(res_err[~und].max()), constraint_resid_max=cons,
                         best_gpu=bg, best_oracle=bo,
                         best_match=bool(near), undetermined=np.flatnonzero(und).tolist()))
        print(json.dumps(rows[-1]))
    with open(report_path("bf16x3_precision_report.json"), "w") as f:
        json.dump(rows, f, indent=1)
    assert sum(r["best_match"] for r in rows) >= 9
    assert max(r["coef_err_max"] for r in rows) <= TOL_BF16X3
    assert max(r["constraint_resid_max"] for r in rows) <= 1e-3
