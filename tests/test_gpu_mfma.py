"""Matrix-core kernel: FP32 parity with the oracle, invariances, and the split-BF16 precision report.

The FP32 form runs the same gate as the wave kernel (1e-4 per goal and axis;
bifurcating goals checked by one oracle iteration from the GPU's own state). The
split-BF16 form (basis evaluations and x/y contractions in two-way split BF16,
the x/y and heading applies in three-way split BF16, FP32 accumulation, no FP64)
is held to 1e-3 on the same measure; its coefficient, multiplier and residual
errors against the FP64 oracle are reported per scene.
"""

import numpy as np
import pytest

from paper_2109_10392_amd import scenes as S
from tests.test_gpu_parity import (DENSE_SAMPLE, TOL, TOL_BF16X3, TOL_BF16X3_LARGE, coef_err, gate_batch, gpu_solve,
                                   oracle_scene, precision_report, ragged_batch)

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
    print(f"seed {seed}:")
    gate_batch(T, batch, 100, out, kernel="mfma")


_DENSE_ORACLE = {}


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_mfma_dense_sampled(T, precision):
    """Dense scene (1024 goals, 50 obstacles), sampled goals against the oracle:
    FP32 at 1e-4, the split-BF16 form at 1e-3."""
    batch = S.workload_dense(0)
    out = gpu_solve(T, batch, 100, kernel="mfma", precision=precision)
    print(f"dense, sampled goals ({precision}):")
    gate_batch(T, batch, 100, out, goals={0: DENSE_SAMPLE}, oracle_cache=_DENSE_ORACLE, kernel="mfma",
               precision=precision, tol=TOL if precision == "fp32" else TOL_BF16X3_LARGE)
    assert np.all(np.isfinite(out["c"]))


_RAGGED_ORACLE = {}


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_mfma_ragged(T, precision):
    """Scenes of different horizons, obstacle and goal counts in one launch, each
    against the oracle: FP32 at 1e-4, the split-BF16 form at 1e-3."""
    batch = ragged_batch()
    out = gpu_solve(T, batch, 40, kernel="mfma", precision=precision)
    print(precision)
    gate_batch(T, batch, 40, out, oracle_cache=_RAGGED_ORACLE, kernel="mfma",
               precision=precision, tol=TOL if precision == "fp32" else TOL_BF16X3_LARGE)


def test_mfma_group_size_does_not_change_results(T):
    batch = S.Batch([S.make_scene(21, 37, 12, n_lanes=6), S.make_scene(22, 5, 3, n_lanes=4)])
    ref = gpu_solve(T, batch, 30, kernel="mfma", group=16)
    for group in (1, 4, 7):
        out = gpu_solve(T, batch, 30, kernel="mfma", group=group)
        for k in ("c", "lam", "resid"):
            assert np.array_equal(out[k], ref[k]), (group, k)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_mfma_resume_equals_continuous_bitwise(T, precision):
    batch = S.workload_small(5)
    full = gpu_solve(T, batch, 100, kernel="mfma", precision=precision)
    part = gpu_solve(T, batch, 40, kernel="mfma", precision=precision)
    rest = gpu_solve(T, batch, 60, init=dict(c=part["c"], lam=part["lam"]), kernel="mfma", precision=precision)
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


@pytest.mark.parametrize("chunk", range(10))
def test_bf16x3_precision_report(T, chunk):
    """Precision form (config 3: the 11-goal scenes, seeds 0-99) on the mfma kernel:
    the gate at 1e-3 and the per-scene errors against the FP64 oracle in
    bf16x3_precision_report.json."""
    precision_report(T, "mfma", "bf16x3", range(10 * chunk, 10 * chunk + 10), "bf16x3_precision_report.json",
                     TOL_BF16X3)
