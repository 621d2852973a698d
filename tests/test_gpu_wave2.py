"""Wave kernel with two wavefronts per goal (each holds half of the time samples;
partial contractions are added through LDS in a fixed order): the same parity
gate against the oracle as one wave per goal, at the dense size (the tile the
benchmark uses) and on ragged shapes up to 150 samples."""
import numpy as np
import pytest

from paper_2109_10392_amd import scenes as S
from tests.test_gpu_parity import TOL, check_gate, coef_err, gpu_solve, oracle_scene, ragged_batch

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
def test_two_waves_small_parity(T, seed):
    batch = S.workload_small(seed)
    out = gpu_solve(T, batch, 100, kernel="wave", waves=2)
    prob, st = oracle_scene(batch.scenes[0], 100)
    print(f"seed {seed}:")
    check_gate(out["c"], prob, batch.scenes[0], st, 100)


def test_two_waves_dense_sampled(T):
    batch = S.workload_dense(0)
    out = gpu_solve(T, batch, 100, kernel="wave", waves=2)
    sample = [0, 1, 2, 3, 4, 5, 63, 64, 255, 256, 511, 700, 1000, 1021, 1022, 1023]
    prob, st = oracle_scene(batch.scenes[0], 100, goals=sample)
    print("dense, sampled goals:")
    check_gate(out["c"][:, :, sample], prob, batch.scenes[0], st, 100, goals=sample)
    assert np.all(np.isfinite(out["c"])) and np.all(np.isfinite(out["resid"]))


def test_two_waves_ragged(T):
    batch = ragged_batch()
    out = gpu_solve(T, batch, 40, kernel="wave", waves=2)
    off = batch.goal_off()
    for i, sc in enumerate(batch.scenes):
        prob, st = oracle_scene(sc, 40)
        print(f"scene {i} (n={sc.n_time}, m={sc.obs.shape[0]}, B={sc.goals.shape[0]}):")
        check_gate(out["c"][:, :, off[i]:off[i + 1]], prob, sc, st, 40, max_undetermined=0.5)


def test_two_waves_resume_and_zero_iterations(T):
    batch = S.workload_small(5)
    full = gpu_solve(T, batch, 100, kernel="wave", waves=2)
    part = gpu_solve(T, batch, 40, kernel="wave", waves=2)
    rest = gpu_solve(T, batch, 60, init=dict(c=part["c"], lam=part["lam"]), kernel="wave", waves=2)
    for k in ("c", "lam", "resid"):
        assert np.array_equal(full[k], rest[k]), k
    zero = gpu_solve(T, S.workload_small(3), 0, kernel="wave", waves=2)
    _, st = oracle_scene(S.workload_small(3).scenes[0], 0)
    assert coef_err(zero["c"], st).max() <= TOL and np.all(zero["lam"] == 0)


def test_two_waves_tolerance_stop(T):
    batch = S.workload_small(2)
    out = gpu_solve(T, batch, 300, tol=1e-3, kernel="wave", waves=2)
    it = out["iters"]
    assert np.all(it % 5 == 0) and np.all((it > 0) & (it <= 300))
    stopped = it < 300
    assert stopped.any()
    assert np.all(out["resid"][:3, stopped].max(0) <= 1e-3)
