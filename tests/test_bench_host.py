"""Host logic of bench.py (CPU): the measured HBM traffic is reported only for the
kernel, tile and precision form its counters were taken on."""
import bench


def test_traffic_only_for_the_profiled_configuration():
    assert bench.measured_traffic("uneven", "group", None, "bf16x3") is None
    assert bench.measured_traffic("uneven", "mfma", None, "fp32") is None
    assert bench.measured_traffic("dense", "wave", 1, "fp32") is None
    assert bench.measured_traffic("dense", "mfma", 2, "fp32") is None
    for workload, kernel, waves in (("dense", "wave", 2), ("uneven", "group", None)):
        m = bench.MEASURED_TRAFFIC[workload]
        got = bench.measured_traffic(workload, kernel, waves, "fp32")
        # the profiled configuration: the figure while its sources are unchanged, else nothing
        assert got == (m["bytes_per_launch"] if bench.sources_hash(m["sources"]) == m["sha256"] else None)


def test_more_than_one_gpu_exits_with_a_message():
    import subprocess
    import sys
    out = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert out.returncode != 0 and "one GPU" in out.stdout + out.stderr


def test_parity_statement_splits_determined_goals():
    """parity_vs_oracle: per-goal relative coefficient error on the measure of the
    parity tests (max over axes of max |dc| / max(max |c_ref|, 1)), reported over
    all goals and over the determined ones."""
    import numpy as np
    rng = np.random.default_rng(0)
    c_ref = rng.normal(0.0, 5.0, (3, 11, 6))
    c = c_ref.copy()
    c[1, 3, 0] += 1e-5 * max(np.abs(c_ref[1, :, 0]).max(), 1.0)   # goal 0: 1e-5
    c[2, 7, 1] += 0.5 * max(np.abs(c_ref[2, :, 1]).max(), 1.0)    # goal 1: 0.5, at a bifurcation
    c[0, 0, 2] += 3e-4 * max(np.abs(c_ref[0, :, 2]).max(), 1.0)   # goal 2: 3e-4, determined
    bif = np.array([False, True, False, False, False, False])
    err = bench._rel_coef_err(c, c_ref)
    assert np.allclose(err, [1e-5, 0.5, 3e-4, 0, 0, 0], rtol=1e-9, atol=1e-15)
    out = bench.parity_vs_oracle(c, c_ref, bif, 4, 4)
    assert out["goals"] == 6 and out["within_1e-4"] == 4 and out["within_1e-3"] == 5
    assert out["determined_goals"] == 5 and out["determined_within_1e-4"] == 4
    assert out["determined_within_1e-3"] == 5
    assert abs(out["determined_max"] - 3e-4) < 1e-9 and abs(out["max"] - 0.5) < 1e-9
    assert out["best_goal_gpu"] == out["best_goal_oracle"] == 4
