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
