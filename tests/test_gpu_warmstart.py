"""What the trained warm start gains over the method without it.

A network is trained on the GPU (the library's forward, backward and Adam
kernels) on solutions of held-apart template scenes, then the solver runs to
the stopping rule (best goal of each scene at max(r_obs, r_acc, r_nh) <= 1e-3,
checked every 5 iterations, at most 300) on 4096 unseen scenes from the cold
start (FP32) and from the network's prediction (split-BF16 solver; the cold start
as fallback per goal after one iteration and per scene after 10). The warm
start must need fewer iterations on average at the same FP32 precision, take
less wall-clock time per scene than the cold FP32 start, both over all scenes
and over the scenes both bring to the tolerance, and bring at least as many
scenes to the tolerance. The report goes to warmstart_report.json in the test
report directory.
"""
import json

import numpy as np
import pytest

from tests.conftest import report_path

pytestmark = pytest.mark.gpu


def test_trained_warm_start_gains_over_the_cold_start():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_10392_amd import warmstart as W
    prob = W.Problem()
    net, mean, std, info = W.fit(prob, range(1000, 1000 + 32768), epochs=30, lr=2e-3, log=None)
    print("training:", json.dumps(info))
    assert np.isfinite(info["final_loss"])
    res = W.evaluate(prob, net, mean, std, list(range(4096)))
    res["training"] = info
    print(json.dumps(res, indent=1))
    with open(report_path("warmstart_report.json"), "w") as f:
        json.dump(res, f, indent=1)
    assert res["warm_fp32"]["iters_mean"] < 0.97 * res["cold"]["iters_mean"]
    assert res["warm"]["iters_mean"] < res["cold"]["iters_mean"]
    assert res["ms_ratio"] < 1.0
    assert res["common"]["ms_ratio"] < 1.0
    assert res["warm"]["converged"] >= res["cold"]["converged"]
