"""The benchmark's extra legs on small inputs (GPU): the residual curve over the
iterations and the single-plan latency workload run end to end through the
library and report well-formed figures."""
import math
import types

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bench():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import bench as B
    return B


def test_residual_curve_on_three_scenes(bench):
    r = bench.residual_curve(range(3), chunk=5, total=20)
    assert r["iterations"] == [5, 10, 15, 20]
    med, share = r["best_goal_max_residual_median"], r["share_at_or_below_1e-3"]
    assert len(med) == len(share) == 4
    assert all(m >= 0.0 and not math.isnan(m) for m in med)
    assert all(0.0 <= s <= 1.0 for s in share)
    # the chunks resume one solve: the share of converged scenes never falls
    assert all(a <= b for a, b in zip(share, share[1:]))


def test_plan_leg_on_two_seeds(bench):
    args = types.SimpleNamespace(steps=2, warmup=1, iters=60)
    out = bench.run_plan(args)
    assert out["steps"] == 2 and out["unit"] == "ms" and out["higher_is_better"] is False
    lo, med, hi = out["plan_ms_p10_median_p90"]
    assert 0.0 < lo <= med <= hi
    # 60 iterations of one goal's chain take ~0.14 ms; a plain solve that skipped its
    # scene (a stale skip mask from the chunked runs) and the scoring take ~0.03 ms
    assert med > 0.07
    rule = out["to_rule"]
    assert 0 <= rule["converged"] <= rule["of"] == 2
    assert rule["ms_median_all"] > 0.0
