"""The ablation driver on a small diagonal Gaussian: the bias metric agrees
with a direct evaluation from the final positions, a run with more chains and
the defaults reaches the threshold, and a fixed step size holds."""
import numpy as np
import pytest

from paper_2601_16696_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "gpu tests need a GPU"
    from paper_2601_16696_amd import ablation, laps
    laps.lib()
    return ablation


def test_grads_to_bias_reaches_threshold(gpu):
    w = workloads.gaussian(n_chains=1024, d=20, x0_scale=1.0)
    r = gpu.grads_to_bias(w, w["sigma2"], "f64", max_unadj=400, max_total=1000)
    assert r["reached"] and r["min_b2"] < 0.01
    assert 0 < r["grads_per_chain"] <= r["final_grads"]
    assert r["n_unadj"] + r["n_adj"] > 0


def test_fixed_eps_run_stays_unadjusted(gpu):
    w = workloads.gaussian(n_chains=256, d=20, x0_scale=1.0)
    r = gpu.grads_to_bias(w, w["sigma2"], "f64", unadjusted_only=True, max_total=60, stop_at_hit=False,
                          eps_fixed=0.05)
    assert r["final_eps"] == 0.05 and r["switch"] is None and r["final_grads"] == 61
    assert np.isfinite(r["min_b2"])


def test_relative_column(gpu):
    rows = gpu._relative([dict(reached=True, grads_per_chain=200), dict(reached=False),
                          dict(reached=True, grads_per_chain=100)])
    assert [r["relative"] for r in rows] == [2.0, None, 1.0]
