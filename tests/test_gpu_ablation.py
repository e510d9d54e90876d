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


def test_batched_sweep_equals_sequential_runs(gpu):
    """The batched driver (configurations advancing together on their own
    streams) gives exactly the sequential driver's results: each run is
    deterministic and independent of the others."""
    w = workloads.gaussian(n_chains=256, d=20, x0_scale=1.0)
    base = dict(max_unadj=300, max_total=800)
    specs = [dict(C=0.01), dict(alpha=1.0), dict(integrator_adj=2, acc_target=0.9),
             dict(switch_policy=1, max_unadj=50), dict(which="avg"),
             dict(unadjusted_only=True, max_total=100, stop_at_hit=False, eps_fixed=0.05)]
    seq = [gpu.grads_to_bias(w, w["sigma2"], "f64", **dict(base, **sp)) for sp in specs]
    bat = gpu.grads_to_bias_many([dict(w=w, s2=w["sigma2"], **dict(base, **sp)) for sp in specs], "f64",
                                 concurrent=4)
    assert len(bat) == len(seq)
    for a, b in zip(seq, bat):
        for key in ("reached", "min_b2", "final_eps", "final_grads", "switch", "grads_per_chain", "n_unadj",
                    "n_adj", "phase"):
            assert a.get(key) == b.get(key), (key, a.get(key), b.get(key))
