"""The launch-shape autotuner: it returns a valid shape, keeps it in its
cache under (kind, d, n, N, precision), returns the cached entry without
timing, and a sampler made with the returned fields runs."""
import json

import pytest

from paper_2601_16696_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "gpu tests need a GPU"
    from paper_2601_16696_amd import laps
    laps.lib()
    return laps


@pytest.mark.parametrize("name", ["gauss", "logreg"])
def test_autotune_picks_and_caches_a_shape(gpu, tmp_path, name):
    w = workloads.gaussian(n_chains=64, d=40) if name == "gauss" else workloads.logreg(n_chains=128, n=300, d=20)
    prec = "f64" if name == "gauss" else "bf16"
    cache = str(tmp_path / "tune.json")
    r = gpu.autotune(w, prec, cache=cache, n_steps=5)
    assert r["cached"] is False and r["ms_per_step"] > 0
    table = json.load(open(cache))
    key = gpu._tune_key(w, prec)
    assert key in table and table[key]["ms_per_step"] == r["ms_per_step"]
    again = gpu.autotune(w, prec, cache=cache, n_steps=5)
    assert again["cached"] is True and again["ms_per_step"] == r["ms_per_step"]
    fields = {k: v for k, v in r.items() if k not in ("cached", "ms_per_step", "trials")}
    s = gpu.Sampler(w, prec, switch_policy=1, max_steps_unadj=5, **fields)
    s.step_unadjusted(5)
    assert s.stats()["t"] == 5
