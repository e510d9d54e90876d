"""Full-rank equipartition loss (Hutchinson's estimator, section
"Equipartition condition") on the GPU against the oracle.

With full_rank_probes = P the controller's D~ is the mean of |(I - V) z|^2 / d
over P Rademacher probes drawn from the Philox stream of the step; the GPU
and the oracle draw the same probes, so D~ and everything the controller
derives from it are compared per step as in the diagonal-loss tests."""
import numpy as np
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


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    return oracle


def _rel_rows(a, b):
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


CASES = {
    # name: (workload, precision, probes, steps)
    "gauss": (lambda: workloads.gaussian(n_chains=64, d=50, x0_scale=1.0), "f64", 16, 12),
    # two probe blocks per probe (d > 256, ragged) and three chain chunks (N > 1024, ragged)
    "gauss_wide": (lambda: workloads.gaussian(n_chains=1100, d=300, x0_scale=1.0), "f64", 6, 3),
    "logreg": (lambda: workloads.logreg(n_chains=64, n=200, d=20), "f64", 32, 10),
    "gauss_f32": (lambda: workloads.gaussian(n_chains=64, d=50, x0_scale=1.0), "f32", 16, 10),
}


@pytest.mark.parametrize("name", list(CASES))
def test_full_rank_loss_matches_oracle(gpu, orc, name):
    import torch
    make, prec, P, steps = CASES[name]
    w = make()
    cfg = dict(switch_policy=1, max_steps_unadj=1000, full_rank_probes=P)
    if w["kind"] == "logreg":
        cfg["integrator_adj"] = 1
    s = gpu.Sampler(w, prec, **cfg)
    o = orc.Ensemble(orc.Target.from_workload(w), w["n_chains"], w["seed"], **cfg)
    o.init(w["x0"])
    replay = prec == "f32"
    for k in range(steps):
        if replay:
            st = s.stats()
            o.set_hyper(st["eps"], st["L"])
        s.step_unadjusted(1)
        o.step_unadjusted(1)
        sg, so = s.stats(), o.stats()
        assert sg["t"] == so["t"] == k + 1
        if replay:
            # FP32 positions differ from the oracle's at ~1e-6; D~ follows them
            assert abs(sg["dtilde"] - so["dtilde"]) <= 2e-3 * so["dtilde"], (k, sg["dtilde"], so["dtilde"])
        else:
            assert abs(sg["dtilde"] - so["dtilde"]) <= 1e-9 * so["dtilde"], (k, sg["dtilde"], so["dtilde"])
            for key in ("eevpd_target", "eps", "L"):
                assert abs(sg[key] - so[key]) <= 1e-9 * abs(so[key]), (k, key, sg[key], so[key])
    torch.cuda.synchronize()
    x = s.positions().cpu().numpy()
    tol = 1e-4 if replay else 1e-10
    assert np.max(_rel_rows(x, o.array("x"))) < tol


def test_full_rank_differs_from_diagonal(gpu):
    """The option changes D~ (and so eps) relative to the diagonal loss on a
    correlated target, and P = 0 keeps the diagonal loss."""
    w = workloads.logreg(n_chains=64, n=200, d=20)
    base = dict(switch_policy=1, max_steps_unadj=1000, integrator_adj=1)
    a = gpu.Sampler(w, "f64", **base)
    b = gpu.Sampler(w, "f64", full_rank_probes=64, **base)
    a.step_unadjusted(5)
    b.step_unadjusted(5)
    da, db = a.stats()["dtilde"], b.stats()["dtilde"]
    assert da > 0 and db > 0 and da != db
