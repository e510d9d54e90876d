"""The underdamped Langevin variant of the dynamics (dynamics = 1; the
dynamics ablation of appendix "Ablation studies") against the oracle: 20
unadjusted steps with the adaptive controller, the switch, and 3 adjusted
transitions, on every kernel family (per-chain Gaussian, stochastic volatility,
phi^4 with MN2 and MN4, the logistic-regression and dense-Gaussian update
kernels)."""
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


def _close(a, b, tol):
    return abs(a - b) <= tol * max(abs(b), 1e-300)


CASES = {
    "gauss": (lambda: workloads.gaussian(n_chains=96, d=40, x0_scale=2.0), {}),
    "gauss_mn4": (lambda: workloads.gaussian(n_chains=64, d=37, x0_scale=2.0), dict(integrator_adj=2)),
    "stochvol": (lambda: workloads.stochvol(n_chains=64, T=120), {}),
    "phi4": (lambda: workloads.phi4(n_chains=40, side=12), {}),
    "logreg": (lambda: workloads.logreg(n_chains=64, n=300, d=20), {}),
    "ill_gauss": (lambda: workloads.ill_gaussian(n_chains=64, d=24), {}),
}


@pytest.mark.parametrize("name", list(CASES))
def test_langevin_run_matches_oracle(gpu, orc, name):
    gen, extra = CASES[name]
    w = gen()
    cfg = dict(dynamics=1, switch_policy=1, max_steps_unadj=20, max_steps_total=20 + 15 * 3, **extra)
    o = orc.Ensemble(orc.Target.from_workload(w), w["n_chains"], w["seed"], **cfg)
    o.init(w["x0"])
    s = gpu.Sampler(w, "f64", **cfg)
    for k in range(20):
        o.step_unadjusted(1)
        s.step_unadjusted(1)
        so, sg = o.stats(), s.stats()
        assert sg["t"] == so["t"]
        for key in ("eps", "L", "dtilde"):
            assert _close(sg[key], so[key], 1e-9), (k, key, sg[key], so[key])
    err = _rel_rows(s.positions().cpu().numpy(), o.array("x"))
    assert np.max(err) < 1e-10, np.max(err)
    u_err = _rel_rows(s.buffer("u").cpu().numpy(), o.array("u"))
    assert np.max(u_err) < 1e-10, np.max(u_err)
    assert o.stats()["phase"] == s.stats()["phase"] == 1
    for k in range(3):
        o.step_adjusted(1)
        s.step_adjusted(1)
        so, sg = o.stats(), s.stats()
        assert so["integrator"] == sg["integrator"]
        assert _close(sg["acc_mean"], so["acc_mean"], 1e-8), (k, sg["acc_mean"], so["acc_mean"])
        assert _close(sg["eps"], so["eps"], 1e-9), (k, sg["eps"], so["eps"])
    err = _rel_rows(s.positions().cpu().numpy(), o.array("x"))
    assert np.max(err) < 1e-10, np.max(err)


def test_langevin_fp32_state_replayed(gpu, orc):
    """FP32 state: the oracle takes the GPU's (eps, L) before every step."""
    w = workloads.gaussian(n_chains=96, d=40, x0_scale=2.0)
    cfg = dict(dynamics=1, switch_policy=1, max_steps_unadj=20)
    o = orc.Ensemble(orc.Target.from_workload(w), w["n_chains"], w["seed"], **cfg)
    o.init(w["x0"])
    s = gpu.Sampler(w, "f32", **cfg)
    for _ in range(20):
        sg = s.stats()
        o.set_hyper(sg["eps"], sg["L"])
        o.step_unadjusted(1)
        s.step_unadjusted(1)
    err = _rel_rows(s.positions().cpu().numpy().astype(np.float64), o.array("x"))
    assert np.max(err) < 1e-4, np.max(err)


def test_langevin_differs_from_microcanonical(gpu):
    w = workloads.gaussian(n_chains=64, d=30, x0_scale=2.0)
    a = gpu.Sampler(w, "f64", switch_policy=1, max_steps_unadj=5)
    b = gpu.Sampler(w, "f64", switch_policy=1, max_steps_unadj=5, dynamics=1)
    a.step_unadjusted(5)
    b.step_unadjusted(5)
    ua = a.buffer("u").cpu().numpy()
    ub = b.buffer("u").cpu().numpy()
    assert np.allclose(np.linalg.norm(ua, axis=1), 1.0, atol=1e-12)
    assert not np.allclose(np.linalg.norm(ub, axis=1), 1.0, atol=1e-3)
