"""The fixed step size of the unadjusted phase (eps_fixed; the fixed-step
comparison of the step-size appendix) against the oracle: eps stays at the
given value, positions, L and the diagnostics follow the oracle, and after the
switch the bisection starts from that value."""
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
    "gauss": (lambda: workloads.gaussian(n_chains=96, d=40, x0_scale=2.0), 0.4),
    "stochvol": (lambda: workloads.stochvol(n_chains=64, T=120), 0.05),
    "logreg": (lambda: workloads.logreg(n_chains=64, n=300, d=20), 0.03),
}


@pytest.mark.parametrize("name", list(CASES))
def test_fixed_eps_run_matches_oracle(gpu, orc, name):
    gen, E = CASES[name]
    w = gen()
    cfg = dict(eps_fixed=E, switch_policy=1, max_steps_unadj=20, max_steps_total=20 + 15 * 3)
    o = orc.Ensemble(orc.Target.from_workload(w), w["n_chains"], w["seed"], **cfg)
    o.init(w["x0"])
    s = gpu.Sampler(w, "f64", **cfg)
    assert s.stats()["eps"] == E == o.stats()["eps"]
    for k in range(20):
        o.step_unadjusted(1)
        s.step_unadjusted(1)
        so, sg = o.stats(), s.stats()
        assert sg["eps"] == E and so["eps"] == E
        for key in ("L", "dtilde"):
            assert _close(sg[key], so[key], 1e-10), (k, key, sg[key], so[key])
        assert _close(sg["eevpd"], so["eevpd"], 1e-7), (k, sg["eevpd"], so["eevpd"])
    err = _rel_rows(s.positions().cpu().numpy(), o.array("x"))
    assert np.max(err) < 1e-10, np.max(err)
    assert o.stats()["phase"] == s.stats()["phase"] == 1
    for k in range(3):
        o.step_adjusted(1)
        s.step_adjusted(1)
        so, sg = o.stats(), s.stats()
        assert _close(sg["eps"], so["eps"], 1e-12), (k, sg["eps"], so["eps"])
        assert _close(sg["acc_mean"], so["acc_mean"], 1e-8), (k, sg["acc_mean"], so["acc_mean"])
    err = _rel_rows(s.positions().cpu().numpy(), o.array("x"))
    assert np.max(err) < 1e-10, np.max(err)
