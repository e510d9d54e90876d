"""The differentiable log density (laps.log_density, forward and backward in
the library's target kernels) against the oracle's log p and gradient."""
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


@pytest.mark.parametrize("name", ["gauss", "stochvol", "phi4"])
def test_log_density_forward_and_backward(gpu, orc, name):
    import torch
    w = {"gauss": lambda: workloads.gaussian(n_chains=20, d=37, x0_scale=1.0),
         "stochvol": lambda: workloads.stochvol(n_chains=12, T=150),
         "phi4": lambda: workloads.phi4(n_chains=10, side=12)}[name]()
    tgt = gpu.Target(w, "f64")
    x = torch.as_tensor(w["x0"], device="cuda:0").clone().requires_grad_(True)
    lp = gpu.log_density(tgt, x)
    wts = torch.linspace(0.5, 2.0, x.shape[0], device="cuda:0", dtype=torch.float64)
    (wts * lp).sum().backward()
    ot = orc.Target.from_workload(w)
    ref = [ot.logp_grad(r) for r in w["x0"]]
    lref = np.array([r[0] for r in ref])
    gref = np.array([r[1] for r in ref]) * wts.cpu().numpy()[:, None]
    assert np.max(np.abs(lp.detach().cpu().numpy() - lref) / np.maximum(np.abs(lref), 1.0)) < 1e-12
    g = x.grad.cpu().numpy()
    assert np.max(np.abs(g - gref)) <= 1e-12 * np.max(np.abs(gref))
