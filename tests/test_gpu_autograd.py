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


def _fd_check(f, x, n_dirs=3, h=1e-5, seed=0):
    """Central differences of the forward pass along random directions
    against the backward pass (both on the GPU, FP64)."""
    import torch
    gen = torch.Generator(device="cpu").manual_seed(seed)
    xx = x.detach().clone().requires_grad_(True)
    f(xx).sum().backward()
    g = xx.grad
    for _ in range(n_dirs):
        v = torch.randn(x.shape, generator=gen, dtype=torch.float64).to(x.device)
        with torch.no_grad():
            fp = f(x + h * v)
            fm = f(x - h * v)
        fd = (fp - fm) / (2 * h)
        an = (g * v).sum(1)
        scale = (g.abs() * v.abs()).sum(1) + 1.0
        assert torch.all((fd - an).abs() <= 1e-6 * scale), torch.max((fd - an).abs() / scale)


@pytest.mark.parametrize("name", ["gauss", "stochvol", "phi4"])
def test_log_density_finite_differences(gpu, name):
    import torch
    w = {"gauss": lambda: workloads.gaussian(n_chains=8, d=37, x0_scale=1.0),
         "stochvol": lambda: workloads.stochvol(n_chains=6, T=150),
         "phi4": lambda: workloads.phi4(n_chains=5, side=12)}[name]()
    tgt = gpu.Target(w, "f64")
    x = torch.as_tensor(w["x0"], device="cuda:0")
    _fd_check(lambda y: gpu.log_density(tgt, y), x)


@pytest.mark.parametrize("name", ["logreg", "ill_gauss"])
def test_log_density_through_the_context(gpu, orc, name):
    """Targets whose gradient needs the context (logistic regression's split
    matrix-core kernels, the dense precision product): forward and backward
    against the oracle at positions other than the sampler's state, and
    central differences."""
    import torch
    w = workloads.logreg(n_chains=24, n=300, d=20) if name == "logreg" else workloads.ill_gaussian(n_chains=16, d=24)
    s = gpu.Sampler(w, "f64", integrator_adj=1)
    before = s.positions().clone()
    x = torch.as_tensor(np.asarray(w["x0"]) * 0.7 + 0.1, device="cuda:0").requires_grad_(True)
    lp = gpu.log_density(s, x)
    wts = torch.linspace(0.5, 2.0, x.shape[0], device="cuda:0", dtype=torch.float64)
    (wts * lp).sum().backward()
    ot = orc.Target.from_workload(w)
    ref = [ot.logp_grad(r) for r in x.detach().cpu().numpy()]
    lref = np.array([r[0] for r in ref])
    gref = np.array([r[1] for r in ref]) * wts.cpu().numpy()[:, None]
    assert np.max(np.abs(lp.detach().cpu().numpy() - lref) / np.maximum(np.abs(lref), 1.0)) < 1e-12
    g = x.grad.cpu().numpy()
    assert np.max(np.abs(g - gref)) <= 1e-11 * np.max(np.abs(gref))
    assert torch.equal(s.positions(), before)  # the sampler's state is untouched
    _fd_check(lambda y: gpu.log_density(s, y), x.detach())
    s.step_unadjusted(2)  # the sampler still steps after an evaluation
    assert s.stats()["t"] == 2


def test_log_density_bf16_logistic_through_the_context(gpu, orc):
    import torch
    w = workloads.logreg(n_chains=32, n=400, d=30)
    s = gpu.Sampler(w, "bf16")
    x = torch.as_tensor(w["x0"], device="cuda:0", dtype=torch.float32)
    lp, g = s.eval(x)
    ot = orc.Target.from_workload(w)
    X, y = w["X"], w["y"]
    th_all = x.cpu().numpy().astype(np.float64)
    for m in range(0, 32, 5):
        l_ref, g_ref = ot.logp_grad(th_all[m])
        z = X @ th_all[m]
        zabs = np.abs(X) @ np.abs(th_all[m])
        dz = 2.0**-17 * zabs + 2.0**-22 * zabs * 2
        sig = 1 / (1 + np.exp(-z))
        bound_l = np.sum(np.abs(y - sig) * dz + 0.25 * dz**2) + 1e-6 * np.sum(np.abs(z) + 1.0)
        assert abs(lp[m].item() - l_ref) <= bound_l
        dr = 2.0**-9 * np.abs(y - sig) + 0.25 * dz + 1e-7
        bound_g = np.abs(X).T @ dr + 1e-5 * (np.abs(X).T @ np.abs(y - sig)) + 1e-6 * np.abs(th_all[m])
        assert np.all(np.abs(g[m].cpu().numpy().astype(np.float64) - g_ref) <= bound_g)


def test_log_density_mixed_sampler_double_input(gpu):
    """A bf16/FP32-state sampler evaluated at FP64 positions: the gradient
    comes back in the input's dtype."""
    import torch
    w = workloads.logreg(n_chains=16, n=200, d=20)
    s = gpu.Sampler(w, "bf16")
    x = s.positions().double().clone().requires_grad_(True)
    lp = gpu.log_density(s, x)
    lp.sum().backward()
    assert lp.dtype == torch.float64 and x.grad.dtype == torch.float64
    _, g = s.eval(x.detach())
    assert torch.allclose(x.grad, g.double())
