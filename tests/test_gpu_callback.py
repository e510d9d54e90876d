"""Caller-supplied targets (LAPS_CALLBACK) on the GPU.

The caller's gradient (here the diagonal Gaussian written in torch) feeds the
library's per-chain update kernels; the run is compared with the FP64 oracle
of the same Gaussian, as the built-in targets are."""
import numpy as np
import pytest

from paper_2601_16696_amd import workloads

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-4}


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


def _gauss_callback(w, dtype):
    import torch
    d = w["d"]
    inv = torch.as_tensor(1.0 / np.asarray(w["sigma2"]), device="cuda:0").to(dtype)
    calls = [0]

    def fn(x, g, lp):
        calls[0] += 1
        xd = x[:, :d]
        g[:, :d] = -xd * inv
        lp.copy_((-0.5 * (xd * xd * inv).sum(1)).to(torch.float64))

    return dict(w, kind="callback", fn=fn), calls


def _rel_rows(a, b):
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("N,d", [(64, 50), (40, 300)])
def test_callback_gaussian_matches_oracle(gpu, orc, prec, N, d):
    """d = 50 runs one oct per lane and MN2; d = 300 runs 16-lane update teams
    with 3 octs per lane and the MN4 integrator (the automatic choice above
    d = 200), whose FP32 positions are held to 2.5 x the MN2 bound (five
    gradient stages per step instead of two)."""
    import torch
    w = workloads.gaussian(n_chains=N, d=d, x0_scale=1.0)
    wc, calls = _gauss_callback(w, torch.float64 if prec == "f64" else torch.float32)
    cfg = dict(switch_policy=1, max_steps_unadj=12, max_steps_total=12 + 15 * 3)
    s = gpu.Sampler(wc, prec, **cfg)
    o = orc.Ensemble(orc.Target.from_workload(w), w["n_chains"], w["seed"], **cfg)
    o.init(w["x0"])
    for _ in range(12):
        if prec == "f32":  # FP32 state against the FP64 oracle: replay the GPU's step size and L
            st = s.stats()
            o.set_hyper(st["eps"], st["L"])
        s.step_unadjusted(1)
        o.step_unadjusted(1)
    so, sg = o.stats(), s.stats()
    assert sg["t"] == so["t"] == 12
    if prec == "f64":
        assert abs(sg["eps"] - so["eps"]) <= 1e-9 * so["eps"] and abs(sg["L"] - so["L"]) <= 1e-9 * so["L"]
    x = s.positions().cpu().numpy()
    assert np.max(_rel_rows(x, o.array("x"))) < TOL[prec]
    for k in range(2):
        if prec == "f32" and k > 0:
            o.set_hyper(s.stats()["eps"], 0.0)
        s.step_adjusted(1)
        o.step_adjusted(1)
    torch.cuda.synchronize()
    sg, so = s.stats(), o.stats()
    integ = 2 if d > 200 else 1
    tol = TOL[prec] * (2.5 if integ == 2 and prec == "f32" else 1.0)
    assert sg["phase"] == so["phase"] == 2 and sg["integrator"] == so["integrator"] == integ
    acc_o, acc_g = o.array("acc"), s.buffer("acc").cpu().numpy()
    x = s.positions().cpu().numpy()
    err = _rel_rows(x, o.array("x"))
    flipped = err > 1e-2  # an accept decision within rounding of the threshold
    if prec == "f64":
        assert not flipped.any()
    assert flipped.mean() <= 0.05
    assert np.max(err[~flipped]) < tol
    assert np.max(np.abs(acc_g - acc_o)[~flipped]) < (1e-8 if prec == "f64" else 2e-3)
    # one gradient at init, one per unadjusted step, two (MN2) or five (MN4) per step of the two
    # 15-step trajectories
    assert calls[0] == 1 + 12 + 2 * (5 if integ == 2 else 2) * 15


def test_callback_error_fails_the_step(gpu):
    """A callback that fails (here: raises on its fourth call) fails the step
    that called it with LAPS_EDEVICE and names the callback."""
    import torch
    w = workloads.gaussian(n_chains=16, d=20, x0_scale=1.0)
    wc, calls = _gauss_callback(w, torch.float64)
    ok = wc["fn"]

    def flaky(x, g, lp):
        if calls[0] >= 3:
            raise ValueError("planted failure in the caller's gradient")
        ok(x, g, lp)

    wc["fn"] = flaky
    s = gpu.Sampler(wc, "f64", switch_policy=1, max_steps_unadj=5, max_steps_total=5 + 15)  # call 1 (init)
    s.step_unadjusted(2)                                                                     # calls 2, 3
    with pytest.raises(gpu.LapsError, match="gradient callback returned 1"):
        s.step_unadjusted(1)


def test_callback_eval_through_the_context(gpu):
    """laps_eval on a callback target calls the callback at the caller's
    positions (not the sampler's state) and returns its log p and gradient."""
    import torch
    w = workloads.gaussian(n_chains=32, d=24, x0_scale=1.0)
    wc, calls = _gauss_callback(w, torch.float64)
    s = gpu.Sampler(wc, "f64")
    n0 = calls[0]
    before = s.positions().clone()
    x = torch.as_tensor(np.asarray(w["x0"]) * 0.5 - 0.2, device="cuda:0")
    lp, g = s.eval(x)
    torch.cuda.synchronize()
    assert calls[0] == n0 + 1
    inv = torch.as_tensor(1.0 / np.asarray(w["sigma2"]), device="cuda:0")
    assert torch.allclose(g, -x * inv, rtol=1e-15, atol=0)
    assert torch.allclose(lp, -0.5 * (x * x * inv).sum(1), rtol=1e-14, atol=0)
    assert torch.equal(s.positions(), before)
