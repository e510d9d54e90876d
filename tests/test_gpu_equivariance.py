"""The GPU's unadjusted phase under a change of units, without the oracle.

Scaling a diagonal Gaussian's standard deviations, the start and the initial
step size by f leaves every quantity the controllers read unchanged (the
energy errors, D~, EEVPD and the moving window's relative fluctuations of
E[x_i^2], section "Switch to adjustment") and scales eps and
L = alpha (sum Var)^{1/2} by f.  With f a power of two every floating-point
operation of the path scales exactly, in FP64 and in FP32 state, so the
whole trajectory (eps(t), L(t), the window-triggered switch step and the
positions) must scale bit for bit.  This checks the units of the device
controllers and maps independently of the oracle.
"""
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


def _run(gpu, prec, sc):
    w = workloads.gaussian(n_chains=512, d=20, seed_data=7, seed_x0=8, x0_scale=3.0)
    w["sigma2"] = w["sigma2"] * sc * sc
    w["x0"] = w["x0"] * sc
    s = gpu.Sampler(w, prec, switch_policy=0, switch_tol=0.1, max_steps_unadj=600, max_steps_total=720,
                    eps0_factor=0.01 * sc)
    hist = [s.stats()]
    while hist[-1]["phase"] == 0:
        s.step_unadjusted(1)
        hist.append(s.stats())
    return hist, s.positions().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("f", [2.0, 0.5])
def test_unadjusted_phase_is_scale_equivariant(gpu, prec, f):
    h1, x1 = _run(gpu, prec, 1.0)
    hf, xf = _run(gpu, prec, f)
    assert len(h1) == len(hf)
    # the switch came from the window criterion, not from the step limit
    assert h1[-1]["switch_ready"] == 1 and 20 < h1[-1]["t"] < 600, h1[-1]
    for a, b in zip(h1, hf):
        assert (a["t"], a["phase"], a["switch_ready"]) == (b["t"], b["phase"], b["switch_ready"])
        assert b["eps"] == f * a["eps"] and b["L"] == f * a["L"], (a["t"], a["eps"], b["eps"], a["L"], b["L"])
        for key in ("dtilde", "eevpd", "max_delta"):
            assert a[key] == b[key] or (np.isinf(a[key]) and np.isinf(b[key])), (a["t"], key, a[key], b[key])
    np.testing.assert_array_equal(xf, f * x1)
