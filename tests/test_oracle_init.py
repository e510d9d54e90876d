"""Pins of the oracle's initialisation (section "Initialization" and Algorithm
"LAPS Pseudocode"): the initial velocity is the unit vector along the gradient
of log p at the start, the first step size is 0.01 sqrt(d), and L is
alpha (sum_i Var[x_i])^{1/2} over the initial ensemble.

The gradient is taken from the closed form of the diagonal Gaussian
(grad log p = -x / sigma^2), not from the oracle.  Where the gradient is zero
or not finite the oracle falls back to a uniform direction: the normals of the
stream with tag 5 (whose words and Box-Muller layout are pinned in
test_oracle_rng.py), normalised.
"""
import numpy as np
import pytest

TAG_INIT_DIR = 5


def _gauss(orc, N=64, d=37, seed=5, scale=3.0):
    rng = np.random.default_rng(seed)
    s2 = 10.0 ** rng.uniform(-2, 2, size=d)
    x0 = rng.normal(size=(N, d)) * scale
    return s2, x0, orc.Target(orc.GAUSS_DIAG, d, a=s2)


@pytest.mark.parametrize("d", [2, 5, 37, 100])
def test_initial_velocity_is_the_normalised_gradient(orc, d):
    s2, x0, tgt = _gauss(orc, d=d)
    N = x0.shape[0]
    e = orc.Ensemble(tgt, N, 11)
    e.init(x0)
    g = -x0 / s2
    ref = g / np.linalg.norm(g, axis=1, keepdims=True)
    u = e.array("u")
    assert np.max(np.abs(u - ref)) < 1e-15
    np.testing.assert_allclose(np.linalg.norm(u, axis=1), 1.0, rtol=0, atol=2e-15)
    # u points along +grad log p (uphill), not along its negative
    assert np.all(np.sum(u * g, axis=1) > 0)
    np.testing.assert_allclose(e.array("g"), g, rtol=1e-15, atol=0)
    np.testing.assert_allclose(e.array("logp"), -0.5 * np.sum(x0 * x0 / s2, axis=1), rtol=1e-14)


@pytest.mark.parametrize("bad", ["zero", "overflow"])
def test_zero_or_nonfinite_gradient_takes_a_uniform_direction(orc, bad):
    s2, x0, tgt = _gauss(orc, N=16, d=37)
    seed = 4242
    rows = [3, 9]
    for m in rows:
        # the gradient -x / s2 is exactly zero at x = 0; at |x| = 1e308 with s2 < 1 it overflows
        x0[m] = 0.0 if bad == "zero" else np.where(s2 < 1.0, 1e308, 0.0)
    e = orc.Ensemble(tgt, x0.shape[0], seed)
    e.init(x0)
    u = e.array("u")
    for m in range(x0.shape[0]):
        if m in rows:
            z = orc.normals(seed, m, 0, TAG_INIT_DIR, 0, x0.shape[1])
            ref = z / np.linalg.norm(z)
        else:
            g = -x0[m] / s2
            ref = g / np.linalg.norm(g)
        assert np.max(np.abs(u[m] - ref)) < 1e-15, m
        assert abs(np.linalg.norm(u[m]) - 1.0) < 2e-15
    # the fallback directions of two chains are different draws
    assert not np.allclose(u[rows[0]], u[rows[1]])


def test_caller_velocity_is_used_verbatim(orc):
    s2, x0, tgt = _gauss(orc, N=8, d=10)
    u0 = np.random.default_rng(1).normal(size=x0.shape)
    e = orc.Ensemble(tgt, x0.shape[0], 3)
    e.init(x0, u0)
    assert np.array_equal(e.array("u"), u0)


@pytest.mark.parametrize("d,factor,alpha", [(37, 0.01, 2.0), (100, 0.01, 2.0), (7, 0.05, 0.5)])
def test_initial_step_size_and_trajectory_scale(orc, d, factor, alpha):
    s2, x0, tgt = _gauss(orc, N=50, d=d)
    e = orc.Ensemble(tgt, x0.shape[0], 1, eps0_factor=factor, alpha=alpha)
    e.init(x0)
    st = e.stats()
    assert st["eps"] == factor * np.sqrt(d)
    # ensemble variances with 1/M, two-pass, summed over dimensions
    var = np.mean((x0 - x0.mean(axis=0)) ** 2, axis=0)
    assert abs(st["L"] - alpha * np.sqrt(var.sum())) <= 1e-13 * st["L"]
    assert st["t"] == 0 and st["grads_per_chain"] == 1 and st["phase"] == 0
    assert np.all(e.array("delta") == 0.0)
