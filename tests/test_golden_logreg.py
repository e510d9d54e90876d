"""The stored reference moments of the logistic-regression posterior
(tests/golden/logreg_n5000_d100_moments.json, written by the FP64 oracle via
tests/golden/logreg_moments.py) against an independent approximation: the
Laplace approximation at the posterior mode (Newton's method on the log
posterior, Hessian X^T W X + I), whose E[x_i^2] = mode_i^2 + C_ii agrees to a
few percent for n = 5000 observations in d = 100 (the posterior is close to
Gaussian; the skew left by the logistic likelihood is what remains).  Also
the Monte Carlo precision of the reference, which must be well below the
bias threshold 0.01 it is used against."""
import json
import os

import numpy as np

from paper_2601_16696_amd import workloads

PATH = os.path.join(os.path.dirname(__file__), "golden", "logreg_n5000_d100_moments.json")


def test_reference_moments_against_laplace():
    r = json.load(open(PATH))
    e, v, se = np.array(r["E_x2"]), np.array(r["Var_x2"]), np.array(r["se_E_x2"])
    w = workloads.logreg()
    X, y = w["X"], w["y"]
    assert e.shape == v.shape == se.shape == (w["d"],)
    th = np.zeros(w["d"])
    for _ in range(50):
        p = 1.0 / (1.0 + np.exp(-(X @ th)))
        g = X.T @ (y - p) - th
        H = (X.T * (p * (1 - p))) @ X + np.eye(w["d"])
        step = np.linalg.solve(H, g)
        th += step
        if np.max(np.abs(step)) < 1e-13:
            break
    c = np.diag(np.linalg.inv(H))
    lap = th**2 + c
    lap_var = 4 * th**2 * c + 2 * c**2
    assert np.max(np.abs(e - lap) / lap) < 0.1
    assert np.median(np.abs(v - lap_var) / lap_var) < 0.15
    # reference noise: b^2 contribution (se / std)^2 well below 0.01
    assert np.all(v > 0) and np.max(se / np.sqrt(v)) < 0.03
    assert all(0.55 < a < 0.85 for a in r["acceptance"])


def test_stochvol_reference_is_stationary_and_precise():
    """The stochastic-volatility reference (tests/golden/stochvol_moments.py,
    FP64 oracle): the first and second halves of the pooled transitions agree
    within their Monte Carlo error across all 2429 dimensions (no drift left
    after burn-in), and the reference's own noise stays well below the bias
    threshold it is used against."""
    r = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "stochvol_T2427_moments.json")))
    e, v, se = np.array(r["E_x2"]), np.array(r["Var_x2"]), np.array(r["se_E_x2"])
    assert e.shape == v.shape == se.shape == (2429,)
    assert np.all(e > 0) and np.all(v > 0)
    assert r["halves_z_max"] < 4.5 and 0.4 < r["halves_z_median"] < 0.9
    assert r["max_se_over_std"] < 0.05
