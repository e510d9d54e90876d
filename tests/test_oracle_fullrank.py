"""Pins of the oracle's full-rank equipartition loss (section "Equipartition
condition", full-rank paragraph: Hutchinson's trace estimator with Rademacher
probes).

- Over all 2^d sign vectors a Rademacher average of |A z|^2 is exactly the
  squared Frobenius norm of A, so with every sign vector as a probe the
  estimator must equal (1/d)|I - V|_F^2 computed from the matrix V of its
  definition (V_ij = -mean_m (x_i - xbar_i) g_j), written here from scratch.
- The probes are +-1 with zero mean and identity second moment.
- With the paper's 100 random probes the estimate is close to the exact value.
- The sampler uses the probes of the step being controlled.
"""
import itertools

import numpy as np
import pytest

from paper_2601_16696_amd import workloads


def _ensemble(N, d, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(d, d)) / np.sqrt(d)
    x = rng.normal(size=(N, d)) @ A + rng.normal(size=d)
    prec = np.linalg.inv(A.T @ A + 0.5 * np.eye(d))
    g = -(x - x.mean(0)) @ prec.T + 0.3 * rng.normal(size=(N, d))  # correlated, not exact
    return x, g


def _exact(x, g):
    N, d = x.shape
    xc = x - x.mean(0)
    V = -(xc.T @ g) / N
    return float(np.sum((np.eye(d) - V) ** 2) / d)


@pytest.mark.parametrize("d", [2, 3, 5])
def test_all_sign_vectors_give_the_frobenius_norm(orc, d):
    x, g = _ensemble(40, d, 11 + d)
    z = np.array(list(itertools.product([-1.0, 1.0], repeat=d)))
    got = orc.dtilde_full(x, g, z)
    want = _exact(x, g)
    assert abs(got - want) <= 1e-12 * want, (got, want)


def test_exact_at_equipartition(orc):
    """V = I exactly (x and g = -x whitened) makes every probe's (I - V) z vanish."""
    rng = np.random.default_rng(5)
    N, d = 64, 6
    x = rng.normal(size=(N, d))
    xc = x - x.mean(0)
    C = xc.T @ xc / N
    g = -xc @ np.linalg.inv(C)          # then -mean (x - xbar) g^T = I
    z = np.array([orc.rademacher(3, 0, p, d) for p in range(20)])
    assert orc.dtilde_full(x, g, z) < 1e-24


def test_probes_are_rademacher(orc):
    P, d = 3000, 300                    # two Philox blocks per probe (dims 256..299 in the second)
    z = np.array([orc.rademacher(17, 4, p, d) for p in range(P)])
    assert set(np.unique(z)) == {-1.0, 1.0}
    assert np.max(np.abs(z.mean(0))) < 5 / np.sqrt(P)
    M = z.T @ z / P
    assert np.allclose(np.diag(M), 1.0)
    off = M - np.diag(np.diag(M))
    assert np.max(np.abs(off)) < 6 / np.sqrt(P)
    # another step or seed gives other probes
    assert not np.array_equal(z[0], orc.rademacher(17, 5, 0, d))
    assert not np.array_equal(z[0], orc.rademacher(18, 4, 0, d))


def test_hundred_probes_are_close(orc):
    x, g = _ensemble(200, 30, 3)
    want = _exact(x, g)
    z = np.array([orc.rademacher(9, 0, p, 30) for p in range(100)])
    got = orc.dtilde_full(x, g, z)
    assert abs(got - want) < 0.2 * want, (got, want)
    z4k = np.array([orc.rademacher(9, 1, p, 30) for p in range(4000)])
    assert abs(orc.dtilde_full(x, g, z4k) - want) < 0.03 * want


def test_sampler_uses_the_probes_of_the_step(orc):
    w = workloads.gaussian(n_chains=32, d=12, x0_scale=1.0)
    P = 7
    e = orc.Ensemble(orc.Target.from_workload(w), w["n_chains"], w["seed"], switch_policy=1,
                     max_steps_unadj=10, full_rank_probes=P)
    e.init(w["x0"])
    for t in range(3):
        e.step_unadjusted(1)
        z = np.array([orc.rademacher(w["seed"], t, p, w["d"]) for p in range(P)])
        want = orc.dtilde_full(e.array("x"), e.array("g"), z)
        assert e.stats()["dtilde"] == pytest.approx(want, rel=1e-13)
