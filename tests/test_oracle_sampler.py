"""Pins of the oracle's whole transitions and of the sampler end to end.

MAMS exactness: exact Gaussian draws stay exact in distribution after
transitions at a deliberately large step (moments within Monte Carlo error),
and one transition satisfies detailed balance on a 2-D target (brute-force
histogram symmetry).  The unadjusted energy error scales as eps^6 and obeys
the Gaussian bias bound D~(p, p_eps) <= F^{-1}(EEVPD).  A full LAPS run on the
diagonal Gaussian workload ends with b_i^2 M distributed as chi^2_1.
"""
import numpy as np
import pytest
from scipy import stats

from paper_2601_16696_amd import workloads


def _gauss_ens(orc, s2, M, seed=1, **cfg):
    d = s2.size
    e = orc.Ensemble(orc.Target(orc.GAUSS_DIAG, d, a=s2), M, seed, **cfg)
    return e


def _uniform_u(rng, M, d):
    u = rng.normal(size=(M, d))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def test_eevpd_scales_as_eps6(orc):
    """One unadjusted step from an exact ensemble (x ~ p, u uniform): the
    slope of log EEVPD against log eps is close to 6 for small eps."""
    rng = np.random.default_rng(0)
    M, d = 4000, 50
    s2 = np.linspace(0.5, 2.0, d)
    x = rng.normal(size=(M, d)) * np.sqrt(s2)
    u = _uniform_u(rng, M, d)
    vals = []
    epss = [0.05, 0.1, 0.2]
    for eps in epss:
        e = _gauss_ens(orc, s2, M, eevpd_mode=0)
        e.init(x, u)
        e.set_hyper(eps, 1e9)  # no noise: isolate the integrator's energy error
        e.unadj_move()
        dl = e.array("delta")
        vals.append(np.var(dl) / d)
    slope = np.polyfit(np.log(epss), np.log(vals), 1)[0]
    assert abs(slope - 6) < 0.5, slope


def test_unadjusted_bias_bound_on_gaussian(orc):
    """At fixed eps and L the stationary unadjusted ensemble's D~_diag stays
    below F^{-1}(EEVPD) (bias bound, rigorous for Gaussians)."""
    rng = np.random.default_rng(1)
    M, d = 4096, 10
    s2 = np.linspace(0.5, 2.0, d)
    x = rng.normal(size=(M, d)) * np.sqrt(s2)
    e = _gauss_ens(orc, s2, M, eevpd_mode=0, switch_tol=-1.0, max_steps_unadj=10**6, max_steps_total=10**6)
    e.init(x)
    eps, L = 3.0, 3.0
    D_hist, E_hist = [], []
    for k in range(600):
        e.set_hyper(eps, L)
        e.unadj_move()
        e.unadj_control()
        if k >= 300:
            s = e.stats()
            D_hist.append(s["dtilde"])
            E_hist.append(s["eevpd"])
    D = np.mean(D_hist)
    E = np.mean(E_hist)
    # F^{-1} by bisection on the closed form
    lo, hi = 0.0, 100.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if orc.F(mid) < E else (lo, mid)
    # finite-M estimator noise of D~ is about 2/M per term
    assert D - 3 * 2.0 / M <= lo, (D, lo)
    assert D > 10 * 2.0 / M  # the bias is resolved, not just noise


@pytest.mark.parametrize("which_d,eps,integ", [(4, 3.2, 0), (30, 11.0, 0), (30, 16.0, 2)])
def test_mams_preserves_exact_gaussian(orc, which_d, eps, integ):
    """Start from exact draws; transitions at a large step (low acceptance)
    leave E[x_i^2] at sigma_i^2 within Monte Carlo error.  integ 0 takes the
    default (MN2 at these d); integ 2 forces the fourth-order MN4, whose
    negative kick coefficient the energy accounting must also cover."""
    rng = np.random.default_rng(which_d)
    d = which_d
    M = 60000 if d == 4 else 12000
    s2 = np.linspace(0.3, 3.0, d)
    x = rng.normal(size=(M, d)) * np.sqrt(s2)
    e = _gauss_ens(orc, s2, M, seed=7, acc_tol=2.0, max_steps_total=10**6, integrator_adj=integ)
    e.init(x)
    e.do_switch()
    e.set_array("sigma", np.sqrt(s2) * np.linspace(0.7, 1.4, d))  # any fixed preconditioner is valid
    e.set_hyper(eps, 1.0)
    accs = []
    for _ in range(3):
        e.mams_move()
        e.adj_control()
        accs.append(e.stats()["acc_mean"])
    assert 0.05 < np.mean(accs) < 0.75, accs
    xf = e.array("x")
    m2 = (xf**2).mean(axis=0)
    z = (m2 - s2) / (s2 * np.sqrt(2.0 / M))
    assert np.max(np.abs(z)) < 4.5, z
    # chains actually moved
    assert np.mean(np.any(xf != x, axis=1)) > 0.05


def test_mams_detailed_balance_2d(orc):
    """x ~ p exactly on a 2-D Gaussian; after one transition the joint
    histogram of (bin(x_1), bin(x'_1)) is symmetric."""
    rng = np.random.default_rng(3)
    M = 150000
    s2 = np.array([1.0, 4.0])
    x = rng.normal(size=(M, 2)) * np.sqrt(s2)
    e = _gauss_ens(orc, s2, M, seed=11, acc_tol=2.0, max_steps_total=10**6, n_steps_traj=3)
    e.init(x)
    e.do_switch()
    e.set_array("sigma", np.ones(2))
    e.set_hyper(3.5, 1.0)
    e.mams_move()
    e.adj_control()
    acc = e.stats()["acc_mean"]
    assert 0.2 < acc < 0.95
    xf = e.array("x")
    edges = stats.norm.ppf(np.linspace(0, 1, 7)[1:-1])
    a = np.digitize(x[:, 0], edges)
    b = np.digitize(xf[:, 0], edges)
    n = np.zeros((6, 6))
    np.add.at(n, (a, b), 1)
    iu = np.triu_indices(6, 1)
    num = (n[iu] - n.T[iu]) ** 2
    den = n[iu] + n.T[iu]
    chi2 = np.sum(num / den)
    assert stats.chi2.sf(chi2, len(num)) > 1e-3, chi2
    # the marginal of x' is still the target
    assert stats.kstest(xf[:, 1] / 2.0, "norm").pvalue > 1e-3


def test_mams_reject_restores_state(orc):
    # a huge step makes every proposal fail: state, gradient and log p come back bit-exact
    rng = np.random.default_rng(4)
    M, d = 64, 8
    s2 = np.linspace(0.1, 1.0, d)
    x = rng.normal(size=(M, d)) * np.sqrt(s2)
    e = _gauss_ens(orc, s2, M, acc_tol=2.0, max_steps_total=10**6)
    e.init(x)
    g0, l0 = e.array("g"), e.array("logp")
    e.do_switch()
    e.set_hyper(1e3, 1.0)
    e.mams_move()
    acc = e.array("acc")
    rejected = acc < 1e-12
    assert rejected.sum() > M // 2
    np.testing.assert_array_equal(e.array("x")[rejected], x[rejected])
    np.testing.assert_array_equal(e.array("g")[rejected], g0[rejected])
    np.testing.assert_array_equal(e.array("logp")[rejected], l0[rejected])


def test_nonfinite_chain_is_rejected(orc):
    M, d = 16, 4
    s2 = np.ones(d)
    e = _gauss_ens(orc, s2, M, acc_tol=2.0, max_steps_total=10**6)
    x = np.random.default_rng(5).normal(size=(M, d))
    x[3, 1] = np.nan
    e.init(x)
    e.do_switch()
    e.set_array("sigma", np.ones(d))
    e.set_hyper(0.5, 1.0)
    e.mams_move()
    s = e.stats()
    assert e.array("acc")[3] == 0.0 and s["n_nonfinite"] >= 1 and (s["status_bits"] & 1)
    assert np.isnan(e.array("x")[3, 1])  # restored, not propagated to others
    assert np.all(np.isfinite(np.delete(e.array("x"), 3, axis=0)))


@pytest.mark.slow
def test_full_laps_run_gaussian_chi2(orc):
    """Full LAPS on the diagonal Gaussian workload (N=1024, d=100, cold start
    N(0, 10^2 I), 1000 unadjusted + 67 adjusted transitions): b_i^2 M ~ chi^2_1
    across the 100 dimensions (E_p x_i^2 = sigma_i^2, Var_p x_i^2 = 2 sigma_i^4)."""
    w = workloads.gaussian()
    e = orc.Ensemble(orc.Target.from_workload(w), w["n_chains"], w["seed"], switch_policy=1)
    e.init(w["x0"])
    e.run()
    s = e.stats()
    assert s["t"] == 2005 and s["phase"] == 2 and s["grads_per_chain"] == 1 + 1000 + 67 * 30
    x = e.array("x")
    m2 = (x**2).mean(axis=0)
    b2M = (m2 - w["sigma2"]) ** 2 / (2 * w["sigma2"] ** 2) * w["n_chains"]
    assert stats.kstest(b2M, stats.chi2(1).cdf).pvalue > 1e-3
    assert abs(s["acc_mean"] - 0.7) < 0.03 + 0.02
