"""Pins of the oracle's underdamped Langevin variant (the dynamics ablation of
appendix "Ablation studies"): the microcanonical velocity replaced by a
Gaussian one, u ~ N(0, I/d) with kinetic energy (d/2)|u|^2.

The kick is checked against RK4 of Hamilton's equations du/dt = g/d,
dK/dt = g.u and against the kinetic-energy difference in 50-digit arithmetic;
the refresh through the Ornstein-Uhlenbeck transition (its limits, its
conditional mean and variance, stationarity of N(0, I/d)); the leapfrog built
from them through reversibility and second-order energy error; the adjusted
transition through exactness on Gaussian draws and detailed balance; and the
ensemble's unadjusted step against the maps composed by hand.
"""
import mpmath
import numpy as np
import pytest
from scipy import stats


def _rk4_kick(u, g, h, nsteps=50):
    d = u.size

    def f(state):
        return np.concatenate([g / d, [state[:d] @ g]])

    s = np.concatenate([u, [0.0]])
    dt = h / nsteps
    for _ in range(nsteps):
        k1 = f(s)
        k2 = f(s + 0.5 * dt * k1)
        k3 = f(s + 0.5 * dt * k2)
        k4 = f(s + dt * k3)
        s = s + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return s[:d], s[d]


@pytest.mark.parametrize("d,h,gscale", [(2, 0.3, 1.0), (9, -0.7, 5.0), (100, 0.05, 300.0)])
def test_kick_matches_hamilton_equations(orc, d, h, gscale):
    rng = np.random.default_rng(d)
    u = rng.normal(size=d) / np.sqrt(d)
    g = gscale * rng.normal(size=d)
    u1, dk = orc.map_B_lang(u, g, h)
    ur, kr = _rk4_kick(u, g, h)
    np.testing.assert_allclose(u1, ur, rtol=1e-12, atol=1e-14)
    assert abs(dk - kr) <= 1e-11 * max(abs(kr), 1.0)


def test_kick_energy_is_the_kinetic_difference(orc):
    mpmath.mp.dps = 50
    rng = np.random.default_rng(4)
    for d, h in [(3, 1e-6), (40, 0.2), (500, 3.0)]:
        u = rng.normal(size=d) / np.sqrt(d)
        g = rng.normal(size=d) * 7.0
        u1, dk = orc.map_B_lang(u, g, h)
        uu = [mpmath.mpf(float(v)) for v in u]
        un = [a + mpmath.mpf(h) / d * mpmath.mpf(float(b)) for a, b in zip(uu, g)]
        ref = mpmath.mpf(d) / 2 * (sum(v * v for v in un) - sum(v * v for v in uu))
        assert abs(dk - float(ref)) <= 1e-13 * abs(float(ref)), (d, h, dk, float(ref))


def test_refresh_limits_and_conditional_moments(orc):
    rng = np.random.default_rng(8)
    d = 6
    u = rng.normal(size=d)
    xi = rng.normal(size=d)
    np.testing.assert_array_equal(orc.map_O_lang(u, xi, 0.0, 1.0), u)
    np.testing.assert_allclose(orc.map_O_lang(u, xi, 1e4, 1.0), xi / np.sqrt(d), rtol=1e-15)
    # conditional law of one step: mean c1 u, variance (1 - c1^2)/d per component
    h, L, n = 0.3, 0.8, 200000
    c1 = np.exp(-h / L)
    xis = rng.normal(size=(n, d))
    out = np.array([orc.map_O_lang(u, x, h, L) for x in xis[:20000]])
    z = (out.mean(0) - c1 * u) / np.sqrt((1 - c1**2) / d / len(out))
    assert np.max(np.abs(z)) < 4.5
    v = out.var(0) * d / (1 - c1**2)
    assert np.max(np.abs(v - 1)) < 0.05


def test_refresh_keeps_the_gaussian_velocity_stationary(orc):
    rng = np.random.default_rng(9)
    d, n = 5, 40000
    u = rng.normal(size=(n, d)) / np.sqrt(d)
    xi = rng.normal(size=(n, d))
    out = np.array([orc.map_O_lang(u[i], xi[i], 0.7, 1.3) for i in range(n)])
    for j in range(d):
        assert stats.kstest(out[:, j] * np.sqrt(d), "norm").pvalue > 1e-3
    c = np.cov(out.T) * d
    assert np.max(np.abs(c - np.eye(d))) < 0.05


def _flow_lang(orc, tgt, x, u, eps, nsteps, which):
    b, a = orc.integrator_coeffs(which)
    lp, g = tgt.logp_grad(x)
    E = 0.0
    for _ in range(nsteps):
        for k in range(b.size):
            u, dk = orc.map_B_lang(u, g, b[k] * eps)
            E += dk
            if k == b.size - 1:
                break
            x = orc.map_A(x, u, a[k] * eps)
            l2, g = tgt.logp_grad(x)
            E += lp - l2
            lp = l2
    return x, u, E


@pytest.mark.parametrize("which", [0, 1, 2])
def test_langevin_flow_reversible(orc, which):
    rng = np.random.default_rng(20 + which)
    d = 10
    tgt = orc.Target(orc.GAUSS_DIAG, d, a=10 ** rng.uniform(-0.5, 0.5, size=d))
    x = rng.normal(size=d)
    u = rng.normal(size=d) / np.sqrt(d)
    x1, u1, E1 = _flow_lang(orc, tgt, x, u, 0.2, 15, which)
    x2, u2, E2 = _flow_lang(orc, tgt, x1, -u1, 0.2, 15, which)
    np.testing.assert_allclose(x2, x, atol=1e-12)
    np.testing.assert_allclose(-u2, u, atol=1e-12)
    assert abs(E1 + E2) < 1e-10


@pytest.mark.parametrize("which,order", [(0, 2), (1, 2), (2, 4)])
def test_langevin_flow_energy_error_order(orc, which, order):
    rng = np.random.default_rng(31)
    d = 8
    tgt = orc.Target(orc.GAUSS_DIAG, d, a=np.linspace(0.5, 2.0, d))
    x = rng.normal(size=d)
    u = rng.normal(size=d) / np.sqrt(d)
    epss = [0.1, 0.05, 0.025]
    errs = [abs(_flow_lang(orc, tgt, x, u, eps, int(round(1.0 / eps)), which)[2]) for eps in epss]
    slopes = np.diff(np.log(errs)) / np.diff(np.log(epss))
    assert np.all(np.abs(slopes - order) < 0.35), slopes


def _gauss_ens(orc, s2, M, seed=1, **cfg):
    return orc.Ensemble(orc.Target(orc.GAUSS_DIAG, s2.size, a=s2), M, seed, dynamics=1, **cfg)


def test_unadjusted_step_composes_the_maps(orc):
    """One unadjusted step of the ensemble equals O_lang, leapfrog with the
    Langevin kick, O_lang composed by hand from the same normals."""
    rng = np.random.default_rng(12)
    d, M, seed = 7, 5, 21
    s2 = np.linspace(0.5, 3.0, d)
    e = _gauss_ens(orc, s2, M, seed=seed)
    x0 = rng.normal(size=(M, d)) * 2.0
    u0 = rng.normal(size=(M, d)) / np.sqrt(d)
    e.init(x0, u0)
    st = e.stats()
    eps, L = st["eps"], st["L"]
    e.unadj_move()
    tgt = orc.Target(orc.GAUSS_DIAG, d, a=s2)
    for m in range(M):
        u = orc.map_O_lang(u0[m], orc.normals(seed, m, 0, orc.TAG_O_FIRST, 0, d), 0.5 * eps, L)
        x, u, E = _flow_lang(orc, tgt, x0[m], u, eps, 1, 0)
        u = orc.map_O_lang(u, orc.normals(seed, m, 0, orc.TAG_O_SECOND, 0, d), 0.5 * eps, L)
        np.testing.assert_allclose(e.array("x")[m], x, rtol=1e-15, atol=1e-15)
        np.testing.assert_allclose(e.array("u")[m], u, rtol=1e-15, atol=1e-15)
        assert abs(e.array("delta")[m] - E) <= 1e-14 * max(abs(E), 1.0)


@pytest.mark.parametrize("d,eps", [(4, 3.5), (30, 9.0)])
def test_adjusted_langevin_preserves_exact_gaussian(orc, d, eps):
    rng = np.random.default_rng(40 + d)
    M = 60000 if d == 4 else 12000
    s2 = np.linspace(0.3, 3.0, d)
    x = rng.normal(size=(M, d)) * np.sqrt(s2)
    e = _gauss_ens(orc, s2, M, seed=7, acc_tol=2.0, max_steps_total=10**6)
    e.init(x)
    e.do_switch()
    e.set_array("sigma", np.sqrt(s2) * np.linspace(0.7, 1.4, d))
    e.set_hyper(eps, 1.0)
    accs = []
    for _ in range(3):
        e.mams_move()
        e.adj_control()
        accs.append(e.stats()["acc_mean"])
    assert 0.05 < np.mean(accs) < 0.9, accs
    xf = e.array("x")
    z = ((xf**2).mean(axis=0) - s2) / (s2 * np.sqrt(2.0 / M))
    assert np.max(np.abs(z)) < 4.5, z
    assert np.mean(np.any(xf != x, axis=1)) > 0.05


def test_adjusted_langevin_detailed_balance_2d(orc):
    rng = np.random.default_rng(5)
    M = 150000
    s2 = np.array([1.0, 4.0])
    x = rng.normal(size=(M, 2)) * np.sqrt(s2)
    e = _gauss_ens(orc, s2, M, seed=13, acc_tol=2.0, max_steps_total=10**6, n_steps_traj=3)
    e.init(x)
    e.do_switch()
    e.set_array("sigma", np.ones(2))
    e.set_hyper(3.6, 1.0)
    e.mams_move()
    e.adj_control()
    assert 0.2 < e.stats()["acc_mean"] < 0.95
    xf = e.array("x")
    edges = stats.norm.ppf(np.linspace(0, 1, 7)[1:-1])
    a = np.digitize(x[:, 0], edges)
    b = np.digitize(xf[:, 0], edges)
    n = np.zeros((6, 6))
    np.add.at(n, (a, b), 1)
    iu = np.triu_indices(6, 1)
    num, den = (n[iu] - n.T[iu]) ** 2, n[iu] + n.T[iu]
    seen = den > 0  # bin pairs never joined in either direction are trivially symmetric
    assert seen.sum() >= 5
    chi2 = np.sum(num[seen] / den[seen])
    assert stats.chi2.sf(chi2, int(seen.sum())) > 1e-3, chi2
    assert stats.kstest(xf[:, 1] / 2.0, "norm").pvalue > 1e-3


def test_dynamics_field_validated(orc):
    with pytest.raises(ValueError):
        orc.Ensemble(orc.Target(orc.GAUSS_DIAG, 3, a=np.ones(3)), 4, 1, dynamics=2)
