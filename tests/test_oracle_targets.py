"""Pins of the oracle's targets: log p differences against scipy's densities of
the generative models, gradients against central finite differences, and
closed-form special cases."""
import numpy as np
import pytest
from scipy import sparse, stats
from scipy.special import expit

from paper_2601_16696_amd import workloads


def _fd_grad(tgt, x, h=1e-5):
    g = np.zeros_like(x)
    for i in range(x.size):
        e = np.zeros_like(x)
        e[i] = h
        g[i] = (tgt.logp(x + e) - tgt.logp(x - e)) / (2 * h)
    return g


def _check_fd(tgt, x, rtol=1e-7):
    _, g = tgt.logp_grad(x)
    gf = _fd_grad(tgt, x)
    scale = np.max(np.abs(g)) + 1e-300
    assert np.max(np.abs(g - gf)) / scale < rtol


def test_gauss_against_scipy_and_fd(orc):
    rng = np.random.default_rng(0)
    s2 = 10 ** rng.uniform(-2, 2, size=30)
    tgt = orc.Target(orc.GAUSS_DIAG, 30, a=s2)
    x1, x2 = rng.normal(size=30), rng.normal(size=30)
    ref = stats.norm.logpdf(x1, scale=np.sqrt(s2)).sum() - stats.norm.logpdf(x2, scale=np.sqrt(s2)).sum()
    assert abs((tgt.logp(x1) - tgt.logp(x2)) - ref) < 1e-9 * max(1, abs(ref))
    _check_fd(tgt, x1)


def test_logreg_against_bernoulli_likelihood_and_fd(orc):
    w = workloads.logreg(n_chains=4, n=300, d=17, seed_data=7)
    tgt = orc.Target.from_workload(w)
    X, y = w["X"], w["y"]

    def ref_logp(th):
        p = expit(X @ th)
        return (stats.bernoulli.logpmf(y, p).sum() + stats.norm.logpdf(th).sum())

    th1, th2 = w["x0"][0], w["x0"][1]
    assert abs((tgt.logp(th1) - tgt.logp(th2)) - (ref_logp(th1) - ref_logp(th2))) < 1e-8
    _check_fd(tgt, th1)


def test_logreg_without_data_is_standard_normal(orc):
    d, n = 9, 50
    tgt = orc.Target(orc.LOGREG, d, a=np.zeros((n, d)), b=np.ones(n), n=n)
    th = np.random.default_rng(1).normal(size=d)
    l, g = tgt.logp_grad(th)
    np.testing.assert_allclose(g, -th, rtol=0, atol=1e-15)
    # softplus(0) = log 2 per row, y z = 0
    assert abs(l - (-0.5 * th @ th - n * np.log(2.0))) < 1e-12


def test_logreg_extreme_logits_finite(orc):
    d, n = 3, 4
    X = np.array([[400.0, 0, 0], [-400.0, 0, 0], [0, 800.0, 0], [0, 0, -900.0]])
    tgt = orc.Target(orc.LOGREG, d, a=X, b=np.array([1.0, 0.0, 0.0, 1.0]), n=n)
    l, g = tgt.logp_grad(np.ones(d))
    assert np.isfinite(l) and np.all(np.isfinite(g))


def _sv_ref_logp(theta, y):
    T = y.size
    h, s, r = theta[:T], theta[T], theta[T + 1]
    sig, phi = np.exp(s), np.tanh(r)
    lp = stats.norm.logpdf(s, -2.0, 0.5) + stats.norm.logpdf(r, 2.0, 0.5)
    lp += stats.norm.logpdf(h[0], 0.0, sig / np.sqrt(1 - phi**2))
    lp += stats.norm.logpdf(h[1:], phi * h[:-1], sig).sum()
    lp += stats.norm.logpdf(y, 0.0, np.exp(0.5 * h)).sum()
    return lp


def test_stochvol_against_generative_model_and_fd(orc):
    w = workloads.stochvol(n_chains=3, T=40)
    tgt = orc.Target.from_workload(w)
    a, b = w["x0"][0], w["x0"][1]
    ref = _sv_ref_logp(a, w["y"]) - _sv_ref_logp(b, w["y"])
    assert abs((tgt.logp(a) - tgt.logp(b)) - ref) < 1e-8 * max(1, abs(ref))
    _check_fd(tgt, a, rtol=2e-7)


def test_stochvol_single_step_series(orc):
    # T = 1: only the stationary prior of h_1 and the likelihood remain
    y = np.array([0.3])
    tgt = orc.Target(orc.STOCHVOL, 3, a=y, n=1)
    a, b = np.array([0.2, -1.7, 1.5]), np.array([-0.4, -2.3, 2.2])
    ref = _sv_ref_logp(a, y) - _sv_ref_logp(b, y)
    assert abs((tgt.logp(a) - tgt.logp(b)) - ref) < 1e-10
    _check_fd(tgt, a)


def _phi4_free_field_precision(L, m2):
    """K = m2 I + graph Laplacian of the periodic L x L lattice."""
    n = L * L
    rows, cols, vals = [], [], []
    for r in range(L):
        for c in range(L):
            i = r * L + c
            rows.append(i); cols.append(i); vals.append(4.0 + m2)
            for j in (r * L + (c + 1) % L, r * L + (c - 1) % L, ((r + 1) % L) * L + c, ((r - 1) % L) * L + c):
                rows.append(i); cols.append(j); vals.append(-1.0)
    return sparse.csr_matrix((vals, (rows, cols)), shape=(n, n))


def test_phi4_free_field_is_gaussian(orc):
    L, m2 = 6, 0.7
    tgt = orc.Target(orc.PHI4, L * L, n=L, p0=m2, p1=0.0)
    K = _phi4_free_field_precision(L, m2)
    x = np.random.default_rng(2).normal(size=L * L)
    l, g = tgt.logp_grad(x)
    assert abs(l - (-0.5 * x @ (K @ x))) < 1e-11 * max(1, abs(l))
    np.testing.assert_allclose(g, -(K @ x), rtol=0, atol=1e-12)


def test_phi4_constant_field_and_fd(orc):
    L, m2, lam = 5, -4.0, 8.0
    tgt = orc.Target(orc.PHI4, L * L, n=L, p0=m2, p1=lam)
    c = 0.37
    l = tgt.logp(np.full(L * L, c))
    # gradient terms vanish for a constant field
    assert abs(l - (-(L * L) * (0.5 * m2 * c * c + lam * c**4))) < 1e-12
    x = np.random.default_rng(3).normal(size=L * L)
    _check_fd(tgt, x)


def test_phi4_rectangular_indexing_is_periodic(orc):
    # shifting the field by one lattice site in either direction leaves log p unchanged
    L = 7
    tgt = orc.Target(orc.PHI4, L * L, n=L, p0=-1.0, p1=0.5)
    x = np.random.default_rng(4).normal(size=(L, L))
    l0 = tgt.logp(x.ravel())
    assert abs(tgt.logp(np.roll(x, 1, axis=0).ravel()) - l0) < 1e-11
    assert abs(tgt.logp(np.roll(x, 1, axis=1).ravel()) - l0) < 1e-11
    assert abs(tgt.logp(x.T.copy().ravel()) - l0) < 1e-11


def test_dense_gauss_against_scipy_and_fd(orc):
    w = workloads.ill_gaussian(n_chains=4, d=20)
    tgt = orc.Target.from_workload(w)
    mvn = stats.multivariate_normal(mean=np.zeros(20), cov=w["cov"])
    x1, x2 = w["x0"][0], w["x0"][1]
    ref = mvn.logpdf(x1) - mvn.logpdf(x2)
    assert abs((tgt.logp(x1) - tgt.logp(x2)) - ref) < 1e-8 * max(1, abs(ref))
    _check_fd(tgt, x1, rtol=1e-6)


def test_dense_gauss_with_diagonal_precision_is_the_diagonal_target(orc):
    rng = np.random.default_rng(4)
    s2 = 10 ** rng.uniform(-2, 2, size=12)
    dense = orc.Target(orc.GAUSS_DENSE, 12, a=np.diag(1.0 / s2))
    diag = orc.Target(orc.GAUSS_DIAG, 12, a=s2)
    x = rng.normal(size=12)
    ld, gd = dense.logp_grad(x)
    l0, g0 = diag.logp_grad(x)
    assert abs(ld - l0) <= 1e-13 * abs(l0) and np.allclose(gd, g0, rtol=1e-14, atol=0)


def test_ill_gaussian_workload_is_ill_conditioned():
    w = workloads.ill_gaussian()
    assert 1e4 < w["cond"] < 1e7
    assert np.allclose(w["prec"] @ w["cov"], np.eye(100), atol=1e-6 * w["cond"])
