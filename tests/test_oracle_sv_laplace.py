"""Pins of the Laplace-method reference for the stochastic-volatility posterior
(oracle/sv_laplace.py).

- Without the likelihood the conditional of h given (s, r) is the AR(1)
  prior, which the Laplace method integrates exactly: the grid marginal of
  (s, r) must be the prior N(-2, 0.5^2) x N(2, 0.5^2), and E[h_t^2],
  E[h_t^4] must equal their closed forms E[e^{2s}] E[cosh^2 r] and
  3 E[e^{4s}] E[cosh^4 r] (h_t ~ N(0, sigma^2 / (1 - phi^2)) stationary).
  This checks every normalisation term (-T s, log(1 - phi^2) / 2, the
  log-determinant) of the marginal.
- With the likelihood, the conditional mode is a zero of the gradient of the
  oracle's own log density (oracle/laps_oracle.c) with respect to h, and the
  tridiagonal negative Hessian matches central differences of that gradient;
  its log-determinant and the diagonal of its inverse match dense linear
  algebra.
"""
import math

import numpy as np

from oracle import sv_laplace


def _gauss_moment(mu, var, k):
    """E[e^{k x}] for x ~ N(mu, var)."""
    return math.exp(k * mu + 0.5 * k * k * var)


def test_without_likelihood_the_marginal_is_the_prior():
    T = 50
    y = np.zeros(T)
    S = np.linspace(-2.0 - 3.5, -2.0 + 3.5, 141)
    R = np.linspace(2.0 - 3.5, 2.0 + 3.5, 141)
    out = sv_laplace.posterior_moments(y, S, R, likelihood=False)
    P = out["weights"]
    prior = np.exp(-2.0 * (S[:, None] + 2.0) ** 2 - 2.0 * (R[None, :] - 2.0) ** 2)
    prior /= prior.sum()
    assert np.max(np.abs(P - prior)) < 1e-12
    assert abs(out["E_s"] + 2.0) < 1e-9 and abs(out["E_r"] - 2.0) < 1e-9
    e2, v2 = out["E_x2"], out["Var_x2"]
    assert abs(e2[T] - 4.25) < 1e-6 and abs(e2[T + 1] - 4.25) < 1e-6
    # E[h^2] = E[e^{2s}] E[cosh^2 r], E[h^4] = 3 E[e^{4s}] E[cosh^4 r]
    Ee2s = _gauss_moment(-2.0, 0.25, 2.0)
    Ee4s = _gauss_moment(-2.0, 0.25, 4.0)
    Ech2 = 0.5 + 0.25 * (_gauss_moment(2.0, 0.25, 2.0) + _gauss_moment(2.0, 0.25, -2.0))
    Ech4 = (3.0 + 2.0 * (_gauss_moment(2.0, 0.25, 2.0) + _gauss_moment(2.0, 0.25, -2.0))
            + 0.5 * (_gauss_moment(2.0, 0.25, 4.0) + _gauss_moment(2.0, 0.25, -4.0))) / 8.0
    Eh2 = Ee2s * Ech2
    Eh4 = 3.0 * Ee4s * Ech4
    np.testing.assert_allclose(e2[:T], Eh2, rtol=1e-4)
    np.testing.assert_allclose(v2[:T], Eh4 - Eh2 ** 2, rtol=1e-3)


def _sv_target(orc, y):
    T = y.size
    return orc.Target(orc.STOCHVOL, T + 2, a=y, n=T), T


def test_mode_is_a_zero_of_the_oracle_gradient(orc):
    from paper_2601_16696_amd import workloads
    y = np.asarray(workloads.stochvol(n_chains=2, T=60)["y"])
    tgt, T = _sv_target(orc, y)
    for s, r in ((-2.7, 2.0), (-2.0, 1.5), (-3.2, 2.6)):
        _, h, _, a, b = sv_laplace.conditional(y, s, r)
        _, g = tgt.logp_grad(np.concatenate([h, [s, r]]))
        assert np.max(np.abs(g[:T])) < 1e-7 * max(1.0, np.max(np.abs(a))), (s, r, np.max(np.abs(g[:T])))
        # negative Hessian in h from central differences of the oracle gradient
        x0 = np.concatenate([h, [s, r]])
        H = np.zeros((T, T))
        step = 1e-5
        for t in range(T):
            xp, xm = x0.copy(), x0.copy()
            xp[t] += step
            xm[t] -= step
            H[:, t] = -(tgt.logp_grad(xp)[1][:T] - tgt.logp_grad(xm)[1][:T]) / (2.0 * step)
        A = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        np.testing.assert_allclose(H, A, rtol=1e-5, atol=1e-5 * np.max(np.abs(a)))


def test_log_determinant_and_inverse_diagonal_against_dense_algebra():
    from paper_2601_16696_amd import workloads
    y = np.asarray(workloads.stochvol(n_chains=2, T=40)["y"])
    T = y.size
    s, r = -2.4, 1.8
    lw, h, dinv, a, b = sv_laplace.conditional(y, s, r)
    A = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    sign, logdet = np.linalg.slogdet(A)
    assert sign > 0
    np.testing.assert_allclose(dinv, np.diag(np.linalg.inv(A)), rtol=1e-10)
    # the returned weight is log p(h*, s, r) + (T/2) log 2 pi - log det(A) / 2
    sig2, phi = math.exp(2 * s), math.tanh(r)
    P = np.diag(np.r_[1.0, np.full(T - 2, 1 + phi * phi), 1.0]) + np.diag(np.full(T - 1, -phi), 1) \
        + np.diag(np.full(T - 1, -phi), -1)
    logp = (-2 * (s + 2) ** 2 - 2 * (r - 2) ** 2 - T * s + 0.5 * math.log(1 - phi * phi)
            - h @ P @ h / (2 * sig2) + np.sum(-0.5 * h - 0.5 * y * y * np.exp(-h)))
    assert abs(lw - (logp + 0.5 * T * math.log(2 * math.pi) - 0.5 * logdet)) < 1e-8 * abs(lw)
