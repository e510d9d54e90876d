"""Reference posterior moments of the stochastic-volatility target by the
Laplace method.

TEST INFRASTRUCTURE ONLY: used by tests/ and by the script that writes the
stored reference (tests/golden/stochvol_laplace.py); never by the product
path.  It shares no code with the GPU library.

Target (the benchmark's stochastic-volatility model): theta = (h_1..h_T, s, r),
sigma = e^s, phi = tanh r, s ~ N(-2, 0.5^2), r ~ N(2, 0.5^2),
h_1 ~ N(0, sigma^2 / (1 - phi^2)), h_t ~ N(phi h_{t-1}, sigma^2),
y_t ~ N(0, e^{h_t}); log p is the oracle's (additive constants dropped):
    log p = -2 (s + 2)^2 - 2 (r - 2)^2 - T s + log(1 - phi^2) / 2
            - h^T P h / (2 sigma^2) - sum_t [h_t / 2 + y_t^2 e^{-h_t} / 2],
with P the tridiagonal AR(1) precision (diagonal 1, 1 + phi^2, ..., 1 + phi^2, 1;
off-diagonal -phi).

Method.  The hyperparameters (s, r) are integrated on a grid.  For each grid
point the latent h is integrated by the Laplace approximation at its
conditional mode h* (Newton's method; the negative Hessian
A = P / sigma^2 + diag(y^2 e^{-h*} / 2) is tridiagonal):
    log p(s, r | y) ~ log p(h*, s, r) + (T/2) log 2 pi - log det(A) / 2,
and h given (s, r) is taken as N(h*, A^{-1}), whose marginal variances are
the diagonal of A^{-1}.  Moments of x_i^2 follow by mixing these Gaussians
over the grid weights.  Without the likelihood terms the conditional of h is
exactly Gaussian and the method is exact (the grid marginal is then the
prior): that case pins the normalisation.

Parity: pinned by the CPU tests in tests/test_oracle_sv_laplace.py (prior
recovered exactly without the likelihood; the mode is a zero of the oracle
target's gradient; Hessian, its log-determinant and the diagonal of its
inverse against dense linear algebra on a short series).  The Laplace error
itself (the departure of h | s, r, y from a Gaussian) is not bounded by a
test: parity unpinned for that approximation; it is small here because the
AR(1) prior's precision (~(1 + phi^2) / sigma^2 ~ 400) dominates the
likelihood's curvature (~1/2) in every h_t.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded


def _precision(T: int, phi: float):
    dP = np.full(T, 1.0 + phi * phi)
    dP[0] = 1.0
    dP[-1] = 1.0
    oP = np.full(T - 1, -phi)
    return dP, oP


def _tri_mul(dP, oP, h):
    v = dP * h
    v[:-1] += oP * h[1:]
    v[1:] += oP * h[:-1]
    return v


def conditional(y, s: float, r: float, h0=None, likelihood: bool = True, tol: float = 1e-12):
    """Laplace approximation of h | s, r, y: returns (log of the grid weight
    of (s, r) up to a constant, the mode h*, the diagonal of A^{-1}, the
    diagonal and off-diagonal of A)."""
    y = np.asarray(y, dtype=np.float64)
    T = y.size
    sig2 = np.exp(2.0 * s)
    phi = np.tanh(r)
    omp = 1.0 - phi * phi
    dP, oP = _precision(T, phi)
    y2 = y * y
    h = np.zeros(T) if h0 is None else np.array(h0, dtype=np.float64)
    for _ in range(200):
        e = y2 * np.exp(-h) if likelihood else np.zeros(T)
        g = -_tri_mul(dP, oP, h) / sig2 + ((-0.5 + 0.5 * e) if likelihood else 0.0)
        ab = np.zeros((3, T))
        ab[0, 1:] = oP / sig2
        ab[1] = dP / sig2 + 0.5 * e
        ab[2, :-1] = oP / sig2
        step = solve_banded((1, 1), ab, g)
        h = h + step
        if np.max(np.abs(step)) < tol:
            break
    e = y2 * np.exp(-h) if likelihood else np.zeros(T)
    E = float(h @ _tri_mul(dP, oP, h))
    lik = float(np.sum(-0.5 * h - 0.5 * e)) if likelihood else 0.0
    logp = -2.0 * (s + 2.0) ** 2 - 2.0 * (r - 2.0) ** 2 - T * s + 0.5 * np.log(omp) - E / (2.0 * sig2) + lik
    a = dP / sig2 + 0.5 * e
    b = oP / sig2
    # forward and backward pivots of the tridiagonal A; log det from the forward
    # ones, diag(A^{-1})_t = 1 / (fwd_t + bwd_t - a_t)
    fwd = np.empty(T)
    fwd[0] = a[0]
    for t in range(1, T):
        fwd[t] = a[t] - b[t - 1] ** 2 / fwd[t - 1]
    bwd = np.empty(T)
    bwd[-1] = a[-1]
    for t in range(T - 2, -1, -1):
        bwd[t] = a[t] - b[t] ** 2 / bwd[t + 1]
    logdet = float(np.sum(np.log(fwd)))
    dinv = 1.0 / (fwd + bwd - a)
    return logp + 0.5 * T * np.log(2.0 * np.pi) - 0.5 * logdet, h, dinv, a, b


def posterior_moments(y, S, R, likelihood: bool = True) -> dict:
    """E[x_i^2] and Var[x_i^2] for x = (h_1..h_T, s, r) on the (s, r) grid S x R
    (rectangle rule), with h | s, r ~ N(h*, diag(A^{-1})) per grid point."""
    y = np.asarray(y, dtype=np.float64)
    T = y.size
    S = np.asarray(S, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    L = np.empty((S.size, R.size))
    m2 = np.zeros((S.size, R.size, T))
    m4 = np.zeros((S.size, R.size, T))
    for i, s in enumerate(S):
        hprev = None
        for j, r in enumerate(R):
            lw, h, v, _, _ = conditional(y, s, r, h0=hprev, likelihood=likelihood)
            hprev = h
            L[i, j] = lw
            m2[i, j] = h * h + v
            m4[i, j] = h ** 4 + 6.0 * h * h * v + 3.0 * v * v
    L -= L.max()
    P = np.exp(L)
    P /= P.sum()
    Ps, Pr = P.sum(1), P.sum(0)
    e2 = np.concatenate([np.einsum("ij,ijt->t", P, m2), [np.sum(Ps * S ** 2), np.sum(Pr * R ** 2)]])
    e4 = np.concatenate([np.einsum("ij,ijt->t", P, m4), [np.sum(Ps * S ** 4), np.sum(Pr * R ** 4)]])
    edge = float(P[0].sum() + P[-1].sum() + P[:, 0].sum() + P[:, -1].sum())
    return dict(E_x2=e2, Var_x2=e4 - e2 * e2, E_s=float(np.sum(Ps * S)), E_r=float(np.sum(Pr * R)),
                grid_edge_mass=edge, weights=P)
