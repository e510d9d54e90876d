"""Seeded synthetic inputs for the LAPS hot path.

This module is the only code shared by the GPU path's tests/benchmark and the
CPU oracle.  It draws targets' data and initial positions with numpy's
``default_rng`` and holds none of the sampler's arithmetic.  The paper's
benchmark datasets are not available, so these inputs stand in for them with
the shapes and distributions stated per workload.
"""
from __future__ import annotations

import numpy as np


def round_to_bf16(a: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even); returns float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    r = ((bits + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def gaussian(n_chains: int = 1024, d: int = 100, seed_data: int = 1001, seed_x0: int = 2001,
             seed_rng: int = 3001, x0_scale: float = 10.0) -> dict:
    """Diagonal Gaussian, variances log-uniform in [1e-2, 1e2]; cold start N(0, 10^2 I)."""
    sigma2 = 10.0 ** np.random.default_rng(seed_data).uniform(-2.0, 2.0, size=d)
    x0 = np.random.default_rng(seed_x0).normal(0.0, x0_scale, size=(n_chains, d))
    return dict(kind="gauss", d=d, n_chains=n_chains, sigma2=sigma2, x0=x0, seed=seed_rng,
                name=f"gaussian_diag_d{d}_N{n_chains}")


def ill_gaussian(n_chains: int = 1024, d: int = 100, seed_data: int = 1006, seed_x0: int = 2006,
                 seed_rng: int = 3006, shape: float = 0.5) -> dict:
    """Randomly rotated ill-conditioned Gaussian (zero mean): covariance eigenvalues ~ Gamma(shape, 1)
    (condition number ~1e5 at d = 100), orientation Haar-random (QR of a Gaussian matrix with the sign
    of R's diagonal folded in); start N(0, I).  prec = covariance^-1, cov_diag = diag(covariance)."""
    rng = np.random.default_rng(seed_data)
    lam = rng.gamma(shape, 1.0, size=d)
    q, r = np.linalg.qr(rng.normal(size=(d, d)))
    q = q * np.sign(np.diag(r))
    cov = (q * lam) @ q.T
    prec = (q / lam) @ q.T
    cov, prec = 0.5 * (cov + cov.T), 0.5 * (prec + prec.T)
    x0 = np.random.default_rng(seed_x0).normal(size=(n_chains, d))
    return dict(kind="gauss_dense", d=d, n_chains=n_chains, prec=prec, cov=cov, cov_diag=np.diag(cov).copy(),
                cond=float(lam.max() / lam.min()), x0=x0, seed=seed_rng, name=f"ill_gaussian_d{d}_N{n_chains}")


def logreg(n_chains: int = 4096, n: int = 5000, d: int = 100, seed_data: int = 1002, seed_x0: int = 2002,
           seed_rng: int = 3002) -> dict:
    """Bayesian logistic regression: X ~ N(0,1) rounded to bf16 (those values define the problem),
    true weights ~ N(0, 1/d), labels ~ Bernoulli(sigmoid(X w)), prior N(0, I); x0 from the prior."""
    rng = np.random.default_rng(seed_data)
    X = round_to_bf16(rng.normal(size=(n, d)))
    w = rng.normal(0.0, 1.0 / np.sqrt(d), size=d)
    p = 1.0 / (1.0 + np.exp(-(X @ w)))
    y = (rng.uniform(size=n) < p).astype(np.float64)
    x0 = np.random.default_rng(seed_x0).normal(size=(n_chains, d))
    return dict(kind="logreg", d=d, n_chains=n_chains, X=X, y=y, w_true=w, x0=x0, seed=seed_rng,
                name=f"logreg_n{n}_d{d}_N{n_chains}")


def _sv_prior(rng, T: int, count: int) -> np.ndarray:
    s = rng.normal(-2.0, 0.5, size=count)
    r = rng.normal(2.0, 0.5, size=count)
    sig = np.exp(s)
    phi = np.tanh(r)
    h = np.empty((count, T))
    h[:, 0] = rng.normal(size=count) * sig / np.sqrt(1.0 - phi * phi)
    eta = rng.normal(size=(count, T))
    for t in range(1, T):
        h[:, t] = phi * h[:, t - 1] + sig * eta[:, t]
    return np.concatenate([h, s[:, None], r[:, None]], axis=1)


def stochvol(n_chains: int = 4096, T: int = 2427, seed_data: int = 1003, seed_x0: int = 2003,
             seed_rng: int = 3003) -> dict:
    """Stochastic volatility: theta = (h_1..h_T, s, r), sigma = e^s, phi = tanh r,
    s ~ N(-2, 0.5^2), r ~ N(2, 0.5^2), AR(1) log-volatility, y_t ~ N(0, e^{h_t}).
    Returns y are drawn from the model's own prior (one draw); x0 from the prior."""
    rng = np.random.default_rng(seed_data)
    truth = _sv_prior(rng, T, 1)[0]
    y = rng.normal(size=T) * np.exp(0.5 * truth[:T])
    x0 = _sv_prior(np.random.default_rng(seed_x0), T, n_chains)
    return dict(kind="stochvol", d=T + 2, n_chains=n_chains, y=y, truth=truth, x0=x0, seed=seed_rng,
                name=f"stochvol_T{T}_N{n_chains}")


def phi4(n_chains: int = 2048, side: int = 64, m2: float = -4.0, lam: float = 8.0, seed_x0: int = 2004,
         seed_rng: int = 3004) -> dict:
    """2-D periodic lattice phi^4, L x L sites, x0 ~ N(0, 1) i.i.d."""
    x0 = np.random.default_rng(seed_x0).normal(size=(n_chains, side * side))
    return dict(kind="phi4", d=side * side, n_chains=n_chains, side=side, m2=m2, lam=lam, x0=x0,
                seed=seed_rng, name=f"phi4_L{side}_N{n_chains}")


def batched_mix(scale: float = 1.0) -> list[dict]:
    """Sixteen targets in one launch: 8 Gaussians with d log-spaced in 10..2000 and 8 logistic
    regressions with (n, d) log-spaced in (1000, 20)..(20000, 300); chain counts log-spaced in
    512..8192 assigned by a seeded permutation.  ``scale`` < 1 shrinks every size for tests."""
    gd = [10, 21, 45, 97, 206, 440, 938, 2000]
    ln = [(1000, 20), (1534, 29), (2354, 43), (3611, 64), (5539, 94), (8498, 138), (13037, 204), (20000, 300)]
    counts = [512, 616, 741, 891, 1072, 1290, 1552, 1867, 2246, 2702, 3251, 3911, 4705, 5660, 6810, 8192]
    perm = np.random.default_rng(5).permutation(16)
    out = []
    for k in range(16):
        N = max(8, int(round(counts[perm[k]] * scale)))
        if k < 8:
            d = max(2, int(round(gd[k] * (scale if scale < 1 else 1))))
            w = gaussian(N, d, seed_data=1005 + k, seed_x0=2005 + k, seed_rng=3005 + k)
        else:
            n, d = ln[k - 8]
            if scale < 1:
                n, d = max(16, int(round(n * scale))), max(2, int(round(d * scale)))
            w = logreg(N, n, d, seed_data=1005 + k, seed_x0=2005 + k, seed_rng=3005 + k)
        out.append(w)
    return out
