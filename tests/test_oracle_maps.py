"""Pins of the oracle's integrator maps (Appendix D of the paper).

Phi^B is checked against an RK4 solution of the Riccati velocity equation and
of the energy rate g.u it induces, and through its exact-flow group property;
Phi^O through norm preservation, its two limits and the noise strength
eta = sqrt(2/(L d)) of the SDE; the compositions through reversibility and the
convergence order of their energy error.
"""
import numpy as np
import pytest


def _unit(v):
    return v / np.linalg.norm(v)


# ------------------------------------------------------------------ Phi^B
def _rk4_velocity(u, g, h, nsteps=4000):
    """RK4 of du/dt = (I - u u^T) g/(d-1), dK/dt = g.u over time h."""
    d = u.size

    def f(state):
        uu = state[:d]
        du = (g - uu * (uu @ g)) / (d - 1)
        return np.concatenate([du, [uu @ g]])

    s = np.concatenate([u, [0.0]])
    dt = h / nsteps
    for _ in range(nsteps):
        k1 = f(s)
        k2 = f(s + 0.5 * dt * k1)
        k3 = f(s + 0.5 * dt * k2)
        k4 = f(s + dt * k3)
        s = s + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return s[:d], s[d]


@pytest.mark.parametrize("d,h,gscale", [(2, 0.3, 1.0), (7, 0.5, 3.0), (50, 0.2, 40.0), (50, -0.25, 40.0)])
def test_B_matches_rk4_of_riccati_flow(orc, d, h, gscale):
    rng = np.random.default_rng(d)
    u = _unit(rng.normal(size=d))
    g = gscale * rng.normal(size=d)
    u1, dk = orc.map_B(u, g, h)
    ur, kr = _rk4_velocity(u, g, h)
    np.testing.assert_allclose(u1, ur, rtol=0, atol=1e-10)
    assert abs(dk - kr) < 1e-9 * max(1.0, abs(kr))


def test_B_unit_norm_and_group_property(orc):
    rng = np.random.default_rng(1)
    d = 33
    u = _unit(rng.normal(size=d))
    g = 25 * rng.normal(size=d)
    ua, ka = orc.map_B(u, g, 0.37)
    uab, kb = orc.map_B(ua, g, 0.81)
    uc, kc = orc.map_B(u, g, 1.18)
    assert abs(np.linalg.norm(ua) - 1) < 1e-14
    np.testing.assert_allclose(uab, uc, atol=1e-13)
    assert abs(ka + kb - kc) < 1e-12 * max(1, abs(kc))
    # the reverse-time map undoes the forward map (exact flow)
    ub, kback = orc.map_B(uc, g, -1.18)
    np.testing.assert_allclose(ub, u, atol=1e-13)
    assert abs(kback + kc) < 1e-11 * max(1, abs(kc))


def test_B_zero_gradient_is_identity(orc):
    u = _unit(np.arange(1.0, 6.0))
    u1, dk = orc.map_B(u, np.zeros(5), 0.7)
    assert np.array_equal(u1, u) and dk == 0.0


def test_B_first_order_energy(orc):
    rng = np.random.default_rng(4)
    d = 20
    u = _unit(rng.normal(size=d))
    g = rng.normal(size=d)
    h = 1e-3
    _, dk = orc.map_B(u, g, h)
    # Taylor expansion of the energy rate: dK = h u.g + h^2 |g_perp|^2 / (2 (d-1)) + O(h^3)
    gperp2 = g @ g - (u @ g) ** 2
    expect = h * (u @ g) + h * h * gperp2 / (2 * (d - 1))
    assert abs(dk - expect) < 1e-7 * abs(expect)


def test_B_collinear_velocity_does_not_turn(orc):
    g = np.array([3.0, 4.0, 0.0])
    u = g / 5.0
    u1, dk = orc.map_B(u, g, 0.9)
    np.testing.assert_allclose(u1, u, atol=1e-15)
    # e.u = 1: Delta K = (d-1) log(cosh + sinh) = (d-1) delta = h |g|
    assert abs(dk - 0.9 * 5.0) < 1e-13


# ------------------------------------------------------------------ Phi^O
def test_O_unit_norm_and_limits(orc):
    rng = np.random.default_rng(2)
    d = 40
    u = _unit(rng.normal(size=d))
    xi = rng.normal(size=d)
    u1 = orc.map_O(u, xi, 0.3, 2.0)
    assert abs(np.linalg.norm(u1) - 1) < 1e-14
    # h -> 0: c1 = 1, c2 = 0: identity
    np.testing.assert_allclose(orc.map_O(u, xi, 0.0, 2.0), u, atol=1e-15)
    # h/L -> infinity: c1 = 0: a direction drawn from xi alone
    np.testing.assert_allclose(orc.map_O(u, xi, 1e6, 1.0), _unit(xi), atol=1e-14)


def test_O_noise_strength_matches_sde(orc):
    """For small h the perpendicular increment of u has variance eta^2 h per
    unit of the (d-1)-dimensional tangent space times d-1 in total, with
    eta = sqrt(2/(L d)) (eq. SDE)."""
    rng = np.random.default_rng(3)
    d, h, L = 10, 1e-4, 0.5
    u = _unit(rng.normal(size=d))
    incs = []
    for _ in range(20000):
        xi = rng.normal(size=d)
        u1 = orc.map_O(u, xi, h, L)
        du = u1 - u
        perp = du - u * (u @ du)
        incs.append(perp @ perp)
    eta2 = 2.0 / (L * d)
    expect = eta2 * h * (d - 1)
    got = np.mean(incs)
    assert abs(got / expect - 1) < 0.05


def test_O_full_refresh_is_uniform_on_sphere(orc):
    rng = np.random.default_rng(5)
    d = 6
    us = np.array([orc.map_O(np.eye(d)[0], rng.normal(size=d), 1e6, 1.0) for _ in range(20000)])
    # uniform direction: E u_i^2 = 1/d, E u_i = 0
    np.testing.assert_allclose((us**2).mean(axis=0), 1 / d, atol=0.01)
    np.testing.assert_allclose(us.mean(axis=0), 0, atol=0.02)


# ------------------------------------------------------------------ Phi^A
def test_A_position_update(orc):
    x = np.array([1.0, -2.0, 3.0])
    u = np.array([0.6, 0.8, 0.0])
    np.testing.assert_allclose(orc.map_A(x, u, 0.5), x + 0.5 * u, rtol=0, atol=0)
    s = np.array([2.0, 0.5, 1.0])
    np.testing.assert_allclose(orc.map_A(x, u, 0.5, s), x + 0.5 * s * u, rtol=0, atol=1e-15)


# ------------------------------------------------------------------ compositions
def test_integrator_tables(orc):
    for which, K in ((0, 2), (1, 3), (2, 6)):
        b, a = orc.integrator_coeffs(which)
        assert b.size == K and a.size == K - 1
        assert abs(b.sum() - 1) < 1e-15 and abs(a.sum() - 1) < 1e-15
        np.testing.assert_array_equal(b, b[::-1])
        np.testing.assert_array_equal(a, a[::-1])
    b, a = orc.integrator_coeffs(2)
    assert abs(b[2] - (-0.2662196861)) < 1e-10 and abs(a[2] - 0.5566487124) < 1e-10
    b, a = orc.integrator_coeffs(1)
    assert b[0] == 0.1931833275 and a[0] == 0.5


def _flow(orc, tgt, x, u, eps, nsteps, which):
    """Deterministic integrator only (no refresh); returns x, u, total energy error."""
    b, a = orc.integrator_coeffs(which)
    lp, g = tgt.logp_grad(x)
    E = 0.0
    for _ in range(nsteps):
        for k in range(b.size):
            u, dk = orc.map_B(u, g, b[k] * eps)
            E += dk
            if k == b.size - 1:
                break
            x = orc.map_A(x, u, a[k] * eps)
            l2, g = tgt.logp_grad(x)
            E += lp - l2
            lp = l2
    return x, u, E


@pytest.mark.parametrize("which", [0, 1, 2])
def test_composition_reversible(orc, which):
    rng = np.random.default_rng(which)
    d = 12
    tgt = orc.Target(orc.GAUSS_DIAG, d, a=10 ** rng.uniform(-1, 1, size=d))
    x = rng.normal(size=d)
    u = _unit(rng.normal(size=d))
    x1, u1, E1 = _flow(orc, tgt, x, u, 0.1, 20, which)
    x2, u2, E2 = _flow(orc, tgt, x1, -u1, 0.1, 20, which)
    np.testing.assert_allclose(x2, x, atol=1e-12)
    np.testing.assert_allclose(-u2, u, atol=1e-12)
    assert abs(E1 + E2) < 1e-10


@pytest.mark.parametrize("which,order", [(0, 2), (1, 2), (2, 4)])
def test_composition_energy_error_order(orc, which, order):
    """At fixed total time the energy error of the deterministic flow decays as
    eps^order; a wrong coefficient in a table breaks the fourth order."""
    rng = np.random.default_rng(11)
    d = 8
    tgt = orc.Target(orc.GAUSS_DIAG, d, a=np.linspace(0.5, 2.0, d))
    x = rng.normal(size=d)
    u = _unit(rng.normal(size=d))
    Ttot = 1.0
    errs = []
    epss = [0.1, 0.05, 0.025]
    for eps in epss:
        _, _, E = _flow(orc, tgt, x, u, eps, int(round(Ttot / eps)), which)
        errs.append(abs(E))
    slopes = np.diff(np.log(errs)) / np.diff(np.log(epss))
    assert np.all(np.abs(slopes - order) < 0.35), slopes


@pytest.mark.parametrize("d,h,gscale,cmix", [(3, 0.05, 1500.0, 0.3), (10, 2.0, 400.0, -0.6), (4, 0.9, 3000.0, 0.9),
                                             (50, 0.4, 2600.0, 0.0), (5, 0.012, 7000.0, -0.2)])
def test_B_large_delta_against_multiprecision(orc, d, h, gscale, cmix):
    """|delta| from about 20 to beyond cosh overflow: the oracle matches the
    paper's closed form evaluated in 60-digit arithmetic."""
    import mpmath as mp
    mp.mp.dps = 60
    rng = np.random.default_rng(d)
    g = gscale * _unit(rng.normal(size=d))
    w = rng.normal(size=d)
    w -= g * (w @ g) / (g @ g)
    u = cmix * g / np.linalg.norm(g) + np.sqrt(1 - cmix**2) * _unit(w)
    u1, dk = orc.map_B(u, g, h)
    n = mp.sqrt(mp.fsum(mp.mpf(v) ** 2 for v in g))
    delta = mp.mpf(h) * n / (d - 1)
    assert float(delta) > 19.0
    c = mp.fsum(mp.mpf(a) * mp.mpf(b) for a, b in zip(g, u)) / n
    den = mp.cosh(delta) + c * mp.sinh(delta)
    coef = mp.sinh(delta) + c * (mp.cosh(delta) - 1)
    ref = [float((mp.mpf(u[i]) + coef * mp.mpf(g[i]) / n) / den) for i in range(d)]
    np.testing.assert_allclose(u1, ref, rtol=0, atol=1e-12)
    kref = float((d - 1) * mp.log(den))
    assert abs(dk - kref) < 1e-12 * abs(kref)


def test_B_branch_continuity(orc):
    # the direct form below |delta| = 20 and the cosh-divided form above agree across the switch
    d = 6
    g = np.array([3.0, -1.0, 2.0, 0.5, 0.0, 1.0]) * 20.0
    u = _unit(np.array([0.2, 1.0, -0.3, 0.0, 0.4, 0.1]))
    n = np.linalg.norm(g)
    h0 = 20.0 * (d - 1) / n
    ua, ka = orc.map_B(u, g, h0 * (1 - 1e-12))
    ub, kb = orc.map_B(u, g, h0 * (1 + 1e-12))
    np.testing.assert_allclose(ua, ub, atol=1e-10)
    assert abs(ka - kb) < 1e-9 * abs(ka)
