"""Pins of the oracle's ensemble statistics and controllers.

Equipartition and D~_diag are checked on exact Gaussian draws against their
closed forms for zero-mean Gaussians (appendix "Equipartition condition");
F against its closed form and inverse; the eps rule through its fixed point and
its scaling law; the moving-window switch and the bisection through
hand-derived worked examples.
"""
import math

import numpy as np
import pytest

from paper_2601_16696_amd import workloads


def test_F_closed_form_and_inverse(orc):
    assert orc.F(0.0) == 0.0
    assert abs(orc.F(1.0) - 1.0) < 1e-15           # 4 * 1 / (1 + 1)^2
    assert abs(orc.F(0.25) - 4 * 0.125 / 2.25) < 1e-15
    xs = np.logspace(-8, 4, 200)
    fs = np.array([orc.F(x) for x in xs])
    assert np.all(np.diff(fs) > 0)                  # monotonically increasing
    for D in (1e-6, 0.01, 0.3, 5.0):
        y = orc.F(D)
        lo, hi = 0.0, 1e6
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            lo, hi = (mid, hi) if orc.F(mid) < y else (lo, mid)
        assert abs(lo - D) < 1e-9 * max(1, D)
    # small-D asymptote 4 D^{3/2}
    assert abs(orc.F(1e-10) / (4e-15) - 1) < 1e-4


def test_compensated_sum_matches_fsum(orc):
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.normal(size=1000) * 10.0 ** rng.integers(-10, 16, size=1000), [1e16, 1.0, -1e16]])
    assert orc.fsum(v) == math.fsum(v)
    assert orc.fsum([1e16, 1.0, -1e16]) == 1.0


def _ensemble_on_draws(orc, s2_target, s2_draw, M, seed=0, **cfg):
    d = s2_target.size
    tgt = orc.Target(orc.GAUSS_DIAG, d, a=s2_target)
    x = np.random.default_rng(seed).normal(size=(M, d)) * np.sqrt(s2_draw)
    e = orc.Ensemble(tgt, M, 1, **cfg)
    e.init(x)
    return e, x


def test_equipartition_on_exact_gaussian_draws(orc):
    """V_ii -> Sigma'_ii / Sigma_ii and D~_diag -> (1/d) sum (1 - Sigma'/Sigma)^2."""
    M = 40000
    s2 = np.array([0.5, 1.0, 2.0, 4.0, 0.1])
    s2p = s2 * np.array([1.0, 2.0, 0.5, 1.3, 3.0])
    e, x = _ensemble_on_draws(orc, s2, s2p, M)
    e.unadj_control()
    V = e.array("Vii")
    np.testing.assert_allclose(V, s2p / s2, rtol=6 * np.sqrt(2.0 / M))
    D = e.stats()["dtilde"]
    Dref = np.mean((1 - s2p / s2) ** 2)
    assert abs(D - Dref) < 0.03 * Dref
    # moments reported alongside
    np.testing.assert_allclose(e.array("var"), s2p, rtol=6 * np.sqrt(2.0 / M))
    np.testing.assert_allclose(e.array("m2"), s2p, rtol=6 * np.sqrt(2.0 / M))


def test_equipartition_is_identity_at_stationarity(orc):
    M = 40000
    s2 = np.array([0.01, 1.0, 100.0])
    e, _ = _ensemble_on_draws(orc, s2, s2, M, seed=3)
    e.unadj_control()
    np.testing.assert_allclose(e.array("Vii"), 1.0, atol=6 * np.sqrt(2.0 / M))
    assert e.stats()["dtilde"] < 3 * 2.0 / M * 3


def test_L_rule_on_exact_draws(orc):
    M = 40000
    s2 = np.array([0.3, 2.0, 7.0, 1.0])
    e, _ = _ensemble_on_draws(orc, s2, s2, M, seed=5)
    L = e.stats()["L"]
    assert abs(L / (2.0 * np.sqrt(s2.sum())) - 1) < 0.02


def _set_delta_and_control(e, delta):
    e.set_array("delta", delta)
    e.unadj_control()
    return e.stats()


def test_eps_rule_fixed_point_and_scaling(orc):
    """eps is unchanged when the measured EEVPD equals F(C D~); scaling every
    Delta by s multiplies the next eps by s^{-1/3} (EEVPD ~ s^2, 1/6 power)."""
    M, d = 64, 4
    s2 = np.ones(d)
    rng = np.random.default_rng(8)
    x = rng.normal(size=(M, d)) * 1.7
    base = rng.normal(size=M)
    for mode in (0, 1):
        e = orc.Ensemble(orc.Target(orc.GAUSS_DIAG, d, a=s2), M, 1, eevpd_mode=mode)
        e.init(x)
        e.set_hyper(0.3, 1.0)
        s = _set_delta_and_control(e, base)
        W = s["eevpd_target"]
        E = s["eevpd"]
        # rescale Delta so that the measured EEVPD hits the target exactly
        e2 = orc.Ensemble(orc.Target(orc.GAUSS_DIAG, d, a=s2), M, 1, eevpd_mode=mode)
        e2.init(x)
        e2.set_hyper(0.3, 1.0)
        s2_ = _set_delta_and_control(e2, base * np.sqrt(W / E))
        assert abs(s2_["eps"] / 0.3 - 1) < 1e-12
        for sc in (0.1, 3.0):
            e3 = orc.Ensemble(orc.Target(orc.GAUSS_DIAG, d, a=s2), M, 1, eevpd_mode=mode)
            e3.init(x)
            e3.set_hyper(0.3, 1.0)
            s3 = _set_delta_and_control(e3, base * np.sqrt(W / E) * sc)
            assert abs(s3["eps"] / 0.3 - sc ** (-1.0 / 3.0)) < 1e-12


def test_eevpd_modes_differ_by_the_mean(orc):
    # mean square = variance + mean^2: a common offset only shows in mode 1
    M, d = 32, 3
    e0 = orc.Ensemble(orc.Target(orc.GAUSS_DIAG, d, a=np.ones(d)), M, 1, eevpd_mode=0)
    e1 = orc.Ensemble(orc.Target(orc.GAUSS_DIAG, d, a=np.ones(d)), M, 1, eevpd_mode=1)
    x = np.random.default_rng(1).normal(size=(M, d))
    delta = np.full(M, 0.25)
    delta[::2] += 0.5
    for e in (e0, e1):
        e.init(x)
        _set_delta_and_control(e, delta)
    # mean 0.5, variance 0.0625: both are exact binary fractions
    assert e0.stats()["eevpd"] == 0.0625 / d
    assert e1.stats()["eevpd"] == (0.0625 + 0.25) / d


def test_eps_kept_when_eevpd_is_zero(orc):
    M, d = 16, 2
    e = orc.Ensemble(orc.Target(orc.GAUSS_DIAG, d, a=np.ones(d)), M, 1, eevpd_mode=0)
    e.init(np.random.default_rng(2).normal(size=(M, d)))
    e.set_hyper(0.7, 1.0)
    s = _set_delta_and_control(e, np.full(M, 3.0))  # zero variance
    assert s["eps"] == 0.7 and (s["status_bits"] & 2)


def _window_ensemble(orc, max_total=25):
    """Two chains at +-sqrt(v) make E[x_i^2] = v exactly; window length
    round(0.2 * 25) = 5."""
    d = 2
    e = orc.Ensemble(orc.Target(orc.GAUSS_DIAG, d, a=np.ones(d)), 2, 1, max_steps_total=max_total,
                     max_steps_unadj=10**6, switch_policy=0)
    e.init(np.zeros((2, d)) + 1.0)
    return e


def _push(e, v0, v1):
    x = np.array([[np.sqrt(v0), np.sqrt(v1)], [-np.sqrt(v0), -np.sqrt(v1)]])
    e.set_array("x", x)
    e.set_array("g", np.zeros((2, 2)))
    e.set_array("delta", np.array([0.1, -0.1]))
    e.unadj_control()
    return e.stats()


def test_window_worked_example(orc):
    """Hand-derived: window [1,2,3,4,5] has mean 3 and sample variance 2.5, so
    delta = sqrt(2.5)/3; then [2,3,4,5,5] -> sqrt(1.7)/3.8, [3,4,5,5,5] ->
    sqrt(0.8)/4.4, [4,5,5,5,5] -> sqrt(0.2)/4.8, [5,5,5,5,5] -> 0 and the
    switch fires on that step."""
    e = _window_ensemble(orc)
    seq = [1, 2, 3, 4, 5, 5, 5, 5, 5]
    expect = [None, None, None, None, math.sqrt(2.5) / 3, math.sqrt(1.7) / 3.8, math.sqrt(0.8) / 4.4,
              math.sqrt(0.2) / 4.8, 0.0]
    for k, v in enumerate(seq):
        s = _push(e, float(v), 4.0)
        if expect[k] is None:
            assert s["ring_full"] == 0 and s["switch_ready"] == 0 and s["phase"] == 0
        else:
            assert abs(s["max_delta"] - expect[k]) < 1e-14
            wd = e.array("wdelta")
            assert wd[1] == 0.0
            if k < len(seq) - 1:
                assert s["phase"] == 0
    assert s["switch_ready"] == 1 and s["phase"] == 1 and s["t"] == 9


def test_window_constant_sequence_switches_when_full(orc):
    e = _window_ensemble(orc)
    for k in range(5):
        s = _push(e, 2.0, 3.0)
    assert s["max_delta"] == 0.0 and s["phase"] == 1 and s["t"] == 5


def test_fixed_switch_policy(orc):
    d = 3
    e = orc.Ensemble(orc.Target(orc.GAUSS_DIAG, d, a=np.ones(d)), 8, 1, max_steps_unadj=7, max_steps_total=20,
                     switch_policy=1)
    e.init(np.random.default_rng(0).normal(size=(8, d)))
    e.step_unadjusted(100)
    s = e.stats()
    assert s["t"] == 7 and s["phase"] == 1


def _bisect_trace(orc, a_of_eps, eps0, a_star, tol, n):
    d = 4
    e = orc.Ensemble(orc.Target(orc.GAUSS_DIAG, d, a=np.ones(d)), 8, 1, acc_target=a_star, acc_tol=tol,
                     max_steps_total=10**6)
    e.init(np.random.default_rng(0).normal(size=(8, d)))
    e.do_switch()
    e.set_hyper(eps0, 1.0)
    out = []
    for _ in range(n):
        eps = e.stats()["eps"]
        e.set_array("acc", np.full(8, a_of_eps(eps)))
        e.adj_control()
        out.append(e.stats()["eps"])
    return out, e.stats()


def test_bisection_worked_example_short(orc):
    """a(eps) = exp(-eps), target 0.7, tol 0.03, start 1: a = 0.368 -> halve to
    0.5; a = 0.607 -> halve to 0.25; a = 0.779 -> bracket (0.25, 0.5) -> 0.375;
    a = 0.687 within tolerance -> frozen."""
    tr, s = _bisect_trace(orc, lambda e: math.exp(-e), 1.0, 0.7, 0.03, 6)
    assert tr == [0.5, 0.25, 0.375, 0.375, 0.375, 0.375]
    assert s["adapt"] == 0


def test_bisection_worked_example_long(orc):
    """a(eps) = exp(-3 eps), target 0.9, tol 0.01, start 1: halvings to
    0.03125 (a = 0.9105), then midpoints 0.046875, 0.0390625, 0.03515625
    (a = 0.89990, within tolerance)."""
    tr, s = _bisect_trace(orc, lambda e: math.exp(-3 * e), 1.0, 0.9, 0.01, 10)
    assert tr == [0.5, 0.25, 0.125, 0.0625, 0.03125, 0.046875, 0.0390625, 0.03515625, 0.03515625, 0.03515625]
    assert s["have_lo"] == 1 and s["have_hi"] == 1 and s["adapt"] == 0


def test_bisection_doubling_from_small_eps(orc):
    tr, _ = _bisect_trace(orc, lambda e: math.exp(-e), 0.01, 0.7, 0.03, 7)
    # doubling 0.01 -> 0.32, where a = exp(-0.32) = 0.726 is within 0.03 of 0.7 and eps freezes
    assert tr[:5] == [0.02, 0.04, 0.08, 0.16, 0.32]
    assert tr[5] == 0.32 and tr[6] == 0.32


def test_switch_sets_preconditioner_and_integrator(orc):
    for d, integ, astar in ((100, 1, 0.7), (201, 2, 0.9), (200, 1, 0.7)):
        M = 64
        s2 = np.linspace(0.5, 3.0, d)
        e, x = _ensemble_on_draws(orc, s2, s2, M, seed=d)
        e.unadj_control()
        e.do_switch()
        s = e.stats()
        assert s["integrator"] == integ and s["a_star"] == astar and s["phase"] == 2 and s["adapt"] == 1
        np.testing.assert_allclose(e.array("sigma") ** 2, x.var(axis=0), rtol=1e-12)


def test_fixed_step_size_holds_eps_and_changes_nothing_else(orc):
    """eps_fixed (the fixed-step comparison of the step-size appendix): eps
    stays at the given value through the unadjusted phase, and the run is the
    adaptive run with eps reset to that value before every move (L, the
    diagnostics and the window follow the ensemble exactly as before)."""
    d, M, E = 12, 16, 0.37
    s2 = 10.0 ** np.linspace(-1.0, 1.0, d)
    x0 = np.random.default_rng(5).normal(0.0, 3.0, size=(M, d))
    fixed = orc.Ensemble(orc.Target(orc.GAUSS_DIAG, d, a=s2), M, 9, eps_fixed=E)
    adapt = orc.Ensemble(orc.Target(orc.GAUSS_DIAG, d, a=s2), M, 9)
    fixed.init(x0)
    adapt.init(x0)
    assert fixed.stats()["eps"] == E
    for _ in range(25):
        adapt.set_hyper(E, adapt.stats()["L"])
        adapt.unadj_move()
        adapt.unadj_control()
        fixed.unadj_move()
        fixed.unadj_control()
        sf, sa = fixed.stats(), adapt.stats()
        assert sf["eps"] == E and sa["eps"] != E
        assert sf["L"] == sa["L"] and sf["eevpd"] == sa["eevpd"] and sf["dtilde"] == sa["dtilde"]
        assert sf["status_bits"] & 2 == 0
    assert np.array_equal(fixed.array("x"), adapt.array("x"))
    assert np.array_equal(fixed.array("u"), adapt.array("u"))


def test_fixed_step_size_at_eps0_matches_the_first_adaptive_step(orc):
    """With eps_fixed = 0.01 sqrt(d) (the adaptive run's eps_0) the first step
    of both runs is identical; the adaptive eps then moves off eps_0."""
    d, M = 9, 12
    x0 = np.random.default_rng(6).normal(0.0, 5.0, size=(M, d))
    e0 = 0.01 * math.sqrt(d)
    a = orc.Ensemble(orc.Target(orc.GAUSS_DIAG, d, a=np.ones(d)), M, 4)
    f = orc.Ensemble(orc.Target(orc.GAUSS_DIAG, d, a=np.ones(d)), M, 4, eps_fixed=e0)
    a.init(x0)
    f.init(x0)
    a.step_unadjusted(1)
    f.step_unadjusted(1)
    assert np.array_equal(a.array("x"), f.array("x")) and np.array_equal(a.array("delta"), f.array("delta"))
    assert a.stats()["eps"] != e0 and f.stats()["eps"] == e0


def test_fixed_step_size_rejects_negative(orc):
    with pytest.raises(ValueError):
        orc.Ensemble(orc.Target(orc.GAUSS_DIAG, 3, a=np.ones(3)), 4, 1, eps_fixed=-1.0)


@pytest.mark.parametrize("f", [2.0, 0.5])
def test_unadjusted_trajectory_is_scale_equivariant(orc, f):
    """The unadjusted controller's whole trajectory under a change of units.
    Scaling a diagonal Gaussian's standard deviations, the start and the
    initial step size by f leaves every quantity the controller reads
    unchanged: the energy errors (eq. (discrete update): eps |g| and h / L
    are unit-free), D~ (V_ii = -E[(x_i - xbar_i) d_i log p]), EEVPD and the
    moving window's relative fluctuations of E[x_i^2] (section "Switch to
    adjustment"); it scales eps and L = alpha (sum Var)^{1/2} by f and
    sum Var by f^2.  With f a power of two every FP64 operation scales
    exactly, so the eps(t), L(t) schedule, the window switch's step and the
    final positions must be the unscaled run's times f bit for bit.  A slip
    in the units of a controller formula (L without its square root, a drift
    not multiplied by eps, a window spread not divided by its mean) breaks
    this; a wrong exponent inside a unit-free ratio does not, and is pinned
    by the single-update tests above."""
    d, N = 20, 512
    rng = np.random.default_rng(7)
    s2 = 10.0 ** rng.uniform(-1, 1, size=d)
    x0 = rng.normal(size=(N, d)) * 3.0
    cfg = dict(switch_policy=0, switch_tol=0.1, max_steps_unadj=600, max_steps_total=720)
    runs = []
    for sc in (1.0, f):
        e = orc.Ensemble(orc.Target(orc.GAUSS_DIAG, d, a=s2 * sc * sc), N, 11, eps0_factor=0.01 * sc, **cfg)
        e.init(x0 * sc)
        hist = [e.stats()]
        while hist[-1]["phase"] == 0:
            e.step_unadjusted(1)
            hist.append(e.stats())
        runs.append((hist, e.array("x"), e.array("delta")))
    (h1, x1, D1), (hf, xf, Df) = runs
    assert len(h1) == len(hf)
    last = h1[-1]
    # the switch came from the window criterion, not from the step limit
    assert last["switch_ready"] == 1 and 20 < last["t"] < cfg["max_steps_unadj"], last
    same = ("t", "phase", "switch_ready", "status_bits", "n_nonfinite", "ring_full", "dtilde", "eevpd",
            "eevpd_target", "max_delta")
    for a, b in zip(h1, hf):
        for key in same:
            assert a[key] == b[key] or (a[key] != a[key] and b[key] != b[key]), (a["t"], key, a[key], b[key])
        assert b["eps"] == f * a["eps"] and b["L"] == f * a["L"], (a["t"], a["eps"], b["eps"], a["L"], b["L"])
        assert b["sum_var"] == f * f * a["sum_var"], (a["t"], a["sum_var"], b["sum_var"])
    np.testing.assert_array_equal(xf, f * x1)
    np.testing.assert_array_equal(Df, D1)
